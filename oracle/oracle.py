"""Python face of the CPU oracle (test infrastructure only).

Only the test suite, the smoke entry and the benchmark's CPU-baseline leg use
this module; the GPU library never imports it. It loads liboracle.so, built by
g++ from qsv_oracle.cpp (complex128 throughout), and strings its per-gate
update (section 4.3.2, Eq. update_mat) into circuits, observables and
gradients:

  run_circuit        apply a gate list in order to |0...0> (section 4.4)
  expectation        <psi|O|psi> for O a real combination of Pauli strings (4.5)
  apply_observable   O|psi>
  param_shift_grad   exact derivative of <O> for every parameter: each
                     parametric gate is exp(+i t P / 2) with P^2 = I, so
                     dE/dt = [E(t + pi/2) - E(t - pi/2)] / 2
  fd_grad            central finite differences (cross-check of the above)
  marginal_probability  probability of a Z-basis outcome on a subset of the
                     qubits, the others left unmeasured (section 4.2.2)
  sample             Z-basis samples by inverse CDF over the cumulative
                     distribution of |psi_x|^2 (section 4.2.2)

Parity status: every function here is pinned by tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsv_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NAMED = {"i": 0, "x": 1, "y": 2, "z": 3, "h": 4, "rx": 5, "ry": 6, "rz": 7,
         "cnot": 8, "cz": 9, "swap": 10}


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP for the outer B0 loop only)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = ctypes.c_int
        L.orc_set_basis.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
        L.orc_apply_matrix.argtypes = [dp, ctypes.c_int, dp, ip, ctypes.c_int, ip, ip, ctypes.c_int]
        L.orc_apply_matrix.restype = ctypes.c_int
        L.orc_named_matrix.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_named_matrix.restype = ctypes.c_int
        L.orc_norm2.argtypes = [dp, ctypes.c_int]
        L.orc_norm2.restype = ctypes.c_double
        L.orc_inner.argtypes = [dp, dp, ctypes.c_int, dp, dp]
        L.orc_expectation.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, ip, ip, ip, dp, dp]
        L.orc_expectation.restype = ctypes.c_int
        L.orc_apply_observable.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ip, ip, ip]
        L.orc_apply_observable.restype = ctypes.c_int
        L.orc_pauli_rotation.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, ctypes.c_double]
        L.orc_pauli_rotation.restype = ctypes.c_int
        L.orc_transition.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ip, ip, ip, dp, dp]
        L.orc_transition.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def zero_state(n: int) -> np.ndarray:
    return basis_state(n, 0)


def basis_state(n: int, k: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_set_basis(_dp(psi), n, k)
    return psi


def named_matrix(name: str, theta: float = 0.0) -> np.ndarray:
    out = np.zeros(16, dtype=np.complex128)
    d = lib().orc_named_matrix(NAMED[name], float(theta), _dp(out))
    if d < 0:
        raise ValueError(name)
    return out[: d * d].reshape(d, d).copy()


def apply_matrix(psi: np.ndarray, mat, targets, controls=(), ctrl_vals=()) -> None:
    """In-place psi <- K psi (section 4.3.2, Eq. update_mat)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    n = int(psi.size).bit_length() - 1
    m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(list(controls) or [0], dtype=np.int32))
    v = np.ascontiguousarray(np.asarray(list(ctrl_vals) or [0], dtype=np.int32))
    rc = lib().orc_apply_matrix(_dp(psi), n, _dp(m), _ip(t), len(targets), _ip(c), _ip(v),
                                len(controls))
    if rc != 0:
        raise ValueError("oracle rejected gate")


def gate_matrix_and_qubits(g, theta=None):
    """(matrix, targets, controls, ctrl_vals) of a gate record."""
    op = g["op"]
    q = list(g["q"])
    if op in ("rx", "ry", "rz"):
        ang = theta[g["slot"]] if "slot" in g else g["angle"]
        return named_matrix(op, ang), q, [], []
    if op in ("h", "x", "y", "z"):
        return named_matrix(op), q, [], []
    if op == "cnot":
        # record lists [control, target]; the oracle matrix has bit 0 = target
        return named_matrix("cnot"), [q[1], q[0]], [], []
    if op in ("cz", "swap"):
        return named_matrix(op), q, [], []
    if op == "dense":
        return np.asarray(g["mat"], dtype=np.complex128), q, list(g.get("controls", [])), \
            list(g.get("ctrl_vals", []))
    raise ValueError(op)


def pauli_rotation(psi: np.ndarray, qubits, paulis, theta: float) -> None:
    """psi <- exp(+i theta P / 2) psi for the Pauli string P (ids 1..3 on qubits)."""
    n = int(psi.size).bit_length() - 1
    q = np.asarray(qubits, dtype=np.int32)
    p = np.asarray(paulis, dtype=np.int32)
    if lib().orc_pauli_rotation(_dp(psi), n, len(q), _ip(q), _ip(p), float(theta)) != 0:
        raise ValueError("oracle rejected Pauli rotation")


def apply_gate(psi, g, theta=None):
    if g["op"] == "pauli_rot":
        ang = theta[g["slot"]] if "slot" in g else g["angle"]
        pauli_rotation(psi, g["q"], g["paulis"], ang)
        return
    m, t, c, v = gate_matrix_and_qubits(g, theta)
    apply_matrix(psi, m, t, c, v)


def run_circuit(n: int, gates, theta=None, psi=None) -> np.ndarray:
    """Apply the gates in order (section 4.4) to psi (default |0...0>)."""
    if psi is None:
        psi = zero_state(n)
    for g in gates:
        apply_gate(psi, g, theta)
    return psi


def _encode_obs(obs):
    coefs = np.asarray([t[0] for t in obs], dtype=np.float64)
    lens = np.asarray([len(t[1]) for t in obs], dtype=np.int32)
    qs = np.asarray([qp[0] for t in obs for qp in t[1]] or [0], dtype=np.int32)
    ps = np.asarray([qp[1] for t in obs for qp in t[1]] or [0], dtype=np.int32)
    return coefs, lens, qs, ps


def expectation_complex(psi: np.ndarray, obs) -> complex:
    n = int(psi.size).bit_length() - 1
    coefs, lens, qs, ps = _encode_obs(obs)
    re = ctypes.c_double()
    im = ctypes.c_double()
    rc = lib().orc_expectation(_dp(psi), n, len(obs), _dp(coefs), _ip(lens), _ip(qs), _ip(ps),
                               ctypes.byref(re), ctypes.byref(im))
    if rc != 0:
        raise ValueError("oracle rejected observable")
    return complex(re.value, im.value)


def expectation(psi: np.ndarray, obs) -> float:
    return expectation_complex(psi, obs).real


def transition_amplitude(a: np.ndarray, b: np.ndarray, obs) -> complex:
    """<a|O|b> (complex)."""
    n = int(a.size).bit_length() - 1
    coefs, lens, qs, ps = _encode_obs(obs)
    re = ctypes.c_double()
    im = ctypes.c_double()
    rc = lib().orc_transition(_dp(a), _dp(b), n, len(obs), _dp(coefs), _ip(lens), _ip(qs), _ip(ps),
                              ctypes.byref(re), ctypes.byref(im))
    if rc != 0:
        raise ValueError("oracle rejected observable")
    return complex(re.value, im.value)


def apply_observable(psi: np.ndarray, obs) -> np.ndarray:
    n = int(psi.size).bit_length() - 1
    coefs, lens, qs, ps = _encode_obs(obs)
    out = np.empty_like(psi)
    rc = lib().orc_apply_observable(_dp(psi), _dp(out), n, len(obs), _dp(coefs), _ip(lens),
                                    _ip(qs), _ip(ps))
    if rc != 0:
        raise ValueError("oracle rejected observable")
    return out


def norm2(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return lib().orc_norm2(_dp(psi), n)


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = int(a.size).bit_length() - 1
    re = ctypes.c_double()
    im = ctypes.c_double()
    lib().orc_inner(_dp(a), _dp(b), n, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def energy(n, gates, theta, obs) -> float:
    return expectation(run_circuit(n, gates, theta), obs)


def param_shift_grad(n, gates, theta, obs, slots=None) -> np.ndarray:
    """Exact gradient by the two-term shift rule. Valid because each slot
    drives exactly one gate exp(+i t P/2) with P^2 = I."""
    theta = np.asarray(theta, dtype=np.float64)
    slots = list(range(theta.size)) if slots is None else list(slots)
    g = np.zeros(len(slots))
    for i, s in enumerate(slots):
        tp = theta.copy()
        tp[s] += np.pi / 2
        tm = theta.copy()
        tm[s] -= np.pi / 2
        g[i] = 0.5 * (energy(n, gates, tp, obs) - energy(n, gates, tm, obs))
    return g


def fd_grad(n, gates, theta, obs, h=1e-5, slots=None) -> np.ndarray:
    theta = np.asarray(theta, dtype=np.float64)
    slots = list(range(theta.size)) if slots is None else list(slots)
    g = np.zeros(len(slots))
    for i, s in enumerate(slots):
        tp = theta.copy()
        tp[s] += h
        tm = theta.copy()
        tm[s] -= h
        g[i] = (energy(n, gates, tp, obs) - energy(n, gates, tm, obs)) / (2 * h)
    return g


def marginal_probability(psi: np.ndarray, values) -> float:
    """Sum of |psi_x|^2 over the basis indices x whose bit q equals values[q]
    for every qubit q with values[q] in {0, 1}; values[q] == 2 leaves qubit q
    unmeasured (section 4.2.2, the marginal-probability utility: one list
    entry per qubit, entry q for qubit q, 2 a wild card). Plain definition,
    FP64, no normalisation."""
    n = int(psi.size).bit_length() - 1
    if len(values) != n:
        raise ValueError("one value per qubit")
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    x = np.arange(psi.size, dtype=np.uint64)
    keep = np.ones(psi.size, dtype=bool)
    for q, v in enumerate(values):
        if v == 2:
            continue
        if v not in (0, 1):
            raise ValueError("values must be 0, 1 or 2")
        keep &= ((x >> np.uint64(q)) & np.uint64(1)) == np.uint64(v)
    return float(p[keep].sum())


def sample(psi: np.ndarray, u) -> np.ndarray:
    """Z-basis samples (section 4.2.2: sampling goes through the cumulative
    distribution of the outcome probabilities). For each uniform u_i in
    [0, 1) the sample is the smallest index x with C(x) > u_i * C(N - 1),
    C(x) = sum_{y <= x} |psi_y|^2 accumulated in order in FP64; the uniforms
    are inputs, drawn by the caller."""
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    c = np.cumsum(p)
    u = np.asarray(u, dtype=np.float64)
    if np.any(~(u >= 0.0)) or np.any(~(u < 1.0)):
        raise ValueError("uniforms must lie in [0, 1)")
    if c[-1] <= 0.0:
        raise ValueError("zero-norm state")
    return np.searchsorted(c, u * c[-1], side="right").astype(np.int64)

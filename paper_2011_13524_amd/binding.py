"""Thin ctypes binding of libqsv (include/qsv.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libqsv.so. Missing library -> ImportError at first use; there is no
fallback path.

The functions keep the C names (qsv_state_alloc, qsv_apply_gate, ...). A few
small classes (State, Circuit, Observable, Plan) own the handles and convert
numpy arrays / gate records into the C arguments.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

QSV_C64 = 1
QSV_C128 = 2
QSV_PLAN_HEAVY = 1
GATE = {"x": 1, "y": 2, "z": 3, "h": 4, "rx": 5, "ry": 6, "rz": 7, "cnot": 8, "cz": 9, "swap": 10}
PAULI_ID = {"rx": 1, "ry": 2, "rz": 3}

_c = ctypes
_vp = _c.c_void_p
_ip = _c.POINTER(_c.c_int)
_dp = _c.POINTER(_c.c_double)

# name -> (restype, argtypes)
_SIGS = {
    "qsv_last_error": (_c.c_char_p, []),
    "qsv_version": (_c.c_int, []),
    "qsv_state_alloc": (_c.c_int, [_c.c_int, _c.c_int, _vp, _c.POINTER(_vp)]),
    "qsv_state_wrap": (_c.c_int, [_vp, _c.c_int, _c.c_int, _vp, _c.POINTER(_vp)]),
    "qsv_state_free": (_c.c_int, [_vp]),
    "qsv_state_info": (_c.c_int, [_vp, _ip, _ip, _c.POINTER(_vp)]),
    "qsv_state_sync": (_c.c_int, [_vp]),
    "qsv_set_basis": (_c.c_int, [_vp, _c.c_uint64]),
    "qsv_load": (_c.c_int, [_vp, _dp]),
    "qsv_store": (_c.c_int, [_vp, _dp]),
    "qsv_copy": (_c.c_int, [_vp, _vp]),
    "qsv_apply_gate": (_c.c_int, [_vp, _dp, _ip, _c.c_int, _ip, _ip, _c.c_int]),
    "qsv_apply_named": (_c.c_int, [_vp, _c.c_int, _ip, _c.c_int, _c.c_double]),
    "qsv_norm2": (_c.c_int, [_vp, _dp]),
    "qsv_inner": (_c.c_int, [_vp, _vp, _dp, _dp]),
    "qsv_observable_create": (_c.c_int, [_c.c_int, _c.POINTER(_vp)]),
    "qsv_observable_free": (_c.c_int, [_vp]),
    "qsv_observable_add_term": (_c.c_int, [_vp, _c.c_double, _ip, _ip, _c.c_int]),
    "qsv_observable_info": (_c.c_int, [_vp, _ip, _ip, _ip]),
    "qsv_observable_passes": (_c.c_int, [_vp, _c.c_int, _ip]),
    "qsv_expectation": (_c.c_int, [_vp, _vp, _dp]),
    "qsv_expectation_noalloc": (_c.c_int, [_vp, _vp, _dp]),
    "qsv_circuit_create": (_c.c_int, [_c.c_int, _c.POINTER(_vp)]),
    "qsv_circuit_free": (_c.c_int, [_vp]),
    "qsv_circuit_add_gate": (_c.c_int, [_vp, _dp, _ip, _c.c_int, _ip, _ip, _c.c_int]),
    "qsv_circuit_add_named": (_c.c_int, [_vp, _c.c_int, _ip, _c.c_int, _c.c_double]),
    "qsv_circuit_add_rotation": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int]),
    "qsv_circuit_add_pauli_rotation": (_c.c_int, [_vp, _ip, _ip, _c.c_int, _c.c_int, _c.c_double]),
    "qsv_apply_pauli_rotation": (_c.c_int, [_vp, _ip, _ip, _c.c_int, _c.c_double]),
    "qsv_transition_amplitude": (_c.c_int, [_vp, _vp, _vp, _dp, _dp]),
    "qsv_marginal_probability": (_c.c_int, [_vp, _ip, _dp]),
    "qsv_sample": (_c.c_int, [_vp, _dp, _c.c_int64, _c.POINTER(_c.c_int64)]),
    "qsv_circuit_info": (_c.c_int, [_vp, _ip, _ip, _ip]),
    "qsv_apply_circuit": (_c.c_int, [_vp, _vp, _dp]),
    "qsv_plan_fused": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.POINTER(_vp)]),
    "qsv_circuit_commute": (_c.c_int, [_vp, _c.c_int, _c.c_int, _ip]),
    "qsv_plan_fused_ex": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int,
                                     _c.POINTER(_vp)]),
    "qsv_plan_autotune": (_c.c_int, [_vp, _vp, _dp, _c.c_int, _c.POINTER(_vp), _ip]),
    "qsv_plan_info": (_c.c_int, [_vp, _ip, _ip, _ip]),
    "qsv_plan_free": (_c.c_int, [_vp]),
    "qsv_plan_stats": (_c.c_int, [_vp, _ip, _ip, _ip]),
    "qsv_apply_fused": (_c.c_int, [_vp, _vp, _dp]),
    "qsv_apply_observable": (_c.c_int, [_vp, _vp, _vp]),
    "qsv_adjoint_gradient": (_c.c_int, [_vp, _vp, _dp, _vp, _vp, _vp, _dp, _dp]),
    "qsv_batch_create": (_c.c_int, [_c.POINTER(_vp)]),
    "qsv_batch_free": (_c.c_int, [_vp]),
    "qsv_batch_add": (_c.c_int, [_vp, _vp, _vp, _dp]),
    "qsv_batch_set_theta": (_c.c_int, [_vp, _c.c_int, _dp]),
    "qsv_batch_info": (_c.c_int, [_vp, _ip, _ip]),
    "qsv_batch_run": (_c.c_int, [_vp, _c.c_int, _vp, _dp, _dp]),
    "qsv_batch_set_graph": (_c.c_int, [_vp, _c.c_int]),
    "qsv_batch_autotune": (_c.c_int, [_vp, _c.c_int, _vp, _c.c_int, _ip]),
    "qsv_prof_enable": (_c.c_int, [_c.c_int]),
    "qsv_prof_read": (_c.c_int, [_c.c_char_p, _ip, _dp, _dp]),
}

_lib = None


class QsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqsv error {code}: {msg}")
        self.code = code


def lib():
    """Load libqsv.so (built in-tree by paper_2011_13524_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2011_13524_amd.build`")
        # One HIP runtime per process: torch ships its own copy of the HIP
        # runtime, and a second copy loaded beside it finds no device. With
        # torch imported first, the library's libamdhip64.so.7 dependency
        # resolves to the copy torch loaded, so the library and torch share
        # one runtime (and can share streams and memory).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGS)


def check(rc: int) -> None:
    if rc != 0:
        raise QsvError(rc, lib().qsv_last_error().decode())


def _ints(xs):
    a = np.ascontiguousarray(np.asarray(list(xs) if xs is not None else [], dtype=np.int32))
    if a.size == 0:
        a = np.zeros(1, dtype=np.int32)
    return a


def _iptr(a):
    return a.ctypes.data_as(_ip)


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class State:
    """A device state vector (qsv_state)."""

    def __init__(self, n: int, dtype: str = "c128", stream=None, _handle=None, _keep=None):
        self.n = n
        self.dtype = dtype
        self._keep = _keep
        if _handle is not None:
            self.h = _handle
            return
        h = _vp()
        check(lib().qsv_state_alloc(n, QSV_C64 if dtype == "c64" else QSV_C128,
                                    _stream_handle(stream), _c.byref(h)))
        self.h = h

    @classmethod
    def wrap(cls, tensor, stream=None):
        """Borrow a contiguous torch complex64/complex128 CUDA tensor of 2^n elements."""
        import torch
        assert tensor.is_contiguous() and tensor.dim() == 1
        n = int(tensor.numel()).bit_length() - 1
        assert (1 << n) == tensor.numel()
        dt = {torch.complex64: "c64", torch.complex128: "c128"}[tensor.dtype]
        h = _vp()
        check(lib().qsv_state_wrap(_c.c_void_p(tensor.data_ptr()), n,
                                   QSV_C64 if dt == "c64" else QSV_C128,
                                   _stream_handle(stream), _c.byref(h)))
        return cls(n, dt, _handle=h, _keep=tensor)

    def free(self):
        if self.h is not None and lib is not None:
            check(lib().qsv_state_free(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib().qsv_state_free(self.h)
                self.h = None
        except Exception:
            pass

    def set_basis(self, k: int):
        check(lib().qsv_set_basis(self.h, k))

    def load(self, vec):
        v = np.ascontiguousarray(np.asarray(vec, dtype=np.complex128))
        assert v.size == (1 << self.n)
        check(lib().qsv_load(self.h, _dptr(v.view(np.float64))))

    def store(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex128)
        check(lib().qsv_store(self.h, _dptr(out.view(np.float64))))
        return out

    def copy_from(self, other: "State"):
        check(lib().qsv_copy(self.h, other.h))

    def apply_gate(self, mat, targets, controls=(), ctrl_vals=()):
        m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128))
        t, c, v = _ints(targets), _ints(controls), _ints(ctrl_vals)
        check(lib().qsv_apply_gate(self.h, _dptr(m.view(np.float64)), _iptr(t), len(targets),
                                   _iptr(c), _iptr(v), len(controls)))

    def apply_named(self, name: str, qubits, theta: float = 0.0):
        q = _ints(qubits)
        check(lib().qsv_apply_named(self.h, GATE[name], _iptr(q), len(qubits), float(theta)))

    def sync(self):
        """Wait for the work enqueued on the state's stream."""
        check(lib().qsv_state_sync(self.h))

    def norm2(self) -> float:
        out = _c.c_double()
        check(lib().qsv_norm2(self.h, _c.byref(out)))
        return out.value

    def marginal_probability(self, values) -> float:
        """Probability of the outcome `values` (one entry per qubit: 0, 1, or 2
        for unmeasured) (qsv_marginal_probability)."""
        if len(values) != self.n:
            raise ValueError("one value per qubit")
        v = (_c.c_int * len(values))(*[int(x) for x in values])
        out = _c.c_double()
        check(lib().qsv_marginal_probability(self.h, v, _c.byref(out)))
        return out.value

    def sample(self, u) -> np.ndarray:
        """Basis indices for the uniforms `u` in [0, 1) (qsv_sample)."""
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
        out = np.empty(u.size, dtype=np.int64)
        check(lib().qsv_sample(self.h, u.ctypes.data_as(_dp), int(u.size),
                               out.ctypes.data_as(_c.POINTER(_c.c_int64))))
        return out

    def inner(self, ket: "State") -> complex:
        re, im = _c.c_double(), _c.c_double()
        check(lib().qsv_inner(self.h, ket.h, _c.byref(re), _c.byref(im)))
        return complex(re.value, im.value)


class Observable:
    """Real combination of Pauli strings: terms = [(coef, [(qubit, pauli_id), ...]), ...]."""

    def __init__(self, n: int, terms=()):
        self.n = n
        h = _vp()
        check(lib().qsv_observable_create(n, _c.byref(h)))
        self.h = h
        for coef, qp in terms:
            self.add_term(coef, qp)

    def add_term(self, coef: float, qp):
        q = _ints([a for a, _ in qp])
        p = _ints([b for _, b in qp])
        check(lib().qsv_observable_add_term(self.h, float(coef), _iptr(q), _iptr(p), len(qp)))

    def info(self):
        n, t, g = _c.c_int(), _c.c_int(), _c.c_int()
        check(lib().qsv_observable_info(self.h, _c.byref(n), _c.byref(t), _c.byref(g)))
        return n.value, t.value, g.value

    def passes(self, dtype: str = "c64") -> int:
        """State passes an expectation of this observable takes (host-only)."""
        p = _c.c_int()
        check(lib().qsv_observable_passes(self.h, QSV_C64 if dtype == "c64" else QSV_C128, _c.byref(p)))
        return p.value

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib().qsv_observable_free(self.h)
                self.h = None
        except Exception:
            pass


def expectation(state: State, obs: Observable) -> float:
    out = _c.c_double()
    check(lib().qsv_expectation(state.h, obs.h, _c.byref(out)))
    return out.value


def expectation_noalloc(state: State, obs: Observable) -> float:
    """qsv_expectation_noalloc: the expectation with no device allocation."""
    out = _c.c_double()
    check(lib().qsv_expectation_noalloc(state.h, obs.h, _c.byref(out)))
    return out.value


class Circuit:
    """Host-side gate list (qsv_circuit). Build from gate records with
    Circuit.from_records(n, gates)."""

    def __init__(self, n: int):
        self.n = n
        h = _vp()
        check(lib().qsv_circuit_create(n, _c.byref(h)))
        self.h = h

    @classmethod
    def from_records(cls, n: int, gates):
        c = cls(n)
        for g in gates:
            c.add_record(g)
        return c

    def add_record(self, g):
        op = g["op"]
        if op in ("rx", "ry", "rz") and "slot" in g:
            check(lib().qsv_circuit_add_rotation(self.h, PAULI_ID[op], int(g["q"][0]), int(g["slot"])))
        elif op in GATE:
            q = _ints(g["q"])
            check(lib().qsv_circuit_add_named(self.h, GATE[op], _iptr(q), len(g["q"]),
                                              float(g.get("angle", 0.0))))
        elif op == "pauli_rot":
            q, p = _ints(g["q"]), _ints(g["paulis"])
            check(lib().qsv_circuit_add_pauli_rotation(self.h, _iptr(q), _iptr(p), len(g["q"]),
                                                       int(g.get("slot", -1)), float(g.get("angle", 0.0))))
        elif op == "dense":
            m = np.ascontiguousarray(np.asarray(g["mat"], dtype=np.complex128))
            t = _ints(g["q"])
            ctrl = list(g.get("controls", ()))
            vals = list(g.get("ctrl_vals", ()))
            c, v = _ints(ctrl), _ints(vals)
            check(lib().qsv_circuit_add_gate(self.h, _dptr(m.view(np.float64)), _iptr(t),
                                             len(g["q"]), _iptr(c), _iptr(v), len(ctrl)))
        else:
            raise ValueError(op)

    def commute(self, gate: int, qubit: int) -> int:
        """Paulis gate `gate` commutes with on `qubit` (bit 0 X, 1 Y, 2 Z)."""
        m = _c.c_int()
        check(lib().qsv_circuit_commute(self.h, gate, qubit, _c.byref(m)))
        return m.value

    def info(self):
        n, g, p = _c.c_int(), _c.c_int(), _c.c_int()
        check(lib().qsv_circuit_info(self.h, _c.byref(n), _c.byref(g), _c.byref(p)))
        return n.value, g.value, p.value

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib().qsv_circuit_free(self.h)
                self.h = None
        except Exception:
            pass


def _theta_ptr(theta):
    if theta is None:
        return None, None
    t = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    if t.size == 0:
        t = np.zeros(1)
    return t, _dptr(t)


def apply_circuit(state: State, circ: Circuit, theta=None):
    keep, tp = _theta_ptr(theta)
    check(lib().qsv_apply_circuit(state.h, circ.h, tp))


class Plan:
    """Fused execution plan (qsv_plan) of a circuit for one dtype."""

    def __init__(self, circ: Circuit, dtype: str = "c128", max_k: int = 2, tile_qubits: int = 0,
                 low_qubits: int = 0, heavy: bool = False):
        h = _vp()
        check(lib().qsv_plan_fused_ex(circ.h, QSV_C64 if dtype == "c64" else QSV_C128, max_k,
                                      tile_qubits, low_qubits, QSV_PLAN_HEAVY if heavy else 0,
                                      _c.byref(h)))
        self.h = h
        self.dtype = dtype

    @classmethod
    def autotune(cls, circ: Circuit, scratch: "State", theta=None, reps: int = 3) -> "Plan":
        """Fastest plan over fusion widths and tile shapes (qsv_plan_autotune);
        overwrites `scratch`. The choice is in `plan.choice`."""
        keep, tp = _theta_ptr(theta)
        h = _vp()
        ch = (_c.c_int * 4)()
        check(lib().qsv_plan_autotune(circ.h, scratch.h, tp, reps, _c.byref(h), ch))
        self = cls.__new__(cls)
        self.h = h
        self.dtype = scratch.dtype
        self.choice = {"max_k": ch[0], "tile_qubits": ch[1], "thread_bits": ch[2], "reg_bits": ch[3]}
        return self

    def info(self):
        p, b, g = _c.c_int(), _c.c_int(), _c.c_int()
        check(lib().qsv_plan_info(self.h, _c.byref(p), _c.byref(b), _c.byref(g)))
        s, lo, km = _c.c_int(), _c.c_int(), _c.c_int()
        check(lib().qsv_plan_stats(self.h, _c.byref(s), _c.byref(lo), _c.byref(km)))
        return {"passes": p.value, "blocks": b.value, "gates": g.value, "segments": s.value,
                "lds_ops": lo.value, "kmax": km.value}

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib().qsv_plan_free(self.h)
                self.h = None
        except Exception:
            pass


def apply_fused(state: State, plan: Plan, theta=None):
    keep, tp = _theta_ptr(theta)
    check(lib().qsv_apply_fused(state.h, plan.h, tp))


def apply_observable(src: State, obs: Observable, dst: State):
    check(lib().qsv_apply_observable(src.h, obs.h, dst.h))


def adjoint_gradient(circ: Circuit, theta, obs: Observable, psi: State, lam: State,
                     plan: "Plan | None" = None):
    """(energy, grad ndarray) through qsv_adjoint_gradient."""
    _, _, npar = circ.info()
    t = np.ascontiguousarray(np.asarray(theta if theta is not None else [], dtype=np.float64))
    if t.size == 0:
        t = np.zeros(1)
    grad = np.zeros(max(npar, 1))
    e = _c.c_double()
    check(lib().qsv_adjoint_gradient(circ.h, plan.h if plan is not None else None, _dptr(t),
                                     obs.h, psi.h, lam.h, _c.byref(e), _dptr(grad)))
    return e.value, grad[:npar]


class Batch:
    """Batched energies + adjoint gradients in one persistent launch (qsv_batch)."""

    def __init__(self):
        h = _vp()
        check(lib().qsv_batch_create(_c.byref(h)))
        self.h = h
        self._nparams = []

    def add(self, circ: Circuit, obs: Observable, theta=None):
        keep, tp = _theta_ptr(theta)
        check(lib().qsv_batch_add(self.h, circ.h, obs.h, tp))
        self._nparams.append(circ.info()[2])

    def set_theta(self, item: int, theta):
        keep, tp = _theta_ptr(theta)
        check(lib().qsv_batch_set_theta(self.h, item, tp))

    def autotune(self, dtype: str = "c64", stream=None, reps: int = 2) -> dict:
        """Pick the launch shape (LDS per workgroup, threads) by timing runs."""
        ch = (_c.c_int * 2)()
        check(lib().qsv_batch_autotune(self.h, QSV_C64 if dtype == "c64" else QSV_C128,
                                       _stream_handle(stream), reps, ch))
        return {"lds_kib": ch[0], "threads": ch[1]}

    def set_graph(self, enable: bool):
        """Replay the launch as a captured HIP graph (default) or launch plainly."""
        check(lib().qsv_batch_set_graph(self.h, 1 if enable else 0))

    def run(self, dtype: str = "c64", stream=None):
        """Returns (energies ndarray, list of per-item gradient ndarrays)."""
        items, tot = _c.c_int(), _c.c_int()
        check(lib().qsv_batch_info(self.h, _c.byref(items), _c.byref(tot)))
        e = np.zeros(max(items.value, 1))
        g = np.zeros(max(tot.value, 1))
        check(lib().qsv_batch_run(self.h, QSV_C64 if dtype == "c64" else QSV_C128,
                                  _stream_handle(stream), _dptr(e), _dptr(g)))
        out, off = [], 0
        for p in self._nparams:
            out.append(g[off:off + p].copy())
            off += p
        return e[:items.value], out

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None:
                lib().qsv_batch_free(self.h)
                self.h = None
        except Exception:
            pass


def prof_enable(on: bool):
    check(lib().qsv_prof_enable(1 if on else 0))


def prof_read(name: str):
    """(launches, total_ms, algorithmic bytes) for a kernel family."""
    n, ms, by = _c.c_int(), _c.c_double(), _c.c_double()
    check(lib().qsv_prof_read(name.encode(), _c.byref(n), _c.byref(ms), _c.byref(by)))
    return n.value, ms.value, by.value


def apply_record(state: State, g, theta=None):
    """Apply one gate record (see workloads.py) through the C ABI."""
    op = g["op"]
    if op in ("rx", "ry", "rz"):
        ang = theta[g["slot"]] if "slot" in g else g["angle"]
        state.apply_named(op, g["q"], ang)
    elif op in GATE:
        state.apply_named(op, g["q"])
    elif op == "dense":
        state.apply_gate(g["mat"], g["q"], g.get("controls", ()), g.get("ctrl_vals", ()))
    elif op == "pauli_rot":
        ang = theta[g["slot"]] if "slot" in g else g["angle"]
        apply_pauli_rotation(state, g["q"], g["paulis"], ang)
    else:
        raise ValueError(op)


def apply_pauli_rotation(state: State, qubits, paulis, theta: float):
    """psi <- exp(+i theta P / 2) psi (qsv_apply_pauli_rotation)."""
    q, p = _ints(qubits), _ints(paulis)
    check(lib().qsv_apply_pauli_rotation(state.h, _iptr(q), _iptr(p), len(qubits), float(theta)))


def transition_amplitude(bra: State, obs: "Observable", ket: State) -> complex:
    """<bra|O|ket> (qsv_transition_amplitude)."""
    re, im = _c.c_double(), _c.c_double()
    check(lib().qsv_transition_amplitude(bra.h, obs.h, ket.h, _c.byref(re), _c.byref(im)))
    return complex(re.value, im.value)

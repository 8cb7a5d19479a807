"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own formulas: each one compares it
with a closed form, a printed fixture from the paper, or an independent library
route (numpy Kronecker products / tensordot, scipy's matrix exponential), so
that a dropped term, a wrong sign, a wrong bit order or a transposed operand in
the oracle fails at least one of them.
"""
import json
import os
import re

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_2011_13524_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")

# ---------------------------------------------------------------- helpers (independent of the oracle)

PAULI_NP = {
    0: np.eye(2, dtype=complex),
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def kron_op(n, ops):
    """Dense 2^n x 2^n operator from {qubit: 2x2}; qubit 0 is the right-most
    Kronecker factor, matching 'the right-most digit is qubit 0'."""
    m = np.eye(1, dtype=complex)
    for q in range(n - 1, -1, -1):
        m = np.kron(m, ops.get(q, np.eye(2, dtype=complex)))
    return m


def dense_observable(n, obs):
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for coef, qp in obs:
        ops = {}
        for q, p in qp:
            ops[q] = PAULI_NP[p]
        H += coef * kron_op(n, ops)
    return H


def tensordot_apply(psi, mat, targets):
    """psi' = K psi through numpy tensordot on the (2,)*n view of psi.
    Axis a of the view is qubit n-1-a. Matrix index bit j <-> targets[j]."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    t = psi.reshape([2] * n)
    m = np.asarray(mat).reshape([2] * (2 * k))  # axes (r_{k-1}..r_0, c_{k-1}..c_0)
    col_axes = list(range(k, 2 * k))
    psi_axes = [n - 1 - targets[k - 1 - a] for a in range(k)]  # c_{k-1}..c_0
    out = np.tensordot(m, t, axes=(col_axes, psi_axes))
    # out axes: r_{k-1}..r_0 followed by the remaining psi axes in order
    rest = [a for a in range(n) if a not in psi_axes]
    src_order = [n - 1 - targets[k - 1 - a] for a in range(k)] + rest
    out = np.moveaxis(out, list(range(n)), src_order)
    return out.reshape(-1)


def rand_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------- fixtures from the paper

def test_pauli_matrices_match_printed():
    g = json.load(open(os.path.join(GOLD, "pauli_matrices.json")))
    for name, pid in g["ids"].items():
        printed = np.array([[complex(*e) for e in row] for row in g["matrices"][name]])
        if name == "I":
            continue
        np.testing.assert_array_equal(O.named_matrix(name.lower()), printed)
        np.testing.assert_array_equal(PAULI_NP[pid], printed)


def test_basis_index_convention():
    # section 4.2.1: index 2 of a 2-qubit state is |10>, qubit 0 right-most.
    psi = O.basis_state(2, 2)
    O.apply_gate(psi, {"op": "x", "q": [1]})
    np.testing.assert_array_equal(psi, [1, 0, 0, 0])
    psi = O.basis_state(2, 2)
    O.apply_gate(psi, {"op": "x", "q": [0]})
    np.testing.assert_array_equal(psi, [0, 0, 0, 1])


def test_appA_dense_matrix_is_cnot():
    g = json.load(open(os.path.join(GOLD, "appA_dense_cnot.json")))
    rng = np.random.default_rng(7)
    for n in (2, 3, 5):
        for (t, c) in [(0, 1), (1, 0), (0, n - 1), (n - 1, 0)]:
            if t == c:
                continue
            psi = rand_state(rng, n)
            a = psi.copy()
            O.apply_matrix(a, np.array(g["matrix"], dtype=complex), [t, c])
            b = psi.copy()
            O.apply_gate(b, {"op": "cnot", "q": [c, t]})
            # closed form: swap amplitudes of x and x^(1<<t) where bit c is set
            ref = psi.copy()
            for x in range(1 << n):
                if (x >> c) & 1:
                    ref[x] = psi[x ^ (1 << t)]
            np.testing.assert_array_equal(a, ref)
            np.testing.assert_array_equal(b, ref)


def test_appA_printed_output_norm():
    rows = [l.split() for l in open(os.path.join(GOLD, "appA_output_state.txt"))
            if l.strip() and not l.startswith("#")]
    v = np.array([complex(float(r), float(i)) for r, i in rows])
    assert abs(O.norm2(v) - 1.0) < 5e-6
    w = v.copy()
    O.apply_gate(w, {"op": "swap", "q": [0, 1]})
    np.testing.assert_array_equal(w, v[[0, 2, 1, 3]])


def _parse_openfermion(path):
    obs = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        m = re.match(r"\(([-0-9.e]+)\+0j\) \[(.*)\]", line.strip())
        coef = float(m.group(1))
        qp = []
        for tok in m.group(2).split():
            qp.append((int(tok[1:]), {"X": 1, "Y": 2, "Z": 3}[tok[0]]))
        obs.append((coef, qp))
    return obs


def test_openfermion_observable_on_basis_states():
    obs = _parse_openfermion(os.path.join(GOLD, "openfermion_h4.txt"))
    assert len(obs) == 15
    for b in range(16):
        psi = O.basis_state(4, b)
        # closed form: terms with an X or Y vanish on a basis state; a Z-only
        # term contributes coef * prod_q (-1)^{b_q}.
        ref = 0.0
        for coef, qp in obs:
            if any(p in (1, 2) for _, p in qp):
                continue
            ref += coef * np.prod([(-1) ** ((b >> q) & 1) for q, _ in qp])
        assert abs(O.expectation(psi, obs) - ref) < 1e-14
    assert abs(O.expectation(O.basis_state(4, 0), obs)) < 1e-14


# ---------------------------------------------------------------- definitions and closed forms

@pytest.mark.parametrize("name,pid", [("rx", 1), ("ry", 2), ("rz", 3)])
def test_rotation_is_exp_plus_i_theta_p_over_2(name, pid):
    # table of named gates: R_P(theta) = exp(+i theta P / 2)
    for th in np.linspace(-7, 7, 15):
        ref = scipy.linalg.expm(1j * th / 2 * PAULI_NP[pid])
        np.testing.assert_allclose(O.named_matrix(name, th), ref, atol=1e-15)


def test_hadamard_swap_cz():
    h = O.named_matrix("h")
    np.testing.assert_allclose(h @ h, np.eye(2), atol=1e-15)
    np.testing.assert_allclose(h @ PAULI_NP[3] @ h, PAULI_NP[1], atol=1e-15)
    rng = np.random.default_rng(1)
    psi = rand_state(rng, 3)
    a = psi.copy()
    O.apply_gate(a, {"op": "cz", "q": [0, 2]})
    ref = psi * np.array([-1 if (x & 1) and (x >> 2) & 1 else 1 for x in range(8)])
    np.testing.assert_allclose(a, ref, atol=0)


def test_rotation_expectations_closed_form():
    for th in np.linspace(0, 2 * np.pi, 9):
        psi = O.run_circuit(1, [{"op": "ry", "q": [0], "angle": th}])
        assert abs(O.expectation(psi, [(1.0, [(0, 3)])]) - np.cos(th)) < 1e-14
        assert abs(O.expectation(psi, [(1.0, [(0, 1)])]) + np.sin(th)) < 1e-14
        psi = O.run_circuit(1, [{"op": "rx", "q": [0], "angle": th}])
        assert abs(O.expectation(psi, [(1.0, [(0, 2)])]) - np.sin(th)) < 1e-14
        psi = O.run_circuit(1, [{"op": "h", "q": [0]}, {"op": "rz", "q": [0], "angle": th}])
        assert abs(O.expectation(psi, [(1.0, [(0, 1)])]) - np.cos(th)) < 1e-14
        assert abs(O.expectation(psi, [(1.0, [(0, 2)])]) + np.sin(th)) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_ghz(n):
    g = [{"op": "h", "q": [0]}] + [{"op": "cnot", "q": [0, i]} for i in range(1, n)]
    psi = O.run_circuit(n, g)
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    np.testing.assert_allclose(psi, ref, atol=1e-15)


def test_bell_states():
    s = 1 / np.sqrt(2)
    cases = {
        (): [s, 0, 0, s],
        ("z",): [s, 0, 0, -s],
        ("x",): [0, s, s, 0],
        ("x", "z"): [0, s, -s, 0],
    }
    for pre, ref in cases.items():
        g = [{"op": "h", "q": [1]}, {"op": "cnot", "q": [1, 0]}]
        # apply Pauli corrections on qubit 1 after preparing (|00>+|11>)/sqrt2
        g += [{"op": p, "q": [1]} for p in pre]
        psi = O.run_circuit(2, g)
        # X on qubit 1 maps |00>+|11> to |10>+|01>, Z on qubit 1 flips the sign of
        # components with qubit 1 set; the expected vectors follow from that.
        np.testing.assert_allclose(psi, np.array(ref, dtype=complex), atol=1e-15)


def test_controlled_x_with_control_values_bruteforce():
    # section 4.3.2 example: X on qubit 1, acting when qubit 2 is 0 and qubit 3 is 1
    rng = np.random.default_rng(3)
    X = PAULI_NP[1]
    P0 = np.diag([1.0, 0.0]).astype(complex)
    P1 = np.diag([0.0, 1.0]).astype(complex)
    for n in (4, 5, 6):
        psi = rand_state(rng, n)
        Kf = kron_op(n, {2: P0, 3: P1, 1: X}) + (np.eye(1 << n) - kron_op(n, {2: P0, 3: P1}))
        a = psi.copy()
        O.apply_matrix(a, X, [1], [2, 3], [0, 1])
        np.testing.assert_allclose(a, Kf @ psi, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_dense_k_matches_tensordot(k):
    rng = np.random.default_rng(10 + k)
    for n in (k, k + 2, 8):
        for _ in range(4):
            targets = list(rng.choice(n, size=k, replace=False))
            # deliberately non-unitary and non-symmetric (section 4.3.2: K need not be unitary)
            mat = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
            psi = rand_state(rng, n)
            a = psi.copy()
            O.apply_matrix(a, mat, targets)
            np.testing.assert_allclose(a, tensordot_apply(psi, mat, targets), atol=1e-12)


def test_dense_controlled_k_matches_projector_bruteforce():
    rng = np.random.default_rng(5)
    n = 6
    for _ in range(6):
        qs = list(rng.choice(n, size=4, replace=False))
        targets, controls = qs[:2], qs[2:]
        vals = list(rng.integers(0, 2, size=2))
        mat = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        psi = rand_state(rng, n)
        a = psi.copy()
        O.apply_matrix(a, mat, targets, controls, vals)
        proj = {c: np.diag([1.0 - v, float(v)]).astype(complex) for c, v in zip(controls, vals)}
        Pm = kron_op(n, proj)
        # K_full = P_c (x) K on targets + (1 - P_c)
        ref = Pm @ tensordot_apply(psi, mat, targets) + (psi - Pm @ psi)
        np.testing.assert_allclose(a, ref, atol=1e-12)


def test_one_qubit_layer_is_kronecker_product():
    rng = np.random.default_rng(11)
    n = 6
    us = {q: W.haar_unitary(rng, 2) for q in range(n)}
    psi = rand_state(rng, n)
    a = psi.copy()
    for q in range(n):
        O.apply_matrix(a, us[q], [q])
    np.testing.assert_allclose(a, kron_op(n, us) @ psi, atol=1e-13)


def _qft_gates(n):
    g = []
    for i in range(n - 1, -1, -1):
        g.append({"op": "h", "q": [i]})
        for j in range(i - 1, -1, -1):
            ph = np.exp(2j * np.pi / 2 ** (i - j + 1))
            g.append({"op": "dense", "q": [i], "mat": np.diag([1.0, ph]),
                      "controls": [j], "ctrl_vals": [1]})
    for q in range(n // 2):
        g.append({"op": "swap", "q": [q, n - 1 - q]})
    return g


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_qft_of_basis_states(n):
    N = 1 << n
    g = _qft_gates(n)
    for k in sorted({0, 1, N // 3, N - 1}):
        psi = O.run_circuit(n, g, psi=O.basis_state(n, k))
        ref = np.exp(2j * np.pi * np.arange(N) * k / N) / np.sqrt(N)
        np.testing.assert_allclose(psi, ref, atol=1e-13)


def test_qft_unitary_is_dft_matrix():
    n = 4
    N = 1 << n
    g = _qft_gates(n)
    U = np.zeros((N, N), dtype=complex)
    for k in range(N):
        U[:, k] = O.run_circuit(n, g, psi=O.basis_state(n, k))
    np.testing.assert_allclose(U, np.fft.ifft(np.eye(N), axis=0) * np.sqrt(N), atol=1e-13)


def test_norm_preserved_random_circuit():
    n = 9
    g = W.random_u_cz(n, 6, seed_key=(1, 99))
    psi = O.run_circuit(n, g)
    assert abs(O.norm2(psi) - 1.0) < 1e-13
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


def test_norm_and_inner_vs_numpy():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    b = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    assert abs(O.norm2(a) - np.vdot(a, a).real) < 1e-12
    assert abs(O.inner(a, b) - np.vdot(a, b)) < 1e-12


@pytest.mark.parametrize("n", [1, 3, 6])
def test_expectation_vs_dense_matrix(n):
    rng = np.random.default_rng(20 + n)
    obs = W.random_pauli_observable(n, 12, (1, n), seed_key=(9, n))
    obs.append((0.37, []))  # identity term
    obs.append((0.5, [(0, 2)]))
    H = dense_observable(n, obs)
    for _ in range(3):
        psi = rand_state(rng, n) * 1.3  # unnormalised on purpose: no division by <psi|psi>
        e = O.expectation_complex(psi, obs)
        ref = np.vdot(psi, H @ psi)
        assert abs(e - ref) < 1e-12
        assert abs(e.imag) < 1e-12
        np.testing.assert_allclose(O.apply_observable(psi, obs), H @ psi, atol=1e-12)


def test_pure_z_and_x_strings_on_product_state():
    # product state (x)_q RY(t_q)|0>: <Z_q> = cos t_q, <X_q> = -sin t_q, strings multiply
    rng = np.random.default_rng(4)
    n = 5
    th = rng.uniform(0, 2 * np.pi, n)
    psi = O.run_circuit(n, [{"op": "ry", "q": [q], "angle": th[q]} for q in range(n)])
    for qs in ([0], [1, 3], [0, 2, 4], list(range(n))):
        for p, f in ((3, np.cos), (1, lambda t: -np.sin(t))):
            e = O.expectation(psi, [(1.0, [(q, p) for q in qs])])
            assert abs(e - np.prod([f(th[q]) for q in qs])) < 1e-13
    e = O.expectation(psi, [(1.0, [(0, 1), (2, 3)])])
    assert abs(e - (-np.sin(th[0]) * np.cos(th[2]))) < 1e-13


def test_gradient_one_qubit_closed_form():
    for th in np.linspace(0.1, 6.0, 7):
        g = [{"op": "ry", "q": [0], "slot": 0}]
        ps = O.param_shift_grad(1, g, [th], [(1.0, [(0, 3)])])
        assert abs(ps[0] + np.sin(th)) < 1e-14


def test_param_shift_matches_finite_difference_and_closed_form():
    n = 4
    gates, npar = W.ry_rz_cnot_ring(n, 2)
    theta = W.uniform_angles(npar, (4, 0))
    obs = W.random_pauli_observable(n, 10, (1, 4), seed_key=(4, 1))
    ps = O.param_shift_grad(n, gates, theta, obs)
    fd = O.fd_grad(n, gates, theta, obs, h=1e-5)
    scale = sum(abs(c) for c, _ in obs)
    assert np.max(np.abs(ps - fd)) < 1e-8 * scale
    # product ansatz: H = Z0 Z1, circuit RY(a) on 0, RY(b) on 1 -> E = cos a cos b
    g = [{"op": "ry", "q": [0], "slot": 0}, {"op": "ry", "q": [1], "slot": 1}]
    a, b = 0.7, 2.1
    ps = O.param_shift_grad(2, g, [a, b], [(1.0, [(0, 3), (1, 3)])])
    np.testing.assert_allclose(ps, [-np.sin(a) * np.cos(b), -np.cos(a) * np.sin(b)], atol=1e-14)


def test_oracle_rejects_bad_gates():
    psi = O.zero_state(3)
    with pytest.raises(ValueError):
        O.apply_matrix(psi, np.eye(2), [3])
    with pytest.raises(ValueError):
        O.apply_matrix(psi, np.eye(4), [1, 1])
    with pytest.raises(ValueError):
        O.apply_matrix(psi, np.eye(2), [0], [0], [1])


# ---------------------------------------------------------------- Pauli rotations, transition amplitudes

_PAULI = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]


def _string_matrix(n, qubits, paulis):
    # qubit 0 is the right-most Kronecker factor (index x = sum x_q 2^q)
    mats = [np.eye(2)] * n
    for q, p in zip(qubits, paulis):
        mats[q] = _PAULI[p]
    full = np.array(mats[n - 1], dtype=complex)
    for q in range(n - 2, -1, -1):
        full = np.kron(full, mats[q])
    return full


def test_pauli_rotation_one_qubit_is_the_named_rotation():
    rng = np.random.default_rng(41)
    for p, name in ((1, "rx"), (2, "ry"), (3, "rz")):
        for q in range(3):
            psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
            th = rng.uniform(0, 6.3)
            a = psi.copy()
            O.pauli_rotation(a, [q], [p], th)
            b = psi.copy()
            O.apply_matrix(b, O.named_matrix(name, th), [q])
            assert np.max(np.abs(a - b)) <= 1e-14


def test_pauli_rotation_is_the_matrix_exponential():
    from scipy.linalg import expm
    rng = np.random.default_rng(42)
    for n in (2, 3, 4):
        for _ in range(6):
            w = int(rng.integers(1, n + 1))
            qs = [int(q) for q in rng.choice(n, size=w, replace=False)]
            ps = [int(p) for p in rng.integers(1, 4, size=w)]
            th = rng.uniform(-6.3, 6.3)
            psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
            ref = expm(0.5j * th * _string_matrix(n, qs, ps)) @ psi
            got = psi.copy()
            O.pauli_rotation(got, qs, ps, th)
            assert np.max(np.abs(got - ref)) <= 1e-13


def test_zz_rotation_phases_on_basis_states():
    th = 0.83
    for k in range(16):
        psi = O.basis_state(4, k)
        O.pauli_rotation(psi, [1, 3], [3, 3], th)
        s = 1 - 2 * (((k >> 1) & 1) ^ ((k >> 3) & 1))
        assert abs(psi[k] - np.exp(0.5j * th * s)) <= 1e-15
        assert np.sum(np.abs(psi) > 0) == 1


def test_transition_amplitude_pins():
    rng = np.random.default_rng(43)
    n = 4
    obs = [(float(rng.standard_normal()), [(int(q), int(p)) for q, p in
                                           zip(rng.choice(n, size=2, replace=False), rng.integers(1, 4, size=2))])
           for _ in range(5)] + [(0.3, [])]
    a = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    b = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    # <a|a> form equals the expectation
    assert abs(O.transition_amplitude(a, a, obs) - O.expectation_complex(a, obs)) <= 1e-13
    # brute force a^dagger O b
    full = sum(c * _string_matrix(n, [q for q, _ in t], [p for _, p in t]) for c, t in obs)
    ref = np.vdot(a, full @ b)
    assert abs(O.transition_amplitude(a, b, obs) - ref) <= 1e-12


# ------------------------------------------------- marginals and sampling (4.2.2)

def test_marginal_worked_example_wildcard_pattern():
    # Section 4.2.2 example: values [1, 2, 0] on 3 qubits (entry q for qubit q,
    # 2 a wild card) is the outcome written |0?1> with qubit 0 rightmost, i.e.
    # the indices 0b001 and 0b011.
    p = np.arange(1, 9, dtype=np.float64)
    p /= p.sum()
    psi = np.sqrt(p) * np.exp(1j * np.arange(8))
    assert O.marginal_probability(psi, [1, 2, 0]) == pytest.approx(p[1] + p[3], abs=1e-15)
    assert O.marginal_probability(psi, [2, 2, 2]) == pytest.approx(1.0, abs=1e-14)
    for x in range(8):
        bits = [(x >> q) & 1 for q in range(3)]
        assert O.marginal_probability(psi, bits) == pytest.approx(p[x], abs=1e-15)


def test_marginal_product_state_closed_form():
    # prod_q (cos a_q |0> + e^{i b_q} sin a_q |1>): the marginal of any pattern
    # is the product of cos^2 / sin^2 over the measured qubits.
    rng = np.random.default_rng(11)
    n = 6
    a, b = rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n)
    psi = np.ones(1, dtype=np.complex128)
    for q in range(n):
        psi = np.kron(np.array([np.cos(a[q]), np.exp(1j * b[q]) * np.sin(a[q])]), psi)
    for _ in range(20):
        vals = [int(v) for v in rng.integers(0, 3, n)]
        want = 1.0
        for q, v in enumerate(vals):
            if v != 2:
                want *= np.cos(a[q]) ** 2 if v == 0 else np.sin(a[q]) ** 2
        assert O.marginal_probability(psi, vals) == pytest.approx(want, rel=1e-12, abs=1e-15)
    with pytest.raises(ValueError):
        O.marginal_probability(psi, [0, 1, 3, 2, 2, 2])


def test_sample_inverse_cdf_pins():
    # probabilities 1/4 on the even indices (exact in binary); the sample is
    # the first index whose running sum exceeds u, so u on a boundary goes up
    psi = np.array([0.5, 0, 0.5, 0, 0.5j, 0, -0.5, 0], dtype=np.complex128)
    u = [0.0, 0.2499, 0.25, 0.5, 0.74, 0.75, 0.9999999]
    assert [int(v) for v in O.sample(psi, u)] == [0, 0, 2, 4, 4, 6, 6]
    # a basis state is always sampled as itself; scaling the state changes nothing
    e = np.zeros(16, dtype=np.complex128)
    e[11] = 1j
    assert set(O.sample(e, np.linspace(0, 0.999, 50))) == {11}
    rng = np.random.default_rng(5)
    s = rng.normal(size=32) + 1j * rng.normal(size=32)
    uu = rng.uniform(size=200)
    assert np.array_equal(O.sample(s, uu), O.sample(3.0 * s, uu))
    with pytest.raises(ValueError):
        O.sample(psi, [1.0])
    with pytest.raises(ValueError):
        O.sample(np.zeros(4, dtype=np.complex128), [0.5])


def test_sample_matches_linear_scan_and_frequencies():
    rng = np.random.default_rng(9)
    psi = rng.normal(size=16) + 1j * rng.normal(size=16)
    psi[[3, 7]] = 0.0
    p = np.abs(psi) ** 2
    u = rng.uniform(size=4000)
    got = O.sample(psi, u)
    for ui, g in zip(u[:300], got[:300]):
        acc, pick = 0.0, None
        for x in range(16):  # brute force: first x whose running sum passes u * total
            acc += p[x]
            if acc > ui * p.sum():
                pick = x
                break
        assert g == pick
    assert not np.isin(got, [3, 7]).any()
    freq = np.bincount(got, minlength=16) / got.size
    sigma = np.sqrt(p / p.sum() * (1 - p / p.sum()) / got.size)
    assert np.all(np.abs(freq - p / p.sum()) <= 5 * sigma + 1e-12)

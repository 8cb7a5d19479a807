"""GPU parity of single-gate application, state set-up and reductions against
the CPU oracle (element by element, on the same seeded inputs).

Bars: complex128 max-abs amplitude error <= 1e-12, complex64 <= 1e-5 (scaled
by the largest amplitude for non-unitary gates); expectations
|dE| <= 1e-11 * sum|alpha| (c128) and 1e-5 * sum|alpha| (c64).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import Observable, State, expectation
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
DTYPES = ["c128", "c64"]


def rand_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def check_close(got, ref, dt, scale=1.0):
    err = np.max(np.abs(got - ref))
    assert err <= TOL[dt] * max(1.0, scale), f"max-abs error {err:.3e} ({dt})"


def gpu_apply(dt, psi, fn):
    n = int(psi.size).bit_length() - 1
    s = State(n, dt)
    s.load(psi)
    fn(s)
    return s.store()


def ref_input(psi, dt):
    # the complex64 path starts from the rounded input; compare against the
    # oracle run on exactly that input
    return psi.astype(np.complex64).astype(np.complex128) if dt == "c64" else psi.copy()


@pytest.mark.parametrize("dt", DTYPES)
def test_set_basis_load_store(dt):
    for n in (1, 2, 5, 11):
        s = State(n, dt)
        np.testing.assert_array_equal(s.store(), O.zero_state(n))
        for k in {0, 1, (1 << n) - 1, (1 << n) // 3}:
            s.set_basis(k)
            np.testing.assert_array_equal(s.store(), O.basis_state(n, k))
        rng = np.random.default_rng(n)
        v = rand_state(rng, n)
        s.load(v)
        check_close(s.store(), v, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_one_qubit_every_target_every_n(dt):
    rng = np.random.default_rng(100)
    for n in range(1, 13):
        psi = rand_state(rng, n)
        for t in range(n):
            u = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
            ref = ref_input(psi, dt)
            O.apply_matrix(ref, u, [t])
            got = gpu_apply(dt, psi, lambda s: s.apply_gate(u, [t]))
            check_close(got, ref, dt, np.max(np.abs(ref)) * 4)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("name", ["x", "y", "z", "h", "rx", "ry", "rz"])
def test_named_one_qubit(dt, name):
    rng = np.random.default_rng(7)
    for n in (1, 3, 8):
        psi = rand_state(rng, n)
        for t in range(n):
            th = rng.uniform(0, 2 * np.pi)
            g = {"op": name, "q": [t], "angle": th} if name.startswith("r") else {"op": name, "q": [t]}
            ref = ref_input(psi, dt)
            O.apply_gate(ref, g)
            got = gpu_apply(dt, psi, lambda s: s.apply_named(name, [t], th))
            check_close(got, ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_two_qubit_named_all_pairs(dt):
    # (8 qubits: the streamed kernels for low targets and low phase masks)
    rng = np.random.default_rng(8)
    for n in (2, 3, 6, 8):
        psi = rand_state(rng, n)
        for a, b in itertools.permutations(range(n), 2):
            for name in ("cnot", "cz", "swap"):
                ref = ref_input(psi, dt)
                O.apply_gate(ref, {"op": name, "q": [a, b]})
                got = gpu_apply(dt, psi, lambda s: s.apply_named(name, [a, b]))
                check_close(got, ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_controlled_with_values(dt):
    rng = np.random.default_rng(9)
    for n in (3, 5, 9, 12):
        psi = rand_state(rng, n)
        for _ in range(12):
            nc = int(rng.integers(1, min(4, n - 1) + 1))
            qs = [int(q) for q in rng.choice(n, size=1 + nc, replace=False)]
            t, ctrl = qs[0], qs[1:]
            vals = [int(v) for v in rng.integers(0, 2, size=nc)]
            kind = rng.integers(0, 4)
            if kind == 0:
                u = W.haar_unitary(rng, 2)
            elif kind == 1:
                u = np.array([[0, 1], [1, 0]], dtype=complex)
            elif kind == 2:
                u = np.diag([1.0, np.exp(1j * rng.uniform(0, 6))])
            else:
                u = np.diag(np.exp(1j * rng.uniform(0, 6, 2)))
            ref = ref_input(psi, dt)
            O.apply_matrix(ref, u, [t], ctrl, vals)
            got = gpu_apply(dt, psi, lambda s: s.apply_gate(u, [t], ctrl, vals))
            check_close(got, ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_dense_k(dt, k):
    rng = np.random.default_rng(20 + k)
    for n in (k, k + 1, 10, 12):
        psi = rand_state(rng, n)
        for _ in range(4):
            qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
            u = W.haar_unitary(rng, 1 << k)
            ref = ref_input(psi, dt)
            O.apply_matrix(ref, u, qs)
            got = gpu_apply(dt, psi, lambda s: s.apply_gate(u, qs))
            check_close(got, ref, dt)
        # with a control
        if n > k:
            qs = [int(q) for q in rng.choice(n, size=k + 1, replace=False)]
            u = W.haar_unitary(rng, 1 << k)
            ref = ref_input(psi, dt)
            O.apply_matrix(ref, u, qs[:k], qs[k:], [1])
            got = gpu_apply(dt, psi, lambda s: s.apply_gate(u, qs[:k], qs[k:], [1]))
            check_close(got, ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("k", [6, 7, 8, 10])
def test_dense_wide_k(dt, k):
    # the generic path (6 <= k <= 10 targets, temporal vector in LDS):
    # non-unitary, non-symmetric matrices (a transposed or conjugated operand
    # fails), targets in random order, with and without controls of either
    # value, several B0 groups and a ragged last grid stride
    rng = np.random.default_rng(40 + k)
    for n in (k, k + 2, 13):
        psi = rand_state(rng, n)
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        m = (rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))) / (1 << (k // 2))
        ref = ref_input(psi, dt)
        O.apply_matrix(ref, m, qs)
        got = gpu_apply(dt, psi, lambda s: s.apply_gate(m, qs))
        check_close(got, ref, dt)
        if n >= k + 2:
            qc = [int(q) for q in rng.choice(n, size=k + 2, replace=False)]
            vals = [int(v) for v in rng.integers(0, 2, size=2)]
            ref = ref_input(psi, dt)
            O.apply_matrix(ref, m, qc[:k], qc[k:], vals)
            got = gpu_apply(dt, psi, lambda s: s.apply_gate(m, qc[:k], qc[k:], vals))
            check_close(got, ref, dt)
    # a wide diagonal gate takes the same path
    n = k + 1
    psi = rand_state(rng, n)
    d = np.diag(np.exp(1j * rng.uniform(0, 6, 1 << k)))
    qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
    ref = ref_input(psi, dt)
    O.apply_matrix(ref, d, qs)
    check_close(gpu_apply(dt, psi, lambda s: s.apply_gate(d, qs)), ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_diagonal_and_structured_k(dt):
    rng = np.random.default_rng(33)
    n = 9
    psi = rand_state(rng, n)
    for k in (2, 3, 4):
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        d = np.diag(np.exp(1j * rng.uniform(0, 6, 1 << k)))
        ref = ref_input(psi, dt)
        O.apply_matrix(ref, d, qs)
        got = gpu_apply(dt, psi, lambda s: s.apply_gate(d, qs))
        check_close(got, ref, dt)
    # Toffoli as a dense 3-qubit matrix: reduces to X with two controls
    tof = np.eye(8, dtype=complex)
    tof[[6, 7]] = tof[[7, 6]]
    for qs in ([0, 1, 2], [5, 0, 8], [8, 7, 6]):
        ref = ref_input(psi, dt)
        O.apply_matrix(ref, tof, qs)
        got = gpu_apply(dt, psi, lambda s: s.apply_gate(tof, qs))
        check_close(got, ref, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_norm_inner(dt):
    rng = np.random.default_rng(44)
    for n in (1, 4, 13, 16):
        a, b = rand_state(rng, n) * 1.7, rand_state(rng, n)
        sa, sb = State(n, dt), State(n, dt)
        sa.load(a)
        sb.load(b)
        ra, rb = ref_input(a, dt), ref_input(b, dt)
        assert abs(sa.norm2() - O.norm2(ra)) <= 1e-12 * O.norm2(ra)
        assert abs(sa.inner(sb) - O.inner(ra, rb)) <= 1e-12


@pytest.mark.parametrize("dt", DTYPES)
def test_expectation_random_observables(dt):
    rng = np.random.default_rng(55)
    for n in (1, 2, 6, 11, 14):
        psi = rand_state(rng, n)
        ref = ref_input(psi, dt)
        obs = W.random_pauli_observable(n, 40, (1, min(n, 6)), seed_key=(55, n))
        obs += [(0.3, []), (0.2, [(0, 3)]), (-0.4, [(n - 1, 2)])]
        s = State(n, dt)
        s.load(psi)
        e = expectation(s, Observable(n, obs))
        e_ref = O.expectation(ref, obs)
        scale = sum(abs(c) for c, _ in obs)
        # complex64: FP32 pair products (relative error <= 2^-23) and FP32
        # sums of a thread's 8 products per tile (7 roundings of 2^-24) before
        # the FP64 sums, relative to <psi|psi>; complex128: FP64 throughout
        tol = 1e-12 if dt == "c128" else 9 * 2.0 ** -24 + 1e-12
        assert abs(e - e_ref) <= tol * scale, (e, e_ref)


def test_abi_errors_on_device():
    from paper_2011_13524_amd import QsvError
    s = State(4, "c128")
    with pytest.raises(QsvError) as ei:
        s.apply_gate(np.eye(2), [4])
    assert ei.value.code == -2
    with pytest.raises(QsvError) as ei:
        s.apply_gate(np.eye(4), [1, 1])
    assert ei.value.code == -3
    with pytest.raises(QsvError):
        s.apply_gate(np.eye(2), [0], [1], [2])
    with pytest.raises(QsvError):
        s.set_basis(16)
    np.testing.assert_array_equal(s.store(), O.zero_state(4))

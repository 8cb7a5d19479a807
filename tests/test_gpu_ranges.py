"""Oracle parity of the persistent multi-tile paths.

The expectation pass (k_expect_tile), the lambda = O psi pass
(k_apply_obs_tile) and the register-resident reverse sweep (k_adj_reg) run on
a bounded persistent grid: a workgroup takes a contiguous range of several
tiles only when the state has more tiles than the grid (at the default grids
from 24 or 25 qubits, depending on the pass and the dtype), and only then do
the next-tile prefetch and the carry of the next tile's base across local bit
positions run. Here the grids are
overridden (QSV_EXPECT_GRID, QSV_ADJOINT_GRID) to small odd values at 14-16
qubits, so every workgroup takes a ragged range of several tiles, with X/Y
strings on high qubits (non-contiguous local sets: the carry skips local bit
positions); and the default grids are checked at 24 qubits on seeded inputs
against the oracle.

Bars (section 4.5 expectation, the adjoint of section 4.4's parametric
circuits): expectations of a loaded state <= 1e-12 * sum|alpha| (c128) and
(9 * 2^-24 + 1e-12) * sum|alpha| (c64: each pair product is formed in FP32
with relative error <= 2^-23, a thread's 8 products of a tile are summed in
FP32, at most 7 more roundings of 2^-24, then everything in FP64; the pairs
partition the amplitudes, so the bound is relative to <psi|psi>; the oracle
reduces the same rounded amplitudes); O psi <= 1e-13 * sum|alpha| (c128) and 1e-6 * sum|alpha| (c64,
lambda stored in complex64); energies and gradients of circuits <= 1e-10 *
sum|alpha| (c128) and 2e-5 * sum|alpha| (c64).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import (Circuit, Observable, Plan, State, adjoint_gradient,
                                  apply_observable, expectation)
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

# expectation of a loaded (unit-norm) state against the oracle on the same
# rounded amplitudes, per unit of sum|alpha|
E_LOADED = {"c128": 1e-12, "c64": 9 * 2.0 ** -24 + 1e-12}

GRAD_TOL = {"c128": 1e-10, "c64": 2e-5}
LAM_TOL = {"c128": 1e-13, "c64": 1e-6}


def rand_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def high_observable(n, terms, seed):
    """Random strings of weight 1..6 plus strings whose X/Y sit on the highest
    qubits (flip masks far from the low local bits), a pure-Z string across
    the range, a multi-term flip-mask group and the identity."""
    obs = W.random_pauli_observable(n, terms, (1, 6), seed_key=(21, n, seed))
    obs += [(0.7, [(n - 1, 1)]), (-0.4, [(n - 1, 2), (n - 3, 1), (2, 3)]),
            (0.3, [(n - 2, 1), (n - 5, 2), (0, 3), (n - 1, 3)]),
            (0.9, [(n - 2, 2), (n - 5, 1), (1, 3)]),  # same flip mask as the line above
            (-0.6, [(0, 3), (n // 2, 3), (n - 1, 3)]), (0.25, [])]
    return obs


def as_loaded(psi, dt):
    return psi.astype(np.complex64).astype(np.complex128) if dt == "c64" else psi


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("grid", [3, 5])
def test_expectation_and_lambda_ragged_ranges(dt, grid, monkeypatch):
    monkeypatch.setenv("QSV_EXPECT_GRID", str(grid))
    rng = np.random.default_rng(100 + grid)
    for n in (14, 16):
        psi = rand_state(rng, n)
        ref_in = as_loaded(psi, dt)
        obs_t = high_observable(n, 24, grid)
        obs = Observable(n, obs_t)
        scale = sum(abs(c) for c, _ in obs_t)
        s, out = State(n, dt), State(n, dt)
        s.load(psi)
        e = expectation(s, obs)
        assert abs(e - O.expectation(ref_in, obs_t)) <= E_LOADED[dt] * scale, (n, dt, grid)
        apply_observable(s, obs, out)
        err = np.max(np.abs(out.store() - O.apply_observable(ref_in, obs_t)))
        assert err <= LAM_TOL[dt] * scale, (n, dt, grid, err)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("grid", [3, 5])
def test_adjoint_ragged_ranges(dt, grid, monkeypatch):
    # the tile-pass reverse sweep forced on, with every workgroup of the
    # sweep, of lambda = O psi and of the energy taking several tiles
    monkeypatch.setenv("QSV_ADJOINT_TILED_MIN", "1")
    monkeypatch.setenv("QSV_ADJOINT_GRID", str(grid))
    monkeypatch.setenv("QSV_EXPECT_GRID", str(grid))
    for n, (gates, npar) in ((14, W.ry_rz_cnot_ring(14, 2)), (16, W.hea_ry_rz_cz(16, 1))):
        theta = W.uniform_angles(npar, (22, n, grid))
        obs_t = high_observable(n, 10, grid)
        c = Circuit.from_records(n, gates)
        psi, lam = State(n, dt), State(n, dt)
        e, g = adjoint_gradient(c, theta, Observable(n, obs_t), psi, lam, Plan(c, dt, max_k=2))
        scale = sum(abs(cf) for cf, _ in obs_t)
        slots = sorted({0, 1, npar // 3, npar // 2, npar - 2, npar - 1})
        assert abs(e - O.energy(n, gates, theta, obs_t)) <= GRAD_TOL[dt] * scale, (n, dt, grid)
        g_ref = O.param_shift_grad(n, gates, theta, obs_t, slots=slots)
        err = np.max(np.abs(g[slots] - g_ref))
        assert err <= GRAD_TOL[dt] * scale, (n, dt, grid, err)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_expectation_and_lambda_24q_default_grid(dt):
    # 24 qubits at the default grid of 2048 persistent workgroups: 2048
    # (c64) / 4096 (c128) tiles, 1 / 2 per workgroup; seeded random state,
    # strings of weight <= 6
    n = 24
    psi = rand_state(np.random.default_rng(24), n)
    ref_in = as_loaded(psi, dt)
    obs_t = high_observable(n, 14, 0)
    obs = Observable(n, obs_t)
    scale = sum(abs(c) for c, _ in obs_t)
    s, out = State(n, dt), State(n, dt)
    s.load(psi)
    e = expectation(s, obs)
    assert abs(e - O.expectation(ref_in, obs_t)) <= E_LOADED[dt] * scale, dt
    apply_observable(s, obs, out)
    err = np.max(np.abs(out.store() - O.apply_observable(ref_in, obs_t)))
    assert err <= LAM_TOL[dt] * scale, (dt, err)


_ORACLE_24Q = {}


def _adjoint_24q_case():
    n = 24
    gates, npar = W.ry_rz_cnot_ring(n, 2)
    theta = W.uniform_angles(npar, (23, n))
    obs_t = high_observable(n, 4, 1)
    slots = [0, npar - 1]
    if not _ORACLE_24Q:  # (one oracle run serves both dtypes)
        _ORACLE_24Q["e"] = O.energy(n, gates, theta, obs_t)
        _ORACLE_24Q["g"] = O.param_shift_grad(n, gates, theta, obs_t, slots=slots)
    return n, gates, theta, obs_t, slots, _ORACLE_24Q["e"], _ORACLE_24Q["g"]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_adjoint_24q_vs_oracle(dt):
    # the 24-qubit adjoint at its default launch shape (register-resident
    # sweep at its default persistent grid), on two layers of the
    # workload's circuit family, against the oracle's energy and exact shift
    # rule on sampled parameters
    n, gates, theta, obs_t, slots, e_ref, g_ref = _adjoint_24q_case()
    c = Circuit.from_records(n, gates)
    psi, lam = State(n, dt), State(n, dt)
    e, g = adjoint_gradient(c, theta, Observable(n, obs_t), psi, lam, Plan(c, dt, max_k=2))
    scale = sum(abs(cf) for cf, _ in obs_t)
    assert abs(e - e_ref) <= GRAD_TOL[dt] * scale, dt
    err = np.max(np.abs(g[slots] - g_ref))
    assert err <= GRAD_TOL[dt] * scale, (dt, err)


def wide_observable(n, seed):
    """Strings whose X/Y factors cover more qubits than a tile holds beside
    the low ones (10 and 11 flip qubits above qubit 3; a tile holds 9 more
    for both dtypes), one of them twice with
    other Z/Y signs (a multi-term group), mixed with ordinary strings."""
    rng = np.random.default_rng(seed)
    hi = list(range(4, n))
    obs = W.random_pauli_observable(n, 8, (1, 4), seed_key=(25, n, seed))
    for w in (10, 11):
        qs = [int(q) for q in rng.choice(hi, size=w, replace=False)]
        ps = [int(p) for p in rng.integers(1, 3, size=w)]
        obs.append((float(rng.standard_normal()), list(zip(qs, ps)) + [(0, 3)]))
    flips = obs[-1][1][:-1]  # the same flip mask, X and Y swapped, other Z factors
    obs.append((0.45, [(q, 2 if p == 1 else 1) for q, p in flips] + [(1, 3), (2, 3)]))
    return obs


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("grid", ["0", "3"])
def test_wide_flip_masks(dt, grid, monkeypatch):
    # flip masks with more qubits than a tile holds are evaluated on their
    # own, pairs read straight from the state, after the tiled passes (the
    # same persistent partials): expectation, the no-allocation expectation,
    # lambda = O psi and the adjoint, against the oracle; also an observable
    # with wide masks only (no tiled pass: the first wide group writes)
    from paper_2011_13524_amd.binding import expectation_noalloc
    if grid != "0":
        monkeypatch.setenv("QSV_EXPECT_GRID", grid)
    rng = np.random.default_rng(140)
    for n in (15, 17):
        psi = rand_state(rng, n)
        ref_in = as_loaded(psi, dt)
        full = wide_observable(n, n)
        for obs_t in (full, full[-3:]):
            obs = Observable(n, obs_t)
            assert obs.passes(dt) >= 2
            scale = sum(abs(c) for c, _ in obs_t)
            s, out = State(n, dt), State(n, dt)
            s.load(psi)
            e_ref = O.expectation(ref_in, obs_t)
            assert abs(expectation(s, obs) - e_ref) <= E_LOADED[dt] * scale, (n, dt, len(obs_t))
            assert abs(expectation_noalloc(s, obs) - e_ref) <= E_LOADED[dt] * scale, (n, dt, len(obs_t))
            apply_observable(s, obs, out)
            err = np.max(np.abs(out.store() - O.apply_observable(ref_in, obs_t)))
            assert err <= LAM_TOL[dt] * scale, (n, dt, len(obs_t), err)
    n = 15
    gates, npar = W.ry_rz_cnot_ring(n, 1)
    theta = W.uniform_angles(npar, (26, n))
    obs_t = wide_observable(n, 3)
    c = Circuit.from_records(n, gates)
    psi, lam = State(n, dt), State(n, dt)
    e, g = adjoint_gradient(c, theta, Observable(n, obs_t), psi, lam, Plan(c, dt, max_k=2))
    scale = sum(abs(cf) for cf, _ in obs_t)
    slots = [0, npar // 2, npar - 1]
    assert abs(e - O.energy(n, gates, theta, obs_t)) <= GRAD_TOL[dt] * scale
    err = np.max(np.abs(g[slots] - O.param_shift_grad(n, gates, theta, obs_t, slots=slots)))
    assert err <= GRAD_TOL[dt] * scale, err


def shared_mask_observable(n, seed):
    """Flip masks shared by 2, 3, 4, 5, 8 and 9 strings (the X/Y pattern fixed,
    the Z qubits varied): masks of at most eight strings run as single-term
    records, larger sets as one shared record; with 60 more random strings
    the planner takes several passes and moves groups between them."""
    rng = np.random.default_rng(seed)
    obs = W.random_pauli_observable(n, 60, (2, 5), seed_key=(23, n, seed))
    for count in (2, 3, 4, 5, 8, 9):
        flips = rng.choice(n, size=int(rng.integers(1, 4)), replace=False)
        xy = [(int(q), int(rng.integers(1, 3))) for q in flips]
        others = [q for q in range(n) if q not in set(int(f) for f in flips)]
        for _ in range(count):
            zs = rng.choice(others, size=int(rng.integers(0, 4)), replace=False)
            obs.append((float(rng.standard_normal()), xy + [(int(q), 3) for q in zs]))
    # the pure-Z mask shared by several strings too
    for k in range(3):
        obs.append((0.2 * (k + 1), [(k, 3), (n - 1 - k, 3)]))
    return obs


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("grid", [0, 5])
def test_shared_flip_masks_vs_oracle(dt, grid, monkeypatch):
    if grid:
        monkeypatch.setenv("QSV_EXPECT_GRID", str(grid))
    rng = np.random.default_rng(300 + grid)
    for n in (14, 16):
        psi = rand_state(rng, n)
        ref_in = as_loaded(psi, dt)
        obs_t = shared_mask_observable(n, 7 + n)
        obs = Observable(n, obs_t)
        assert obs.passes(dt) >= 2
        scale = sum(abs(c) for c, _ in obs_t)
        s, out = State(n, dt), State(n, dt)
        s.load(psi)
        e = expectation(s, obs)
        assert abs(e - O.expectation(ref_in, obs_t)) <= E_LOADED[dt] * scale, (n, dt, grid)
        apply_observable(s, obs, out)
        err = np.max(np.abs(out.store() - O.apply_observable(ref_in, obs_t)))
        assert err <= LAM_TOL[dt] * scale, (n, dt, grid, err)

"""GPU parity of marginal probabilities and Z-basis sampling (section 4.2.2)
against the CPU oracle, whose marginal is pinned to the paper's wild-card
example and a product-state closed form and whose sampler is pinned to exact
boundary cases, a linear scan and outcome frequencies.

The sampler's cumulative table is summed in another order than the oracle's
sequential running sum, so an index may differ only where u * total lies
within rounding of a boundary: such samples are checked for validity (the
oracle's running sum brackets u * total up to that rounding, and the index
has nonzero probability); all others must agree exactly.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import QsvError, State

pytestmark = pytest.mark.gpu

RED = {"c128": 1e-12, "c64": 1e-12}  # relative, FP64 sums of exact products


def rand_state(rng, n, zero_frac=0.0):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    if zero_frac:
        v[rng.uniform(size=v.size) < zero_frac] = 0.0
    return v / np.linalg.norm(v)


def loaded(psi, dt):
    s = State(int(psi.size).bit_length() - 1, dt)
    s.load(psi)
    return s, s.store()  # the amplitudes as stored (complex64 rounded for c64)


def check_samples(psi_stored, u, got, rel=1e-12):
    p = np.abs(psi_stored.astype(np.complex128)) ** 2
    c = np.cumsum(p)
    r = np.asarray(u) * c[-1]
    want = O.sample(psi_stored, u)
    tol = rel * c[-1]
    near = np.zeros(len(u), dtype=bool)
    for k in (want - 1, want):  # boundaries around the oracle's pick
        kk = np.clip(k, 0, c.size - 1)
        near |= np.abs(c[kk] - r) <= tol
    assert np.array_equal(got[~near], want[~near])
    assert np.all((got >= 0) & (got < c.size))
    assert np.all(p[got] > 0.0)
    lo = np.where(got > 0, c[np.maximum(got - 1, 0)], 0.0)
    assert np.all(lo <= r + tol) and np.all(r < c[got] + tol)
    return int(near.sum())


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_marginal_vs_oracle(dt):
    rng = np.random.default_rng(71)
    for n in (1, 2, 5, 11, 12, 14):
        psi = rand_state(rng, n)
        s, st = loaded(psi, dt)
        pats = [[2] * n, [int(b) for b in rng.integers(0, 2, n)]]
        pats += [[int(v) for v in rng.integers(0, 3, n)] for _ in range(6)]
        for vals in pats:
            want = O.marginal_probability(st, vals)
            got = s.marginal_probability(vals)
            assert abs(got - want) <= RED[dt] * max(want, 1e-300) + 1e-300, (n, vals)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_marginal_large_sampled(dt):
    # 24 qubits: patterns with few and many measured qubits against the oracle,
    # and the sum rule P(q = 0) + P(q = 1) = P(q unmeasured)
    rng = np.random.default_rng(72)
    n = 24
    psi = rand_state(rng, n)
    s, st = loaded(psi, dt)
    for m in (1, 3, 12, 23, 24):
        vals = [2] * n
        for q in rng.choice(n, size=m, replace=False):
            vals[int(q)] = int(rng.integers(0, 2))
        want = O.marginal_probability(st, vals)
        assert abs(s.marginal_probability(vals) - want) <= 1e-12 * want + 1e-300
    vals = [int(v) for v in rng.integers(0, 3, n)]
    q = 7
    a, b, c = (s.marginal_probability(vals[:q] + [v] + vals[q + 1:]) for v in (0, 1, 2))
    assert abs(a + b - c) <= 1e-12 * c


def test_marginal_rejects_bad_values():
    s = State(3, "c64")
    s.set_basis(0)
    with pytest.raises(QsvError):
        s.marginal_probability([0, 1, 5])
    with pytest.raises(ValueError):
        s.marginal_probability([0, 1])


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_sample_vs_oracle_ragged_sizes(dt):
    # one chunk short of 4096, exactly one, two, and several tree levels
    rng = np.random.default_rng(73)
    near = 0
    for n in (1, 3, 11, 12, 13, 17):
        psi = rand_state(rng, n, zero_frac=0.3 if n > 3 else 0.0)
        s, st = loaded(psi, dt)
        u = rng.uniform(size=3000)
        near += check_samples(st, u, s.sample(u))
    assert near < 30


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_sample_25_qubits_three_levels(dt):
    rng = np.random.default_rng(74)
    n = 25
    psi = rand_state(rng, n, zero_frac=0.5)
    s, st = loaded(psi, dt)
    u = rng.uniform(size=20000)
    assert check_samples(st, u, s.sample(u)) < 50


def test_sample_special_cases():
    s = State(20, "c64")
    s.set_basis(12345)
    u = np.linspace(0.0, 0.999999, 1000)
    assert set(s.sample(u).tolist()) == {12345}
    assert s.sample([]).size == 0
    # unnormalised states sample from |psi|^2 / <psi|psi>
    rng = np.random.default_rng(75)
    psi = rand_state(rng, 10)
    a, sa = loaded(psi, "c128")
    b, _ = loaded(5.0 * psi, "c128")
    uu = rng.uniform(size=2000)
    ga = a.sample(uu)
    check_samples(sa, uu, ga)
    check_samples(5.0 * sa, uu, b.sample(uu))
    z = State(6, "c128")
    z.load(np.zeros(64, dtype=np.complex128))
    with pytest.raises(QsvError):
        z.sample([0.5])
    with pytest.raises(QsvError):
        a.sample([1.0])


def test_sample_frequencies_match_probabilities():
    rng = np.random.default_rng(76)
    psi = rand_state(rng, 6, zero_frac=0.25)
    s, st = loaded(psi, "c64")
    u = rng.uniform(size=200000)
    got = s.sample(u)
    p = np.abs(st.astype(np.complex128)) ** 2
    p /= p.sum()
    freq = np.bincount(got, minlength=64) / got.size
    sigma = np.sqrt(p * (1 - p) / got.size)
    assert np.all(np.abs(freq - p) <= 5 * sigma + 1e-12)
    assert np.all(freq[p == 0] == 0)


def test_sample_and_marginals_28_qubit_product_state():
    # full-size check through properties: RY(t_q) on every qubit of |0...0>
    # gives P(bit q = 1) = sin^2(t_q / 2) independently per qubit
    rng = np.random.default_rng(77)
    n = 28
    t = rng.uniform(0.3, 2.8, n)
    s = State(n, "c64")
    s.set_basis(0)
    for q in range(n):
        s.apply_named("ry", [q], float(t[q]))
    p1 = np.sin(t / 2) ** 2
    for q in (0, 5, 13, 27):
        vals = [2] * n
        vals[q] = 1
        assert s.marginal_probability(vals) == pytest.approx(p1[q], rel=1e-5)
    vals = [2] * n
    vals[1], vals[20] = 0, 1
    assert s.marginal_probability(vals) == pytest.approx((1 - p1[1]) * p1[20], rel=1e-5)
    m = 1 << 18
    got = s.sample(rng.uniform(size=m))
    assert got.min() >= 0 and got.max() < (1 << n)
    bits = (got[:, None] >> np.arange(n)) & 1
    freq = bits.mean(axis=0)
    sigma = np.sqrt(p1 * (1 - p1) / m)
    assert np.all(np.abs(freq - p1) <= 5 * sigma)

"""GPU parity of fused execution (merged blocks applied in LDS tile passes)
against the unfused CPU oracle. Fusion is an exact rewrite, so only rounding
differs: bars as for unfused circuits (1e-12 c128, 1e-5 c64 max-abs).

Small tiles (few local qubits) force many passes, non-local controls and
diagonal gates on non-local qubits at sizes the oracle runs in milliseconds.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import Circuit, Plan, State, apply_fused
from paper_2011_13524_amd.binding import QsvError
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-12, "c64": 1e-5}


def mixed_circuit(n, count, seed):
    """Every gate kind the library recognises, on random qubits."""
    rng = np.random.default_rng(seed)
    g = []
    for _ in range(count):
        r = rng.integers(0, 10)
        qs = [int(q) for q in rng.choice(n, size=min(n, 4), replace=False)]
        if r == 0:
            g.append({"op": "dense", "q": qs[:1], "mat": W.haar_unitary(rng, 2)})
        elif r == 1 and n >= 2:
            g.append({"op": "dense", "q": qs[:2], "mat": W.haar_unitary(rng, 4)})
        elif r == 2 and n >= 3:
            g.append({"op": "dense", "q": qs[:3], "mat": W.haar_unitary(rng, 8)})
        elif r == 3 and n >= 3:
            g.append({"op": "dense", "q": qs[:1], "mat": W.haar_unitary(rng, 2),
                      "controls": qs[1:3], "ctrl_vals": [int(v) for v in rng.integers(0, 2, 2)]})
        elif r == 4 and n >= 2:
            g.append({"op": "cnot", "q": qs[:2]})
        elif r == 5 and n >= 2:
            g.append({"op": "cz", "q": qs[:2]})
        elif r == 6 and n >= 2:
            g.append({"op": "swap", "q": qs[:2]})
        elif r == 7:
            g.append({"op": ["rx", "ry", "rz"][int(rng.integers(0, 3))], "q": qs[:1],
                      "angle": float(rng.uniform(0, 6.3))})
        elif r == 8 and n >= 2:
            g.append({"op": "dense", "q": qs[:2], "mat": np.diag(np.exp(1j * rng.uniform(0, 6, 4)))})
        else:
            g.append({"op": "h", "q": qs[:1]})
    return g


def fused_state(n, gates, dt, theta=None, **plan_kw):
    c = Circuit.from_records(n, gates)
    p = Plan(c, dt, **plan_kw)
    s = State(n, dt)
    apply_fused(s, p, theta)
    return s.store(), p.info()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kw", [dict(max_k=1), dict(max_k=2), dict(max_k=3),
                                dict(max_k=2, tile_qubits=6, low_qubits=2),
                                dict(max_k=3, tile_qubits=7, low_qubits=1),
                                dict(max_k=5, tile_qubits=8, low_qubits=3)])
def test_mixed_gates(dt, kw):
    for n, seed in ((10, 1), (12, 2)):
        gates = mixed_circuit(n, 150, seed)
        got, info = fused_state(n, gates, dt, **kw)
        ref = O.run_circuit(n, gates)
        err = np.max(np.abs(got - ref))
        assert err <= AMP_TOL[dt], (err, info)


# register-resident tile shapes (thread bits, tile qubits; 0 = default 12):
# 256 threads x 16 amplitudes (default), 512 x 16, 256 x 32 (complex64), 128 x 16
WG = [("c128", "8", 0), ("c128", "7", 11), ("c64", "8", 0), ("c64", "9", 13), ("c64", "8", 13),
      ("c64", "7", 11)]


@pytest.mark.parametrize("dt,tb,tile", WG)
@pytest.mark.parametrize("max_k", [1, 2, 3])
def test_register_resident_tiles(dt, tb, tile, max_k, monkeypatch):
    # tiles run register-resident once the state is at least one tile; max_k=3
    # also exercises blocks applied through LDS inside a register-resident pass
    monkeypatch.setenv("QSV_TILE_THREAD_BITS", tb)
    for n, seed in ((13, 3), (14, 4), (16, 5)):
        gates = mixed_circuit(n, 220, seed)
        got, info = fused_state(n, gates, dt, max_k=max_k, tile_qubits=tile)
        assert info["segments"] > 0  # the register-resident kernel ran
        ref = O.run_circuit(n, gates)
        err = np.max(np.abs(got - ref))
        assert err <= AMP_TOL[dt], (n, err, info)


@pytest.mark.parametrize("dt,tb,tile", WG)
def test_register_resident_layered_and_random(dt, tb, tile, monkeypatch):
    monkeypatch.setenv("QSV_TILE_THREAD_BITS", tb)
    n = 16
    for gates in (W.layered_rx_rz_cnot(n, 10, seed_key=(2, n)), W.random_u_cz(n, 20, seed_key=(1, n))):
        for max_k in (1, 2):
            got, info = fused_state(n, gates, dt, max_k=max_k, tile_qubits=tile)
            assert np.max(np.abs(got - O.run_circuit(n, gates))) <= AMP_TOL[dt], info


def test_layered_10q_single_pass():
    n = 10
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(0,))
    got, info = fused_state(n, gates, "c128", max_k=2)
    assert info["passes"] == 1
    assert np.max(np.abs(got - O.run_circuit(n, gates))) <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_layered_many_passes(dt):
    n = 15
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(2, n))
    got, info = fused_state(n, gates, dt, max_k=2, tile_qubits=9, low_qubits=3)
    assert info["passes"] > 3
    assert np.max(np.abs(got - O.run_circuit(n, gates))) <= AMP_TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("max_k", [1, 2, 4])
def test_random_u_cz_fused(dt, max_k):
    n = 14
    gates = W.random_u_cz(n, 20, seed_key=(1, n))
    got, info = fused_state(n, gates, dt, max_k=max_k, tile_qubits=10, low_qubits=4)
    assert np.max(np.abs(got - O.run_circuit(n, gates))) <= AMP_TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_parametric_fused_reapply(dt):
    # the same plan applied with two parameter vectors
    n = 11
    gates, npar = W.ry_rz_cnot_ring(n, 4)
    c = Circuit.from_records(n, gates)
    p = Plan(c, dt, max_k=2, tile_qubits=8, low_qubits=2)
    for key in (0, 1):
        theta = W.uniform_angles(npar, (4, key))
        s = State(n, dt)
        apply_fused(s, p, theta)
        ref = O.run_circuit(n, gates, theta)
        assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt]


def test_qft_fused_matches_closed_form():
    n = 9
    N = 1 << n
    g = []
    for i in range(n - 1, -1, -1):
        g.append({"op": "h", "q": [i]})
        for j in range(i - 1, -1, -1):
            g.append({"op": "dense", "q": [i], "mat": np.diag([1.0, np.exp(2j * np.pi / 2 ** (i - j + 1))]),
                      "controls": [j], "ctrl_vals": [1]})
    for q in range(n // 2):
        g.append({"op": "swap", "q": [q, n - 1 - q]})
    c = Circuit.from_records(n, g)
    p = Plan(c, "c128", max_k=3, tile_qubits=6, low_qubits=2)
    for k in (0, 5, N - 1):
        s = State(n, "c128")
        s.set_basis(k)
        apply_fused(s, p)
        ref = np.exp(2j * np.pi * np.arange(N) * k / N) / np.sqrt(N)
        assert np.max(np.abs(s.store() - ref)) <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_autotuned_plan_matches_oracle(dt):
    # the autotuner times candidate plans on a scratch state and returns the
    # fastest; whichever it picks, the result is the circuit's
    n = 16
    gates, npar = W.ry_rz_cnot_ring(n, 3)
    theta = W.uniform_angles(npar, (7, n))
    c = Circuit.from_records(n, gates)
    scratch = State(n, dt)
    p = Plan.autotune(c, scratch, theta, reps=2)
    ch = p.choice
    assert ch["max_k"] in (1, 2, 3)
    assert ch["tile_qubits"] in ((12, 11, 13) if dt == "c64" else (12, 11))
    assert ch["thread_bits"] in (7, 8, 9)
    assert ch["reg_bits"] == ch["tile_qubits"] - ch["thread_bits"]  # register-resident at 16 qubits
    s = State(n, dt)
    apply_fused(s, p, theta)
    ref = O.run_circuit(n, gates, theta)
    assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt], ch
    # the scratch state holds a unit vector (the circuit applied several times)
    assert abs(np.linalg.norm(scratch.store()) - 1.0) <= 1e-4


def test_autotune_rejects_mismatched_state():
    c = Circuit.from_records(8, [{"op": "h", "q": [0]}])
    with pytest.raises(QsvError):
        Plan.autotune(c, State(9, "c64"))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_commuting_diagonal_blocks_run_ahead(dt):
    # QAOA-like layers (two-qubit diagonal phases on a random graph, then RX
    # on every qubit) with small tiles: diagonal blocks may pass deferred
    # diagonal blocks on shared qubits; the result is the circuit's
    rng = np.random.default_rng(17)
    n = 12
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.uniform() < 0.3]
    gates = []
    for _ in range(3):
        for i, j in edges:
            ph = float(rng.uniform(0, 3))
            gates.append({"op": "dense", "q": [i, j], "mat": np.diag(np.exp(1j * ph * np.array([1, -1, -1, 1])))})
        for q in range(n):
            gates.append({"op": "rx", "q": [q], "angle": float(rng.uniform(0, 3))})
    ref = O.run_circuit(n, gates)
    for kw in (dict(max_k=2, tile_qubits=6, low_qubits=2), dict(max_k=1, tile_qubits=8, low_qubits=3)):
        got, info = fused_state(n, gates, dt, **kw)
        assert info["passes"] > 1
        assert np.max(np.abs(got - ref)) <= AMP_TOL[dt], (kw, info)


@pytest.mark.parametrize("layers", ["1", "0"])
@pytest.mark.parametrize("mfma", ["1", "0"])
@pytest.mark.parametrize("tb,tile", [("8", 0), ("9", 13), ("8", 13), ("7", 11)])
def test_one_qubit_ops_matrix_cores_and_vector_alu(layers, mfma, tb, tile, monkeypatch):
    # complex64 register tiles run uncontrolled dense one-qubit ops on the
    # matrix cores by default (QSV_TILE_MFMA=0: vector ALU), grouped into
    # layer ops of up to four register bits (QSV_TILE_LAYERS=0: one op per
    # dispatch); Haar gates on every qubit (every register bit of every
    # segment) with CZ and CNOT layers between them, every form against the
    # oracle
    monkeypatch.setenv("QSV_TILE_LAYERS", layers)
    monkeypatch.setenv("QSV_TILE_MFMA", mfma)
    monkeypatch.setenv("QSV_TILE_THREAD_BITS", tb)
    n = 16
    rng = np.random.default_rng(int(tb) * 10 + int(mfma))
    gates = []
    for layer in range(6):
        for q in range(n):
            gates.append({"op": "dense", "q": [q], "mat": W.haar_unitary(rng, 2)})
        for q in range(layer % 2, n - 1, 2):
            gates.append({"op": "cz" if layer % 3 else "cnot", "q": [q, q + 1]})
    got, info = fused_state(n, gates, "c64", max_k=1, tile_qubits=tile)
    assert info["segments"] > 0
    ref = O.run_circuit(n, gates)
    assert np.max(np.abs(got - ref)) <= AMP_TOL["c64"], info


def commuting_mix(n, count, seed):
    """Random gates rich in commuting pairs (rotations about Z and X, CNOT and
    CZ on few qubits, some H), so heavy planning moves gates past others."""
    rng = np.random.default_rng(seed)
    g = []
    for _ in range(count):
        r = int(rng.integers(0, 7))
        a, b = (int(q) for q in rng.choice(min(n, 5), size=2, replace=False))
        t = float(rng.uniform(0, 6.3))
        if r == 0:
            g.append({"op": "rz", "q": [a], "angle": t})
        elif r == 1:
            g.append({"op": "rx", "q": [a], "angle": t})
        elif r == 2:
            g.append({"op": "cnot", "q": [a, b]})
        elif r == 3:
            g.append({"op": "cz", "q": [a, b]})
        elif r == 4:
            g.append({"op": "dense", "q": [a, b], "mat": np.diag(np.exp(1j * rng.uniform(0, 6, 4)))})
        elif r == 5:
            g.append({"op": "ry", "q": [a], "angle": t})
        else:
            g.append({"op": "h", "q": [int(rng.integers(0, n))]})
    return g


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kw", [dict(max_k=2), dict(max_k=3), dict(max_k=2, tile_qubits=6, low_qubits=2),
                                dict(max_k=4, tile_qubits=8, low_qubits=3)])
def test_heavy_plans_match_oracle(dt, kw):
    # commutation-aware merging (section 5.4) is an exact rewrite: the fused
    # state equals the unfused oracle state up to rounding
    cases = [(12, commuting_mix(12, 300, 31)), (13, mixed_circuit(13, 200, 32)),
             (16, W.iqp_rz_cz(16, 12, seed_key=(5, 16))),
             (14, W.layered_rx_rz_cnot(14, 6, seed_key=(2, 14)))]
    for n, gates in cases:
        got, info = fused_state(n, gates, dt, heavy=True, **kw)
        ref = O.run_circuit(n, gates)
        assert np.max(np.abs(got - ref)) <= AMP_TOL[dt], (n, kw, info)


def test_heavy_compresses_commuting_circuit():
    n = 16
    gates = W.iqp_rz_cz(n, 20, seed_key=(5, 20))
    light = fused_state(n, gates, "c64", max_k=2)
    heavy = fused_state(n, gates, "c64", max_k=2, heavy=True)
    assert heavy[1]["blocks"] <= 2 * n < light[1]["blocks"]
    assert np.max(np.abs(heavy[0] - light[0])) <= 2e-6
    assert np.max(np.abs(heavy[0] - O.run_circuit(n, gates))) <= AMP_TOL["c64"]

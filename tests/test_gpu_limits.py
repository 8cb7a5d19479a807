"""Edge cases of the GPU path: the largest state (34 qubits, 2^34 amplitudes:
indices beyond 32 bits, 2^22 tiles per pass), the smallest (1-3 qubits, tiles
smaller than a workgroup), empty circuits and observables.

Bars as elsewhere: amplitudes max-abs <= 1e-12 (c128) / 1e-5 (c64) against the
oracle; closed forms at 34 qubits to 1e-5 (complex64 amplitudes, FP64 sums).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import (Circuit, Observable, Plan, State, apply_circuit, apply_fused,
                                  apply_observable, expectation)
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.mark.timeout(600)
def test_max_size_34q_c64_closed_forms():
    # RY(t_q) on every qubit, then a CZ ladder (diagonal: Z expectations keep
    # their product-state values); fused, then one unfused X on the top qubit
    n = 34
    rng = np.random.default_rng(34)
    t = rng.uniform(0.1, 3.0, n)
    gates = [{"op": "ry", "q": [q], "angle": float(t[q])} for q in range(n)]
    gates += [{"op": "cz", "q": [q, q + 1]} for q in range(n - 1)]
    s = State(n, "c64")
    apply_fused(s, Plan(Circuit.from_records(n, gates), "c64", max_k=2))
    assert abs(s.norm2() - 1.0) <= 1e-5
    qs = (0, 1, 17, 31, 32, 33)
    obs = [(1.0, [(q, 3)]) for q in qs]
    for q in qs:
        assert abs(expectation(s, Observable(n, [(1.0, [(q, 3)])])) - np.cos(t[q])) <= 1e-5, q
    zz = expectation(s, Observable(n, [(1.0, [(0, 3), (33, 3)])]))
    assert abs(zz - np.cos(t[0]) * np.cos(t[33])) <= 1e-5
    e = expectation(s, Observable(n, obs))
    assert abs(e - sum(np.cos(t[q]) for q in qs)) <= 1e-5 * len(qs)
    apply_circuit(s, Circuit.from_records(n, [{"op": "x", "q": [33]}]))
    assert abs(expectation(s, Observable(n, [(1.0, [(33, 3)])])) + np.cos(t[33])) <= 1e-5


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_smallest_states_fused_and_unfused(dt):
    for n in (1, 2, 3):
        rng = np.random.default_rng(n)
        gates = [{"op": "dense", "q": [q], "mat": W.haar_unitary(rng, 2)} for q in range(n)] * 3
        if n >= 2:
            gates += [{"op": "cnot", "q": [0, n - 1]}, {"op": "cz", "q": [n - 1, 0]},
                      {"op": "dense", "q": [0, 1], "mat": W.haar_unitary(rng, 4)}]
        ref = O.run_circuit(n, gates)
        for mk in (1, 2):
            s = State(n, dt)
            apply_fused(s, Plan(Circuit.from_records(n, gates), dt, max_k=mk))
            assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt], (n, mk)
        s = State(n, dt)
        apply_circuit(s, Circuit.from_records(n, gates))
        assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt], n
        obs = [(0.5, [(0, 1)]), (-0.25, [(n - 1, 2)]), (0.75, [])]
        e_ref = O.expectation(ref, obs)
        assert abs(expectation(s, Observable(n, obs)) - e_ref) <= 1e-6


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_empty_circuit_and_observable(dt):
    n = 13
    s = State(n, dt)
    s.set_basis(5)
    p = Plan(Circuit(n), dt, max_k=2)
    assert p.info()["passes"] == 0
    apply_fused(s, p)
    apply_circuit(s, Circuit(n))
    v = s.store()
    assert v[5] == 1 and np.count_nonzero(v) == 1
    assert expectation(s, Observable(n, [])) == 0.0
    out = State(n, dt)
    out.set_basis(0)
    apply_observable(s, Observable(n, []), out)
    assert np.count_nonzero(out.store()) == 0

"""GPU parity of whole circuits (unfused and fused) against the CPU oracle on
the seeded workloads, at sizes the oracle finishes in seconds.

Bars: amplitudes max-abs <= 1e-12 (c128) / 1e-5 (c64, vs the complex128
oracle); expectations |dE| <= 1e-11 * sum|alpha| (c128) / 1e-5 * sum|alpha|
(c64).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import Circuit, Observable, State, apply_circuit, expectation
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-12, "c64": 1e-5}
E_TOL = {"c128": 1e-11, "c64": 1e-5}


def run_gpu(n, gates, dt, theta=None, mode="unfused", **kw):
    s = State(n, dt)
    c = Circuit.from_records(n, gates)
    apply_circuit(s, c, theta)
    return s


def test_layered_rx_rz_cnot_10q_c128():
    # 10 qubits, complex128, 10 layers: full state and <Z_0>
    n = 10
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(0,))
    assert len(gates) == 290
    s = run_gpu(n, gates, "c128")
    ref = O.run_circuit(n, gates)
    assert np.max(np.abs(s.store() - ref)) <= 1e-12
    z0 = [(1.0, [(0, 3)])]
    assert abs(expectation(s, Observable(n, z0)) - O.expectation(ref, z0)) <= 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 7, 12])
def test_random_u_cz(dt, n):
    gates = W.random_u_cz(n, 20, seed_key=(1, n))
    s = run_gpu(n, gates, dt)
    ref = O.run_circuit(n, gates)
    got = s.store()
    assert np.max(np.abs(got - ref)) <= AMP_TOL[dt]
    assert abs(s.norm2() - 1.0) <= (1e-12 if dt == "c128" else 1e-5)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_layered_with_weight4_observable(dt):
    # structure of the 30-qubit headline workload at 14 qubits
    n = 14
    gates = W.layered_rx_rz_cnot(n, 10, seed_key=(2, n))
    obs = W.random_pauli_observable(n, 200, 4, seed_key=(2, 1, n))
    s = run_gpu(n, gates, dt)
    ref = O.run_circuit(n, gates)
    assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt]
    scale = sum(abs(c) for c, _ in obs)
    e = expectation(s, Observable(n, obs))
    assert abs(e - O.expectation(ref, obs)) <= E_TOL[dt] * scale


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_parametric_ring(dt):
    n = 9
    gates, npar = W.ry_rz_cnot_ring(n, 3)
    theta = W.uniform_angles(npar, (4, 9))
    s = run_gpu(n, gates, dt, theta)
    ref = O.run_circuit(n, gates, theta)
    assert np.max(np.abs(s.store() - ref)) <= AMP_TOL[dt]

"""The boundary with torch: a state borrowed from a torch CUDA tensor
(qsv_state_wrap) on torch's stream, and the autograd.Function on a side
stream. torch supplies the memory and the stream; every step runs in the
library's kernels. Checked against the oracle (amplitudes max-abs 1e-12 c128
/ 1e-5 c64; expectations 1e-12 / 2e-5 x sum|alpha|).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_13524_amd import Circuit, Observable, Plan, State, apply_fused, apply_record, expectation
from paper_2011_13524_amd import workloads as W

pytestmark = pytest.mark.gpu

AMP_TOL = {"c128": 1e-12, "c64": 1e-5}
E_TOL = {"c128": 1e-12, "c64": 2e-5}


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("side_stream", [False, True])
def test_wrapped_torch_tensor(dt, side_stream):
    import torch
    n = 13
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    gates = W.layered_rx_rz_cnot(n, 3, seed_key=(40, n))
    obs_t = W.random_pauli_observable(n, 12, (1, 4), seed_key=(40, 1)) + [(0.5, [])]
    ref = O.run_circuit(n, gates)
    e_ref = O.expectation(ref, obs_t)
    scale = sum(abs(c) for c, _ in obs_t)
    stream = torch.cuda.Stream() if side_stream else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        # torch work on the stream before the library's: the wrapped state
        # starts from what torch wrote
        t = torch.full((1 << n,), 3.0 + 1.0j, dtype=tdt, device="cuda")
        t.zero_()
        t[0] = 1.0
        s = State.wrap(t, stream=stream)
        for g in gates[: len(gates) // 2]:
            apply_record(s, g)  # per-gate kernels
        c = Circuit.from_records(n, gates[len(gates) // 2:])
        apply_fused(s, Plan(c, dt, max_k=2))  # tile passes
        e = expectation(s, Observable(n, obs_t))
        # torch reads the same storage, ordered after the library's kernels
        got = t.to("cpu").numpy().astype(np.complex128)
    torch.cuda.synchronize()
    assert np.max(np.abs(got - ref)) <= AMP_TOL[dt]
    assert np.array_equal(got, s.store())
    assert abs(e - e_ref) <= E_TOL[dt] * scale
    s.free()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_autograd_on_side_stream(dt):
    import torch
    from paper_2011_13524_amd.autograd import circuit_energy
    n = 6
    gates, npar = W.hea_ry_rz_cz(n, 2)
    obs_t = W.tfim_chain(n)
    c = Circuit.from_records(n, gates)
    obs = Observable(n, obs_t)
    theta0 = W.uniform_angles(npar, (41, n))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        theta = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
        e = circuit_energy(theta, c, obs, dt)
        (2.0 * e).backward()
        grad = theta.grad.to("cpu").numpy()
    scale = sum(abs(cf) for cf, _ in obs_t)
    tol = 1e-10 if dt == "c128" else 2e-5
    assert abs(e.item() - O.energy(n, gates, theta0, obs_t)) <= tol * scale
    np.testing.assert_allclose(grad, 2.0 * O.param_shift_grad(n, gates, theta0, obs_t),
                               atol=2.0 * tol * scale)

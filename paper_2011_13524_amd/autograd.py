"""torch.autograd.Function over the library's adjoint gradient.

    energy = circuit_energy(theta, circuit, observable, dtype="c64")
    energy.backward()          # theta.grad = dE/dtheta from qsv_adjoint_gradient

The forward pass runs the circuit and the observable on the GPU through the C
ABI; backward returns grad_output * dE/dtheta computed by the same call (the
reverse sweep runs in forward and its result is kept for backward). torch is
used for the parameter tensor and the autograd graph only.
"""
from __future__ import annotations

import torch

from .binding import Circuit, Observable, Plan, State, adjoint_gradient


class _Workspace:
    """Two device states (psi, lambda) reused across calls for one (n, dtype,
    stream): the library enqueues on torch's current stream, so the energy and
    gradient are ordered with the caller's other work on that stream."""

    _cache: dict = {}

    @classmethod
    def get(cls, n: int, dtype: str):
        stream = torch.cuda.current_stream() if torch.cuda.is_available() else None
        key = (n, dtype, None if stream is None else int(stream.cuda_stream))
        if key not in cls._cache:
            cls._cache[key] = (State(n, dtype, stream=stream), State(n, dtype, stream=stream))
        return cls._cache[key]


class CircuitEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, circuit: Circuit, observable: Observable, dtype: str, plan):
        n = circuit.info()[0]
        psi, lam = _Workspace.get(n, dtype)
        th = theta.detach().to("cpu", torch.float64).numpy()
        e, g = adjoint_gradient(circuit, th, observable, psi, lam, plan)
        ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
        return theta.new_tensor(e)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None


def circuit_energy(theta: torch.Tensor, circuit: Circuit, observable: Observable,
                   dtype: str = "c64", plan: Plan | None = None) -> torch.Tensor:
    return CircuitEnergy.apply(theta, circuit, observable, dtype, plan)

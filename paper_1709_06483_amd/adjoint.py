"""torch.autograd bridge for the fidelity gradient computed by the library.

``FidelityLoss.apply(theta, problem)`` maps real control parameters theta
(a CPU float64 tensor) to the loss 1 - |<psi_target, psi(T)>|^2 of a Cf4
propagation under the field f(t) = sum_k theta_k s_k(t).  The forward call
runs ``magnus_propagate_adjoint`` (forward sweep with checkpoints, backward
Magnus-Leja sweep with Frechet block exponentials) and keeps the gradient
for ``backward``.  Only marshalling happens here: the basis values s_k at the
quadrature nodes are the problem's parametrisation of the field.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import binding as B


@dataclass
class ControlProblem:
    ctx: B.Context
    ham: B.DeviceHamiltonian
    tau: float
    basis_nodes: np.ndarray  # (nsteps, 2, P): s_k(t_n + c_j tau)
    psi0: object             # device complex128 state
    psi_target: object       # device complex128 state
    every_k: int = 16
    opts: B.LejaOpts | None = None

    @staticmethod
    def with_basis(ctx, ham, tau, nsteps, basis, psi0, psi_target, t0=0.0, every_k=16, opts=None):
        """basis(t) -> array of the P basis values at time t."""
        t = B.magnus_quadrature_nodes(B.CF4, t0, tau, nsteps)
        S = np.stack([np.stack([np.asarray(basis(t[n, j]), dtype=np.float64) for j in range(2)])
                      for n in range(nsteps)])
        return ControlProblem(ctx, ham, tau, S, psi0, psi_target, every_k, opts)

    def loss_and_grad(self, theta: np.ndarray):
        f = self.basis_nodes @ np.asarray(theta, dtype=np.float64)
        return B.magnus_propagate_adjoint(self.ctx, self.ham, self.tau, f, self.basis_nodes, self.psi0,
                                          self.psi_target, every_k=self.every_k, opts=self.opts)


def _function():
    import torch

    class FidelityLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, theta, problem: ControlProblem):
            loss, grad = problem.loss_and_grad(theta.detach().cpu().numpy())
            fctx.save_for_backward(torch.from_numpy(grad).to(theta.dtype))
            return torch.tensor(loss, dtype=theta.dtype)

        @staticmethod
        def backward(fctx, gout):
            (grad,) = fctx.saved_tensors
            return gout * grad, None

    return FidelityLoss


_FL = None


def fidelity_loss(theta, problem: ControlProblem):
    """Differentiable loss (torch scalar) of the control parameters theta."""
    global _FL
    if _FL is None:
        _FL = _function()
    return _FL.apply(theta, problem)

"""Differentiating through a sketched TT-GMRES solve of a parametric Kronecker sum.

A(theta) = sum_k theta_k (I x .. x L_k x .. x I), the Laplacian-like operators of
Sec. 5.1 with one weight per mode.  For the loss ||x(theta) - x_t||^2 with
A(theta) x = b:

  lambda = A(theta)^-T 2 (x - x_t)            (adjoint solve, transposed L_k)
  dLoss/dtheta_k = -<lambda, L_k x>           (environment sweeps of <lambda, x>)
  dLoss/db       = lambda.

Both solves are the enhanced sketched TT-GMRES of Alg. 4 (restarted, FP64 true
residual); every contraction runs in the HIP library.  The accuracy of the
gradient follows that of the two solves: with forward and adjoint residuals
below tol the relative gradient error is of order cond(A) * tol.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import ttsg


@dataclass
class KronSumProblem:
    """Inputs of the parametric solve; cores are CUDA float64 tensors."""
    Ls: List[np.ndarray]                   # unscaled 1-D operators, one per mode (n_k x n_k)
    b: List[torch.Tensor]
    x_target: List[torch.Tensor]
    S: List[torch.Tensor]                  # Khatri-Rao factors (s x n_k)
    X: List[torch.Tensor]                  # STTA right sketch cores
    Y: List[torch.Tensor]                  # STTA left sketch cores
    rx: List[int]
    rho: List[int]
    maxit: int = 500
    tol: float = 1e-6
    q: int = 1
    round_tol: float = 1e-8
    final_tol: float = 1e-10
    maxrank: int = 64
    stop_safety: float = 0.3
    restart: int = 0
    precision: int = ttsg.PREC_F64
    adjoint_rhs_tol: float = 1e-13
    last: dict = field(default_factory=dict)


def _operator(Ls: Sequence[np.ndarray], theta: np.ndarray, transpose: bool, device) -> List[torch.Tensor]:
    mats = [theta[k] * (np.asarray(L).T if transpose else np.asarray(L)) for k, L in enumerate(Ls)]
    return ttsg.kron_sum_operator([mats], device)


def _solve(P: KronSumProblem, A, rhs) -> ttsg.SolveResult:
    r = ttsg.sgmres_solve(A, rhs, P.S, P.X, P.Y, P.rx, P.rho, maxit=P.maxit, tol=P.tol, q=P.q,
                          round_tol=P.round_tol, maxrank=P.maxrank, stop_safety=P.stop_safety,
                          restart=P.restart, final_tol=P.final_tol, precision=P.precision)
    if r.status != ttsg.OK:
        raise ttsg.TTSGError(f"parametric solve did not converge (status {r.status}, true residual "
                             f"{r.true_residual:.3e} after {r.iterations} iterations)")
    return r


def forward_loss(P: KronSumProblem, theta: np.ndarray):
    """x(theta) and ||x - x_t||^2 (dot products on the GPU)."""
    dev = P.b[0].device
    fwd = _solve(P, _operator(P.Ls, theta, False, dev), P.b)
    x = fwd.x
    loss = ttsg.dot(x, x) - 2.0 * ttsg.dot(x, P.x_target) + ttsg.dot(P.x_target, P.x_target)
    return x, loss, fwd


def backward_grad(P: KronSumProblem, theta: np.ndarray, x: List[torch.Tensor]):
    """(dLoss/dtheta, lambda) from one adjoint solve and one pair of environment sweeps."""
    dev = x[0].device
    rhs = ttsg.tt_axpby(2.0, x, -2.0, P.x_target)
    rhs = ttsg.round_svd(rhs, P.adjoint_rhs_tol, P.maxrank)
    adj = _solve(P, _operator(P.Ls, theta, True, dev), rhs)
    lam = adj.x
    Ls_dev = [torch.as_tensor(np.asarray(L), dtype=torch.float64, device=dev).contiguous() for L in P.Ls]
    g = ttsg.grad_kron_sum(Ls_dev, lam, x)
    return g, lam, adj


class _KronSumSolveLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, problem: KronSumProblem):
        th = theta.detach().cpu().double().numpy()
        x, loss, fwd = forward_loss(problem, th)
        ctx.problem = problem
        ctx.theta = th
        ctx.x = x
        problem.last = dict(x=x, forward=fwd)
        return torch.tensor(loss, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g, lam, adj = backward_grad(ctx.problem, ctx.theta, ctx.x)
        ctx.problem.last.update(lam=lam, adjoint=adj, grad=g)
        gt = torch.as_tensor(g, dtype=grad_out.dtype, device=grad_out.device) * grad_out
        return gt, None


def kron_sum_solve_loss(theta: torch.Tensor, problem: KronSumProblem) -> torch.Tensor:
    """||x(theta) - x_t||^2 with autograd support for theta.

    After backward(), problem.last["lam"] holds lambda = dLoss/db as TT cores."""
    if theta.dim() != 1 or theta.numel() != len(problem.Ls):
        raise ttsg.TTSGError("theta must be a vector with one weight per mode")
    return _KronSumSolveLoss.apply(theta, problem)

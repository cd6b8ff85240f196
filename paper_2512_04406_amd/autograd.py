"""torch.autograd face of the subproblem cost.

The ALM subproblem cost Psi(Y) = <D + Xt, Z> + sigma/2 ||Q(Z)||_F^2 with
Z = Y Y^T + C (eq. reduced-ALM-subproblem) becomes a differentiable function
of Y whose derivatives are the library's hand-written ones:

* first derivative: the Euclidean gradient 2 G Y with G = Xt + D + sigma Q(Z)
  (Lemma lm:suboptimality), from the fused residual/product pass;
* second derivative: the Euclidean Hessian-vector product
  2 G U + 2 sigma Q(Y U^T + U Y^T) Y (Proposition prop), from the HVP kernels.

`alm_cost(prob, Y)` supports `backward()` and double backward
(`torch.autograd.grad(..., create_graph=True)` followed by a second grad),
which is how a Hessian-vector product of Psi is written in PyTorch; both
derivatives run on the GPU kernels, nothing is traced.  Riemannian quantities
on the oblique manifold (Proposition prop, eq. sec4:eq7) are exposed as plain
functions `riemannian_grad` and `riemannian_hvp`.
"""

from __future__ import annotations

import torch

from .problem import FP64, Problem


def _key(Y: torch.Tensor):
    return (Y.data_ptr(), Y._version, tuple(Y.shape))


def _ensure_point(prob: Problem, Y: torch.Tensor) -> None:
    """Make `Y` the problem's current point (the HVP kernels reuse the class
    averages and diag(G S) of the last cost/gradient pass)."""
    if getattr(prob, "_ad_key", None) != _key(Y):
        prob.cost_grad(Y, want_egrad=False, want_rgrad=False)
        prob._ad_key = _key(Y)


class _EGrad(torch.autograd.Function):
    """Y -> 2 G(Y) Y; its vector-Jacobian product is the (symmetric)
    Euclidean Hessian applied to the incoming vector."""

    @staticmethod
    def forward(ctx, prob: Problem, Y: torch.Tensor, prec: int):
        Yc = Y.detach().clone(memory_format=torch.contiguous_format)
        _, eg, _ = prob.cost_grad(Yc, want_egrad=True, want_rgrad=False)
        prob._ad_key = _key(Yc)
        ctx.prob, ctx.prec = prob, prec
        ctx.save_for_backward(Yc)
        return eg

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        (Yc,) = ctx.saved_tensors
        prob = ctx.prob
        _ensure_point(prob, Yc)
        H = prob.hvp(Yc, gout.detach().contiguous(), ctx.prec, riemannian=False)
        return None, H, None


class _Cost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prob: Problem, Y: torch.Tensor, prec: int):
        Yc = Y.detach().clone(memory_format=torch.contiguous_format)
        f, _, _ = prob.cost_grad(Yc, want_egrad=False, want_rgrad=False)
        prob._ad_key = _key(Yc)
        ctx.prob, ctx.prec = prob, prec
        ctx.save_for_backward(Y)
        return f.reshape(())

    @staticmethod
    def backward(ctx, gf: torch.Tensor):
        (Y,) = ctx.saved_tensors
        # routed through _EGrad so that a second differentiation reaches the
        # hand-written HVP
        eg = _EGrad.apply(ctx.prob, Y, ctx.prec)
        return None, gf * eg, None


def alm_cost(prob: Problem, Y: torch.Tensor, hvp_prec: int = FP64) -> torch.Tensor:
    """Psi(Y) as a 0-d float64 tensor, differentiable twice in Y.

    Y: contiguous float64 CUDA tensor n x p (any rows; the cost is defined on
    all of R^{n x p}, the manifold only restricts where the solver looks).
    hvp_prec: tile precision of the second derivative (FP64 or FP32)."""
    if not (Y.is_cuda and Y.dtype == torch.float64):
        raise TypeError("Y must be a float64 CUDA tensor")
    return _Cost.apply(prob, Y, hvp_prec)


def euclidean_grad(prob: Problem, Y: torch.Tensor, hvp_prec: int = FP64) -> torch.Tensor:
    """2 G Y, differentiable once more (its derivative is the Euclidean HVP)."""
    return _EGrad.apply(prob, Y, hvp_prec)


def riemannian_grad(prob: Problem, Y: torch.Tensor) -> torch.Tensor:
    """grad Psi(Y) = 2GY - Diag(rowdot(2GY, Y)) Y on the oblique manifold."""
    Yc = Y.detach().contiguous()
    _, _, rg = prob.cost_grad(Yc, want_egrad=False, want_rgrad=True)
    prob._ad_key = _key(Yc)
    return rg


def riemannian_hvp(prob: Problem, Y: torch.Tensor, U: torch.Tensor, prec: int = FP64) -> torch.Tensor:
    """Hess Psi(Y)[U] (eq. sec4:eq7) for a tangent U."""
    Yc = Y.detach().contiguous()
    _ensure_point(prob, Yc)
    return prob.hvp(Yc, U.detach().contiguous(), prec, riemannian=True)

"""Riemannian trust region with truncated CG (oracle).

The paper solves each Sub-k with the Riemannian trust-region method (section
"Exploiting the manifold structure", and the experiments section: Manopt's
trust-region solver).  This is the textbook method of Absil, Baker and
Gallivan (Found. Comput. Math. 2007), written from its description:

* Steihaug-Toint truncated CG on the model m(eta) = <g, eta> + 1/2 <eta, H eta>
  in the tangent space: stop at negative curvature or at the trust-region
  boundary (then step to the boundary), or when ||r|| <= ||r0|| min(||r0||^theta, kappa).
* ratio rho = (f(x) - f(R_x(eta))) / (m(0) - m(eta)); shrink the radius by 4 when
  rho < 1/4, double it (capped) when rho > 3/4 and tCG stopped on the boundary
  or on negative curvature; accept when rho > rho'.

Constants the paper does not state are arguments (defaults: rho' = 0.1,
kappa = 0.1, theta = 1, Delta_bar = pi sqrt(n), Delta_0 = Delta_bar / 8).

Parity: iterates are not a parity target (rounding changes the path); the
solver's output is pinned through the ALM end-to-end tests (optimal value vs
brute force, KKT residuals).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .subproblem import Subproblem, proj_tangent, retract

__all__ = ["tcg", "rtr", "RTRResult"]


def _inner(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.sum(a * b))


def tcg(sub: Subproblem, Y: np.ndarray, grad: np.ndarray, Delta: float,
        kappa: float = 0.1, theta: float = 1.0, maxinner: int = 200):
    """Return (eta, Heta, n_hvp, stop) with stop in
    {"negcurv", "boundary", "converged", "maxinner"}."""
    eta = np.zeros_like(Y)
    Heta = np.zeros_like(Y)
    r = grad.copy()
    rr = _inner(r, r)
    r0 = math.sqrt(rr)
    delta = -r
    e_Pe = 0.0
    e_Pd = 0.0
    d_Pd = rr
    n_hvp = 0
    stop = "maxinner"
    for _ in range(maxinner):
        Hd = sub.rhess(Y, delta)
        n_hvp += 1
        d_Hd = _inner(delta, Hd)
        alpha = rr / d_Hd if d_Hd != 0.0 else math.inf
        e_Pe_new = e_Pe + 2.0 * alpha * e_Pd + alpha * alpha * d_Pd
        if d_Hd <= 0.0 or e_Pe_new >= Delta * Delta:
            tau = (-e_Pd + math.sqrt(e_Pd * e_Pd + d_Pd * (Delta * Delta - e_Pe))) / d_Pd
            eta = eta + tau * delta
            Heta = Heta + tau * Hd
            stop = "negcurv" if d_Hd <= 0.0 else "boundary"
            break
        e_Pe = e_Pe_new
        eta = eta + alpha * delta
        Heta = Heta + alpha * Hd
        r = proj_tangent(Y, r + alpha * Hd)
        rr_new = _inner(r, r)
        if math.sqrt(rr_new) <= r0 * min(r0 ** theta, kappa):
            stop = "converged"
            break
        beta = rr_new / rr
        rr = rr_new
        delta = proj_tangent(Y, -r + beta * delta)
        e_Pd = beta * (e_Pd + alpha * d_Pd)
        d_Pd = rr + beta * beta * d_Pd
    return eta, Heta, n_hvp, stop


@dataclass
class RTRResult:
    Y: np.ndarray
    f: float
    grad: np.ndarray
    gradnorm: float
    iters: int
    n_hvp: int


def rtr(sub: Subproblem, Y: np.ndarray, gradtol: float, maxiter: int = 50,
        Delta0: float | None = None, Delta_bar: float | None = None,
        rho_prime: float = 0.1, kappa: float = 0.1, theta: float = 1.0,
        maxinner: int = 200, max_stall: int = 0) -> RTRResult:
    """max_stall > 0: also stop after max_stall consecutive iterations that
    leave the gradient norm above 0.9 times the best value of this call (the
    gradient is then at the level of its rounding errors)."""
    n = Y.shape[0]
    if Delta_bar is None:
        Delta_bar = math.pi * math.sqrt(n)
    Delta = Delta_bar / 8.0 if Delta0 is None else Delta0
    f = sub.cost(Y)
    g = sub.rgrad(Y)
    gn = math.sqrt(_inner(g, g))
    n_hvp = 0
    it = 0
    gn_best = gn
    stall = 0
    for it in range(1, maxiter + 1):
        if gn <= gradtol or (max_stall > 0 and stall >= max_stall):
            it -= 1
            break
        eta, Heta, nh, stop = tcg(sub, Y, g, Delta, kappa, theta, maxinner)
        n_hvp += nh
        Yp = retract(Y, eta)
        fp = sub.cost(Yp)
        model_dec = -(_inner(g, eta) + 0.5 * _inner(eta, Heta))
        reg = max(1.0, abs(f)) * np.finfo(float).eps * 1e3
        rho = (f - fp + reg) / (model_dec + reg)
        if rho < 0.25:
            Delta /= 4.0
        elif rho > 0.75 and stop in ("negcurv", "boundary"):
            Delta = min(2.0 * Delta, Delta_bar)
        if rho > rho_prime:
            Y, f = Yp, fp
            g = sub.rgrad(Y)
            gn = math.sqrt(_inner(g, g))
        if gn < 0.9 * gn_best:
            gn_best, stall = gn, 0
        else:
            stall += 1
    return RTRResult(Y=Y, f=f, grad=g, gradnorm=gn, iters=it, n_hvp=n_hvp)

"""Algorithm alg1 (ManiDSDP), FP64 dense oracle.

Steps per outer iteration k (Algorithm alg1, section "The ManiDSDP algorithm"):
 1. approximately solve Sub-k by RTR, warm-started at Y^k and supplied with the
    carried direction U;
 2. y^{k+1} = (AA*)^{-1} A(S^{k+1} + C);
 3. Xt^{k+1} = Xt^k - sigma_k (A* y^{k+1} - S^{k+1} - C)   (= Xt^k + sigma_k Q(Z));
 4. z^{k+1} = diag((Xt^{k+1} + D) S^{k+1});
 5. X^{k+1} = Xt^{k+1} + D - Diag(z^{k+1});
 6. if lambda_min(X^{k+1}) < 0 form U as in Theorem sec5:thm1, else U = 0;
 7. update p (zero-padding Y and U);
 8. update sigma by eq. sec5:eq1;
and the KKT residuals eta_p, eta_d, eta_g of eq. res with the stop at
eta_max <= tol.

Readings of points the paper leaves open:
* Y^0: the paper writes the zero matrix, which is not on the manifold; we take
  the given row-normalised Gaussian start.
* "supplied with the carried direction": from Yhat = [Y, 0] we backtrack
  t = sqrt(n), sqrt(n)/2, ... along R_Yhat(t U) until the new Psi_k decreases,
  then start RTR there (RTR alone cannot leave a saddle along U: the
  gradient vanishes on the new columns).
* rank rule (delegated by the paper to ManiSDP section 5.1, not in the text):
  after each subproblem, drop singular directions of Y below tau_rank * s_1
  (tau_rank = 1e-7; Y <- Y V_r, rows renormalised), then append one zero
  column per carried eigenvector (at most n_neg = 15 of them, p <= p_max;
  near a rank-one solution the factor then has 16 columns).  A column carried
  along a negative-curvature direction of size |lambda| only grows to about
  sqrt(|lambda| / sigma) relative to the leading one, so a larger threshold
  removes it at the next step before it can act on the certificate.
* inner tolerance: RTR for subproblem k stops at ||grad|| <= gtol_k with
  gtol_k = max(gtol_min, min(gtol0, gtol_ratio ||R^k|| / (1 + ||b||))), i.e. the
  subproblem is solved to a fixed fraction of the same scaled primal residual
  that eq. sec5:eq1 weighs against ||grad||; for k = 0 (no R yet) gtol0.  Then
  the two sides of eq. sec5:eq1 are measured on one scale, and the rule
  raises sigma when an outer step leaves the primal residual about where it
  was.  (With
  gtol_ratio <= 0 the older form min(gtol0, 0.1 eta_max^k, gtol_decay * previous)
  is used; there ||grad|| scales with eta_p while the rule divides ||R|| by
  1 + ||b||, so the decrease branch fires whenever 1 + ||b|| is large.)
  Optional stall cap: whenever RTR starts below its tolerance (takes no
  step) every later tolerance is capped at gtol_stall * ||grad|| (off by
  default).
* sigma constants: sigma_0 = 1, sigma_min = 1e-3, sigma_max = 1e6, gamma = 2,
  kappa_1 = 0.1, kappa_2 = 10 (the paper states none).  eq. sec5:eq1 weighs
  the scaled primal residual against ||grad Psi_k(Y^{k+1})|| as the dual
  residual of a (approximately) solved subproblem; when RTR stops at its
  iteration budget that norm measures the unfinished inner solve instead, so
  with sigma_hold (default) the decrease branch is not taken then (the
  increase branch and the rule after a solved subproblem are as printed;
  sigma_hold = False applies the rule as printed after every step).
* inner budget: the subproblem is solved approximately (Algorithm alg1 step
  3): at most rtr_maxiter = 10 RTR iterations of at most tcg_maxinner = 200
  truncated-CG steps, and rtr_maxiter_polish = 50 of at most
  tcg_maxinner_polish = 1000 once eta_max < polish_eta = 1e-4 (the polishing
  phase: near the solution the subproblem Hessian is ill-conditioned, and
  with 200 steps the inner gradient stalls above the tolerance, so the rule
  of eq. sec5:eq1 can never raise sigma).
* carried direction (step 9): formed after every outer step whose
  certificate has an eigenvalue below -max(neg_tol, tol) (1 + |lambda_max|)
  (curvature below the stopping tolerance's scale adds no columns); with
  escape_when_solved only after an RTR call that reached its tolerance.
* direct-DSDP ablation (option direct, section "Why solve DSDP' instead of
  DSDP"): the subproblem is eq. direct-ALM-subproblem with the stale y^k of
  the two-block ADMM; y^0 is the class average of the start point (the paper
  derives the subproblem from the second iteration on); the multiplier,
  sigma, rank and stopping steps are the same as for DSDP'.

Parity: not pinned on iterates; the result is pinned by brute force (q <= 16,
v <= min f, equality when rank S = 1), by the rank-one rounding certificate,
and by the invariants of Lemmas lm1 and sec3:lm1.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .operators import A_adj, D_matrix, Q_op, class_average
from .rtr import rtr
from .subproblem import DirectSubproblem, Subproblem, retract, rowdot

__all__ = ["ALMOptions", "ALMResult", "solve", "kkt_residuals", "rank_one_rounding"]


@dataclass
class ALMOptions:
    tol: float = 1e-8
    max_outer: int = 200
    sigma0: float = 1.0
    sigma_min: float = 1e-3
    sigma_max: float = 1e6
    gamma: float = 2.0
    kappa1: float = 0.1
    kappa2: float = 10.0
    p_max: int = 512
    n_neg: int = 15
    tau_rank: float = 1e-7
    gtol0: float = 1e-2
    gtol_min: float = 1e-10
    gtol_decay: float = 1.0
    gtol_ratio: float = 0.1
    gtol_stall: float = 0.0
    sigma_hold: bool = True
    escape_when_solved: bool = False
    direct: bool = False  # the direct-DSDP ADMM subproblem (ablation), see DirectSubproblem
    rtr_maxiter: int = 10
    rtr_maxiter_polish: int = 50
    tcg_maxinner: int = 200
    tcg_maxinner_polish: int = 1000
    rtr_stall: int = 0  # > 0: RTR also stops after this many iterations without progress
    polish_eta: float = 1e-4
    neg_tol: float = 1e-12
    round_rank_one: bool = True  # rank-one compression test (Remark rem:inexact-near-locking)
    round_eta: float = 1e-3      # ... tried once eta_max is below this
    round_gap: float = 0.1       # ... and s_2 <= round_gap s_1 (singular values of Y)


@dataclass
class ALMResult:
    Y: np.ndarray
    y: np.ndarray
    Xt: np.ndarray
    z: np.ndarray
    X: np.ndarray
    sigma: float
    value: float  # b^T y
    eta: tuple
    history: list = field(default_factory=list)


def kkt_residuals(S, y, X, z, b, cls, C=None, w=None):
    """eq. res: eta_p, eta_d, eta_g (Frobenius norms; eigenvalues by LAPACK)."""
    n = S.shape[0]
    Cm = np.zeros((n, n)) if C is None else C
    R = A_adj(y, cls, w) - S - Cm
    eta_p = float(np.linalg.norm(R) / (1.0 + np.linalg.norm(Cm)))
    ev = np.linalg.eigvalsh(X)
    eta_d = float(max(0.0, -ev[0]) / (1.0 + abs(ev[-1])))
    prim = float(np.sum(Cm * (X + np.diag(z))) + np.sum(z))
    dual = float(b @ y)
    eta_g = abs(prim - dual) / (1.0 + abs(prim) + abs(dual))
    return eta_p, eta_d, eta_g


def _escape(sub: Subproblem, Y: np.ndarray, U: np.ndarray) -> np.ndarray:
    f0 = sub.cost(Y)
    t = math.sqrt(Y.shape[0])
    while t > 1e-8:
        Yt = retract(Y, t * U)
        if sub.cost(Yt) < f0:
            return Yt
        t *= 0.5
    return Y


def _rank_one_candidate(Y, Xt, D, cls, counts, b, C, w, gap):
    """Rank-one compression of the current iterate, checked as a KKT point.

    Theorem thm:finite-locking: once the multiplier Xt is close enough to its
    limit, the rank-one solution S* is the unique minimiser of every later
    subproblem, its residual R is zero (so the multiplier stops moving) and
    (S*, y*, C_{S*}(Xt + D), z) satisfies the KKT system of DSDP.  Remark
    rem:inexact-near-locking: an inexact subproblem only brings S near S*, and
    a rank-one compression step can then land on S* exactly.  Reading: when
    Y's second singular value is at most gap times its first, take the
    leading left singular vector u of Y, the oblique-manifold point
    Y1 = sign(u) (rows of width 1; zeros to +1), and evaluate eq. res at
    S1 = Y1 Y1^T with the current multiplier Xt and no multiplier step:
    y1 = (A A^*)^{-1} A (S1 + C), z1 = diag((Xt + D) S1), X1 = Xt + D - Diag(z1).
    The caller accepts it only when that point meets the stopping tolerance,
    so a wrong guess costs one evaluation and never changes the iteration.
    Returns (Y1, y1, z1, X1, S1, eta1) or None when the gap test fails."""
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    if s.size > 1 and s[1] > gap * s[0]:
        return None
    Y1 = np.where(U[:, 0] >= 0.0, 1.0, -1.0)[:, None]
    S1 = Y1 @ Y1.T
    y1 = class_average(S1 if C is None else S1 + C, cls, counts, w)
    z1 = rowdot((Xt + D) @ Y1, Y1)
    X1 = Xt + D - np.diag(z1)
    return Y1, y1, z1, X1, S1, kkt_residuals(S1, y1, X1, z1, b, cls, C, w)


def rank_one_rounding(Y: np.ndarray, Q: np.ndarray, c: np.ndarray, order_basis: np.ndarray):
    """Read x_hat = sign(S[0, x_i]) from the leading row block of S = YY^T."""
    q = c.size
    s0 = Y[0] @ Y[1:1 + q].T
    x = np.where(s0 >= 0, 1.0, -1.0)
    return x, float(x @ Q @ x + c @ x)


def solve(cls: np.ndarray, counts: np.ndarray, b: np.ndarray, Y0: np.ndarray,
          opts: ALMOptions | None = None, C: np.ndarray | None = None,
          w: np.ndarray | None = None) -> ALMResult:
    opts = opts or ALMOptions()
    n = cls.shape[0]
    Xt = np.zeros((n, n))
    sigma = opts.sigma0
    Y = Y0 / np.linalg.norm(Y0, axis=1, keepdims=True)
    D = D_matrix(b, cls, counts, w)
    U = None
    eta_max = 1.0
    gtol = opts.gtol0 / opts.gtol_decay
    prim_ratio = None
    stall_cap = math.inf
    hist = []
    normb = float(np.linalg.norm(b))
    y = z = X = None
    eta = (np.inf, np.inf, np.inf)
    # direct-DSDP ablation: the stale dual iterate y^k of the two-block ADMM,
    # taken at the start point for k = 0 and after every multiplier update
    yk = class_average(Y @ Y.T + (0.0 if C is None else C), cls, counts, w) if opts.direct else None
    for k in range(opts.max_outer):
        if opts.direct:
            sub = DirectSubproblem(cls, counts, b, Xt, sigma, C, w, yk=yk)
        else:
            sub = Subproblem(cls, counts, b, Xt, sigma, C, w)
        if U is not None:
            Y = _escape(sub, Y, U)
        if opts.gtol_ratio > 0.0:
            g = opts.gtol0 if prim_ratio is None else min(opts.gtol0, opts.gtol_ratio * prim_ratio)
        else:
            g = min(opts.gtol0, 0.1 * eta_max, opts.gtol_decay * gtol)
        gtol = max(opts.gtol_min, min(g, stall_cap))
        polish = eta_max < opts.polish_eta
        budget = max(opts.rtr_maxiter, opts.rtr_maxiter_polish) if polish else opts.rtr_maxiter
        inner = max(opts.tcg_maxinner, opts.tcg_maxinner_polish) if polish else opts.tcg_maxinner
        res = rtr(sub, Y, gtol, maxiter=budget, maxinner=inner, max_stall=opts.rtr_stall)
        if opts.gtol_stall > 0.0 and res.iters == 0 and res.gradnorm > 0.0:
            stall_cap = min(stall_cap, opts.gtol_stall * res.gradnorm)
        Y = res.Y
        S = Y @ Y.T
        Z = S if C is None else S + C
        y = class_average(Z, cls, counts, w)
        if opts.direct:
            yk = y  # the y-update of the two-block ADMM (eq. direct-y-projection)
        Rq = Q_op(Z, cls, counts, w)  # = -(A* y - S - C)
        Xt = Xt + sigma * Rq
        z = rowdot((Xt + D) @ Y, Y)
        X = Xt + D - np.diag(z)
        evals, evecs = np.linalg.eigh(X)
        lmin, lmax = float(evals[0]), float(evals[-1])
        eta = kkt_residuals(S, y, X, z, b, cls, C, w)
        eta_max = max(eta)
        hist.append(dict(k=k, p=Y.shape[1], sigma=sigma, eta=eta, value=float(b @ y),
                         gradnorm=res.gradnorm, rtr_iters=res.iters, n_hvp=res.n_hvp,
                         lmin=lmin, lmax=lmax))
        if eta_max <= opts.tol:
            break
        if opts.round_rank_one and not opts.direct and eta_max < opts.round_eta:
            cand = _rank_one_candidate(Y, Xt, D, cls, counts, b, C, w, opts.round_gap)
            if cand is not None:
                hist[-1]["round_eta"] = cand[5]
                if max(cand[5]) <= opts.tol:
                    Y, y, z, X, S, eta = cand
                    hist.append(dict(k=k, p=1, sigma=sigma, eta=eta, value=float(b @ y), gradnorm=0.0,
                                     rtr_iters=0, n_hvp=0, rounded=True))
                    break
        unsolved = res.gradnorm > gtol  # RTR stopped at its iteration cap
        # negative-curvature directions (Theorem sec5:thm1)
        neg = np.nonzero(evals < -max(opts.neg_tol, opts.tol) * (1.0 + abs(lmax)))[0][: opts.n_neg]
        if opts.escape_when_solved and unsolved:
            neg = neg[:0]
        V = evecs[:, neg]
        for j in range(V.shape[1]):
            i = int(np.argmax(np.abs(V[:, j])))
            if V[i, j] < 0:
                V[:, j] = -V[:, j]
        # rank update
        _, s, Vt = np.linalg.svd(Y, full_matrices=False)
        r = max(1, int(np.sum(s > opts.tau_rank * s[0])))
        if r < Y.shape[1]:
            Y = Y @ Vt[:r].T
            Y = Y / np.linalg.norm(Y, axis=1, keepdims=True)
        d = min(V.shape[1], opts.p_max - Y.shape[1])
        if d > 0:
            Y = np.hstack([Y, np.zeros((n, d))])
            U = np.hstack([np.zeros((n, Y.shape[1] - d)), V[:, :d]])
        else:
            U = None
        # sigma rule, eq. sec5:eq1
        ratio = float(np.linalg.norm(Rq)) / (1.0 + normb)
        prim_ratio = ratio
        if ratio < opts.kappa1 * res.gradnorm and not (opts.sigma_hold and unsolved):
            sigma = max(sigma / opts.gamma, opts.sigma_min)
        elif ratio > opts.kappa2 * res.gradnorm:
            sigma = min(opts.gamma * sigma, opts.sigma_max)
    return ALMResult(Y=Y, y=y, Xt=Xt, z=z, X=X, sigma=sigma, value=float(b @ y),
                     eta=eta, history=hist)

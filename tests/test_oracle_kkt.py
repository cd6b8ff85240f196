"""Direct pins of the oracle's KKT residuals (eq. res), no GPU.

Each residual is compared with a value fixed in closed form at a point built
by hand, so that a wrong normalisation, a sign error or a swapped operand in
one of eta_p, eta_d, eta_g fails:

* a primal-dual optimal point: S = v(x) v(x)^T (a moment matrix, so
  A*(y(S)) = S), X0 = kappa (I - v v^T / ||v||^2) (PSD with X0 v = 0), any z0,
  and the data b := A(X0 + Diag z0) of the dual constraint (Lemma lm1).  Then
  b^T y = <X0 + Diag z0, S> = sum z0, so every eta is zero;
* one entry pair (a, b) of a class gamma moved by eps: Q(E) for
  E = eps (e_a e_b^T + e_b e_a^T) has ||Q(E)||^2 = 2 eps^2 (1 - 2/|gamma|), so
  eta_p = eps sqrt(2 (1 - 2/|gamma|)), and with C = E it is that divided by
  1 + ||C|| = 1 + eps sqrt(2);
* X = X0 - mu v v^T / ||v||^2 has lambda_min = -mu and lambda_max = kappa, so
  eta_d = mu / (1 + kappa);
* z = z0 + delta e_1: the primal value moves by delta and the dual does not, so
  eta_g = |delta| / (1 + |sum z0 + delta| + |sum z0|);
* the lower bound of lambda_min that deflation against range(Y) gives (the
  smaller eigenvalue of a 2 x 2 matrix of block bounds) against LAPACK.
"""

import numpy as np
import pytest

from oracle import bqp
from oracle.alm import kkt_residuals
from oracle.operators import A_op, class_average
from synth import bqp_instance, gaussian, gaussian_vector


def _optimal_point(q=5, order="colex", kappa=3.0):
    Q, c = bqp_instance(q, 11)
    rel = bqp.build_relaxation(Q, c, order)
    x = np.where(gaussian_vector(q, 12) >= 0, 1.0, -1.0)
    v = bqp.monomial_vector(x, order)
    S = np.outer(v, v)
    n = rel.n
    X0 = kappa * (np.eye(n) - np.outer(v, v) / (v @ v))
    z0 = gaussian_vector(n, 13)
    b = A_op(X0 + np.diag(z0), rel.cls, rel.m)
    y = class_average(S, rel.cls, rel.counts)
    return rel, v, S, X0, z0, b, y


def test_eta_zero_at_hand_built_optimal_pair():
    rel, v, S, X0, z0, b, y = _optimal_point()
    eta_p, eta_d, eta_g = kkt_residuals(S, y, X0, z0, b, rel.cls)
    assert eta_p <= 1e-14
    assert eta_d <= 1e-14
    assert eta_g <= 1e-14


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_eta_p_closed_form_one_entry_pair(degree):
    rel, v, S, X0, z0, b, y = _optimal_point()
    counts = rel.counts
    # an off-diagonal entry whose class has the requested degree
    off = bqp.class_offsets(5)
    ids = rel.cls
    a, bb = np.argwhere((ids >= off[degree]) & (ids < (off[degree + 1] if degree < 4 else rel.m))
                        & ~np.eye(rel.n, dtype=bool))[0]
    g = counts[ids[a, bb]]
    eps = 0.37
    E = np.zeros_like(S)
    E[a, bb] = E[bb, a] = eps
    S1 = S + E
    y1 = class_average(S1, rel.cls, counts)
    eta_p, _, _ = kkt_residuals(S1, y1, X0, z0, b, rel.cls)
    assert eta_p == pytest.approx(eps * np.sqrt(2.0 * (1.0 - 2.0 / g)), rel=1e-13)
    # with C = E the normalisation is 1 + ||C||_F and the residual is Q(S + C)
    y2 = class_average(S + E, rel.cls, counts)
    eta_p2, _, _ = kkt_residuals(S, y2, X0, z0, b, rel.cls, C=E)
    assert eta_p2 == pytest.approx(eps * np.sqrt(2.0 * (1.0 - 2.0 / g)) / (1.0 + eps * np.sqrt(2.0)), rel=1e-13)


def test_eta_d_closed_form():
    kappa, mu = 3.0, 0.25
    rel, v, S, X0, z0, b, y = _optimal_point(kappa=kappa)
    X = X0 - mu * np.outer(v, v) / (v @ v)
    _, eta_d, _ = kkt_residuals(S, y, X, z0, b, rel.cls)
    assert eta_d == pytest.approx(mu / (1.0 + kappa), rel=1e-13)


def test_eta_g_closed_form():
    rel, v, S, X0, z0, b, y = _optimal_point()
    delta = -0.8
    z = z0.copy()
    z[0] += delta
    _, _, eta_g = kkt_residuals(S, y, X0, z, b, rel.cls)
    s0 = z0.sum()
    assert eta_g == pytest.approx(abs(delta) / (1.0 + abs(s0 + delta) + abs(s0)), rel=1e-12)


def test_parity_bounds_catch_one_wrong_row():
    """The element-wise gate used by the GPU parity tests: an FP64
    recomputation in another order passes 1e-10, an FP32 one passes 1e-4 but
    not 1e-10, and one row with the penalty term dropped fails both."""
    from oracle.operators import Q_op
    from oracle.subproblem import Subproblem, proj_tangent
    from parity_bounds import bound_rhess, elem_err

    q, p, sigma = 6, 3, 1.4
    Q, c = bqp_instance(q, 2)
    rel = bqp.build_relaxation(Q, c, "colex")
    W = gaussian(rel.n, rel.n, 3)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Y = gaussian(rel.n, p, 4)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 5))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    ref = sub.rhess(Y, U)
    B = bound_rhess(sub, Y, U)
    # the same quantity, summed in reverse row order of the products
    perm = np.arange(rel.n)[::-1]
    sub_r = Subproblem(rel.cls[np.ix_(perm, perm)], rel.counts, rel.b, Xt[np.ix_(perm, perm)], sigma)
    alt = sub_r.rhess(Y[perm], U[perm])[np.argsort(perm)]
    assert elem_err(alt, ref, B) <= 1e-10
    f32 = Subproblem(rel.cls, rel.counts, rel.b, Xt.astype(np.float32).astype(np.float64), sigma)
    lo = f32.rhess(Y.astype(np.float32).astype(np.float64), U.astype(np.float32).astype(np.float64))
    e32 = elem_err(lo, ref, B)
    assert 1e-10 < e32 <= 1e-4
    # one row without the penalty part of the Euclidean Hessian
    bad = ref.copy()
    Wm = Y @ U.T + U @ Y.T
    pen = 2.0 * sigma * Q_op(Wm, rel.cls, rel.counts) @ Y
    row = 7
    bad[row] -= pen[row] - (pen[row] @ Y[row]) * Y[row]
    assert elem_err(bad, ref, B) > 1e-4


def test_deflated_eigenvalue_bound_is_a_lower_bound():
    """The bound a GPU solve ends on (deflation against range(Y)): for an
    orthonormal Q and X = [[A, B^T], [B, C]] in [Q, Q_perp], lambda_min(X) is at
    least the smaller eigenvalue of [[lambda_min(A), -||B||_2], [-||B||_2,
    lambda_min(C)]], which is itself at least Weyl's min(.) - ||B||_2, and is
    tight when B = 0.  Checked by LAPACK on random symmetric matrices, including
    the end-of-solve situation (range(Y) close to the bottom eigenvectors)."""
    rng = np.random.default_rng(17)
    for trial in range(60):
        n, r = 40, 1 + trial % 6
        M = rng.standard_normal((n, n))
        X = 0.5 * (M + M.T)
        if trial % 3 == 0:  # range(Q) near the bottom of the spectrum
            w, V = np.linalg.eigh(X)
            Q, _ = np.linalg.qr(V[:, :r] + 1e-3 * rng.standard_normal((n, r)))
        else:
            Q, _ = np.linalg.qr(rng.standard_normal((n, r)))
        P, _ = np.linalg.qr(np.hstack([Q, rng.standard_normal((n, n - r))]))
        Qp = P[:, r:]
        A = Q.T @ X @ Q
        B = Qp.T @ X @ Q
        Cc = Qp.T @ X @ Qp
        a, c = np.linalg.eigvalsh(A)[0], np.linalg.eigvalsh(Cc)[0]
        b = np.linalg.norm(B, 2)
        bound = 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + b * b)
        lmin = np.linalg.eigvalsh(X)[0]
        assert bound <= lmin + 1e-12
        assert bound >= min(a, c) - b - 1e-12
        # B^T B = (X Q)^T (X Q) - A^2 gives ||B||_2 without Q_perp
        G = (X @ Q).T @ (X @ Q) - A @ A
        assert abs(np.sqrt(max(0.0, np.linalg.eigvalsh(0.5 * (G + G.T))[-1])) - b) <= 1e-9 * (1 + b)
    # B = 0: the bound is exact
    X = np.diag(np.arange(1.0, 9.0))
    Q = np.eye(8)[:, :2]
    a, c = 1.0, 3.0
    assert 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2) == np.linalg.eigvalsh(X)[0]

"""Pins for the oracle's subproblem cost / gradient / Hessian (no GPU).

Each check is chosen so that a dropped term, a wrong sign or a transposed
operand in oracle/subproblem.py fails it:
* central differences of the cost along tangent directions (egrad / rgrad),
* central differences of egrad (ehess, both of its terms),
* second-order Taylor agreement along the retraction (rhess incl. -2 Diag(z) U),
* symmetry of rhess on the tangent space,
* grad = 2 X Y with X built from the certificate definition (Prop. prop),
* tangency of the gradient, and Theorem sec5:thm1 at [Y, 0].
"""

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import Q_op, class_average
from oracle.subproblem import Subproblem, proj_tangent, retract, rowdot
from synth import bqp_instance, gaussian


def _unit_rows(A):
    return A / np.linalg.norm(A, axis=1, keepdims=True)


@pytest.fixture(scope="module", params=[0.7, 3.0])
def setup(request):
    q, p = 6, 3
    Q, c = bqp_instance(q, 11)
    rel = bqp.build_relaxation(Q, c, "lex")
    n = rel.n
    # a multiplier with A(Xt) = 0, as the ALM iterates have (Lemma lm1)
    W = gaussian(n, n, 12)
    Xt = Q_op(W + W.T, rel.cls, rel.counts)
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, request.param)
    Y = _unit_rows(gaussian(n, p, 13))
    U = proj_tangent(Y, gaussian(n, p, 14))
    V = proj_tangent(Y, gaussian(n, p, 15))
    return sub, Y, U, V


def _inner(a, b):
    return float(np.sum(a * b))


def test_egrad_matches_central_difference(setup):
    sub, Y, U, _ = setup
    E = gaussian(*Y.shape, 21)  # any direction (Euclidean gradient)
    g = sub.egrad(Y)
    errs = []
    for h in (1e-3, 5e-4):
        fd = (sub.cost(Y + h * E) - sub.cost(Y - h * E)) / (2 * h)
        errs.append(abs(fd - _inner(g, E)))
    # O(h^2) truncation: halving h divides the error by about 4
    assert errs[1] < errs[0] / 3
    h = 1e-5
    fd = (sub.cost(Y + h * E) - sub.cost(Y - h * E)) / (2 * h)
    assert abs(fd - _inner(g, E)) <= 1e-7 * (1 + abs(fd))


def test_ehess_matches_difference_of_egrad(setup):
    sub, Y, U, _ = setup
    E = gaussian(*Y.shape, 22)
    H = sub.ehess(Y, E)
    h = 1e-5
    fd = (sub.egrad(Y + h * E) - sub.egrad(Y - h * E)) / (2 * h)
    assert np.linalg.norm(fd - H) <= 1e-6 * (1 + np.linalg.norm(H))


def test_rgrad_is_2XY_and_tangent(setup):
    sub, Y, _, _ = setup
    g = sub.rgrad(Y)
    X = sub.certificate(Y)
    np.testing.assert_allclose(g, 2 * X @ Y, rtol=0, atol=1e-11 * (1 + np.abs(g).max()))
    assert np.abs(rowdot(g, Y)).max() <= 1e-12 * (1 + np.abs(g).max())


def test_second_order_taylor_along_retraction(setup):
    sub, Y, U, _ = setup
    f0 = sub.cost(Y)
    g = sub.rgrad(Y)
    HU = sub.rhess(Y, U)
    errs = []
    for t in (1e-2, 5e-3, 2.5e-3):
        ft = sub.cost(retract(Y, t * U))
        model = f0 + t * _inner(g, U) + 0.5 * t * t * _inner(U, HU)
        errs.append(abs(ft - model))
    # third-order remainder: halving t divides the error by about 8
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5


def test_rhess_symmetric_on_tangent_space(setup):
    sub, Y, U, V = setup
    a = _inner(U, sub.rhess(Y, V))
    b = _inner(sub.rhess(Y, U), V)
    assert abs(a - b) <= 1e-10 * (1 + abs(a))
    assert np.abs(rowdot(sub.rhess(Y, U), Y)).max() <= 1e-10 * (1 + np.abs(sub.rhess(Y, U)).max())


def test_negative_curvature_direction_theorem(setup):
    """Theorem sec5:thm1: at Yhat = [Y, 0], U = [0, V] with V eigenvectors of X
    for negative eigenvalues gives <U, grad> = 0 and Hess[U] = 2 X U."""
    sub, Y, _, _ = setup
    n, p = Y.shape
    X = sub.certificate(Y)
    w, Vecs = np.linalg.eigh(X)
    assert w[0] < 0
    V = Vecs[:, :2] if w[1] < 0 else Vecs[:, :1]
    Yh = np.hstack([Y, np.zeros((n, V.shape[1]))])
    Uh = np.hstack([np.zeros((n, p)), V])
    g = sub.rgrad(Yh)
    assert abs(_inner(Uh, g)) <= 1e-12 * (1 + np.abs(g).max())
    H = sub.rhess(Yh, Uh)
    np.testing.assert_allclose(H, 2 * X @ Uh, rtol=0, atol=1e-11 * (1 + np.abs(X).max()))
    assert _inner(Uh, H) < 0


def test_direct_subproblem_pins():
    """Direct-DSDP (ADMM) subproblem of the ablation: its cost exceeds the
    reduced cost by exactly sigma/2 ||P(Z - Z^k)||^2 (eq. penalty-decomposition),
    its Hessian quadratic form by sigma ||P(Y U^T + U Y^T)||^2 (the extra
    sigma P curvature of eq. hessian-comparison, at a point where the
    two gradients' Diag(z) terms are taken into account), and its gradient and
    Hessian agree with central differences."""
    from oracle.operators import P_op
    from oracle.subproblem import DirectSubproblem

    q, p, sigma = 6, 3, 1.7
    Q, c = bqp_instance(q, 3)
    rel = bqp.build_relaxation(Q, c, "colex")
    W = gaussian(rel.n, rel.n, 4)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Yk = gaussian(rel.n, p, 5)
    Yk /= np.linalg.norm(Yk, axis=1, keepdims=True)
    yk = class_average(Yk @ Yk.T, rel.cls, rel.counts)
    red = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    dire = DirectSubproblem(rel.cls, rel.counts, rel.b, Xt, sigma, yk=yk)
    Y = gaussian(rel.n, p, 6)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    Z = Y @ Y.T
    extra = 0.5 * sigma * np.sum(P_op(Z - Yk @ Yk.T, rel.cls, rel.counts) ** 2)
    assert dire.cost(Y) - red.cost(Y) == pytest.approx(extra, rel=1e-11)
    U = proj_tangent(Y, gaussian(rel.n, p, 7))
    Wu = Y @ U.T + U @ Y.T
    de = np.sum(U * dire.ehess(Y, U)) - np.sum(U * red.ehess(Y, U))
    dG = dire.G(Y) - red.G(Y)  # = sigma P(Z - Z^k), class-constant
    assert de == pytest.approx(sigma * np.sum(P_op(Wu, rel.cls, rel.counts) ** 2) + 2 * np.sum(U * (dG @ U)),
                               rel=1e-10)
    # central differences of the cost along U and of egrad
    for h in (1e-3, 1e-4):
        fd = (dire.cost(Y + h * U) - dire.cost(Y - h * U)) / (2 * h)
        assert fd == pytest.approx(np.sum(dire.egrad(Y) * U), rel=1e-5)
        fdg = (dire.egrad(Y + h * U) - dire.egrad(Y - h * U)) / (2 * h)
        assert np.linalg.norm(fdg - dire.ehess(Y, U)) <= 1e-5 * np.linalg.norm(dire.ehess(Y, U))

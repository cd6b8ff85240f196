"""End-to-end pins for the oracle's Algorithm alg1 (no GPU).

* the relaxation value is <= the brute-force minimum of the BQP (it is a
  relaxation), and equals it when the solution has rank one (then S is a
  feasible moment matrix v(x)v(x)^T), which the paper reports for every dense
  BQP; the rounded sign vector attains the minimum;
* the stopping test eta_max <= 1e-8 (eq. res) is met;
* Lemma lm1 (A(Xt) = 0, A(X + Diag z) = b) and Lemma sec3:lm1 (<X, S> = 0) hold
  for the returned iterate;
* after the multiplier update the last subproblem's Riemannian gradient equals
  2 X^{k+1} Y^{k+1} where X^{k+1} uses Xt^{k+1} + D (the remark after the rank
  identification theorem, with D restored).
"""

import numpy as np
import pytest

from oracle import alm, bqp, brute
from oracle.operators import A_op, Q_op
from oracle.subproblem import Subproblem
from synth import bqp_instance, gaussian


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_q10_matches_brute_force(seed):
    q, p0 = 10, 2
    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c)
    res = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, p0, 100 + seed))
    fmin, _ = brute.brute_force_min(Q, c)
    assert max(res.eta) <= 1e-8
    assert res.value <= fmin + 1e-8 * (1 + abs(fmin))
    sv = np.linalg.svd(res.Y, compute_uv=False)
    assert sv.size == 1 or sv[1] <= 1e-3 * sv[0]  # numerically rank one
    assert abs(res.value - fmin) <= 1e-8 * (1 + abs(fmin))
    x, fx = alm.rank_one_rounding(res.Y, Q, c, None)
    assert abs(fx - fmin) <= 1e-9 * (1 + abs(fmin))


def test_invariants_of_returned_iterate():
    q = 8
    Q, c = bqp_instance(q, 5)
    rel = bqp.build_relaxation(Q, c)
    res = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 2, 105))
    S = res.Y @ res.Y.T
    scale = 1 + np.abs(res.Xt).max()
    assert np.abs(A_op(res.Xt, rel.cls, rel.m)).max() <= 1e-11 * scale * rel.n
    np.testing.assert_allclose(A_op(res.X + np.diag(res.z), rel.cls, rel.m), rel.b,
                               rtol=0, atol=1e-10 * scale * rel.n)
    assert abs(np.sum(res.X * S)) <= 1e-10 * scale * rel.n


def test_gradient_identity_after_multiplier_update():
    """grad Psi_k(Y^{k+1}) = 2 X^{k+1} Y^{k+1} with
    X^{k+1} = Xt^{k+1} + D - Diag(z^{k+1}), Xt^{k+1} = Xt^k + sigma Q(Z)."""
    q, p = 6, 3
    Q, c = bqp_instance(q, 9)
    rel = bqp.build_relaxation(Q, c)
    W = gaussian(rel.n, rel.n, 1)
    Xt = Q_op(W + W.T, rel.cls, rel.counts)
    sigma = 2.5
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    Y = gaussian(rel.n, p, 2)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    g = sub.rgrad(Y)
    Xt1 = Xt + sigma * Q_op(Y @ Y.T, rel.cls, rel.counts)
    D = sub.D
    z1 = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    X1 = Xt1 + D - np.diag(z1)
    np.testing.assert_allclose(g, 2 * X1 @ Y, rtol=0, atol=1e-11 * (1 + np.abs(g).max()))


@pytest.mark.parametrize("seed", [3, 4])
def test_q8_value_bounds(seed):
    Q, c = bqp_instance(8, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    res = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 3, 200 + seed))
    fmin, _ = brute.brute_force_min(Q, c)
    assert max(res.eta) <= 1e-8
    assert res.value <= fmin + 1e-8 * (1 + abs(fmin))


def test_adjoint_of_value_in_C_by_central_differences():
    """dv/dC = X + Diag z = Xt + D (Lagrangian duality: C enters the Lagrangian
    of DSDP as <X + Diag z, C>), checked by central differences of oracle
    re-solves at a generic strictly feasible C0 (zero diagonal, ||C0||_2 = 1/2)
    along a zero-diagonal E.  A dropped D or a sign error in the multiplier
    update fails it.  (At C = 0 the tight relaxation is degenerate and v has a
    kink along such E, so the point C0 is generic on purpose.)"""
    from oracle.operators import D_matrix

    q, seed, eps = 6, 3, 1e-4
    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    n = rel.n
    G = gaussian(n, n, 901)
    G = G + G.T
    np.fill_diagonal(G, 0.0)
    G *= 0.5 / np.max(np.abs(np.linalg.eigvalsh(G)))
    E = gaussian(n, n, 900)
    E = E + E.T
    np.fill_diagonal(E, 0.0)
    opts = alm.ALMOptions(tol=1e-11)
    Y0 = gaussian(n, 2, 100 + seed)
    r0 = alm.solve(rel.cls, rel.counts, rel.b, Y0, opts, C=G)
    pred = float(np.sum((r0.Xt + D_matrix(rel.b, rel.cls, rel.counts)) * E))
    vp = alm.solve(rel.cls, rel.counts, rel.b, Y0, opts, C=G + eps * E).value
    vm = alm.solve(rel.cls, rel.counts, rel.b, Y0, opts, C=G - eps * E).value
    fd = (vp - vm) / (2 * eps)
    assert abs(fd - pred) <= 1e-3 * (1 + abs(pred))

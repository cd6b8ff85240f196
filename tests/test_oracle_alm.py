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


def _rel_and_point(q, seed, order="colex"):
    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, order)
    fmin, xmin = brute.brute_force_min(Q, c)
    return Q, c, rel, fmin, np.asarray(xmin, dtype=float)


def test_rank_one_candidate_of_a_near_rank_one_moment_factor():
    """Remark rem:inexact-near-locking: the compression of a factor close to
    v(x) v(x)^T is v(x) itself (exact signs), and S1 = v(x) v(x)^T is a
    feasible moment matrix, so R = A*(y) - S1 = 0 and, for any multiplier Xt in
    the range of Q, <Xt, S1> = 0 and sum z = <D, S1> = b^T y: eta_p = eta_g = 0
    whatever Xt is (only eta_d depends on Xt)."""
    from oracle.operators import D_matrix

    q = 7
    Q, c, rel, fmin, xmin = _rel_and_point(q, 3)
    v = bqp.monomial_vector(xmin, "colex")
    rng = np.random.default_rng(11)
    Y = np.hstack([v[:, None], 0.05 * rng.standard_normal((rel.n, 3))])
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    W = rng.standard_normal((rel.n, rel.n))
    Xt = Q_op(W + W.T, rel.cls, rel.counts)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    cand = alm._rank_one_candidate(Y, Xt, D, rel.cls, rel.counts, rel.b, None, None, 0.1)
    assert cand is not None
    Y1, y1, z1, X1, S1, eta = cand
    assert Y1.shape == (rel.n, 1)
    assert np.array_equal(Y1[:, 0], v) or np.array_equal(Y1[:, 0], -v)
    assert eta[0] <= 1e-14 and eta[2] <= 1e-13
    # b^T y is the BQP objective at x (the relaxation's linear form on v(x) v(x)^T)
    assert abs(float(rel.b @ y1) - float(xmin @ Q @ xmin + c @ xmin)) <= 1e-12 * (1 + abs(fmin))
    # X1 v = 0 exactly (z is the row sum that cancels it), so lambda_min(X1) <= 0
    assert np.max(np.abs(X1 @ Y1[:, 0])) <= 1e-10 * (1 + np.max(np.abs(X1)))


def test_rank_one_candidate_gap_gate_and_infeasible_signs():
    """No candidate while s_2 > gap s_1; a sign pattern that is not a moment
    vector gives a nonzero primal residual, so the test can only reject it."""
    from oracle.operators import D_matrix

    Q, c, rel, fmin, xmin = _rel_and_point(6, 1)
    rng = np.random.default_rng(5)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    Xt = np.zeros((rel.n, rel.n))
    Y = rng.standard_normal((rel.n, 4))
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    assert alm._rank_one_candidate(Y, Xt, D, rel.cls, rel.counts, rel.b, None, None, 0.1) is None
    u = np.where(rng.standard_normal(rel.n) >= 0, 1.0, -1.0)
    u[0] = 1.0
    v = bqp.monomial_vector(xmin, "colex")
    if np.array_equal(u, v) or np.array_equal(u, -v):
        u[-1] = -u[-1]
    cand = alm._rank_one_candidate(u[:, None], Xt, D, rel.cls, rel.counts, rel.b, None, None, 0.1)
    assert cand is not None and cand[5][0] > 1e-3


@pytest.mark.parametrize("seed", [0, 1])
def test_rank_one_compression_does_not_change_the_optimum(seed):
    """With the compression test on (default) and off, the q = 10 solve ends
    at the brute-force minimum; when it accepts the compressed point that
    point meets eta_max <= 1e-8 and its factor is a sign vector."""
    Q, c, rel, fmin, xmin = _rel_and_point(10, seed)
    Y0 = gaussian(rel.n, 2, 100 + seed)
    on = alm.solve(rel.cls, rel.counts, rel.b, Y0, alm.ALMOptions(round_eta=1.0, round_gap=1.0))
    off = alm.solve(rel.cls, rel.counts, rel.b, Y0, alm.ALMOptions(round_rank_one=False))
    for r in (on, off):
        assert max(r.eta) <= 1e-8
        assert abs(r.value - fmin) <= 1e-8 * (1 + abs(fmin))
    if on.history[-1].get("rounded"):
        assert on.Y.shape[1] == 1 and np.all(np.abs(on.Y) == 1.0)
    assert len(on.history) <= len(off.history) + 1


@pytest.mark.parametrize("kw", [dict(sigma_hold=False), dict(escape_when_solved=True),
                                dict(rtr_maxiter=50, rtr_maxiter_polish=50), dict(rtr_stall=3),
                                dict(tcg_maxinner_polish=200, n_neg=16), dict(kappa1=0.01, kappa2=0.1),
                                dict(tau_rank=1e-4)])
def test_readings_of_the_outer_loop_reach_the_same_optimum(kw):
    """The sigma rule as printed (no hold), the escape gated on solved
    subproblems, one fixed RTR budget of 50 iterations, the RTR stall stop,
    the former polish budget and escape width, other sigma-rule constants and
    a lower rank threshold all end at the brute-force minimum at q = 10 with
    eta_max <= 1e-8: the readings change the path of the iteration, not its
    limit."""
    Q, c, rel, fmin, xmin = _rel_and_point(10, 2)
    r = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 2, 102), alm.ALMOptions(**kw))
    assert max(r.eta) <= 1e-8
    assert abs(r.value - fmin) <= 1e-8 * (1 + abs(fmin))

"""Pins of the UCQP (Hermitian) relaxation oracle, no GPU.

* class structure: the number of classes equals the number of distinct
  exponent differences alpha - beta (an independent set enumeration here),
  217,621 at q = 30 (the workload's stated count); every class has the
  coefficient pattern of the real embedding;
* feasibility and objective: for random z on the torus, S(z) = embed(v v^H) is
  a fixed point of P (Q(S) = 0), has unit diagonal, and b^T y(S(z)) = z^H Q z;
* projector identities with signed coefficients at random Z;
* end to end (Algorithm alg1 with the weighted operators): eta_max <= 1e-8 and
  the value is at most the minimum of z^H Q z found by a grid and a local
  refinement (q = 2, 3); when the solution has complex rank one the rounded
  z attains the value.
"""

import itertools

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import alm, ucqp
from oracle.operators import A_op, P_op, Q_op, class_average
from synth import gaussian, ucqp_instance


def _diff_count(q):
    B = [tuple([0] * q)]
    for i in range(q):
        B.append(tuple(1 if k == i else 0 for k in range(q)))
    for i in range(q):
        for j in range(i, q):
            B.append(tuple((k == i) + (k == j) for k in range(q)))
    return len({tuple(x - y for x, y in zip(a, b)) for a in B for b in B})


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6])
def test_class_count_matches_enumeration(q):
    rel = ucqp.build_relaxation(ucqp_instance(q, 0))
    assert rel.m == _diff_count(q)
    assert rel.nc == 1 + q + q * (q + 1) // 2
    # re classes: 2 entries per ordered (alpha, beta) pair; im classes: 2 per
    # pair with a nonzero difference; the 2 n_c imaginary-diagonal entries are free
    assert rel.counts.sum() == 2 * rel.nc ** 2 + 2 * (rel.nc ** 2 - rel.nc)
    assert np.all(rel.counts > 0)
    assert set(np.unique(rel.w)) <= {-1.0, 0.0, 1.0}
    assert np.count_nonzero(rel.w == 0) == 2 * rel.nc


def test_class_count_q30():
    rel = ucqp.build_relaxation(ucqp_instance(30, 0))
    assert rel.n == 992 and rel.m == 217621


@pytest.mark.parametrize("q,seed", [(2, 0), (3, 1), (5, 2)])
def test_feasible_point_and_objective(q, seed):
    Q = ucqp_instance(q, seed)
    rel = ucqp.build_relaxation(Q)
    rng = np.random.default_rng(seed + 10)
    for _ in range(3):
        z = np.exp(1j * rng.uniform(0, 2 * np.pi, q))
        v = ucqp.monomial_vector(z)
        S = ucqp.embed(np.outer(v, v.conj()))
        assert np.allclose(np.diag(S), 1.0, atol=1e-14)
        assert np.abs(Q_op(S, rel.cls, rel.counts, rel.w)).max() <= 1e-13
        y = class_average(S, rel.cls, rel.counts, rel.w)
        assert rel.b @ y == pytest.approx(ucqp.ucqp_value(Q, z), rel=1e-12, abs=1e-12)
        assert np.linalg.eigvalsh(S)[0] >= -1e-12


def test_projector_identities_signed():
    rel = ucqp.build_relaxation(ucqp_instance(3, 4))
    G = gaussian(rel.n, rel.n, 5)
    Z1 = G + G.T
    G = gaussian(rel.n, rel.n, 6)
    Z2 = G + G.T
    P1 = P_op(Z1, rel.cls, rel.counts, rel.w)
    assert np.allclose(P_op(P1, rel.cls, rel.counts, rel.w), P1, atol=1e-13)
    assert np.sum(P1 * Z2) == pytest.approx(np.sum(Z1 * P_op(Z2, rel.cls, rel.counts, rel.w)), rel=1e-12)
    assert np.abs(A_op(Q_op(Z1, rel.cls, rel.counts, rel.w), rel.cls, rel.m, rel.w)).max() <= 1e-12
    # a free (weight-0) entry is left entirely to Q
    Q1 = Q_op(Z1, rel.cls, rel.counts, rel.w)
    assert np.allclose(Q1[rel.w == 0], Z1[rel.w == 0])


def _torus_min(Q):
    q = Q.shape[0]

    def f(t):
        z = np.exp(1j * np.concatenate([[0.0], t]))
        return ucqp.ucqp_value(Q, z)

    grid = np.linspace(0, 2 * np.pi, 181)[:-1]
    best = min((f(np.array(t)), t) for t in itertools.product(grid, repeat=q - 1))
    r = minimize(f, np.array(best[1]), method="BFGS", options={"gtol": 1e-12})
    return min(best[0], r.fun)


@pytest.mark.parametrize("q,seed", [(2, 0), (3, 1), (3, 2)])
def test_solve_small_ucqp(q, seed):
    Q = ucqp_instance(q, seed)
    rel = ucqp.build_relaxation(Q)
    Y0 = gaussian(rel.n, 2, 100 + seed)
    res = alm.solve(rel.cls, rel.counts, rel.b, Y0, alm.ALMOptions(p_max=64), w=rel.w)
    fmin = _torus_min(Q)
    assert max(res.eta) <= 1e-8
    assert res.value <= fmin + 1e-7 * (1 + abs(fmin))
    sv = np.linalg.svd(res.Y, compute_uv=False)
    if sv.size <= 2 or sv[2] <= 1e-4 * sv[0]:  # complex rank one (real rank two)
        z, fz = ucqp.rank_one_rounding(res.Y, Q)
        assert abs(fz - res.value) <= 1e-7 * (1 + abs(res.value))

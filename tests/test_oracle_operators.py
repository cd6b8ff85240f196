"""Pins for the oracle's projector algebra (eq. projection-operators and the
variable projection of section 3), checked on random symmetric matrices."""

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import A_adj, A_op, D_matrix, P_op, Q_op, class_average
from synth import bqp_instance, gaussian


def _sym(n, seed):
    G = gaussian(n, n, seed)
    return G + G.T


@pytest.fixture(scope="module")
def rel():
    Q, c = bqp_instance(6, 3)
    return bqp.build_relaxation(Q, c, "lex")


def test_P_idempotent_and_self_adjoint(rel):
    Z1, Z2 = _sym(rel.n, 1), _sym(rel.n, 2)
    P1 = P_op(Z1, rel.cls, rel.counts)
    np.testing.assert_allclose(P_op(P1, rel.cls, rel.counts), P1, rtol=0, atol=1e-13 * np.abs(P1).max())
    a = np.sum(P1 * Z2)
    b = np.sum(Z1 * P_op(Z2, rel.cls, rel.counts))
    assert abs(a - b) <= 1e-12 * (abs(a) + 1)


def test_pythagoras_and_kernel(rel):
    Z = _sym(rel.n, 4)
    P = P_op(Z, rel.cls, rel.counts)
    Qz = Q_op(Z, rel.cls, rel.counts)
    lhs = np.sum(Z * Z)
    assert abs(lhs - np.sum(P * P) - np.sum(Qz * Qz)) <= 1e-12 * lhs
    # A(QZ) = 0 and Q(A* w) = 0
    assert np.abs(A_op(Qz, rel.cls, rel.m)).max() <= 1e-12 * np.abs(Z).sum()
    w = np.random.default_rng(0).standard_normal(rel.m)
    assert np.abs(Q_op(A_adj(w, rel.cls), rel.cls, rel.counts)).max() <= 1e-13


def test_projection_is_least_squares(rel):
    """y(S) minimises ||A* y - Z|| (footnote of section 3): the optimality
    residual A(A* y - Z) vanishes and perturbing y increases the distance."""
    Z = _sym(rel.n, 5)
    y = class_average(Z, rel.cls, rel.counts)
    base = np.linalg.norm(A_adj(y, rel.cls) - Z)
    rng = np.random.default_rng(1)
    for _ in range(5):
        dy = 1e-3 * rng.standard_normal(rel.m)
        assert np.linalg.norm(A_adj(y + dy, rel.cls) - Z) > base
    assert abs(base - np.linalg.norm(Q_op(Z, rel.cls, rel.counts))) <= 1e-12 * base


def test_D_inner_product_is_b_dot_y(rel):
    Z = _sym(rel.n, 6)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    y = class_average(Z, rel.cls, rel.counts)
    assert abs(np.sum(D * Z) - rel.b @ y) <= 1e-12 * (1 + abs(rel.b @ y))
    # A(D) = b
    np.testing.assert_allclose(A_op(D, rel.cls, rel.m), rel.b, rtol=1e-13, atol=1e-13)


def test_proximal_decomposition(rel):
    """||P(Z^k) - Z||^2 = ||P(Z - Z^k)||^2 + ||Q Z||^2 (section 3.2 comparison)."""
    Z, Zk = _sym(rel.n, 7), _sym(rel.n, 8)
    lhs = np.sum((P_op(Zk, rel.cls, rel.counts) - Z) ** 2)
    PZ = P_op(Z - Zk, rel.cls, rel.counts)
    Qz = Q_op(Z, rel.cls, rel.counts)
    rhs = np.sum(PZ * PZ) + np.sum(Qz * Qz)
    assert abs(lhs - rhs) <= 1e-12 * lhs

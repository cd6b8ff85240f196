"""Pins for the oracle's BQP relaxation builder (no GPU).

* class map == brute-force enumeration with Python frozensets, where the class
  of (alpha, beta) is the symmetric difference of the two index sets (x_i^2 = 1)
  and class ids come from sorting all subsets of size <= 4 by (size, colex);
* class count == eq. bqp-number-moments, moment count == eq.
  bqp-moment-number-constraints (golden file from the printed formulas);
* class sizes per degree; b reproduces f(x) on every sign vector;
* the class sums of a symmetric bilinear form of basis rows, per class degree,
  equal the pairing sums that the structured GPU class-sum kernels evaluate.
"""

import itertools
import os

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import D_matrix
from synth import bqp_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bqp_counts.txt")


def _golden_counts():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(tuple(int(t) for t in line.split()))
    return rows


def _brute_class_map(q, order):
    if order == "lex":
        pairs = [frozenset((i, j)) for i in range(q) for j in range(i + 1, q)]
    else:
        pairs = [frozenset((i, j)) for j in range(q) for i in range(j)]
    mons = [frozenset()] + [frozenset((i,)) for i in range(q)] + pairs
    subsets = [frozenset(s) for d in range(5) for s in itertools.combinations(range(q), d)]
    subsets.sort(key=lambda s: (len(s), sorted(s, reverse=True)))
    ids = {s: k for k, s in enumerate(subsets)}
    n = len(mons)
    full = np.empty((n, n), dtype=np.int64)
    for a in range(n):
        for b in range(n):
            full[a, b] = ids[mons[a] ^ mons[b]]
    return full, len(subsets)


@pytest.mark.parametrize("order", ["lex", "colex"])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 7])
def test_class_map_matches_set_enumeration(q, order):
    full, m = _brute_class_map(q, order)
    got = bqp.class_map_full(q, order)
    assert got.dtype == np.int32
    np.testing.assert_array_equal(got, full)
    assert int(bqp.class_offsets(q)[5]) == m


def test_counts_match_paper_closed_forms():
    for q, n, m_sos, m_mom in _golden_counts():
        assert bqp.m_sos_closed_form(q) == m_sos
        assert bqp.m_mom_closed_form(q) == m_mom
        assert bqp.basis(q).shape[0] == n
        assert int(bqp.class_offsets(q)[5]) == m_sos
        # the moment SDP ties every packed entry to its class moment, minus the
        # classes themselves, plus the normalisation y_{} = 1
        assert n * (n + 1) // 2 - m_sos + 1 == m_mom


@pytest.mark.parametrize("q", [3, 5, 8, 12])
def test_class_sizes_by_degree(q):
    cls = bqp.class_map_full(q)
    n = cls.shape[0]
    off = bqp.class_offsets(q)
    counts = np.bincount(cls.ravel(), minlength=int(off[5]))
    assert counts.sum() == n * n
    assert counts[0] == n
    assert np.all(counts[off[1]:off[2]] == 2 * q)
    assert np.all(counts[off[2]:off[3]] == 2 * q)
    assert np.all(counts[off[3]:off[4]] == 6)
    assert np.all(counts[off[4]:off[5]] == 6)
    # every class present in the packed map too, diagonal only in class 0
    assert np.all(np.diag(cls) == 0)
    assert np.count_nonzero(cls == 0) == n
    np.testing.assert_array_equal(cls, cls.T)


@pytest.mark.parametrize("order", ["lex", "colex"])
@pytest.mark.parametrize("q", [4, 7, 9])
def test_b_reproduces_objective_on_sign_vectors(q, order):
    Q, c = bqp_instance(q, seed=q)
    rel = bqp.build_relaxation(Q, c, order)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    rng = np.random.default_rng(7)
    for _ in range(20):
        x = rng.choice([-1.0, 1.0], size=q)
        v = bqp.monomial_vector(x, order)
        S = np.outer(v, v)
        # S = v v^T is feasible: diag 1 and entries constant on classes
        assert np.allclose(np.diag(S), 1.0)
        for g in range(rel.m):
            vals = S[rel.cls == g]
            assert np.all(vals == vals[0])
        assert abs(np.sum(D * S) - bqp.bqp_value(Q, c, x)) <= 1e-12 * (1 + abs(bqp.bqp_value(Q, c, x)))


def test_orders_are_a_permutation():
    q = 6
    lex = bqp.basis(q, "lex")
    colex = bqp.basis(q, "colex")
    key = lambda r: tuple(r)  # noqa: E731
    assert sorted(map(key, lex)) == sorted(map(key, colex))
    # colex lists pairs by larger index first
    pairs = colex[1 + q:]
    assert np.all(np.diff(pairs[:, 1]) >= 0)


@pytest.mark.parametrize("q", [4, 6, 9])
def test_class_sums_by_pairings(q):
    """The identities the structured class-sum kernels evaluate, checked
    against the oracle's class map: for a symmetric bilinear form
    B(r, s) = y_r . u_s + u_r . y_s of two basis rows (colex basis; rows
    indexed by index sets of size <= 2), the ordered class sum over the
    entries (r, s) with r ^ s = gamma equals
      {}         : sum_r B(r, r)
      {i}        : 2 [B({}, {i}) + sum_{j != i} B({j}, {i, j})]
      {i<j}      : 2 [B({}, {i,j}) + B({i}, {j}) + sum_{l != i,j} B({i,l}, {j,l})]
      {a<b<c}    : 2 [B({a}, {b,c}) + B({b}, {a,c}) + B({c}, {a,b})]
      {a<b<c<d}  : 2 [B({a,b}, {c,d}) + B({a,c}, {b,d}) + B({a,d}, {b,c})]."""
    rng = np.random.default_rng(q)
    rows = bqp.basis(q, "colex")
    n = rows.shape[0]
    mons = []
    for r in range(n):
        mons.append(frozenset(int(v) for v in rows[r] if v >= 0))
    row_of = {s: r for r, s in enumerate(mons)}
    p = 3
    Y = rng.standard_normal((n, p))
    U = rng.standard_normal((n, p))
    Bm = Y @ U.T + U @ Y.T

    def B(s1, s2):
        return Bm[row_of[frozenset(s1)], row_of[frozenset(s2)]]

    cls = bqp.class_map_full(q, "colex")
    m = int(cls.max()) + 1
    sums = np.zeros(m)
    np.add.at(sums, cls.ravel(), Bm.ravel())
    off = bqp.class_offsets(q)
    subsets = [frozenset(s) for d in range(5) for s in itertools.combinations(range(q), d)]
    subsets.sort(key=lambda s: (len(s), sorted(s, reverse=True)))
    assert len(subsets) == m
    for g, s in enumerate(subsets):
        e = sorted(s)
        if len(e) == 0:
            ref = float(np.trace(Bm))
        elif len(e) == 1:
            i = e[0]
            ref = 2 * (B((), (i,)) + sum(B((j,), (i, j)) for j in range(q) if j != i))
        elif len(e) == 2:
            i, j = e
            ref = 2 * (B((), (i, j)) + B((i,), (j,)) + sum(B((i, l), (j, l)) for l in range(q) if l not in (i, j)))
        elif len(e) == 3:
            a, b, c = e
            ref = 2 * (B((a,), (b, c)) + B((b,), (a, c)) + B((c,), (a, b)))
        else:
            a, b, c, d = e
            ref = 2 * (B((a, b), (c, d)) + B((a, c), (b, d)) + B((a, d), (b, c)))
        assert abs(sums[g] - ref) <= 1e-12 * (1 + abs(ref)), (g, e)
    assert off[-1] == m

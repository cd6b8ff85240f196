"""Order-2 moment relaxation of the dense BQP, in the DSDP form (oracle side).

Paper: section "Why solve the dual formulation", paragraph "Binary quadratic
programs" (problem BQP, the basis v(x), the SOS relaxation sec6:sos and the
count eq. bqp-number-moments); DSDP itself is the opening display of the
introduction.

The BQP is   min_x  x^T Q x + c^T x   s.t. x_i^2 = 1.
The basis v(x) lists 1, x_1..x_q, then the products x_i x_j (i < j).  The
paper lists the products lexicographically (x_1x_2, x_1x_3, ..., x_{q-1}x_q);
``order="lex"`` follows it.  ``order="colex"`` lists the same products by their
larger index first (x_1x_2, x_1x_3, x_2x_3, x_1x_4, ...); it is a permutation of
the basis and changes nothing else.

Entry (alpha, beta) of the moment matrix is the monomial x^alpha x^beta, which
modulo x_i^2 = 1 is x^(alpha XOR beta).  Entries sharing that symmetric
difference form one class; class gamma has the 0/1 indicator A_gamma, so
A(Z)_gamma = sum of Z over the class, AA* = Diag(|gamma|) and S = A*(y) is the
moment matrix M(y).  C = 0.  With f(x) = sum_gamma f_gamma x^gamma the
objective of DSDP is b^T y with b = f: b_{} = tr Q, b_{i} = c_i,
b_{ij} = 2 Q_ij, and b_gamma = 0 for |gamma| = 3, 4.

Class numbering (the paper fixes none; this is our convention, shared by the
GPU library through a bit-exact test, not through code): classes are ordered by
degree d = |gamma| in 0..4; within a degree by colex rank of the sorted index
set c_1 < ... < c_d (0-based), i.e.
    id(gamma) = off[d] + sum_{i=1..d} binom(c_i, i),
    off = [0, 1, 1+q, 1+q+C(q,2), 1+q+C(q,2)+C(q,3)].

Parity: the class map is pinned bit-exactly to a brute-force enumeration with
Python sets (tests), the class count to eq. bqp-number-moments, the moment
count to eq. bqp-moment-number-constraints, and b to f(x) = <D, v(x)v(x)^T>.
"""

from __future__ import annotations

from dataclasses import dataclass
from math import comb

import numpy as np

__all__ = [
    "BQPRelaxation",
    "basis",
    "class_offsets",
    "class_map_packed",
    "class_map_full",
    "build_relaxation",
    "m_sos_closed_form",
    "m_mom_closed_form",
    "bqp_value",
    "monomial_vector",
]


def basis(q: int, order: str = "lex") -> np.ndarray:
    """Monomials of v(x) as an (n, 2) int array of 0-based variable indices,
    -1 marking an absent factor.  Row 0 is the constant 1."""
    rows = [(-1, -1)]
    rows += [(i, -1) for i in range(q)]
    if order == "lex":
        rows += [(i, j) for i in range(q) for j in range(i + 1, q)]
    elif order == "colex":
        rows += [(i, j) for j in range(q) for i in range(j)]
    else:
        raise ValueError(f"unknown basis order {order!r}")
    return np.asarray(rows, dtype=np.int64)


def class_offsets(q: int) -> np.ndarray:
    off = np.zeros(6, dtype=np.int64)
    for d in range(5):
        off[d + 1] = off[d] + comb(q, d)
    return off  # off[5] = m


def _xor_class_ids(mon_a: np.ndarray, mon_b: np.ndarray, q: int) -> np.ndarray:
    """Class id of x^a x^b for arrays of monomials (k, 2) x (k, 2) -> (k,)."""
    v = np.concatenate([mon_a, mon_b], axis=1)  # (k, 4), -1 = absent
    v = np.sort(v, axis=1)
    k = v.shape[0]
    big = np.iinfo(np.int64).max
    pad_lo = np.full((k, 1), -2, dtype=np.int64)
    pad_hi = np.full((k, 1), big, dtype=np.int64)
    w = np.concatenate([pad_lo, v, pad_hi], axis=1)  # (k, 6)
    mid = w[:, 1:5]
    # a variable appears at most once in each monomial, so at most twice in
    # total; a repeated variable squares to one and drops out.
    keep = (mid >= 0) & (mid != w[:, 0:4]) & (mid != w[:, 2:6])
    deg = keep.sum(axis=1)
    # remaining indices, ascending, are the set gamma; rank them colex-wise
    rank = np.zeros(k, dtype=np.int64)
    pos = np.cumsum(keep, axis=1)  # 1-based position among kept entries
    binom_tab = np.zeros((q + 1, 5), dtype=np.int64)
    for c in range(q + 1):
        for i in range(5):
            binom_tab[c, i] = comb(c, i)
    for col in range(4):
        sel = keep[:, col]
        rank[sel] += binom_tab[mid[sel, col], pos[sel, col]]
    off = class_offsets(q)
    return off[deg] + rank


def class_map_packed(q: int, order: str = "lex") -> np.ndarray:
    """int32 class ids of the packed upper triangle of the n x n moment matrix,
    row-major (row a, columns a..n-1), length n(n+1)/2."""
    mon = basis(q, order)
    n = mon.shape[0]
    iu = np.triu_indices(n)
    out = np.empty(iu[0].size, dtype=np.int32)
    step = 1 << 22
    for s in range(0, out.size, step):
        a = iu[0][s:s + step]
        b = iu[1][s:s + step]
        out[s:s + step] = _xor_class_ids(mon[a], mon[b], q)
    return out


def class_map_full(q: int, order: str = "lex") -> np.ndarray:
    """Dense symmetric n x n int32 class map."""
    mon = basis(q, order)
    n = mon.shape[0]
    packed = class_map_packed(q, order)
    full = np.empty((n, n), dtype=np.int32)
    iu = np.triu_indices(n)
    full[iu] = packed
    full.T[iu] = packed
    return full


@dataclass
class BQPRelaxation:
    q: int
    order: str
    n: int
    m: int
    cls: np.ndarray  # dense n x n int32 class map
    counts: np.ndarray  # |gamma| = number of ordered entries per class (AA*)
    b: np.ndarray  # float64, length m
    C: np.ndarray | None  # None means C = 0
    Q: np.ndarray
    c: np.ndarray


def build_b(q: int, Q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """b = coefficient vector of f(x) = x^T Q x + c^T x reduced mod x_i^2 = 1."""
    off = class_offsets(q)
    m = int(off[5])
    b = np.zeros(m)
    b[0] = float(np.trace(Q))
    for i in range(q):
        b[off[1] + comb(i, 1)] = c[i]
    for i in range(q):
        for j in range(i + 1, q):
            b[off[2] + comb(i, 1) + comb(j, 2)] = Q[i, j] + Q[j, i]
    return b


def build_relaxation(Q: np.ndarray, c: np.ndarray, order: str = "lex") -> BQPRelaxation:
    q = c.size
    cls = class_map_full(q, order)
    m = int(class_offsets(q)[5])
    counts = np.bincount(cls.ravel(), minlength=m).astype(np.int64)
    b = build_b(q, Q, c)
    return BQPRelaxation(q=q, order=order, n=cls.shape[0], m=m, cls=cls, counts=counts,
                         b=b, C=None, Q=Q, c=c)


def m_sos_closed_form(q: int) -> int:
    """eq. bqp-number-moments: rank of A in the dual SOS form."""
    num = q**4 - 2 * q**3 + 11 * q**2 + 14 * q + 24
    assert num % 24 == 0
    return num // 24


def m_mom_closed_form(q: int) -> int:
    """eq. bqp-moment-number-constraints: affine constraints of the moment SDP."""
    num = q**4 + 4 * q**3 + 5 * q**2 + 2 * q + 12
    assert num % 12 == 0
    return num // 12


def bqp_value(Q: np.ndarray, c: np.ndarray, x: np.ndarray) -> float:
    return float(x @ Q @ x + c @ x)


def monomial_vector(x: np.ndarray, order: str = "lex") -> np.ndarray:
    """v(x) for a sign vector x, in the given basis order."""
    mon = basis(x.size, order)
    xa = np.where(mon[:, 0] >= 0, x[np.maximum(mon[:, 0], 0)], 1.0)
    xb = np.where(mon[:, 1] >= 0, x[np.maximum(mon[:, 1], 0)], 1.0)
    return xa * xb

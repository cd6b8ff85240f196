"""Hermitian order-2 moment relaxation of the unit-modulus quadratic program, as a
real DSDP with signed class coefficients (oracle side).

The problem is  min_z  z^H Q z  s.t. |z_i| = 1, z in C^q, Q Hermitian (the
paper's paragraph on unit-modulus complex quadratic programs; its experiments
use a real-coefficient reformulation, while this relaxation keeps the complex
moments).  The basis is v(z) = (z^alpha) over the exponents alpha in
{0, e_i, e_i + e_j (i <= j)}, n_c = 1 + q + q(q+1)/2, listed 1, z_1..z_q, then
z_i z_j (i <= j) lexicographically.  The moment matrix M = E[v v^H] has
M[alpha, beta] = z^(alpha - beta) on the torus (|z_i| = 1 turns conj(z_i) into
z_i^{-1}), so its entries are classed by the Laurent exponent difference
delta = alpha - beta, with M[beta, alpha] = conj(M[alpha, beta]).

Real embedding (n = 2 n_c): S = [[Re M, -Im M], [Im M, Re M]] is PSD iff M is,
diag S = 1 iff diag M = 1.  For each pair {gamma, -gamma} we keep the
representative gamma whose first nonzero component is positive (0 for
alpha = beta) and two real moments y_re(gamma) = Re z^gamma, y_im(gamma) =
Im z^gamma (gamma != 0).  An entry (alpha, beta) with delta = s gamma,
s = +-1, sits in
  * class re(gamma), coefficient +1, at (alpha, beta) and (n_c + alpha, n_c + beta);
  * class im(gamma), coefficient s at (n_c + alpha, beta) and -s at (alpha, n_c + beta);
and for delta = 0 the imaginary-part entries (n_c + alpha, alpha), (alpha, n_c + alpha)
belong to no class (coefficient 0: A*(y) is zero there, which forces Im M_{alpha alpha} = 0).
The A_gamma have disjoint supports, so AA* is diagonal (the sums of the squared
coefficients) and the variable projection and projectors apply as for 0/1
indicators (see operators.py).

Class ids (our convention; the paper fixes none): the representatives sorted
ascending as integer tuples (gamma = 0 first), re(gamma) = its rank,
im(gamma) = m_re + rank - 1.  m = 2 m_re - 1 (217,621 at q = 30).

Objective: z^H Q z = tr Q + sum_{i<j} 2 Re(Q_ij conj(z_i) z_j) and conj(z_i) z_j =
conj(z^gamma) for gamma = e_i - e_j, so b_re(0) = tr Q, b_re(e_i - e_j) = 2 Re Q_ij,
b_im(e_i - e_j) = 2 Im Q_ij, all other b zero; then b^T y(S(z)) = z^H Q z.

Parity: pinned (tests/test_oracle_ucqp.py) by an independent enumeration of the
exponent differences (class count), feasibility of S(z) = embed(v(z) v(z)^H)
with b^T y = z^H Q z on random points of the torus, the projector identities
with signed coefficients, and end-to-end solves against a grid-and-refine
minimum for q = 2, 3.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["basis", "UCQPRelaxation", "build_relaxation", "embed", "monomial_vector", "ucqp_value",
           "rank_one_rounding"]


def basis(q: int) -> np.ndarray:
    """Exponent vectors (n_c x q, int): 0, e_i, e_i + e_j (i <= j), lex order."""
    rows = [np.zeros(q, dtype=np.int64)]
    for i in range(q):
        e = np.zeros(q, dtype=np.int64)
        e[i] = 1
        rows.append(e)
    for i in range(q):
        for j in range(i, q):
            e = np.zeros(q, dtype=np.int64)
            e[i] += 1
            e[j] += 1
            rows.append(e)
    return np.array(rows)


def _canonical(d: tuple) -> tuple[tuple, int]:
    for x in d:
        if x != 0:
            return (d, 1) if x > 0 else (tuple(-v for v in d), -1)
    return d, 1


@dataclass
class UCQPRelaxation:
    q: int
    nc: int
    n: int          # 2 nc
    m: int
    m_re: int
    cls: np.ndarray     # n x n int32 class ids (0 where w == 0)
    w: np.ndarray       # n x n float64 coefficients in {+1, -1, 0}
    counts: np.ndarray  # m, sum of w^2 per class
    b: np.ndarray       # m
    reps: list          # class representatives gamma (re ids in order)


def build_relaxation(Q: np.ndarray) -> UCQPRelaxation:
    Q = np.asarray(Q, dtype=np.complex128)
    q = Q.shape[0]
    B = basis(q)
    nc = B.shape[0]
    n = 2 * nc
    canon = {}
    sign = np.zeros((nc, nc), dtype=np.int64)
    rep_of = [[None] * nc for _ in range(nc)]
    for a in range(nc):
        for c in range(nc):
            g, s = _canonical(tuple(int(v) for v in (B[a] - B[c])))
            rep_of[a][c] = g
            sign[a, c] = s
            canon[g] = True
    reps = sorted(canon)
    rank = {g: k for k, g in enumerate(reps)}
    m_re = len(reps)
    m = 2 * m_re - 1
    cls = np.zeros((n, n), dtype=np.int32)
    w = np.zeros((n, n), dtype=np.float64)
    for a in range(nc):
        for c in range(nc):
            k = rank[rep_of[a][c]]
            cls[a, c] = cls[nc + a, nc + c] = k
            w[a, c] = w[nc + a, nc + c] = 1.0
            if k != 0:  # gamma != 0 (rank 0 is the zero vector)
                s = float(sign[a, c])
                cls[nc + a, c] = cls[a, nc + c] = m_re + k - 1
                w[nc + a, c] = s
                w[a, nc + c] = -s
    counts = np.bincount(cls.ravel(), weights=(w * w).ravel(), minlength=m)
    b = np.zeros(m)
    b[0] = float(np.real(np.trace(Q)))
    for i in range(q):
        for j in range(i + 1, q):
            g = [0] * q
            g[i], g[j] = 1, -1
            k = rank[tuple(g)]
            b[k] += 2.0 * Q[i, j].real
            b[m_re + k - 1] += 2.0 * Q[i, j].imag
    return UCQPRelaxation(q=q, nc=nc, n=n, m=m, m_re=m_re, cls=cls, w=w, counts=counts, b=b, reps=reps)


def monomial_vector(z: np.ndarray) -> np.ndarray:
    """v(z) = (z^alpha) over the basis."""
    B = basis(z.size)
    return np.prod(np.power(z[None, :], B), axis=1)


def embed(M: np.ndarray) -> np.ndarray:
    """Real embedding [[Re M, -Im M], [Im M, Re M]] of a Hermitian matrix."""
    return np.block([[M.real, -M.imag], [M.imag, M.real]])


def ucqp_value(Q: np.ndarray, z: np.ndarray) -> float:
    return float(np.real(np.conj(z) @ Q @ z))


def rank_one_rounding(Y: np.ndarray, Q: np.ndarray) -> tuple[np.ndarray, float]:
    """z_i from the moment M[e_i, 0] = z_i of S = Y Y^T (entries (1 + i, 0) for
    the real part, (nc + 1 + i, 0) for the imaginary part), put on the unit
    circle; returns (z, z^H Q z)."""
    q = Q.shape[0]
    nc = Y.shape[0] // 2
    re = Y[1:1 + q] @ Y[0]
    im = Y[nc + 1:nc + 1 + q] @ Y[0]
    z = re + 1j * im
    z = z / np.abs(z)
    return z, ucqp_value(Q, z)

"""Linear operators of DSDP for class-indicator constraint matrices (oracle).

For moment relaxations every A_gamma is the 0/1 indicator of one class of
entries, the supports are pairwise disjoint, and so AA* is diagonal with the
class sizes |gamma| on its diagonal (remark list after Algorithm alg1: the
coefficient structure is orthogonal, so AA* is diagonal).  Hence

* A(Z)_gamma     = sum of Z_e over the ordered entries e of class gamma,
* A*(w)          = the matrix with w_gamma(e) in every entry e,
* y(S)           = (AA*)^{-1} A(S + C) = class averages of Z = S + C
                   (section 3 opening, the variable projection and its footnote),
* P = A*(AA*)^{-1}A,  Q = I - P  (eq. projection-operators): P replaces every
                   entry by the average of its class,
* D = A*(AA*)^{-1} b, so <D, S + C> = b^T y(S) (section 3 opening).

All functions take dense n x n float64 matrices and the dense int32 class map.
The optional dense weight matrix w (entries +1, -1 or 0) generalises the 0/1
indicators to A_gamma with signed unit entries on disjoint supports (an entry
of weight 0 is in no A_gamma, so A*(y) is zero there); then AA* = Diag of the
sums of w^2 over each class, and everything above holds with w_e y_gamma(e) in
place of y_gamma(e).  The signed case arises in the real embedding of a
Hermitian moment matrix, whose imaginary parts sit at +-1 in the two
off-diagonal blocks.
Parity: pinned by the identities P^2 = P, <PZ1, Z2> = <Z1, PZ2>,
||Z||^2 = ||PZ||^2 + ||QZ||^2, A(QZ) = 0, Q(A* w) = 0, <D, Z> = b^T y(Z)
(tests/test_oracle_operators.py), which fail for a wrong weight, a dropped
term or a transposed operand.
"""

from __future__ import annotations

import numpy as np

__all__ = ["A_op", "A_adj", "class_counts", "class_average", "P_op", "Q_op", "D_matrix"]


def A_op(Z: np.ndarray, cls: np.ndarray, m: int, w: np.ndarray | None = None) -> np.ndarray:
    """A(Z): class sums over all ordered entries (deterministic bincount),
    each entry weighted by its coefficient w_e in A_gamma (1 when w is None)."""
    vals = Z if w is None else w * Z
    return np.bincount(cls.ravel(), weights=vals.ravel(), minlength=m)


def A_adj(y: np.ndarray, cls: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """A*(y) = sum_gamma y_gamma A_gamma."""
    out = y[cls]
    return out if w is None else w * out


def class_counts(cls: np.ndarray, m: int, w: np.ndarray | None = None) -> np.ndarray:
    """Diagonal of AA*: ||A_gamma||_F^2 = sum of w_e^2 over the class."""
    vals = np.ones(cls.shape) if w is None else w * w
    return np.bincount(cls.ravel(), weights=vals.ravel(), minlength=m)


def class_average(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """(AA*)^{-1} A(Z)."""
    return A_op(Z, cls, counts.size, w) / counts


def P_op(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    return A_adj(class_average(Z, cls, counts, w), cls, w)


def Q_op(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    return Z - P_op(Z, cls, counts, w)


def D_matrix(b: np.ndarray, cls: np.ndarray, counts: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    return A_adj(b / counts, cls, w)

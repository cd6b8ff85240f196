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
Parity: pinned by the identities P^2 = P, <PZ1, Z2> = <Z1, PZ2>,
||Z||^2 = ||PZ||^2 + ||QZ||^2, A(QZ) = 0, Q(A* w) = 0, <D, Z> = b^T y(Z)
(tests/test_oracle_operators.py), which fail for a wrong weight, a dropped
term or a transposed operand.
"""

from __future__ import annotations

import numpy as np

__all__ = ["A_op", "A_adj", "class_average", "P_op", "Q_op", "D_matrix"]


def A_op(Z: np.ndarray, cls: np.ndarray, m: int) -> np.ndarray:
    """A(Z): class sums over all ordered entries (deterministic bincount)."""
    return np.bincount(cls.ravel(), weights=Z.ravel(), minlength=m)


def A_adj(w: np.ndarray, cls: np.ndarray) -> np.ndarray:
    """A*(w) = sum_gamma w_gamma A_gamma."""
    return w[cls]


def class_average(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """(AA*)^{-1} A(Z)."""
    return A_op(Z, cls, counts.size) / counts


def P_op(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray) -> np.ndarray:
    return A_adj(class_average(Z, cls, counts), cls)


def Q_op(Z: np.ndarray, cls: np.ndarray, counts: np.ndarray) -> np.ndarray:
    return Z - P_op(Z, cls, counts)


def D_matrix(b: np.ndarray, cls: np.ndarray, counts: np.ndarray) -> np.ndarray:
    return A_adj(b / counts, cls)

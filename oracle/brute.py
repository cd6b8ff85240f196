"""Exhaustive minimisation of the BQP over {-1, 1}^q (oracle, tiny q only).

The SDP relaxation's optimal value v satisfies v <= min_x f(x) (it is a
relaxation); when the optimal S has rank one it is a feasible moment matrix
v(x)v(x)^T and the two are equal.  Parity: this is the definition itself.
"""

from __future__ import annotations

import numpy as np

__all__ = ["brute_force_min"]


def brute_force_min(Q: np.ndarray, c: np.ndarray, chunk: int = 1 << 16):
    """Return (min value, minimiser x) over x in {-1, 1}^q, q <= 24."""
    q = c.size
    if q > 24:
        raise ValueError("brute force limited to q <= 24")
    best = np.inf
    best_x = None
    total = 1 << q
    bits = np.arange(q, dtype=np.int64)
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        X = 1.0 - 2.0 * ((idx[:, None] >> bits[None, :]) & 1)
        vals = np.einsum("ki,ij,kj->k", X, Q, X) + X @ c
        k = int(np.argmin(vals))
        if vals[k] < best:
            best = float(vals[k])
            best_x = X[k].copy()
    return best, best_x

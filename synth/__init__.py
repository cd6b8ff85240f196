"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no class maps, no projections, no normalisation). Every
consumer (the FP64 oracle, the GPU path, the tests) turns these raw draws into
its own objects with its own code.

Workload recipe (dense BQP of the numerical section, "Dense BQPs"): Q is a
symmetric q x q matrix whose off-diagonal entries are iid N(0,1) and whose
diagonal is zero, c has iid N(0,1) entries.  Draw order: c first (q values),
then the strictly-upper entries of Q in row-major (i < j) order, all from one
``numpy.random.default_rng(seed)`` (PCG64) stream.
"""

from __future__ import annotations

import numpy as np

__all__ = ["bqp_instance", "gaussian", "gaussian_vector", "sparse_bqp_instance", "ucqp_instance"]


def bqp_instance(q: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Return (Q, c): Q symmetric q x q, zero diagonal, iid N(0,1) off-diagonal;
    c iid N(0,1).  Both float64."""
    if q < 1:
        raise ValueError("q must be >= 1")
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(q)
    iu = np.triu_indices(q, k=1)
    vals = rng.standard_normal(iu[0].size)
    Q = np.zeros((q, q))
    Q[iu] = vals
    Q = Q + Q.T
    return Q, c


def sparse_bqp_instance(q: int, density: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Sparse-Q variant: each strictly-upper position is kept with probability
    ``density`` (uniform positions), values N(0,1), symmetric, zero diagonal."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(q)
    iu = np.triu_indices(q, k=1)
    keep = rng.random(iu[0].size) < density
    vals = rng.standard_normal(iu[0].size) * keep
    Q = np.zeros((q, q))
    Q[iu] = vals
    Q = Q + Q.T
    return Q, c


def ucqp_instance(q: int, seed: int) -> np.ndarray:
    """Hermitian q x q complex128 Q: real N(0,1) diagonal, strictly-upper
    entries iid complex Gaussian CN(0,1) (real and imaginary parts iid
    N(0, 1/2)), lower triangle the conjugate.  Draw order: the q diagonal
    values, then (re, im) of each strictly-upper entry in row-major order."""
    if q < 1:
        raise ValueError("q must be >= 1")
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(q)
    iu = np.triu_indices(q, k=1)
    ri = rng.standard_normal((iu[0].size, 2)) / np.sqrt(2.0)
    Q = np.zeros((q, q), dtype=np.complex128)
    Q[iu] = ri[:, 0] + 1j * ri[:, 1]
    Q = Q + Q.conj().T
    Q[np.diag_indices(q)] = d
    return Q


def gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """iid N(0,1) float64 matrix of shape (rows, cols), C order."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols))


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)

"""Element-wise parity gates for the GPU outputs (test helper).

For each output entry the gate compares |gpu - oracle| with a per-entry
magnitude bound built from absolute values of the operands that enter that
entry, so that a wrong entry (a dropped term, a wrong sign, a transposed
operand in one row) fails even when the Frobenius norm of the whole error is
small.  Rounding of any summation order is at most a small multiple of n eps
times this bound, so the 1e-10 bar for FP64 leaves a wide margin for
reordering and still catches a single wrong term.

With W = Y U^T + U Y^T and |.| taken entry-wise:
  |G|      <= |Xt| + |D| + sigma (|Z| + P|Z|)           (G = Xt + D + sigma Q(Z))
  egrad    : B_g = 2 |G| |Y|
  rgrad    : B_g + rowsum(B_g o |Y|) o |Y|
  ehess[U] : B_e = 2 |G| |U| + 2 sigma (|W| + P|W|) |Y|
  rhess[U] : B_e + rowsum(B_e o |Y|) o |Y| + 2 |z| o |U|
where P replaces an entry by its class average (here of absolute values, with
|w_e| for signed class coefficients).
"""

from __future__ import annotations

import numpy as np

from oracle.operators import D_matrix, P_op


def _aw(sub):
    """|w| of signed class coefficients (None for 0/1 indicators)."""
    w = getattr(sub, "w", None)
    return None if w is None else np.abs(w)


def _abs_G(sub, Y):
    Z = Y @ Y.T
    if sub.C is not None:
        Z = Z + sub.C
    aZ = np.abs(Z)
    aw = _aw(sub)
    return (np.abs(sub.Xt) + np.abs(D_matrix(sub.b, sub.cls, sub.counts, aw))
            + sub.sigma * (aZ + P_op(aZ, sub.cls, sub.counts, aw)))


def _project_bound(B, Y):
    aY = np.abs(Y)
    return B + np.sum(B * aY, axis=1, keepdims=True) * aY


def bound_egrad(sub, Y):
    return 2.0 * _abs_G(sub, Y) @ np.abs(Y)


def bound_rgrad(sub, Y):
    return _project_bound(bound_egrad(sub, Y), Y)


def bound_ehess(sub, Y, U):
    aY, aU = np.abs(Y), np.abs(U)
    aW = aY @ aU.T + aU @ aY.T
    return (2.0 * _abs_G(sub, Y) @ aU
            + 2.0 * sub.sigma * (aW + P_op(aW, sub.cls, sub.counts, _aw(sub))) @ aY)


def bound_rhess(sub, Y, U):
    z = np.einsum("ij,ij->i", sub.egrad(Y), Y) / 2.0
    return _project_bound(bound_ehess(sub, Y, U), Y) + 2.0 * np.abs(z)[:, None] * np.abs(U)


def elem_err(out, ref, bound):
    """max over entries of |out - ref| / bound (the gated figure)."""
    out = np.asarray(out)
    return float(np.max(np.abs(out - ref) / np.maximum(bound, 1e-300)))


def frob_rel(out, ref):
    """Frobenius-relative error (reported next to the gate)."""
    return float(np.linalg.norm(np.asarray(out) - ref) / max(np.linalg.norm(ref), 1e-300))

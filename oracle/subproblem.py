"""The factorised ALM subproblem Sub-k on the oblique manifold (oracle).

Paper references:
* cost: eq. reduced-ALM-subproblem,
      Psi(Y) = <D + Xt, Z> + sigma/2 ||Q(Z)||^2,   Z = Y Y^T + C.
  The literal L_sigma(S, y(S), Xt) equals this whenever A(Xt) = 0, which the
  multiplier update keeps (Lemma lm1); the reduced form is the one whose
  Euclidean gradient is exactly the formula of Lemma lm:suboptimality.
* Euclidean gradient in S (Lemma lm:suboptimality):
      G = grad Phi(S) = Xt + D - sigma (A* y(S) - S - C) = Xt + D + sigma Q(Z);
  in Y: egrad = 2 G Y.
* tangent space, projector (Lemma sec4:lm1): P_Y(U) = U - Diag(U Y^T) Y.
* Riemannian gradient (Proposition prop, eq. sec4:eq6): grad = 2 X Y with
      X = G - Diag(diag(G S)),  z = diag(G S) = rowdot(G Y, Y).
* Euclidean Hessian (Proposition prop): Ht = 2 G U + 2 sigma Q(Y U^T + U Y^T) Y.
* Riemannian Hessian (eq. sec4:eq7): Hess[U] = Ht - Diag(Ht Y^T) Y - 2 Diag(z) U.
* retraction: the paper does not name one; we use the standard one for the
  oblique manifold, R_Y(V) = rows of (Y + V) normalised to unit length.

Parity: pinned in tests/test_oracle_subproblem.py by central finite
differences of the cost and of egrad, second-order Taylor agreement along the
retraction, symmetry of Hess, grad = 2XY computed independently, tangency,
and Theorem sec5:thm1 (<U, grad> = 0 and Hess[U] = 2XU exactly at [Y, 0]).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .operators import A_adj, D_matrix, Q_op, class_average

__all__ = ["Subproblem", "DirectSubproblem", "proj_tangent", "retract", "rowdot"]


def rowdot(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    return np.einsum("ij,ij->i", A, B)


def proj_tangent(Y: np.ndarray, U: np.ndarray) -> np.ndarray:
    """P_Y(U) = U - Diag(U Y^T) Y (Lemma sec4:lm1)."""
    return U - rowdot(U, Y)[:, None] * Y


def retract(Y: np.ndarray, V: np.ndarray) -> np.ndarray:
    W = Y + V
    return W / np.linalg.norm(W, axis=1, keepdims=True)


@dataclass
class Subproblem:
    """Psi_k for fixed (Xt, sigma) of one ALM iteration."""

    cls: np.ndarray
    counts: np.ndarray
    b: np.ndarray
    Xt: np.ndarray  # dense symmetric n x n
    sigma: float
    C: np.ndarray | None = None
    w: np.ndarray | None = None  # signed unit coefficients of the A_gamma (None: 0/1 indicators)

    def __post_init__(self):
        self.D = D_matrix(self.b, self.cls, self.counts, self.w)

    # --- plain definitions -------------------------------------------------
    def Z(self, Y: np.ndarray) -> np.ndarray:
        S = Y @ Y.T
        return S if self.C is None else S + self.C

    def cost(self, Y: np.ndarray) -> float:
        Z = self.Z(Y)
        R = Q_op(Z, self.cls, self.counts, self.w)
        return float(np.sum((self.D + self.Xt) * Z) + 0.5 * self.sigma * np.sum(R * R))

    def G(self, Y: np.ndarray) -> np.ndarray:
        Z = self.Z(Y)
        return self.Xt + self.D + self.sigma * Q_op(Z, self.cls, self.counts, self.w)

    def egrad(self, Y: np.ndarray) -> np.ndarray:
        return 2.0 * self.G(Y) @ Y

    def z(self, Y: np.ndarray) -> np.ndarray:
        return rowdot(self.G(Y) @ Y, Y)

    def certificate(self, Y: np.ndarray) -> np.ndarray:
        """X = grad Phi(S) - Diag(diag(grad Phi(S) S))."""
        G = self.G(Y)
        return G - np.diag(np.diag(G @ (Y @ Y.T)))

    def rgrad(self, Y: np.ndarray) -> np.ndarray:
        return proj_tangent(Y, self.egrad(Y))

    def ehess(self, Y: np.ndarray, U: np.ndarray) -> np.ndarray:
        Zu = Y @ U.T + U @ Y.T
        return 2.0 * self.G(Y) @ U + 2.0 * self.sigma * Q_op(Zu, self.cls, self.counts, self.w) @ Y

    def rhess(self, Y: np.ndarray, U: np.ndarray) -> np.ndarray:
        Ht = self.ehess(Y, U)
        return proj_tangent(Y, Ht) - 2.0 * self.z(Y)[:, None] * U

    def class_avg(self, Y: np.ndarray) -> np.ndarray:
        """y(S) = class averages of Z."""
        return class_average(self.Z(Y), self.cls, self.counts, self.w)


@dataclass
class DirectSubproblem(Subproblem):
    """S-subproblem of the two-block ADMM applied directly to DSDP (section
    "Why solve DSDP' instead of DSDP", eq. direct-ALM-subproblem): with the
    multiplier written as D + Xt (eq. shifted-direct-multiplier) and the stale
    dual iterate y^k entering through A*(y^k) = P(Z^k) (eq. direct-y-projection),

        Psi_dir(Y) = <D + Xt, Z> + sigma/2 ||Z - P(Z^k)||^2,

    i.e. the reduced cost plus sigma/2 ||P(Z - Z^k)||^2 (eq. penalty-decomposition).
    Its gradient in S is G = Xt + D + sigma (Z - P(Z^k)) and its Hessian in S is
    sigma I instead of sigma Q (eq. hessian-comparison), so in Y
        egrad = 2 G Y,   ehess[U] = 2 G U + 2 sigma (Y U^T + U Y^T) Y.
    yk holds the class averages y^k of Z^k; the projections use its class map.
    Parity: pinned by the penalty decomposition against the reduced cost, the
    Hessian difference sigma ||P(Y U^T + U Y^T)||^2, and finite differences."""

    yk: np.ndarray | None = None

    def G(self, Y: np.ndarray) -> np.ndarray:
        Z = self.Z(Y)
        PZk = A_adj(self.yk, self.cls, self.w)
        return self.Xt + self.D + self.sigma * (Z - PZk)

    def cost(self, Y: np.ndarray) -> float:
        Z = self.Z(Y)
        E = Z - A_adj(self.yk, self.cls, self.w)
        return float(np.sum((self.D + self.Xt) * Z) + 0.5 * self.sigma * np.sum(E * E))

    def ehess(self, Y: np.ndarray, U: np.ndarray) -> np.ndarray:
        Zu = Y @ U.T + U @ Y.T
        return 2.0 * self.G(Y) @ U + 2.0 * self.sigma * Zu @ Y

"""GPU checks of the failure paths and of the certificate eigensolver.

* non-finite values are values, not faults: NaN written from the host into Y,
  U or the multiplier makes the kernels raise the sticky flag, which
  mdsdp_sync_status reports as MDSDP_ENONFINITE; set_multiplier clears it;
  a solve from a NaN start returns MDSDP_ENONFINITE;
* iteration and time caps: max_outer = 1 and a time limit shorter than one
  outer step end the solve with MDSDP_ENOCONV after exactly one outer step;
* the k smallest eigenpairs of the certificate (eq. res, Theorem sec5:thm1)
  against LAPACK on the oracle's dense X, and the solver's own eigenvalue
  estimate (warm start, gap-based error) against LAPACK at n = 821 and at the
  full size n = 5051: the true lambda_min lies within the reported error of
  the Ritz value.
"""

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import D_matrix, Q_op
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _small(q=8, p=3):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c = bqp_instance(q, 2)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    Y = gaussian(prob.n, p, 3)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    return prob, Y


def test_nan_in_Y_and_U_flagged_and_cleared():
    from paper_2512_04406_amd._lib import MdsdpError
    from paper_2512_04406_amd.problem import FP32, FP64

    prob, Y = _small()
    print("[status] nan in Y / U", flush=True)
    prob.set_multiplier(None, 1.0)
    Yt = _t(Y)
    prob.cost_grad(Yt)
    prob.sync_status()  # clean state
    U = gaussian(prob.n, Y.shape[1], 4)
    U[5, 1] = np.nan
    for prec in (FP64, FP32):
        prob.set_multiplier(None, 1.0)
        prob.cost_grad(Yt)
        prob.hvp(Yt, _t(U), prec)
        with pytest.raises(MdsdpError) as e:
            prob.sync_status()
        assert e.value.code == -5
    Yn = Y.copy()
    Yn[2, 0] = np.nan
    prob.set_multiplier(None, 1.0)
    prob.sync_status()
    prob.cost_grad(_t(Yn))
    with pytest.raises(MdsdpError) as e:
        prob.sync_status()
    assert e.value.code == -5
    prob.set_multiplier(None, 1.0)  # a new multiplier clears the flag
    prob.cost_grad(Yt)
    prob.sync_status()


def test_nan_in_multiplier_flagged():
    from paper_2512_04406_amd._lib import MdsdpError

    prob, Y = _small()
    print("[status] nan in Xt", flush=True)
    X = np.zeros((prob.n, prob.n))
    X[3, 7] = X[7, 3] = np.inf
    prob.set_multiplier(_t(X), 1.0)
    with pytest.raises(MdsdpError) as e:
        prob.sync_status()
    assert e.value.code == -5


def test_solve_from_nan_start_returns_enonfinite():
    from paper_2512_04406_amd._lib import MdsdpError

    prob, Y = _small()
    print("[status] solve from NaN", flush=True)
    Y[0, 0] = np.nan
    with pytest.raises(MdsdpError) as e:
        prob.solve(_t(Y))
    assert e.value.code == -5


@pytest.mark.parametrize("cap", ["max_outer", "time_limit"])
def test_caps_end_with_enoconv(cap):
    prob, Y = _small(q=12, p=2)
    print(f"[status] cap {cap}", flush=True)
    o = prob.default_options()
    if cap == "max_outer":
        o.max_outer = 1
    else:
        o.time_limit_s = 1e-9
    r = prob.solve(_t(Y), o)
    assert r.status == -7
    assert r.outer_iters == 1
    assert max(r.eta) > o.tol


def _certificate(q, p, seed=1):
    """A problem after one multiplier update at a random point, and the
    oracle's dense certificate X there."""
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    W = gaussian(rel.n, rel.n, 5)
    Xt = Q_op(0.2 * (W + W.T), rel.cls, rel.counts)
    del W
    sigma = 1.3
    Y = gaussian(rel.n, p, 6)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), sigma)
    prob.update_multiplier(_t(Y))
    Xt1 = Xt + sigma * Q_op(Y @ Y.T, rel.cls, rel.counts)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    z = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    X = Xt1 + D - np.diag(z)
    return prob, X


@pytest.mark.parametrize("q,p,k", [(8, 2, 4), (12, 3, 3)])
def test_k_smallest_eigenpairs_match_lapack(q, p, k):
    prob, X = _certificate(q, p)
    print(f"[eig-k] q={q} n={X.shape[0]} k={k}", flush=True)
    w, V = np.linalg.eigh(X)
    ev, lmax, vecs, it, conv = prob.min_eigpairs(k, tol=1e-11, maxit=X.shape[0])
    assert conv
    scale = 1 + abs(w[-1])
    np.testing.assert_allclose(ev, w[:k], rtol=0, atol=1e-9 * scale)
    assert abs(lmax - w[-1]) <= 1e-9 * scale
    vv = vecs.cpu().numpy()
    for i in range(k):
        r = X @ vv[i] - ev[i] * vv[i]
        assert np.linalg.norm(r) <= 1e-8 * scale
        assert abs(np.linalg.norm(vv[i]) - 1.0) <= 1e-10


@pytest.mark.parametrize("q,p", [(40, 4), (100, 16)])
def test_solver_eigen_estimate_brackets_lapack(q, p):
    """The estimate the solver feeds into eta_d: theta_min (Ritz value) with
    the error it reports (residual, or residual^2 / certified gap), from a warm
    start.  The true lambda_min must lie in [theta_min - err, theta_min]
    (Ritz values of the smallest end never undershoot), whether or not the
    Lanczos run converged; theta_max must not exceed lambda_max."""
    prob, X = _certificate(q, p)
    n = X.shape[0]
    print(f"[eig-est] q={q} n={n}", flush=True)
    w = np.linalg.eigvalsh(X)
    est = prob.certificate_estimate(tol=1e-10, maxit=300, seed=3, warm=None)
    # a second call warm-started from the first Ritz vector, as in the solver
    est2 = prob.certificate_estimate(tol=1e-10, maxit=60, seed=4, warm=est["evec"])
    for e in (est, est2):
        th, err = e["theta_min"], e["err"]
        print(f"   theta_min={th:.6e} err={err:.2e} conv={e['converged']} lapack={w[0]:.6e}", flush=True)
        assert th >= w[0] - 1e-9 * (1 + abs(w[-1]))
        assert w[0] >= th - err - 1e-9 * (1 + abs(w[-1]))
        # theta_max is a Ritz value too: never above lambda_max, so the
        # denominator 1 + |theta_max| of eta_d errs on the large-eta side
        # (for lambda_max > 0, as here)
        assert e["theta_max"] <= w[-1] + 1e-9 * (1 + abs(w[-1]))


@pytest.mark.parametrize("q,p,near", [(12, 3, False), (20, 4, False), (20, 4, True)])
def test_certificate_bound_below_lapack(q, p, near):
    """mdsdp_certificate_bound (the eta_d a solve ends on): Lanczos on the
    complement of range(Y) combined with the compression to range(Y) through
    the 2 x 2 bound; it must never exceed LAPACK's lambda_min of the dense
    certificate.  `near`: Y spans eigenvectors of X near its bottom (the
    situation at the end of a solve), where the bound must also be close."""
    prob, X = _certificate(q, p)
    n = X.shape[0]
    w, V = np.linalg.eigh(X)
    if near:
        Y = V[:, :p] + 1e-6 * gaussian(n, p, 9)
    else:
        Y = gaussian(n, p, 8)
    print(f"[cert-bound] q={q} n={n} p={p} near={near}", flush=True)
    b = prob.certificate_bound(_t(Y), tol=1e-11, maxit=n)
    scale = 1 + abs(w[-1])
    print(f"   lower={b['lower']:.6e} lapack={w[0]:.6e} conv={b['converged']} iters={b['iters']}", flush=True)
    assert b["lower"] <= w[0] + 1e-9 * scale
    assert b["theta_max"] <= w[-1] + 1e-9 * scale
    if near:
        assert b["lower"] >= w[0] - 1e-5 * scale

"""GPU checks of the direct-DSDP (two-block ADMM) subproblem used for the
ablation of section "Why solve DSDP' instead of DSDP".

* parity against the oracle's DirectSubproblem (eq. direct-ALM-subproblem):
  cost, Euclidean and Riemannian gradients and HVPs entry by entry, with the
  stale class averages y^k taken at another point Y^k;
* the ADMM solve (direct_admm) at a fixed penalty reaches the brute-force
  minimum (q = 8) and the oracle's direct ADMM value.
"""

import numpy as np
import pytest

from oracle import alm, bqp, brute
from oracle.operators import A_adj, D_matrix, Q_op, class_average
from oracle.subproblem import DirectSubproblem, proj_tangent
from parity_bounds import elem_err
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("q,p", [(6, 3), (12, 16), (20, 40)])
def test_direct_subproblem_parity(q, p):
    from paper_2512_04406_amd.problem import FP32, FP64, ORDER_COLEX, Problem

    sigma = 1.4
    Q, c = bqp_instance(q, 2)
    rel = bqp.build_relaxation(Q, c, "colex")
    print(f"[direct] q={q} n={rel.n} p={p}", flush=True)
    W = gaussian(rel.n, rel.n, 3)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Yk = gaussian(rel.n, p, 4)
    Yk /= np.linalg.norm(Yk, axis=1, keepdims=True)
    Y = gaussian(rel.n, p, 5)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 6))
    yk = class_average(Yk @ Yk.T, rel.cls, rel.counts)
    sub = DirectSubproblem(rel.cls, rel.counts, rel.b, Xt, sigma, yk=yk)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), sigma)
    prob.set_direct(True, _t(Yk))
    Yt, Ut = _t(Y), _t(U)
    f, eg, rg = prob.cost_grad(Yt)
    h64 = prob.hvp(Yt, Ut, FP64)
    h32 = prob.hvp(Yt, Ut, FP32)
    torch.cuda.synchronize()
    aY, aU = np.abs(Y), np.abs(U)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    aG = np.abs(Xt) + np.abs(D) + sigma * (np.abs(Y @ Y.T) + np.abs(A_adj(yk, rel.cls)))
    Bg = 2.0 * aG @ aY
    Bg = Bg + np.sum(Bg * aY, axis=1, keepdims=True) * aY
    Be = 2.0 * aG @ aU + 2.0 * sigma * (aY @ aU.T + aU @ aY.T) @ aY
    z = np.einsum("ij,ij->i", sub.G(Y) @ Y, Y)
    Br = Be + np.sum(Be * aY, axis=1, keepdims=True) * aY + 2.0 * np.abs(z)[:, None] * aU
    assert abs(f.item() - sub.cost(Y)) <= 1e-10 * (1 + abs(sub.cost(Y)))
    assert elem_err(eg.cpu().numpy(), sub.egrad(Y), 2.0 * aG @ aY) <= 1e-10
    assert elem_err(rg.cpu().numpy(), sub.rgrad(Y), Bg) <= 1e-10
    rh = sub.rhess(Y, U)
    e64, e32 = elem_err(h64.cpu().numpy(), rh, Br), elem_err(h32.cpu().numpy(), rh, Br)
    print(f"   elem rhess fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
    assert e64 <= 1e-10 and e32 <= 1e-4
    # back to the variable-projected subproblem: the reduced HVP again
    prob.set_direct(False)
    from oracle.subproblem import Subproblem

    red = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    prob.cost_grad(Yt)
    hr = prob.hvp(Yt, Ut, FP64)
    torch.cuda.synchronize()
    assert np.linalg.norm(hr.cpu().numpy() - red.rhess(Y, U)) <= 1e-10 * np.linalg.norm(red.rhess(Y, U))
    prob.close()


def test_direct_admm_solve_q8():
    from paper_2512_04406_amd.problem import FP64, ORDER_COLEX, Problem

    q = 8
    Q, c = bqp_instance(q, 0)
    rel = bqp.build_relaxation(Q, c, "colex")
    fmin, _ = brute.brute_force_min(Q, c)
    kw = dict(sigma0=0.01, kappa1=1e-12, kappa2=1e12, escape_when_solved=False)
    ref = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 2, 100), alm.ALMOptions(direct=True, **kw))
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    o = prob.default_options()
    o.direct_admm = 1
    o.hvp_prec = FP64
    o.sigma0, o.kappa1, o.kappa2, o.escape_when_solved = 0.01, 1e-12, 1e12, 0
    res = prob.solve(_t(gaussian(rel.n, 2, 100)), o)
    print(f"[direct] q=8 value={res.value:.12f} oracle={ref.value:.12f} fmin={fmin:.12f} eta={max(res.eta):.1e} "
          f"outer={res.outer_iters}", flush=True)
    assert res.status == 0 and max(res.eta) <= 1e-8
    assert abs(res.value - fmin) <= 1e-8 * (1 + abs(fmin))
    assert abs(ref.value - fmin) <= 1e-8 * (1 + abs(fmin))
    prob.close()

"""Parity at full size: dense BQP q = 100 (n = 5051, m = 4,087,976), the
headline size, and sparse-Q BQP q = 120 (n = 7261, m = 8,502,671).

The dense FP64 oracle handles this size in seconds (n x n arrays of 204 MB),
so every output is compared element by element, not sampled.  The launch
configuration is the one the benchmark times: structured class sums (colex
basis), factor width p = 16 (staged width 16), and also p = 40 (staged width
64) and p = 128 (the sliced FP64 HVP).  Bars: FP64 results 1e-10 of a
per-entry magnitude bound, entry by entry (tests/parity_bounds.py; the
Frobenius-relative error is printed beside it), class averages 1e-12 absolute,
FP32-tile HVP 1e-4 of the same bound.
"""

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import D_matrix, Q_op, class_average
from oracle.subproblem import Subproblem, proj_tangent
from parity_bounds import bound_egrad, bound_ehess, bound_rgrad, bound_rhess, elem_err
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

Q100 = 100
SIGMA = 1.7


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def big():
    Q, c = bqp_instance(Q100, 0)
    rel = bqp.build_relaxation(Q, c, "colex")
    W = gaussian(rel.n, rel.n, 1000)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    del W
    print(f"[fullsize] q={Q100} n={rel.n} m={rel.m}", flush=True)
    return Q, c, rel, Xt


def _prob(big):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c, rel, Xt = big
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), SIGMA)
    return prob


@pytest.mark.parametrize("p", [16, 40, 128])
def test_fullsize_cost_grad_hvp(big, p):
    from paper_2512_04406_amd.problem import FP32, FP64

    Q, c, rel, Xt = big
    print(f"[fullsize] cost/grad/hvp p={p}", flush=True)
    Y = gaussian(rel.n, p, 2000 + p)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 3000 + p))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, SIGMA)
    prob = _prob(big)
    Yt, Ut = _t(Y), _t(U)
    f, eg, rg = prob.cost_grad(Yt)
    h64 = prob.hvp(Yt, Ut, FP64)
    e64 = prob.hvp(Yt, Ut, FP64, riemannian=False)
    h32 = prob.hvp(Yt, Ut, FP32)
    torch.cuda.synchronize()
    f_ref = sub.cost(Y)
    assert abs(f.item() - f_ref) <= 1e-10 * (1 + abs(f_ref))
    e_eg = elem_err(eg.cpu().numpy(), sub.egrad(Y), bound_egrad(sub, Y))
    e_rg = elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y))
    rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
    e_h = elem_err(h64.cpu().numpy(), rh, brh)
    e_e = elem_err(e64.cpu().numpy(), sub.ehess(Y, U), bound_ehess(sub, Y, U))
    err32 = elem_err(h32.cpu().numpy(), rh, brh)
    print(f"   elem: egrad {e_eg:.2e} rgrad {e_rg:.2e} rhess {e_h:.2e} ehess {e_e:.2e} fp32-tile rhess {err32:.2e}; "
          f"frob rhess {_rel(h64.cpu().numpy(), rh):.2e} fp32 {_rel(h32.cpu().numpy(), rh):.2e}", flush=True)
    assert max(e_eg, e_rg, e_h, e_e) <= 1e-10
    assert err32 <= 1e-4
    # repeated HVPs are bitwise identical (fixed-order reductions)
    h64b = prob.hvp(Yt, Ut, FP64)
    h32b = prob.hvp(Yt, Ut, FP32)
    torch.cuda.synchronize()
    assert torch.equal(h64, h64b) and torch.equal(h32, h32b)
    prob.close()


def test_fullsize_class_average_and_multiplier_update(big):
    Q, c, rel, Xt = big
    p = 16
    Y = gaussian(rel.n, p, 4000)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    prob = _prob(big)
    Yt = _t(Y)
    ya = prob.class_average(Yt)
    y, z, kkt = prob.update_multiplier(Yt)
    torch.cuda.synchronize()
    S = Y @ Y.T
    y_ref = class_average(S, rel.cls, rel.counts)
    assert np.max(np.abs(ya.cpu().numpy() - y_ref)) <= 1e-12
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 1e-12
    R = Q_op(S, rel.cls, rel.counts)
    Xt1 = Xt + SIGMA * R
    del S
    D = D_matrix(rel.b, rel.cls, rel.counts)
    z_ref = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    Bz = (np.abs(Xt1) + np.abs(D)) @ np.ones(rel.n)  # |S_ab| <= 1
    assert np.max(np.abs(z.cpu().numpy() - z_ref) / Bz) <= 1e-10
    k = kkt.cpu().numpy()
    nR = np.linalg.norm(R)
    assert abs(k[0] - nR) <= 1e-10 * (1 + nR)
    assert abs(k[1] - rel.b @ y_ref) <= 1e-10 * (1 + abs(rel.b @ y_ref))
    assert abs(k[2] - z_ref.sum()) <= 1e-10 * (1 + np.abs(z_ref).sum())
    iu = np.triu_indices(rel.n)
    assert _rel(prob.export_multiplier_packed(), Xt1[iu]) <= 1e-13
    prob.close()


def test_sparse_q120_fullsize():
    """Sparse-Q BQP, q = 120 (n = 7261, m = 8,502,671; 5% of the off-diagonal
    positions of Q nonzero): the same relaxation with a sparse b, at full
    size, FP64 and FP32-tile HVP, cost and gradient against the oracle."""
    from paper_2512_04406_amd.problem import FP32, FP64, ORDER_COLEX, Problem
    from synth import sparse_bqp_instance

    q, p = 120, 16
    Q, c = sparse_bqp_instance(q, 0.05, 0)
    rel = bqp.build_relaxation(Q, c, "colex")
    print(f"[fullsize] sparse q={q} n={rel.n} m={rel.m} nnz(Q)={np.count_nonzero(Q)}", flush=True)
    assert rel.n == 7261 and rel.m == 8502671
    W = gaussian(rel.n, rel.n, 1200)
    Xt = Q_op(0.05 * (W + W.T), rel.cls, rel.counts)
    del W
    Y = gaussian(rel.n, p, 1201)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 1202))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, SIGMA)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), SIGMA)
    Yt, Ut = _t(Y), _t(U)
    f, eg, rg = prob.cost_grad(Yt)
    h64 = prob.hvp(Yt, Ut, FP64)
    h32 = prob.hvp(Yt, Ut, FP32)
    torch.cuda.synchronize()
    f_ref = sub.cost(Y)
    assert abs(f.item() - f_ref) <= 1e-10 * (1 + abs(f_ref))
    rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
    e_rg = elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y))
    e_h = elem_err(h64.cpu().numpy(), rh, brh)
    err32 = elem_err(h32.cpu().numpy(), rh, brh)
    print(f"   elem: rgrad {e_rg:.2e} rhess {e_h:.2e} fp32-tile rhess {err32:.2e}", flush=True)
    assert e_rg <= 1e-10 and e_h <= 1e-10
    assert err32 <= 1e-4
    prob.close()

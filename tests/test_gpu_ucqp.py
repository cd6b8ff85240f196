"""GPU parity and solves of the Hermitian UCQP relaxation (signed classes).

The parity cases enter through the sparse-A constructor with coefficients
+-1 (imaginary parts of the real embedding) and entries left in no class (the
imaginary parts of the moment-matrix diagonal), built from the oracle's
structure; the solves use the library's own builder (mdsdp_create_ucqp).  Against the oracle with the
same signed operators: class averages (1e-12), cost, Euclidean/Riemannian
gradients and HVPs entry by entry (1e-10 of the per-entry bound in FP64, 1e-4
with FP32 tiles), the multiplier update; q = 3 (n = 20), 10 (n = 132) and the
workload size q = 30 (n = 992, m = 217,621).  Full solves: eta_max <= 1e-8,
the oracle's optimal value (q = 3 computed here, q = 30 from the golden file)
to 1e-8, mixed and FP64 agreeing, and the oracle recomputing eta from the
GPU's final (Y, Xt).
"""

import os

import numpy as np
import pytest

from oracle import alm, ucqp
from oracle.operators import D_matrix, Q_op, class_average
from oracle.subproblem import Subproblem, proj_tangent
from parity_bounds import bound_egrad, bound_rgrad, bound_rhess, elem_err
from synth import gaussian, ucqp_instance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ucqp_q30_seed0_value.txt")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _problem(rel):
    from paper_2512_04406_amd.problem import Problem

    r, c = np.triu_indices(rel.n)
    keep = rel.w[r, c] != 0
    r, c = r[keep], c[keep]
    return Problem.from_sparse_A(rel.n, rel.m, rel.cls[r, c], r, c, rel.w[r, c], rel.b)


@pytest.mark.parametrize("q,p", [(3, 2), (10, 5), (30, 16)])
def test_ucqp_parity(q, p):
    from paper_2512_04406_amd.problem import FP32, FP64

    Q = ucqp_instance(q, 0)
    rel = ucqp.build_relaxation(Q)
    print(f"[ucqp] q={q} n={rel.n} m={rel.m} p={p}", flush=True)
    sigma = 1.3
    W = gaussian(rel.n, rel.n, 11)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts, rel.w)
    Y = gaussian(rel.n, p, 12)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 13))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma, None, rel.w)
    prob = _problem(rel)
    prob.set_multiplier(_t(Xt), sigma)
    Yt, Ut = _t(Y), _t(U)
    ya = prob.class_average(Yt)
    f, eg, rg = prob.cost_grad(Yt)
    h64 = prob.hvp(Yt, Ut, FP64)
    h32 = prob.hvp(Yt, Ut, FP32)
    torch.cuda.synchronize()
    S = Y @ Y.T
    y_ref = class_average(S, rel.cls, rel.counts, rel.w)
    assert np.max(np.abs(ya.cpu().numpy() - y_ref)) <= 1e-12
    f_ref = sub.cost(Y)
    assert abs(f.item() - f_ref) <= 1e-10 * (1 + abs(f_ref))
    assert elem_err(eg.cpu().numpy(), sub.egrad(Y), bound_egrad(sub, Y)) <= 1e-10
    assert elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y)) <= 1e-10
    rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
    e64, e32 = elem_err(h64.cpu().numpy(), rh, brh), elem_err(h32.cpu().numpy(), rh, brh)
    print(f"   elem rhess fp64 {e64:.2e} fp32 tiles {e32:.2e}", flush=True)
    assert e64 <= 1e-10 and e32 <= 1e-4
    # multiplier update: y, Xt + sigma Q(Z), z, ||Q(Z)||
    y, z, kkt = prob.update_multiplier(Yt)
    torch.cuda.synchronize()
    R = Q_op(S, rel.cls, rel.counts, rel.w)
    Xt1 = Xt + sigma * R
    D = D_matrix(rel.b, rel.cls, rel.counts, rel.w)
    z_ref = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 1e-12
    Bz = (np.abs(Xt1) + np.abs(D)) @ np.ones(rel.n)
    assert np.max(np.abs(z.cpu().numpy() - z_ref) / Bz) <= 1e-10
    assert abs(kkt.cpu().numpy()[0] - np.linalg.norm(R)) <= 1e-10 * (1 + np.linalg.norm(R))
    dC = prob.adjoint_C().cpu().numpy()
    assert np.max(np.abs(dC - (Xt1 + D))) <= 1e-12 * (1 + np.abs(Xt1 + D).max())
    prob.close()


def _certify(rel, Q, res, prob):
    """The oracle recomputes eta (eq. res) from the GPU's final Y and Xt."""
    from oracle.alm import kkt_residuals

    Y = res.Y.cpu().numpy()
    Xt = prob.get_multiplier().cpu().numpy()
    S = Y @ Y.T
    y = class_average(S, rel.cls, rel.counts, rel.w)
    D = D_matrix(rel.b, rel.cls, rel.counts, rel.w)
    z = np.einsum("ij,ij->i", (Xt + D) @ Y, Y)
    X = Xt + D - np.diag(z)
    return max(kkt_residuals(S, y, X, z, rel.b, rel.cls, None, rel.w))


def test_ucqp_q3_solve_matches_oracle():
    from paper_2512_04406_amd.problem import FP32, FP64, Problem

    Q = ucqp_instance(3, 1)
    rel = ucqp.build_relaxation(Q)
    ref = alm.solve(rel.cls, rel.counts, rel.b, gaussian(rel.n, 2, 101), alm.ALMOptions(), w=rel.w)
    for prec in (FP64, FP32):
        prob = Problem.ucqp(Q)  # the library's own builder
        o = prob.default_options()
        o.hvp_prec = prec
        res = prob.solve(_t(gaussian(rel.n, 2, 101)), o)
        print(f"[ucqp] q=3 prec={prec} value={res.value:.12f} oracle={ref.value:.12f} eta={max(res.eta):.1e}",
              flush=True)
        assert res.status == 0 and max(res.eta) <= 1e-8
        assert abs(res.value - ref.value) <= 1e-8 * (1 + abs(ref.value))
        assert _certify(rel, Q, res, prob) <= 2e-8
        prob.close()


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden value not written yet (make_ucqp_q30_value.py)")
def test_ucqp_q30_mixed_and_fp64():
    from paper_2512_04406_amd.problem import FP32, FP64, Problem

    vals = {}
    for line in open(GOLDEN):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    Q = ucqp_instance(30, 0)
    rel = ucqp.build_relaxation(Q)
    out = {}
    for name, prec in (("mixed", FP32), ("fp64", FP64)):
        prob = Problem.ucqp(Q)
        o = prob.default_options()
        o.hvp_prec = prec
        o.time_limit_s = 100.0
        res = prob.solve(_t(gaussian(rel.n, 8, 100)), o)
        print(f"[ucqp] q=30 {name}: value={res.value:.10f} oracle={vals['value']:.10f} eta={max(res.eta):.1e} "
              f"outer={res.outer_iters} t={res.seconds:.1f}s", flush=True)
        assert res.status == 0 and max(res.eta) <= 1e-8
        assert abs(res.value - vals["value"]) <= 1e-8 * (1 + abs(vals["value"]))
        assert _certify(rel, Q, res, prob) <= 2e-8
        out[name] = res.value
        prob.close()
    assert abs(out["mixed"] - out["fp64"]) <= 1e-8 * (1 + abs(out["fp64"]))

"""GPU parity of the HIP hot path against the FP64 oracle (element by element).

Cases span one ragged tile (n = 7, 22), several 64-tiles with ragged tails
(n = 79, 211, 466, 821) and p = 1..128 (staged widths 16, 32, 64 and 128).  Inputs: random (Q, c), Y with unit
rows, tangent U, a multiplier Xt with A(Xt) = 0, sigma > 0.  FP64 outputs must
agree entry by entry to 1e-10 of a per-entry magnitude bound built from the
absolute values of the operands of that entry (tests/parity_bounds.py), with
the Frobenius-relative error reported beside it; class averages to 1e-12
absolute on values of size <= 1; the FP32-tile HVP is gated entry by entry at
1e-4 of the same bound.
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

CASES = [(2, 3), (5, 2), (6, 7), (10, 2), (12, 5), (20, 4), (30, 16), (40, 7),
         (6, 40), (12, 17), (20, 32), (30, 45), (40, 64), (12, 100), (20, 128), (40, 77)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(q, p, seed=0, sigma=1.7, structured=True):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    print(f"[case] q={q} n={rel.n} m={rel.m} p={p} seed={seed} structured={structured}", flush=True)
    W = gaussian(rel.n, rel.n, 1000 + seed)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Y = gaussian(rel.n, p, 2000 + seed)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 3000 + seed))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    prob = Problem.bqp(Q, c, ORDER_COLEX, structured=structured)
    prob.set_multiplier(torch.from_numpy(Xt).cuda(), sigma)
    return rel, sub, prob, Xt, Y, U, sigma


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("q,p", CASES)
@pytest.mark.parametrize("structured", [True, False])
def test_cost_grad_parity(q, p, structured):
    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    f, eg, rg = prob.cost_grad(_t(Y))
    torch.cuda.synchronize()
    f_ref = sub.cost(Y)
    assert abs(f.item() - f_ref) <= 1e-10 * (1 + abs(f_ref))
    e_eg = elem_err(eg.cpu().numpy(), sub.egrad(Y), bound_egrad(sub, Y))
    e_rg = elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y))
    print(f"[cost_grad] q={q} p={p} elem egrad {e_eg:.2e} rgrad {e_rg:.2e} "
          f"(frob {_rel(rg.cpu().numpy(), sub.rgrad(Y)):.2e})")
    assert e_eg <= 1e-10 and e_rg <= 1e-10


@pytest.mark.parametrize("q,p", CASES)
@pytest.mark.parametrize("structured", [True, False])
def test_hvp_parity_fp64(q, p, structured):
    from paper_2512_04406_amd.problem import FP64

    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    Yt, Ut = _t(Y), _t(U)
    prob.cost_grad(Yt)
    Hr = prob.hvp(Yt, Ut, FP64, riemannian=True)
    He = prob.hvp(Yt, Ut, FP64, riemannian=False)
    torch.cuda.synchronize()
    e_r = elem_err(Hr.cpu().numpy(), sub.rhess(Y, U), bound_rhess(sub, Y, U))
    e_e = elem_err(He.cpu().numpy(), sub.ehess(Y, U), bound_ehess(sub, Y, U))
    print(f"[hvp64] q={q} p={p} elem rhess {e_r:.2e} ehess {e_e:.2e} "
          f"(frob {_rel(Hr.cpu().numpy(), sub.rhess(Y, U)):.2e})")
    assert e_r <= 1e-10 and e_e <= 1e-10


@pytest.mark.parametrize("q,p", CASES)
@pytest.mark.parametrize("structured", [True, False])
def test_hvp_parity_fp32_tiles(q, p, structured):
    from paper_2512_04406_amd.problem import FP32

    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    Yt, Ut = _t(Y), _t(U)
    prob.cost_grad(Yt)
    Hr = prob.hvp(Yt, Ut, FP32, riemannian=True)
    torch.cuda.synchronize()
    err = _rel(Hr.cpu().numpy(), sub.rhess(Y, U))
    e_r = elem_err(Hr.cpu().numpy(), sub.rhess(Y, U), bound_rhess(sub, Y, U))
    print(f"[fp32-hvp] q={q} p={p} frob rel err {err:.3e}, elem {e_r:.3e}")
    assert err <= 1e-4 and e_r <= 1e-4


@pytest.mark.parametrize("q,p", CASES[:6])
@pytest.mark.parametrize("structured", [True, False])
def test_class_average_parity(q, p, structured):
    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    y = prob.class_average(_t(Y)).cpu().numpy()
    y_ref = class_average(Y @ Y.T, rel.cls, rel.counts)
    assert np.max(np.abs(y - y_ref)) <= 1e-12


@pytest.mark.parametrize("q,p", [(6, 3), (12, 5), (30, 16), (40, 4), (20, 33), (30, 64), (20, 100)])
@pytest.mark.parametrize("structured", [True, False])
def test_update_multiplier_and_certificate_parity(q, p, structured):
    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    Yt = _t(Y)
    y, z, kkt = prob.update_multiplier(Yt)
    torch.cuda.synchronize()
    S = Y @ Y.T
    y_ref = class_average(S, rel.cls, rel.counts)
    R = Q_op(S, rel.cls, rel.counts)
    Xt1 = Xt + sigma * R
    D = D_matrix(rel.b, rel.cls, rel.counts)
    z_ref = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 1e-12
    Bz = (np.abs(Xt1) + np.abs(D)) @ np.ones(rel.n)  # |S_ab| <= 1
    assert np.max(np.abs(z.cpu().numpy() - z_ref) / Bz) <= 1e-10
    k = kkt.cpu().numpy()
    assert abs(k[0] - np.linalg.norm(R)) <= 1e-10 * (1 + np.linalg.norm(R))
    assert abs(k[1] - rel.b @ y_ref) <= 1e-10 * (1 + abs(rel.b @ y_ref))
    assert abs(k[2] - z_ref.sum()) <= 1e-10 * (1 + np.abs(z_ref).sum())
    iu = np.triu_indices(rel.n)
    Xp = prob.export_multiplier_packed()
    assert _rel(Xp, Xt1[iu]) <= 1e-13
    # certificate matvec X V = (Xt + D) V - z o V
    X = Xt1 + D - np.diag(z_ref)
    V = gaussian(rel.n, 3, 77)
    XV = prob.certificate_matvec(_t(V)).cpu().numpy()
    assert np.max(np.abs(XV - X @ V) / (np.abs(X) @ np.abs(V))) <= 1e-10
    # adjoint dv/dC = Xt + D
    dC = prob.adjoint_C().cpu().numpy()
    assert _rel(dC, Xt1 + D) <= 1e-13


@pytest.mark.parametrize("structured", [True, False])
def test_determinism_bitwise(structured):
    from paper_2512_04406_amd.problem import FP32, FP64

    rel, sub, prob, Xt, Y, U, sigma = _case(30, 16, structured=structured)
    Yt, Ut = _t(Y), _t(U)
    outs = []
    for _ in range(3):
        f, eg, rg = prob.cost_grad(Yt)
        h64 = prob.hvp(Yt, Ut, FP64)
        h32 = prob.hvp(Yt, Ut, FP32)
        torch.cuda.synchronize()
        outs.append([f.cpu().numpy().tobytes(), eg.cpu().numpy().tobytes(), h64.cpu().numpy().tobytes(),
                     h32.cpu().numpy().tobytes()])
    assert outs[0] == outs[1] == outs[2]


def test_retract_and_project_parity():
    from paper_2512_04406_amd import _lib
    from paper_2512_04406_amd.problem import _ptr, _stream

    n, p = 301, 5
    Y = gaussian(n, p, 1)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    V = gaussian(n, p, 2)
    out = torch.empty(n, p, dtype=torch.float64, device="cuda")
    Yt, Vt = _t(Y), _t(V)  # keep the device buffers alive across the async calls
    _lib.call("mdsdp_retract", n, p, _ptr(Yt), _ptr(Vt), 0.3, _ptr(out), _stream())
    ref = (Y + 0.3 * V) / np.linalg.norm(Y + 0.3 * V, axis=1, keepdims=True)
    assert _rel(out.cpu().numpy(), ref) <= 1e-14
    _lib.call("mdsdp_project_tangent", n, p, _ptr(Yt), _ptr(Vt), _ptr(out), _stream())
    assert _rel(out.cpu().numpy(), proj_tangent(Y, V)) <= 1e-14


def test_nonzero_C_parity():
    """Generic class map with C != 0 (DSDP allows any C): cost, gradient, HVP."""
    from paper_2512_04406_amd.problem import FP64, Problem

    q, p, sigma = 6, 3, 0.9
    Q, c = bqp_instance(q, 4)
    rel = bqp.build_relaxation(Q, c, "lex")
    Cm = gaussian(rel.n, rel.n, 5)
    Cm = 0.05 * (Cm + Cm.T)
    W = gaussian(rel.n, rel.n, 6)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma, C=Cm)
    iu = np.triu_indices(rel.n)
    prob = Problem.from_classmap(rel.n, rel.cls[iu].astype(np.int32), rel.b, Cm)
    prob.set_multiplier(_t(Xt), sigma)
    Y = gaussian(rel.n, p, 7)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(rel.n, p, 8))
    f, eg, rg = prob.cost_grad(_t(Y))
    H = prob.hvp(_t(Y), _t(U), FP64)
    torch.cuda.synchronize()
    assert abs(f.item() - sub.cost(Y)) <= 1e-10 * (1 + abs(sub.cost(Y)))
    assert elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y)) <= 1e-10
    assert elem_err(H.cpu().numpy(), sub.rhess(Y, U), bound_rhess(sub, Y, U)) <= 1e-10


@pytest.mark.parametrize("q,p", [(4, 3), (9, 16), (25, 5), (9, 29), (25, 64), (9, 128),
                                 (4, 33), (5, 48), (18, 33), (34, 40), (17, 32)])
def test_structured_matches_generic_class_sums(q, p):
    """The class-map-free BQP kernels and the generic fixed-point class map
    path give the same class averages (both are within rounding of the
    oracle); HVP class averages compared through the HVP output.  Widths up
    to 32 take the single-pass degree-4 kernel, wider ones the two passes;
    q = 4, 5 have one and five degree-4 classes, q = 17, 18, 34 put c on
    either side of a 16-row block boundary."""
    from paper_2512_04406_amd.problem import FP64, ORDER_COLEX, Problem

    Q, c = bqp_instance(q, 8)
    a = Problem.bqp(Q, c, ORDER_COLEX, structured=True)
    b = Problem.bqp(Q, c, ORDER_COLEX, structured=False)
    n = a.n
    Y = gaussian(n, p, 9)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = gaussian(n, p, 10)
    Yt, Ut = _t(Y), _t(U)
    ya, yb = a.class_average(Yt), b.class_average(Yt)
    torch.cuda.synchronize()
    assert float((ya - yb).abs().max()) <= 1e-13
    for P in (a, b):
        P.cost_grad(Yt)
    ha, hb = a.hvp(Yt, Ut, FP64), b.hvp(Yt, Ut, FP64)
    torch.cuda.synchronize()
    assert float((ha - hb).norm() / hb.norm()) <= 1e-12


def test_width_switching_on_one_problem():
    """Calls with different factor widths (and a certificate eigensolve in
    between, which stages width 1) on one problem must each match the
    oracle: no staged width may leak from one call into the next."""
    from paper_2512_04406_amd.problem import FP32, FP64

    rel, sub, prob, Xt, Y0, U0, sigma = _case(20, 3, structured=True)
    for p in (100, 5, 40, 17, 128, 2):
        Y = gaussian(rel.n, p, 7000 + p)
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        U = proj_tangent(Y, gaussian(rel.n, p, 8000 + p))
        Yt, Ut = _t(Y), _t(U)
        print(f"[width] p={p}", flush=True)
        f, eg, rg = prob.cost_grad(Yt)
        h64 = prob.hvp(Yt, Ut, FP64)
        prob.min_eigpair(tol=1e-8, maxit=50)
        h32 = prob.hvp(Yt, Ut, FP32)
        torch.cuda.synchronize()
        rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
        assert elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y)) <= 1e-10
        assert elem_err(h64.cpu().numpy(), rh, brh) <= 1e-10
        assert elem_err(h32.cpu().numpy(), rh, brh) <= 1e-4


@pytest.mark.parametrize("q,p,structured", [(12, 200, True), (20, 256, False), (30, 300, True), (12, 512, True),
                                            (8, 130, False)])
def test_wide_factors(q, p, structured):
    """Factor widths above 64 (64-column slices, S tiles accumulated over
    64-column chunks, the sliced multiplier update into a second buffer, the
    MFMA low-rank term and the width-templated row finalisers), including
    p > n: every output against the oracle."""
    from paper_2512_04406_amd.problem import FP32, FP64

    rel, sub, prob, Xt, Y, U, sigma = _case(q, p, structured=structured)
    Yt, Ut = _t(Y), _t(U)
    f, eg, rg = prob.cost_grad(Yt)
    h64 = prob.hvp(Yt, Ut, FP64)
    e64 = prob.hvp(Yt, Ut, FP64, riemannian=False)
    h32 = prob.hvp(Yt, Ut, FP32)
    h64b = prob.hvp(Yt, Ut, FP64)  # Y^T Y reused from the first HVP at this point
    torch.cuda.synchronize()
    f_ref = sub.cost(Y)
    assert abs(f.item() - f_ref) <= 1e-10 * (1 + abs(f_ref))
    assert elem_err(eg.cpu().numpy(), sub.egrad(Y), bound_egrad(sub, Y)) <= 1e-10
    assert elem_err(rg.cpu().numpy(), sub.rgrad(Y), bound_rgrad(sub, Y)) <= 1e-10
    rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
    assert elem_err(h64.cpu().numpy(), rh, brh) <= 1e-10
    assert elem_err(e64.cpu().numpy(), sub.ehess(Y, U), bound_ehess(sub, Y, U)) <= 1e-10
    assert elem_err(h32.cpu().numpy(), rh, brh) <= 1e-4
    assert torch.equal(h64, h64b)
    # multiplier update and certificate matvec at this width
    y, z, kkt = prob.update_multiplier(Yt)
    torch.cuda.synchronize()
    S = Y @ Y.T
    y_ref = class_average(S, rel.cls, rel.counts)
    R = Q_op(S, rel.cls, rel.counts)
    Xt1 = Xt + sigma * R
    D = D_matrix(rel.b, rel.cls, rel.counts)
    z_ref = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 1e-12
    Bz = (np.abs(Xt1) + np.abs(D)) @ np.ones(rel.n)  # |S_ab| <= 1
    assert np.max(np.abs(z.cpu().numpy() - z_ref) / Bz) <= 1e-10
    assert abs(kkt.cpu().numpy()[0] - np.linalg.norm(R)) <= 1e-10 * (1 + np.linalg.norm(R))
    iu = np.triu_indices(rel.n)
    assert _rel(prob.export_multiplier_packed(), Xt1[iu]) <= 1e-13
    X = Xt1 + D - np.diag(z_ref)
    V = gaussian(rel.n, 70, 77)
    XV = prob.certificate_matvec(_t(V)).cpu().numpy()
    assert np.max(np.abs(XV - X @ V) / (np.abs(X) @ np.abs(V))) <= 1e-10
    # a second update (the sliced update alternates multiplier buffers)
    prob.update_multiplier(Yt)
    assert _rel(prob.export_multiplier_packed(), (Xt1 + sigma * R)[iu]) <= 1e-13


def test_sparse_A_problem_matches_classmap_problem():
    """A problem given as a sparse 0/1 A (COO triplets in shuffled order, lex
    basis) builds the same device layout as the class-map constructor: cost,
    gradient and HVPs bitwise equal, and equal to the oracle."""
    from paper_2512_04406_amd.problem import FP32, FP64, Problem

    q, p, sigma = 9, 5, 1.3
    Q, c = bqp_instance(q, 4)
    rel = bqp.build_relaxation(Q, c, "lex")
    n = rel.n
    r, cc = np.triu_indices(n)
    k = rel.cls[r, cc].astype(np.int32)
    perm = np.random.default_rng(5).permutation(r.size)
    sp = Problem.from_sparse_A(n, rel.m, k[perm], r[perm].astype(np.int32), cc[perm].astype(np.int32),
                               np.ones(r.size), rel.b)
    cm = Problem.from_classmap(n, rel.cls[r, cc], rel.b)
    W = gaussian(n, n, 31)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Y = gaussian(n, p, 32)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    U = proj_tangent(Y, gaussian(n, p, 33))
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    outs = []
    for P in (sp, cm):
        P.set_multiplier(_t(Xt), sigma)
        f, eg, rg = P.cost_grad(_t(Y))
        h64 = P.hvp(_t(Y), _t(U), FP64)
        h32 = P.hvp(_t(Y), _t(U), FP32)
        torch.cuda.synchronize()
        outs.append((f.cpu(), rg.cpu(), h64.cpu(), h32.cpu()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    f, rg, h64, h32 = outs[0]
    assert abs(f.item() - sub.cost(Y)) <= 1e-10 * (1 + abs(sub.cost(Y)))
    rh, brh = sub.rhess(Y, U), bound_rhess(sub, Y, U)
    assert elem_err(rg.numpy(), sub.rgrad(Y), bound_rgrad(sub, Y)) <= 1e-10
    assert elem_err(h64.numpy(), rh, brh) <= 1e-10
    assert elem_err(h32.numpy(), rh, brh) <= 1e-4

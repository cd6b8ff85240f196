"""GPU checks of the differentiable cost and of the adjoints of the optimal value.

* alm_cost: value and backward (Euclidean gradient 2GY) against the FP64
  oracle; double backward (the hand-written HVP) against the oracle's
  Euclidean Hessian; torch.autograd.gradcheck / gradgradcheck (central
  differences of the library's own cost and gradient); an O(h^2) decay of the
  central-difference error of the cost and of the gradient.
* riemannian_grad / riemannian_hvp against the oracle (Proposition prop,
  eq. sec4:eq7).
* adjoints of the optimal value (Lagrangian duality of DSDP and its primal):
  dv/dC = Xt + D against central differences of re-solves with C = C0 +- eps E
  at a generic strictly feasible C0 (v is not differentiable at the
  degenerate C = 0 of the tight BQP relaxation);
  dv/dQ_ij (i < j, both triangles moved) = 2 y_{ij} and dv/dc_i = y_i against
  central differences of re-solves of the perturbed BQP.
"""

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import Q_op
from oracle.subproblem import Subproblem, proj_tangent
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(q, p, seed=0, sigma=1.3):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    print(f"[autograd] q={q} n={rel.n} p={p} seed={seed}", flush=True)
    W = gaussian(rel.n, rel.n, 400 + seed)
    Xt = Q_op(0.1 * (W + W.T), rel.cls, rel.counts)
    Y = gaussian(rel.n, p, 500 + seed)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), sigma)
    sub = Subproblem(rel.cls, rel.counts, rel.b, Xt, sigma)
    return rel, sub, prob, Y


@pytest.mark.parametrize("q,p", [(6, 3), (12, 5), (20, 17)])
def test_cost_backward_and_double_backward(q, p):
    from paper_2512_04406_amd.autograd import alm_cost
    from paper_2512_04406_amd.problem import FP32

    rel, sub, prob, Y = _case(q, p)
    U = gaussian(rel.n, p, 600)
    Yt = _t(Y).requires_grad_(True)
    f = alm_cost(prob, Yt)
    (g,) = torch.autograd.grad(f, Yt, create_graph=True)
    (h,) = torch.autograd.grad(g, Yt, grad_outputs=_t(U))
    assert abs(f.item() - sub.cost(Y)) <= 1e-10 * (1 + abs(sub.cost(Y)))
    assert _rel(g.detach().cpu().numpy(), sub.egrad(Y)) <= 1e-10
    assert _rel(h.cpu().numpy(), sub.ehess(Y, U)) <= 1e-10
    # plain backward accumulates the same gradient
    Y2 = _t(Y).requires_grad_(True)
    alm_cost(prob, Y2).backward()
    assert _rel(Y2.grad.cpu().numpy(), sub.egrad(Y)) <= 1e-10
    # FP32-tile second derivative: reported, gated loosely
    Y3 = _t(Y).requires_grad_(True)
    (g3,) = torch.autograd.grad(alm_cost(prob, Y3, hvp_prec=FP32), Y3, create_graph=True)
    (h3,) = torch.autograd.grad(g3, Y3, grad_outputs=_t(U))
    e32 = _rel(h3.cpu().numpy(), sub.ehess(Y, U))
    print(f"   fp32-tile ehess rel err {e32:.2e}", flush=True)
    assert e32 <= 1e-4


def test_gradcheck_and_gradgradcheck():
    from paper_2512_04406_amd.autograd import alm_cost

    rel, sub, prob, Y = _case(4, 2)
    Yt = _t(Y).requires_grad_(True)
    fn = lambda y: alm_cost(prob, y)  # noqa: E731
    assert torch.autograd.gradcheck(fn, (Yt,), eps=1e-6, atol=1e-6, rtol=1e-6)
    assert torch.autograd.gradgradcheck(fn, (Yt,), eps=1e-6, atol=1e-6, rtol=1e-6)


def test_central_differences_decay_quadratically():
    """Psi is a quartic polynomial of Y: the central-difference error of the
    cost along U and of the gradient along U is O(h^2) (exactly c h^2 for the
    cost, whose third derivative is the only term)."""
    from paper_2512_04406_amd.autograd import alm_cost, euclidean_grad

    rel, sub, prob, Y = _case(12, 4)
    U = gaussian(rel.n, 4, 700)
    Yt = _t(Y).requires_grad_(True)
    (g,) = torch.autograd.grad(alm_cost(prob, Yt), Yt, create_graph=True)
    dirder = float((g.detach() * _t(U)).sum())
    (hu,) = torch.autograd.grad(g, Yt, grad_outputs=_t(U))
    hu = hu.cpu().numpy()
    errs_f, errs_g = [], []
    for h in (1e-2, 5e-3, 2.5e-3):
        fp = alm_cost(prob, _t(Y + h * U)).item()
        fm = alm_cost(prob, _t(Y - h * U)).item()
        errs_f.append(abs((fp - fm) / (2 * h) - dirder))
        gp = euclidean_grad(prob, _t(Y + h * U)).cpu().numpy()
        gm = euclidean_grad(prob, _t(Y - h * U)).cpu().numpy()
        errs_g.append(np.linalg.norm((gp - gm) / (2 * h) - hu))
    print(f"   fd errors cost {errs_f} grad {errs_g}", flush=True)
    for e in (errs_f, errs_g):
        assert 3.0 <= e[0] / e[1] <= 5.0 and 3.0 <= e[1] / e[2] <= 5.0


def test_riemannian_grad_and_hvp():
    from paper_2512_04406_amd.autograd import riemannian_grad, riemannian_hvp
    from paper_2512_04406_amd.problem import FP64

    rel, sub, prob, Y = _case(20, 6)
    U = proj_tangent(Y, gaussian(rel.n, 6, 800))
    Yt = _t(Y)
    rg = riemannian_grad(prob, Yt).cpu().numpy()
    hv = riemannian_hvp(prob, Yt, _t(U), FP64).cpu().numpy()
    assert _rel(rg, sub.rgrad(Y)) <= 1e-10
    assert _rel(hv, sub.rhess(Y, U)) <= 1e-10
    # tangency of the gradient (rowdot with Y vanishes)
    assert np.max(np.abs(np.einsum("ij,ij->i", rg, Y))) <= 1e-10 * max(1.0, np.abs(rg).max())


def _solve_value(prob, n, p0, seed, tol):
    opts = prob.default_options()
    opts.tol = tol
    opts.hvp_prec = 0
    res = prob.solve(_t(gaussian(n, p0, 100 + seed)), opts)
    assert res.status == 0 and max(res.eta) <= tol, (res.status, res.eta)
    return res


def _generic_C(n):
    """A strictly feasible, generic cost matrix C0 (zero diagonal, ||C0||_2 =
    1/2, so S = I - C0 is positive definite) and a zero-diagonal direction E.
    At C = 0 the tight BQP relaxation is primal-degenerate and v(C) has a kink
    along generic off-class directions; at C0 the solution is non-degenerate
    (rank S + rank X = n) and v is differentiable there."""
    G = gaussian(n, n, 901)
    G = G + G.T
    np.fill_diagonal(G, 0.0)
    G *= 0.5 / np.max(np.abs(np.linalg.eigvalsh(G)))
    E = gaussian(n, n, 900)
    E = E + E.T
    np.fill_diagonal(E, 0.0)  # diag(S) = 1 ties the diagonal of C to y_{}
    return G, E


def test_adjoint_C_matches_central_differences_of_resolves():
    from paper_2512_04406_amd.problem import Problem

    q, seed, eps, tol = 6, 3, 1e-4, 1e-11
    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    n = rel.n
    iu = np.triu_indices(n)
    cls_packed = rel.cls[iu].astype(np.int32)
    C0, E = _generic_C(n)
    print(f"[adjoint C] q={q} n={n} eps={eps}", flush=True)
    prob0 = Problem.from_classmap(n, cls_packed, rel.b, C0)
    _solve_value(prob0, n, 2, seed, tol)
    dC = prob0.adjoint_C().cpu().numpy()
    pred = float(np.sum(dC * E))
    vals = []
    for s in (+1.0, -1.0):
        pr = Problem.from_classmap(n, cls_packed, rel.b, C0 + s * eps * E)
        vals.append(_solve_value(pr, n, 2, seed, tol).value)
    fd = (vals[0] - vals[1]) / (2 * eps)
    print(f"   <dv/dC, E> = {pred:.10f}, central difference {fd:.10f}", flush=True)
    assert abs(fd - pred) <= 1e-3 * (1 + abs(pred))


def test_adjoint_Q_and_c_match_central_differences_of_resolves():
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    q, seed, eps, tol = 10, 1, 1e-4, 1e-10
    Q, c = bqp_instance(q, seed)
    n = 1 + q + q * (q - 1) // 2
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    res = _solve_value(prob, n, 2, seed, tol)
    y = prob.class_average(res.Y.contiguous()).cpu().numpy()
    off = bqp.class_offsets(q)
    checks = [("Q", 2, 7), ("Q", 0, 9), ("c", 4, None)]
    for kind, i, j in checks:
        vals = []
        for s in (+1.0, -1.0):
            Qp, cp = Q.copy(), c.copy()
            if kind == "Q":
                Qp[i, j] += s * eps
                Qp[j, i] += s * eps
            else:
                cp[i] += s * eps
            pr = Problem.bqp(Qp, cp, ORDER_COLEX)
            vals.append(_solve_value(pr, n, 2, seed, tol).value)
        fd = (vals[0] - vals[1]) / (2 * eps)
        if kind == "Q":
            pred = 2.0 * y[off[2] + i + j * (j - 1) // 2]
        else:
            pred = y[off[1] + i]
        print(f"   d v / d {kind}[{i},{j}] = {pred:.10f}, central difference {fd:.10f}", flush=True)
        assert abs(fd - pred) <= 1e-5 * (1 + abs(pred))

"""GPU checks of the batched solve (mdsdp_solve_batch) on many small dense BQPs
of uneven size, and of the adjoint d(opt)/dQ on some of them.

* a batch of small relaxations (q uniform in [8, 14], seeded) solved
  concurrently by host workers on separate streams: every problem reaches
  eta_max <= 1e-8 and its value equals the brute-force minimum (rank-one,
  tight relaxation) and the value of the same problem solved alone;
* adjoint: for 8 problems of the batch, d v / d Q_ij (a symmetric
  perturbation of one off-diagonal pair) is 2 y*_{ij} at the optimum (y* the
  class average of the class {i, j}, Lagrangian duality); it is compared with
  central differences of re-solves, themselves run as one batch.
"""

import numpy as np
import pytest

from oracle import brute
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _batch(qs, seeds, Qs=None):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    probs, Y0s, data = [], [], []
    for k, (q, sd) in enumerate(zip(qs, seeds)):
        Q, c = bqp_instance(q, sd) if Qs is None else Qs[k]
        pr = Problem.bqp(Q, c, ORDER_COLEX)
        probs.append(pr)
        Y0s.append(_t(gaussian(pr.n, 2, 100 + sd)))
        data.append((Q, c))
    return probs, Y0s, data


def test_batch_of_small_bqps_matches_brute_force():
    from paper_2512_04406_amd.problem import FP64, Problem

    rng = np.random.default_rng(7)
    qs = list(rng.integers(8, 15, size=24))
    seeds = list(range(24))
    probs, Y0s, data = _batch(qs, seeds)
    print(f"[batch] {len(qs)} problems, n from {min(p.n for p in probs)} to {max(p.n for p in probs)}", flush=True)
    o = probs[0].default_options()
    o.hvp_prec = FP64
    out = Problem.solve_batch(probs, Y0s, o, nworkers=4)
    for k, ((Y, r), (Q, c)) in enumerate(zip(out, data)):
        fmin, _ = brute.brute_force_min(Q, c)
        assert r.status == 0 and max(r.eta_p, r.eta_d, r.eta_g) <= 1e-8, (k, r.status)
        assert abs(r.value - fmin) <= 1e-8 * (1 + abs(fmin)), (k, r.value, fmin)
    # the same problem alone gives the same value
    alone = probs[3].solve(Y0s[3], o)
    assert abs(alone.value - out[3][1].value) <= 1e-10 * (1 + abs(alone.value))
    for pr in probs:
        pr.close()


def test_batch_adjoint_dQ_by_central_differences():
    """d v / d Q_ij = 2 y*_ij for 8 problems, against central differences of
    batched re-solves (v is locally linear in Q at a tight rank-one solution,
    so the differences are exact up to the solve tolerance)."""
    from paper_2512_04406_amd.problem import FP64, Problem

    qs = [8, 9, 10, 11, 12, 10, 9, 8]
    seeds = [31, 32, 33, 34, 35, 36, 37, 38]
    probs, Y0s, data = _batch(qs, seeds)
    o = probs[0].default_options()
    o.hvp_prec = FP64
    o.tol = 1e-11
    out = Problem.solve_batch(probs, Y0s, o, nworkers=4)
    eps = 1e-3
    pert, pred = [], []
    for k, ((Y, r), pr, (Q, c)) in enumerate(zip(out, probs, data)):
        assert r.status == 0
        y = pr.class_average(Y.contiguous()).cpu().numpy()
        i, j = 0, 1 + k % (qs[k] - 1)
        # class {i, j}: degree-2 colex id off2 + C(j, 2) + i with off2 = 1 + q
        g = 1 + qs[k] + j * (j - 1) // 2 + i
        pred.append(2.0 * y[g])
        for sgn in (+1, -1):
            Qp = Q.copy()
            Qp[i, j] += sgn * eps
            Qp[j, i] += sgn * eps
            pert.append((Qp, c))
    probs2, Y0s2, _ = _batch([q for q in qs for _ in (0, 1)], [s for s in seeds for _ in (0, 1)], Qs=pert)
    out2 = Problem.solve_batch(probs2, Y0s2, o, nworkers=4)
    for k in range(8):
        vp, vm = out2[2 * k][1].value, out2[2 * k + 1][1].value
        assert out2[2 * k][1].status == 0 and out2[2 * k + 1][1].status == 0
        fd = (vp - vm) / (2 * eps)
        print(f"[adjoint] k={k} q={qs[k]} fd={fd:.9f} pred={pred[k]:.9f}", flush=True)
        assert abs(fd - pred[k]) <= 1e-5 * (1 + abs(pred[k]))
    for pr in probs + probs2:
        pr.close()

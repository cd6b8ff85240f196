"""GPU check of the allocation-free eigenpair entry point
(mdsdp_min_eigpair_noalloc) against mdsdp_min_eigpair, through the C ABI.

Two calls in a row on one GPU's fixed scratch, the second on a smaller
problem (q = 12, n = 79, then q = 8, n = 37): the k smallest eigenvalues,
lambda_max, the eigenvectors and the iteration counts must equal those of the
allocating entry point bit for bit (same kernels, same seed, same order), and
the eigenvalues must match LAPACK on the oracle's dense certificate.  A size
beyond the scratch is rejected with MDSDP_EINVAL before any work.
"""

import ctypes as C

import numpy as np
import pytest

from oracle import bqp
from oracle.operators import D_matrix, Q_op
from synth import bqp_instance, gaussian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _certificate_problem(q, p, seed):
    from paper_2512_04406_amd.problem import ORDER_COLEX, Problem

    Q, c = bqp_instance(q, seed)
    rel = bqp.build_relaxation(Q, c, "colex")
    W = gaussian(rel.n, rel.n, seed + 5)
    Xt = Q_op(0.2 * (W + W.T), rel.cls, rel.counts)
    Y = gaussian(rel.n, p, seed + 6)
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    prob = Problem.bqp(Q, c, ORDER_COLEX)
    prob.set_multiplier(_t(Xt), 1.3)
    prob.update_multiplier(_t(Y))
    Xt1 = Xt + 1.3 * Q_op(Y @ Y.T, rel.cls, rel.counts)
    D = D_matrix(rel.b, rel.cls, rel.counts)
    z = np.einsum("ij,ij->i", (Xt1 + D) @ Y, Y)
    return prob, Xt1 + D - np.diag(z)


def _call(name, prob, k, tol, maxit, seed):
    from paper_2512_04406_amd import _lib
    from paper_2512_04406_amd.problem import _ptr, _stream

    ev = np.zeros(k)
    lmax = C.c_double()
    it = C.c_int32()
    V = torch.zeros(k, prob.n, dtype=torch.float64, device="cuda")
    code = getattr(_lib.lib(), name)(prob._h, k, tol, maxit, seed, _ptr(ev), C.byref(lmax), _ptr(V), C.byref(it),
                                     _stream())
    torch.cuda.synchronize()
    return code, ev, lmax.value, V.cpu().numpy(), it.value


@pytest.mark.parametrize("rep", [0, 1])
def test_noalloc_matches_allocating_entry_point(rep):
    cases = [(12, 3, 4, 11), (8, 2, 3, 12)]  # (q, p, k, seed): the second problem is smaller
    for q, p, k, seed in cases:
        prob, X = _certificate_problem(q, p, seed)
        n = X.shape[0]
        print(f"[noalloc] q={q} n={n} k={k}", flush=True)
        w = np.linalg.eigvalsh(X)
        a = _call("mdsdp_min_eigpair", prob, k, 1e-11, n, 7)
        b = _call("mdsdp_min_eigpair_noalloc", prob, k, 1e-11, n, 7)
        assert a[0] == 0 and b[0] == 0
        assert np.array_equal(a[1], b[1]) and a[2] == b[2] and a[4] == b[4]
        assert np.array_equal(a[3], b[3])
        np.testing.assert_allclose(b[1], w[:k], rtol=0, atol=1e-9 * (1 + abs(w[-1])))
        prob.close()


def test_noalloc_rejects_sizes_beyond_scratch():
    from paper_2512_04406_amd import _lib

    prob, X = _certificate_problem(100, 2, 3)  # n = 5051
    code, *_ = _call("mdsdp_min_eigpair_noalloc", prob, 1, 1e-8, 900, 1)  # 5051 * 901 doubles > 4 Mi
    assert code == -1
    assert b"scratch" in _lib.lib().mdsdp_last_error()
    code, *_ = _call("mdsdp_min_eigpair_noalloc", prob, 1, 1e-8, 300, 1)  # fits
    assert code in (0, -7)
    prob.close()

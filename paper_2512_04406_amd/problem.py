"""Python face of the library: one `Problem` per DSDP instance.

PyTorch supplies device memory and the current HIP stream; every operation is
a call into libmanidsdp.so (see include/manidsdp.h for the definitions).
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import Options, Result, call, lib

FP64, FP32 = 0, 1
ORDER_LEX, ORDER_COLEX = 0, 1


def _ptr(t) -> C.c_void_p:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    raise TypeError(type(t))


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


def bqp_sizes(q: int) -> tuple[int, int]:
    n = C.c_int32()
    m = C.c_int64()
    call("mdsdp_bqp_sizes", q, C.byref(n), C.byref(m))
    return n.value, m.value


def bqp_classmap(q: int, order: int = ORDER_COLEX) -> np.ndarray:
    """Packed upper-triangle class ids (row-major) of the order-2 BQP relaxation."""
    n, _ = bqp_sizes(q)
    out = np.empty(n * (n + 1) // 2, dtype=np.int32)
    call("mdsdp_bqp_classmap", q, order, _ptr(out))
    return out


def bqp_b(Q: np.ndarray, c: np.ndarray) -> np.ndarray:
    q = c.size
    _, m = bqp_sizes(q)
    Qc = np.ascontiguousarray(Q, dtype=np.float64)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    out = np.empty(m, dtype=np.float64)
    call("mdsdp_bqp_b", q, _ptr(Qc), _ptr(cc), _ptr(out))
    return out


def ucqp_sizes(q: int) -> tuple[int, int]:
    n = C.c_int32()
    m = C.c_int64()
    call("mdsdp_ucqp_sizes", q, C.byref(n), C.byref(m))
    return n.value, m.value


def ucqp_structure(q: int) -> tuple[np.ndarray, np.ndarray]:
    """Packed upper-triangle class ids and coefficients (+1, -1, 0) of the
    Hermitian UCQP relaxation's real embedding."""
    n, _ = ucqp_sizes(q)
    cls_ = np.empty(n * (n + 1) // 2, dtype=np.int32)
    coef = np.empty(n * (n + 1) // 2, dtype=np.int8)
    call("mdsdp_ucqp_structure", q, _ptr(cls_), _ptr(coef))
    return cls_, coef


def ucqp_b(Q: np.ndarray) -> np.ndarray:
    q = Q.shape[0]
    _, m = ucqp_sizes(q)
    out = np.empty(m, dtype=np.float64)
    Qre = np.ascontiguousarray(np.real(Q), dtype=np.float64)
    Qim = np.ascontiguousarray(np.imag(Q), dtype=np.float64)
    call("mdsdp_ucqp_b", q, _ptr(Qre), _ptr(Qim), _ptr(out))
    return out


@dataclass
class SolveResult:
    Y: torch.Tensor
    value: float
    eta: tuple
    status: int
    outer_iters: int
    rtr_iters: int
    hvps: int
    cost_grads: int
    eig_iters: int
    p_final: int
    p_max_reached: int
    sigma: float
    seconds: float
    phases: dict
    history: np.ndarray
    rank_one_round: bool = False  # the final point is the rank-one compression


class Problem:
    """A DSDP instance with class-indicator constraints, resident on the GPU."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        n = C.c_int32()
        m = C.c_int64()
        ns = C.c_int64()
        nt = C.c_int32()
        call("mdsdp_problem_info", self._h, C.byref(n), C.byref(m), C.byref(ns), C.byref(nt))
        self.n, self.m, self.n_slots, self.n_tiles = n.value, m.value, ns.value, nt.value
        self.sigma = 1.0
        self._ad_key = None  # point of the last cost/gradient pass made for autograd

    # ---- construction -------------------------------------------------------
    @classmethod
    def from_classmap(cls, n: int, cls_packed: np.ndarray, b: np.ndarray, C_dense: np.ndarray | None = None):
        clsp = np.ascontiguousarray(cls_packed, dtype=np.int32)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        if clsp.size != n * (n + 1) // 2:
            raise ValueError("class map must hold n(n+1)/2 packed entries")
        Cd = None if C_dense is None else np.ascontiguousarray(C_dense, dtype=np.float64)
        h = C.c_void_p()
        call("mdsdp_create_classmap", n, bb.size, _ptr(clsp), _ptr(bb), _ptr(Cd), C.byref(h))
        return cls(h)

    @classmethod
    def from_sparse_A(cls, n, m, cls_idx, rows, cols, vals, b, C_dense=None):
        ci = np.ascontiguousarray(cls_idx, dtype=np.int32)
        ri = np.ascontiguousarray(rows, dtype=np.int32)
        co = np.ascontiguousarray(cols, dtype=np.int32)
        va = np.ascontiguousarray(vals, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        Cd = None if C_dense is None else np.ascontiguousarray(C_dense, dtype=np.float64)
        h = C.c_void_p()
        call("mdsdp_create_sparse_A", n, m, ci.size, _ptr(ci), _ptr(ri), _ptr(co), _ptr(va), _ptr(bb),
             _ptr(Cd), C.byref(h))
        return cls(h)

    @classmethod
    def ucqp(cls, Q: np.ndarray):
        """Hermitian order-2 relaxation of min z^H Q z, |z_i| = 1 (real
        embedding, signed classes; see mdsdp_ucqp_structure)."""
        q = Q.shape[0]
        Qre = np.ascontiguousarray(np.real(Q), dtype=np.float64)
        Qim = np.ascontiguousarray(np.imag(Q), dtype=np.float64)
        h = C.c_void_p()
        call("mdsdp_create_ucqp", q, _ptr(Qre), _ptr(Qim), C.byref(h))
        return cls(h)

    @classmethod
    def bqp(cls, Q: np.ndarray, c: np.ndarray, order: int = ORDER_COLEX, structured: bool = True):
        """Order-2 BQP relaxation.  structured=True (colex order) uses the
        class-map-free class-sum kernels; False goes through the generic
        class-map path."""
        q = c.size
        if not structured:
            n, _ = bqp_sizes(q)
            return cls.from_classmap(n, bqp_classmap(q, order), bqp_b(Q, c))
        Qc = np.ascontiguousarray(Q, dtype=np.float64)
        cc = np.ascontiguousarray(c, dtype=np.float64)
        h = C.c_void_p()
        call("mdsdp_create_bqp", q, order, _ptr(Qc), _ptr(cc), C.byref(h))
        return cls(h)

    def close(self):
        if self._h:
            call("mdsdp_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().mdsdp_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # ---- multiplier -----------------------------------------------------------
    def set_multiplier(self, Xt: torch.Tensor | None, sigma: float) -> None:
        self._ad_key = None
        if Xt is not None:
            _dev_f64(Xt, "Xt")
            if Xt.shape != (self.n, self.n):
                raise ValueError("Xt must be n x n")
        call("mdsdp_set_multiplier", self._h, _ptr(Xt), float(sigma), _stream())
        self.sigma = float(sigma)

    def set_sigma(self, sigma: float) -> None:
        self._ad_key = None
        call("mdsdp_set_sigma", self._h, float(sigma))
        self.sigma = float(sigma)

    def get_multiplier(self) -> torch.Tensor:
        X = torch.empty(self.n, self.n, dtype=torch.float64, device="cuda")
        call("mdsdp_get_multiplier", self._h, _ptr(X), _stream())
        return X

    # ---- evaluations ------------------------------------------------------------
    def cost_grad(self, Y: torch.Tensor, want_egrad: bool = True, want_rgrad: bool = True):
        self._ad_key = None
        _dev_f64(Y, "Y")
        n, p = Y.shape
        f = torch.empty(1, dtype=torch.float64, device=Y.device)
        eg = torch.empty_like(Y) if want_egrad else None
        rg = torch.empty_like(Y) if want_rgrad else None
        call("mdsdp_cost_grad", self._h, p, _ptr(Y), _ptr(f), _ptr(eg), _ptr(rg), _stream())
        return f, eg, rg

    def hvp(self, Y: torch.Tensor, U: torch.Tensor, prec: int = FP64, riemannian: bool = True,
            out: torch.Tensor | None = None) -> torch.Tensor:
        _dev_f64(Y, "Y")
        _dev_f64(U, "U")
        if out is None:
            out = torch.empty_like(U)
        call("mdsdp_hvp", self._h, Y.shape[1], prec, _ptr(Y), _ptr(U), _ptr(out), 1 if riemannian else 0,
             _stream())
        return out

    def class_average(self, Y: torch.Tensor) -> torch.Tensor:
        self._ad_key = None
        _dev_f64(Y, "Y")
        y = torch.empty(self.m, dtype=torch.float64, device=Y.device)
        call("mdsdp_class_average", self._h, Y.shape[1], _ptr(Y), _ptr(y), _stream())
        return y

    def update_multiplier(self, Y: torch.Tensor):
        self._ad_key = None
        _dev_f64(Y, "Y")
        y = torch.empty(self.m, dtype=torch.float64, device=Y.device)
        z = torch.empty(self.n, dtype=torch.float64, device=Y.device)
        kkt = torch.empty(4, dtype=torch.float64, device=Y.device)
        call("mdsdp_update_multiplier", self._h, Y.shape[1], _ptr(Y), _ptr(y), _ptr(z), _ptr(kkt), _stream())
        return y, z, kkt

    def certificate_matvec(self, V: torch.Tensor) -> torch.Tensor:
        _dev_f64(V, "V")
        XV = torch.empty_like(V)
        call("mdsdp_certificate_matvec", self._h, V.shape[1], _ptr(V), _ptr(XV), _stream())
        return XV

    def min_eigpairs(self, k: int = 1, tol: float = 1e-10, maxit: int = 300, seed: int = 0):
        """The k smallest eigenpairs of the certificate and its largest
        eigenvalue: (evals (k,), lambda_max, evecs (k, n) device, iters,
        converged)."""
        ev = np.empty(k, dtype=np.float64)
        lmax = C.c_double()
        it = C.c_int32()
        V = torch.empty(k, self.n, dtype=torch.float64, device="cuda")
        code = lib().mdsdp_min_eigpair(self._h, k, tol, maxit, seed, _ptr(ev), C.byref(lmax), _ptr(V),
                                        C.byref(it), _stream())
        if code not in (0, -7):
            _lib.check(code, "mdsdp_min_eigpair")
        return ev, lmax.value, V, it.value, code == 0

    def min_eigpair(self, tol: float = 1e-10, maxit: int = 300, seed: int = 0):
        ev, lmax, V, it, conv = self.min_eigpairs(1, tol, maxit, seed)
        return float(ev[0]), lmax, V[0], it, conv

    def certificate_estimate(self, tol: float = 1e-10, maxit: int = 300, seed: int = 0, warm=None) -> dict:
        """The solver's estimate of the certificate's extreme eigenvalues (see
        mdsdp_certificate_estimate)."""
        out = np.zeros(4, dtype=np.float64)
        v = torch.empty(self.n, dtype=torch.float64, device="cuda")
        it = C.c_int32()
        if warm is not None:
            warm = _dev_f64(warm.contiguous(), "warm")
        call("mdsdp_certificate_estimate", self._h, tol, maxit, seed, _ptr(warm), _ptr(out), _ptr(v),
             C.byref(it), _stream())
        return {"theta_min": float(out[0]), "theta_max": float(out[1]), "err": float(out[2]),
                "converged": bool(out[3]), "evec": v, "iters": it.value}

    def certificate_bound(self, Y: torch.Tensor, tol: float = 1e-10, maxit: int = 1200, seed: int = 0) -> dict:
        """The certified lower bound of lambda_min of the certificate that a
        solve ends on, deflated against range(Y) (mdsdp_certificate_bound)."""
        _dev_f64(Y, "Y")
        out = np.zeros(4, dtype=np.float64)
        call("mdsdp_certificate_bound", self._h, Y.shape[1], _ptr(Y), tol, maxit, seed, _ptr(out), _stream())
        return {"lower": float(out[0]), "theta_max": float(out[1]), "iters": int(out[2]),
                "converged": bool(out[3])}

    def set_direct(self, on: bool, Y: torch.Tensor | None = None) -> None:
        """Switch to (or from) the direct-DSDP ADMM subproblem; with Y the
        stale class averages y^k are taken at Y."""
        if Y is not None:
            _dev_f64(Y, "Y")
        call("mdsdp_set_direct", self._h, 1 if on else 0, 0 if Y is None else Y.shape[1], _ptr(Y), _stream())

    def sync_status(self) -> None:
        """Raise MdsdpError(MDSDP_ENONFINITE) if a kernel met a non-finite value
        since the last set_multiplier (synchronises the stream)."""
        call("mdsdp_sync_status", self._h, _stream())

    def adjoint_C(self) -> torch.Tensor:
        X = torch.empty(self.n, self.n, dtype=torch.float64, device="cuda")
        call("mdsdp_adjoint_C", self._h, _ptr(X), _stream())
        return X

    def export_classmap(self) -> np.ndarray:
        out = np.empty(self.n * (self.n + 1) // 2, dtype=np.int32)
        call("mdsdp_export_classmap", self._h, _ptr(out))
        return out

    def export_multiplier_packed(self) -> np.ndarray:
        out = np.empty(self.n * (self.n + 1) // 2, dtype=np.float64)
        call("mdsdp_export_multiplier_packed", self._h, _ptr(out))
        return out

    def time_product_pass(self, reps: int = 50) -> float:
        """Average duration in microseconds of the HVP product pass of the last
        hvp() call, re-launched `reps` times between two HIP events on the
        current stream."""
        us = C.c_double()
        call("mdsdp_time_product_pass", self._h, int(reps), C.byref(us), _stream())
        return us.value

    def enable_timing(self, on: bool = True) -> None:
        call("mdsdp_enable_timing", self._h, 1 if on else 0)

    def kernel_times(self) -> list[tuple[str, float]]:
        cap = 1 << 16
        buf = np.empty(cap, dtype=np.float64)
        cnt = C.c_int32()
        call("mdsdp_kernel_times", self._h, _ptr(buf), cap, C.byref(cnt))
        names = lib().mdsdp_last_error().decode().split(";")[: cnt.value]
        return list(zip(names, buf[: cnt.value].tolist()))

    # ---- solve ------------------------------------------------------------------
    @staticmethod
    def default_options() -> Options:
        o = Options()
        lib().mdsdp_default_options(C.byref(o))
        return o

    @staticmethod
    def solve_batch(problems, Y0s, opts: Options | None = None, nworkers: int = 4):
        """Solve independent problems concurrently (mdsdp_solve_batch): returns
        one (Y, Result) pair per problem."""
        nprob = len(problems)
        opts = opts or problems[0].default_options()
        handles = (C.c_void_p * nprob)(*[pr._h for pr in problems])
        p0 = (C.c_int32 * nprob)(*[int(Y.shape[1]) for Y in Y0s])
        bufs = []
        for pr, Y in zip(problems, Y0s):
            _dev_f64(Y, "Y0")
            b = torch.zeros(pr.n * max(opts.p_max, Y.shape[1]), dtype=torch.float64, device=Y.device)
            b[: pr.n * Y.shape[1]] = Y.reshape(-1)
            bufs.append(b)
        ptrs = (C.c_void_p * nprob)(*[b.data_ptr() for b in bufs])
        res = (Result * nprob)()
        torch.cuda.current_stream().synchronize()
        code = lib().mdsdp_solve_batch(nprob, handles, C.byref(opts), p0, ptrs, res, nworkers)
        if code not in (0, -7):
            _lib.check(code, "mdsdp_solve_batch")
        out = []
        for pr, b, r in zip(problems, bufs, res):
            out.append((b[: pr.n * r.p_final].reshape(pr.n, r.p_final).clone(), r))
        return out

    def solve(self, Y0: torch.Tensor, opts: Options | None = None, history_cap: int = 1000) -> SolveResult:
        self._ad_key = None
        _dev_f64(Y0, "Y0")
        opts = opts or self.default_options()
        n, p0 = Y0.shape
        Ybuf = torch.zeros(n * max(opts.p_max, p0), dtype=torch.float64, device=Y0.device)
        Ybuf[: n * p0] = Y0.reshape(-1)
        res = Result()
        hist = np.zeros((history_cap, 8), dtype=np.float64)
        code = lib().mdsdp_solve(self._h, C.byref(opts), p0, _ptr(Ybuf), C.byref(res), _ptr(hist), history_cap,
                                 _stream())
        if code not in (0, -7):
            _lib.check(code, "mdsdp_solve")
        torch.cuda.current_stream().synchronize()
        Y = Ybuf[: n * res.p_final].reshape(n, res.p_final).clone()
        return SolveResult(Y=Y, value=res.value, eta=(res.eta_p, res.eta_d, res.eta_g), status=res.status,
                           outer_iters=res.outer_iters, rtr_iters=res.rtr_iters, hvps=res.hvps,
                           cost_grads=res.cost_grads, eig_iters=res.eig_iters, p_final=res.p_final,
                           p_max_reached=res.p_max_reached, sigma=res.sigma, seconds=res.seconds,
                           phases=dict(eval=res.t_eval, hvp=res.t_hvp, eig=res.t_eig, update=res.t_update),
                           history=hist[: min(res.outer_iters, history_cap)].copy(),
                           rank_one_round=bool(res.rank_one_round))

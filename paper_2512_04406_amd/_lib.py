"""ctypes binding of libmanidsdp.so (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
device tensors and NumPy host arrays to pointers and checks return codes.  If
the shared library is missing, every call raises: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmanidsdp.so")

_i32, _i64, _u64, _f64, _vp = C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_void_p
_pi32, _pf64, _pi64 = C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int64)

STATUS = {0: "MDSDP_OK", -1: "MDSDP_EINVAL", -2: "MDSDP_ENOMEM", -3: "MDSDP_EHIP", -4: "MDSDP_ENOTORTH",
          -5: "MDSDP_ENONFINITE", -6: "MDSDP_EUNSUPPORTED", -7: "MDSDP_ENOCONV"}


class MdsdpError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("tol", _f64), ("max_outer", _i32), ("sigma0", _f64), ("sigma_min", _f64),
                ("sigma_max", _f64), ("gamma", _f64), ("kappa1", _f64), ("kappa2", _f64),
                ("p_max", _i32), ("n_neg", _i32), ("tau_rank", _f64), ("gtol0", _f64), ("gtol_min", _f64),
                ("gtol_decay", _f64), ("gtol_ratio", _f64),
                ("gtol_stall", _f64), ("sigma_hold", _i32),
                ("rtr_maxiter", _i32), ("tcg_maxinner", _i32), ("hvp_prec", _i32),
                ("polish_fp64", _i32), ("polish_eta", _f64), ("eig_tol", _f64), ("eig_maxit", _i32),
                ("time_limit_s", _f64), ("verbose", _i32), ("seed", _u64),
                ("resume", _i32), ("escape_when_solved", _i32), ("deflate", _i32),
                ("direct_admm", _i32), ("rtr_warm_radius", _i32), ("rtr_maxiter_polish", _i32),
                ("round_rank_one", _i32), ("round_eta", _f64), ("round_gap", _f64),
                ("tcg_maxinner_polish", _i32), ("rtr_stall", _i32)]


class Result(C.Structure):
    _fields_ = [("status", _i32), ("outer_iters", _i32), ("rtr_iters", _i64), ("hvps", _i64),
                ("cost_grads", _i64), ("eig_iters", _i64), ("p_final", _i32), ("p_max_reached", _i32),
                ("value", _f64), ("eta_p", _f64), ("eta_d", _f64), ("eta_g", _f64), ("sigma", _f64),
                ("seconds", _f64), ("t_eval", _f64), ("t_hvp", _f64), ("t_eig", _f64), ("t_update", _f64),
                ("rank_one_round", _i32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "mdsdp_last_error": (C.c_char_p, []),
    "mdsdp_version": (C.c_char_p, []),
    "mdsdp_bqp_sizes": (_i32, [_i32, _pi32, _pi64]),
    "mdsdp_bqp_classmap": (_i32, [_i32, _i32, _vp]),
    "mdsdp_bqp_b": (_i32, [_i32, _vp, _vp, _vp]),
    "mdsdp_create_classmap": (_i32, [_i32, _i64, _vp, _vp, _vp, C.POINTER(_vp)]),
    "mdsdp_create_bqp": (_i32, [_i32, _i32, _vp, _vp, C.POINTER(_vp)]),
    "mdsdp_ucqp_sizes": (_i32, [_i32, _pi32, _pi64]),
    "mdsdp_ucqp_structure": (_i32, [_i32, _vp, _vp]),
    "mdsdp_ucqp_b": (_i32, [_i32, _vp, _vp, _vp]),
    "mdsdp_create_ucqp": (_i32, [_i32, _vp, _vp, C.POINTER(_vp)]),
    "mdsdp_create_sparse_A": (_i32, [_i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "mdsdp_destroy": (_i32, [_vp]),
    "mdsdp_problem_info": (_i32, [_vp, _pi32, _pi64, _pi64, _pi32]),
    "mdsdp_set_multiplier": (_i32, [_vp, _vp, _f64, _vp]),
    "mdsdp_get_multiplier": (_i32, [_vp, _vp, _vp]),
    "mdsdp_set_sigma": (_i32, [_vp, _f64]),
    "mdsdp_cost_grad": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mdsdp_hvp": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp]),
    "mdsdp_class_average": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "mdsdp_retract": (_i32, [_i32, _i32, _vp, _vp, _f64, _vp, _vp]),
    "mdsdp_project_tangent": (_i32, [_i32, _i32, _vp, _vp, _vp, _vp]),
    "mdsdp_update_multiplier": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mdsdp_certificate_matvec": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "mdsdp_min_eigpair": (_i32, [_vp, _i32, _f64, _i32, _u64, _vp, _pf64, _vp, _pi32, _vp]),
    "mdsdp_sync_status": (_i32, [_vp, _vp]),
    "mdsdp_min_eigpair_noalloc": (_i32, [_vp, _i32, _f64, _i32, _u64, _vp, _pf64, _vp, _pi32, _vp]),
    "mdsdp_set_direct": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "mdsdp_certificate_bound": (_i32, [_vp, _i32, _vp, _f64, _i32, _u64, _vp, _vp]),
    "mdsdp_certificate_estimate": (_i32, [_vp, _f64, _i32, _u64, _vp, _vp, _vp, _pi32, _vp]),
    "mdsdp_adjoint_C": (_i32, [_vp, _vp, _vp]),
    "mdsdp_default_options": (None, [C.POINTER(Options)]),
    "mdsdp_solve": (_i32, [_vp, C.POINTER(Options), _i32, _vp, C.POINTER(Result), _vp, _i32, _vp]),
    "mdsdp_solve_batch": (_i32, [_i32, _vp, C.POINTER(Options), _vp, _vp, _vp, _i32]),
    "mdsdp_export_classmap": (_i32, [_vp, _vp]),
    "mdsdp_export_multiplier_packed": (_i32, [_vp, _vp]),
    "mdsdp_kernel_times": (_i32, [_vp, _vp, _i32, _pi32]),
    "mdsdp_enable_timing": (_i32, [_vp, _i32]),
    "mdsdp_time_product_pass": (_i32, [_vp, _i32, _pf64, _vp]),
}

_lib = None


def lib():
    """Load libmanidsdp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2512_04406_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, func: str) -> None:
    if code != 0:
        raise MdsdpError(code, func, lib().mdsdp_last_error().decode(errors="replace"))


def call(name: str, *args) -> int:
    code = getattr(lib(), name)(*args)
    check(code, name)
    return code

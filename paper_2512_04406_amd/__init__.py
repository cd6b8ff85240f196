"""ManiDSDP subproblem hot path on AMD Instinct MI355X (gfx950).

The computation lives in libmanidsdp.so (HIP kernels + C ABI declared in
include/manidsdp.h); `problem.Problem` binds it with ctypes and uses PyTorch
only for device memory and streams.
"""

__all__ = ["Problem", "bqp_classmap", "bqp_b", "bqp_sizes", "FP64", "FP32", "ORDER_LEX", "ORDER_COLEX"]


def __getattr__(name):
    if name in __all__:
        from . import problem

        return getattr(problem, name)
    raise AttributeError(name)

"""ctypes declarations of the kronpcg C ABI (include/kronpcg.h).

Argument marshalling only: no arithmetic of the method lives here.  Loading
fails loudly when the built library is missing; there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkronpcg.so")

KP_OK = 0
KP_NOT_CONVERGED = 1
KP_WARN_RHS_MEAN = 2
KP_ERR_ARG = -1
KP_ERR_HIP = -2
KP_ERR_NOMEM = -3
KP_ERR_BREAKDOWN = -4
KP_ERR_PRECOND_INDEFINITE = -5
KP_ERR_STATE = -6

KP_FP64 = 0
KP_MIXED_BF16 = 1
KP_MIXED_FP16 = 2

PRECISIONS = {"fp64": KP_FP64, "mixed_bf16": KP_MIXED_BF16, "mixed_fp16": KP_MIXED_FP16}


class PrecondInfo(C.Structure):
    _fields_ = [("rank", C.c_int), ("tucker_rank", C.c_int), ("source", C.c_int), ("pad_", C.c_int),
                ("cp_rel_err", C.c_double), ("quad_rel_err", C.c_double), ("rho_min", C.c_double),
                ("rho_max", C.c_double), ("cancellation", C.c_double), ("build_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("replace_every", C.c_int),
                ("use_x0", C.c_int), ("check_every", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("replacements", C.c_int), ("relres_true", C.c_double),
                ("relres_rec", C.c_double), ("rhs_mean", C.c_double), ("ms", C.c_double),
                ("status", C.c_int), ("pad_", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MCStats(C.Structure):
    _fields_ = [("realizations", C.c_int), ("batch", C.c_int), ("chunks", C.c_int), ("status", C.c_int),
                ("iters", C.c_longlong), ("max_relres_true", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TileTiming(C.Structure):
    _fields_ = [("stage", C.c_int), ("bm", C.c_int), ("bn", C.c_int), ("bk", C.c_int), ("order", C.c_int),
                ("circ", C.c_int), ("ms", C.c_double)]


TIMERS = ("stencil", "gemm_mode3", "gemm_mode2", "gemm_mode1", "vector", "assemble", "residual")

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# name -> (restype, argtypes); every symbol declared in include/kronpcg.h.
SIGNATURES = {
    "kp_context_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "kp_context_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kp_context_set_allocator": (C.c_int, [C.c_void_p, ALLOC_FN, RELEASE_FN, C.c_void_p]),
    "kp_context_destroy": (C.c_int, [C.c_void_p]),
    "kp_context_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "kp_context_read_timing": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "kp_coeff_update": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "setup_coeff": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                              C.POINTER(C.c_void_p)]),
    "build_preconditioner_fft": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "setup_coeff_2d": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double),
                                 C.c_int, C.POINTER(C.c_void_p)]),
    "kp_lowrank_factors_2d": (C.c_int, [C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double), C.c_size_t,
                                        C.POINTER(PrecondInfo)]),
    "build_preconditioner_2d": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int,
                                          C.POINTER(C.c_void_p), C.POINTER(PrecondInfo)]),
    "kp_precond_from_factors_2d": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                                             C.POINTER(C.c_void_p)]),
    "setup_coeff_inclusions": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double,
                                         C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_void_p)]),
    "kp_coeff_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "kp_coeff_size": (C.c_int, [C.c_void_p]),
    "kp_free_coeff": (C.c_int, [C.c_void_p]),
    "kp_stiffness_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "kp_lowrank_factors": (C.c_int, [C.c_int, C.c_double, C.c_int, C.POINTER(C.c_double), C.c_size_t,
                                     C.POINTER(PrecondInfo)]),
    "build_preconditioner": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int,
                                       C.POINTER(C.c_void_p), C.POINTER(PrecondInfo)]),
    "kp_precond_from_factors": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                                          C.POINTER(C.c_void_p)]),
    "kp_precond_rank": (C.c_int, [C.c_void_p]),
    "kp_precond_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(TileTiming), C.c_int,
                                      C.POINTER(C.c_int)]),
    "kp_precond_set_tiles": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "kp_precond_get_tiles": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "kp_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "kp_free_precond": (C.c_int, [C.c_void_p]),
    "pcg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                            C.POINTER(SolveOpts), C.POINTER(SolveStats)]),
    "kp_mc_homogenize": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                   C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_int,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.c_void_p]),
    "pcg_solve_batched": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.POINTER(SolveOpts), C.POINTER(SolveStats),
                                    C.POINTER(C.c_double)]),
    "kp_homogenized_matrix": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_double)]),
    "kp_last_error": (C.c_char_p, []),
}

_lib = None


def load() -> C.CDLL:
    """Load libkronpcg.so (built by paper_2007_06524_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_2007_06524_amd/build.py`; the solver has no fallback path")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class KronPCGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kronpcg status {status}: {msg}")
        self.status = status


def check(status: int, allow=(KP_OK,)) -> int:
    if status in allow or status == KP_OK:
        return status
    if status > 0:
        return status
    msg = load().kp_last_error()
    raise KronPCGError(status, msg.decode() if msg else "")

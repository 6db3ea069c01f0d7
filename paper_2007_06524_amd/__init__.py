"""kronpcg: periodic 3D checkerboard PCG solver with a low-Kronecker-rank
preconditioner on MI355X (gfx950).

Python binding of the C ABI in include/kronpcg.h.  PyTorch supplies device
memory (its caching allocator backs the library's allocations) and streams;
every step of the solve runs in the library's HIP kernels.  There is no CPU
fallback: without the built library or a GPU the calls raise.

Method: Khoromskaia & Khoromskij, arXiv:2007.06524 (assembly, Section 3;
preconditioner, Section 4.2; PCG, Section 4.1; homogenized matrix, Section 3.4).
"""

from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _lib
from ._lib import (KP_FP64, KP_MIXED_BF16, KP_MIXED_FP16, KP_NOT_CONVERGED, KP_OK,
                   KP_WARN_RHS_MEAN, PRECISIONS, KronPCGError, PrecondInfo, SolveOpts, SolveStats,
                   check, load)

__all__ = ["Context", "Coeff", "Precond", "solve", "solve_batched", "homogenized_matrix", "stiffness_apply",
           "lowrank_factors", "lowrank_factors_2d", "mc_homogenize", "KronPCGError", "PRECISIONS", "KP_FP64", "KP_MIXED_BF16",
           "KP_MIXED_FP16", "KP_OK", "KP_NOT_CONVERGED", "KP_WARN_RHS_MEAN"]

_live_contexts = weakref.WeakSet()


def _precision(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _ptr(t) -> C.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Context:
    """Device, stream and allocator of the library (kp_context)."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True):
        import torch
        lib = load()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        check(lib.kp_context_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self._cb = None
        if torch_allocator:
            dev, strm = device, self.stream

            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)
                except Exception:
                    return None

            def _release(ptr, user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._cb = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
            check(lib.kp_context_set_allocator(h, self._cb[0], self._cb[1], None))
        self._owned = []
        _live_contexts.add(self)

    def set_timing(self, enable: bool = True):
        """Start (and clear) or stop per-kernel-class HIP event timing."""
        check(load().kp_context_set_timing(self.handle, int(bool(enable))))

    def read_timing(self):
        """{class: (total ms, launches)} accumulated since set_timing(True)."""
        n = len(_lib.TIMERS)
        ms = (C.c_double * n)()
        cnt = (C.c_longlong * n)()
        check(load().kp_context_read_timing(self.handle, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.TIMERS)}

    def close(self):
        if getattr(self, "handle", None) is not None:
            for obj in list(self._owned):
                obj.free()
            load().kp_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@atexit.register
def _close_all():
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Coeff:
    """An assembled coefficient realization (setup_coeff): weights and correctors' RHS.

    inclusion, background: the cell value only on the centred sub-cell of
    `inclusion` voxels per edge, `background` elsewhere (setup_coeff_inclusions)."""

    def __init__(self, ctx: Context, cells: np.ndarray, n0: int, precision="fp64",
                 inclusion: int | None = None, background: float | None = None):
        cells = np.ascontiguousarray(cells, dtype=np.float64)
        if cells.ndim not in (2, 3) or len(set(cells.shape)) != 1:
            raise ValueError("cells must be an (L, L, L) array, or (L, L) for the 2D problem")
        self.ctx = ctx
        self.dim = cells.ndim
        self.L = cells.shape[0]
        self.n0 = int(n0)
        self.precision = _precision(precision)
        self.inclusion = self.n0 if inclusion is None else int(inclusion)
        self.background = 0.0 if background is None else float(background)
        h = C.c_void_p()
        setup = load().setup_coeff_2d if self.dim == 2 else load().setup_coeff_inclusions
        check(setup(ctx.handle, self.L, self.n0, self.inclusion, self.background,
                    cells.ctypes.data_as(C.POINTER(C.c_double)), self.precision, C.byref(h)))
        self.handle = h
        self.N = self.L * self.n0
        ctx._owned.append(self)

    def update(self, cells_dev):
        """Re-assemble from a new realization already on the device (float64 (L, L, L))."""
        import torch
        if tuple(cells_dev.shape) != (self.L,) * self.dim:
            raise ValueError("cells_dev must have shape (L,) * dim")
        check(load().kp_coeff_update(self.ctx.handle, self.handle, _ptr(cells_dev)))

    def fields(self):
        """(w, f): torch float64 tensors of shape (d, N, ..., N) (d = 3 or 2)."""
        import torch
        N = self.N
        w = torch.empty((self.dim,) + (N,) * self.dim, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        f = torch.empty_like(w)
        check(load().kp_coeff_fields(self.ctx.handle, self.handle, _ptr(w), _ptr(f)))
        return w, f

    def free(self):
        if self.handle is not None:
            load().kp_free_coeff(self.handle)
            self.handle = None
            if self in self.ctx._owned:
                self.ctx._owned.remove(self)


class Precond:
    """Low-rank preconditioner (build_preconditioner / kp_precond_from_factors), or with
    fft=True the exact FFT-diagonalized one (build_preconditioner_fft, FP64)."""

    def __init__(self, ctx: Context, N: int, eps: float = 1e-3, rank: int = 0, precision="fp64",
                 factors: np.ndarray | None = None, fft: bool = False, dim: int = 3):
        self.ctx = ctx
        self.N = int(N)
        self.dim = int(dim)
        self.precision = _precision(precision)
        h = C.c_void_p()
        lib = load()
        if self.dim == 2:
            if fft:
                raise ValueError("the FFT preconditioner is 3D")
            if factors is None:
                info = PrecondInfo()
                check(lib.build_preconditioner_2d(ctx.handle, self.N, float(eps), int(rank), self.precision,
                                                  C.byref(h), C.byref(info)))
                self.info = info.as_dict()
            else:
                F = np.ascontiguousarray(factors, dtype=np.float64)
                if F.ndim != 3 or F.shape[0] != 2 or F.shape[2] != self.N:
                    raise ValueError("2D factors must have shape (2, R, N)")
                check(lib.kp_precond_from_factors_2d(ctx.handle, self.N, F.shape[1],
                                                     F.ctypes.data_as(C.POINTER(C.c_double)), self.precision,
                                                     C.byref(h)))
                self.info = {"rank": F.shape[1]}
        elif fft:
            if self.precision != KP_FP64 or factors is not None:
                raise ValueError("the FFT preconditioner is FP64 and takes no factors")
            check(lib.build_preconditioner_fft(ctx.handle, self.N, C.byref(h)))
            self.info = {"rank": 0, "rho_min": 1.0, "rho_max": 1.0, "fft": True}
        elif factors is None:
            info = PrecondInfo()
            check(lib.build_preconditioner(ctx.handle, self.N, float(eps), int(rank), self.precision,
                                           C.byref(h), C.byref(info)))
            self.info = info.as_dict()
        else:
            F = np.ascontiguousarray(factors, dtype=np.float64)
            if F.ndim != 3 or F.shape[0] != 3 or F.shape[2] != self.N:
                raise ValueError("factors must have shape (3, R, N)")
            check(lib.kp_precond_from_factors(ctx.handle, self.N, F.shape[1],
                                              F.ctypes.data_as(C.POINTER(C.c_double)), self.precision,
                                              C.byref(h)))
            self.info = {"rank": F.shape[1]}
        self.handle = h
        self.R = lib.kp_precond_rank(h)
        ctx._owned.append(self)

    def autotune(self, reps: int = 5):
        """Time the tile configurations of the three GEMM stages and keep the fastest.

        Returns [(stage, bm, bn, bk, order, kernel, ms), ...] for every configuration
        timed; kernel 0 streams both operands, 1 builds the circulant operand in LDS,
        2 streams the data operand per wave."""
        cap = 256
        table = (_lib.TileTiming * cap)()
        n = C.c_int(0)
        check(load().kp_precond_autotune(self.ctx.handle, self.handle, int(reps), table, cap, C.byref(n)))
        return [(t.stage, t.bm, t.bn, t.bk, t.order, t.circ, t.ms) for t in table[:min(n.value, cap)]]

    @property
    def tiles(self):
        """Tile configuration index per GEMM stage (-1: size heuristic)."""
        t = (C.c_int * 3)()
        check(load().kp_precond_get_tiles(self.handle, t))
        return tuple(t)

    @tiles.setter
    def tiles(self, value):
        t = (C.c_int * 3)(*[int(v) for v in value])
        check(load().kp_precond_set_tiles(self.handle, t))

    def apply(self, r):
        """z = sum_k (C1^k x C2^k x C3^k) r, r a float64 CUDA tensor (N, N, N)."""
        import torch
        z = torch.empty_like(r)
        check(load().kp_precond_apply(self.ctx.handle, self.handle, _ptr(r), _ptr(z)))
        return z

    def free(self):
        if self.handle is not None:
            load().kp_free_precond(self.handle)
            self.handle = None
            if self in self.ctx._owned:
                self.ctx._owned.remove(self)


def stiffness_apply(ctx: Context, coeff: Coeff, p, precision=None):
    """q = K p for the assembled stiffness (float64 CUDA tensors)."""
    import torch
    q = torch.empty_like(p)
    prec = coeff.precision if precision is None else _precision(precision)
    check(load().kp_stiffness_apply(ctx.handle, coeff.handle, prec, _ptr(p), _ptr(q)))
    return q


def solve(ctx: Context, coeff: Coeff, precond: Precond, rhs: int = 1, f=None, x=None,
          tol: float = 1e-8, maxit: int = 2000, replace_every: int | None = None,
          use_x0: bool = False, check_every: int = 0):
    """pcg_solve: returns (x, stats dict, status)."""
    import torch
    N = coeff.N
    if x is None:
        x = torch.empty((N,) * coeff.dim, dtype=torch.float64, device=f"cuda:{ctx.device}")
    if replace_every is None:
        replace_every = 0 if coeff.precision == KP_FP64 else 25
    opts = SolveOpts(float(tol), int(maxit), int(replace_every), int(bool(use_x0)), int(check_every))
    stats = SolveStats()
    fp = _ptr(f) if f is not None else None
    st = load().pcg_solve(ctx.handle, coeff.handle, precond.handle, int(rhs), fp, _ptr(x),
                          C.byref(opts), C.byref(stats))
    check(st, allow=(KP_OK, KP_NOT_CONVERGED, KP_WARN_RHS_MEAN))
    return x, stats.as_dict(), st


def solve_batched(ctx: Context, coeffs, preconds, xs=None, tol: float = 1e-8, maxit: int = 2000,
                  replace_every: int | None = None, use_x0: bool = False, check_every: int = 0,
                  want_ahom: bool = True):
    """pcg_solve_batched: the three correctors of every instance (coeffs[i], preconds[i]).

    xs: optional list of 3 * len(coeffs) float64 CUDA tensors (N_i, N_i, N_i) (initial
    guesses with use_x0).  Returns (xs, [stats dict per system], ahom (n, 3, 3) or None, status)."""
    import torch
    n = len(coeffs)
    if len(preconds) != n:
        raise ValueError("one preconditioner per coefficient")
    if xs is None:
        xs = [torch.empty((c.N, c.N, c.N), dtype=torch.float64, device=f"cuda:{ctx.device}")
              for c in coeffs for _ in range(3)]
    if len(xs) != 3 * n:
        raise ValueError("xs needs three tensors per instance")
    if replace_every is None:
        replace_every = 0 if coeffs[0].precision == KP_FP64 else 25
    opts = SolveOpts(float(tol), int(maxit), int(replace_every), int(bool(use_x0)), int(check_every))
    stats = (SolveStats * (3 * n))()
    ch = (C.c_void_p * n)(*[c.handle for c in coeffs])
    ph = (C.c_void_p * n)(*[p.handle for p in preconds])
    xp = (C.c_void_p * (3 * n))(*[_ptr(x) for x in xs])
    ah = (C.c_double * (9 * n))() if want_ahom else None
    st = load().pcg_solve_batched(ctx.handle, n, ch, ph, xp, C.byref(opts), stats, ah)
    check(st, allow=(KP_OK, KP_NOT_CONVERGED))
    A = np.frombuffer(ah, dtype=np.float64).reshape(n, 3, 3).copy() if want_ahom else None
    return xs, [s.as_dict() for s in stats], A, st


def mc_homogenize(ctx: Context, cells, n0: int, pc: Precond, inclusion: int | None = None,
                  background: float | None = None, tol: float = 1e-8, maxit: int = 2000,
                  replace_every: int | None = None, check_every: int = 0, batch: int = 0):
    """kp_mc_homogenize: a_hom of M realizations (cells: (M, L, L, L) float64) and the
    empirical mean and standard deviation (M - 1 normalization) of every entry.

    Returns (ahoms (M, 3, 3), mean (3, 3), std (3, 3), stats dict, status)."""
    cells = np.ascontiguousarray(cells, dtype=np.float64)
    if cells.ndim != 4 or len(set(cells.shape[1:])) != 1:
        raise ValueError("cells must be an (M, L, L, L) array")
    M, L = cells.shape[0], cells.shape[1]
    incl = int(n0) if inclusion is None else int(inclusion)
    bg = 0.0 if background is None else float(background)
    if replace_every is None:
        replace_every = 0 if pc.precision == KP_FP64 else 25
    opts = SolveOpts(float(tol), int(maxit), int(replace_every), 0, int(check_every))
    ah = np.zeros((M, 3, 3))
    mean = np.zeros((3, 3))
    sd = np.zeros((3, 3))
    st = _lib.MCStats()
    dp = C.POINTER(C.c_double)
    status = load().kp_mc_homogenize(ctx.handle, L, int(n0), incl, bg, M, cells.ctypes.data_as(dp),
                                     pc.handle, C.byref(opts), int(batch), ah.ctypes.data_as(dp),
                                     mean.ctypes.data_as(dp), sd.ctypes.data_as(dp), C.byref(st))
    check(status, allow=(KP_OK, KP_NOT_CONVERGED))
    return ah, mean, sd, st.as_dict(), status


def homogenized_matrix(ctx: Context, coeff: Coeff, phis) -> np.ndarray:
    """kp_homogenized_matrix: d x d numpy array from the d corrector solutions."""
    d = coeff.dim
    arr = (C.c_void_p * 3)(*([_ptr(p).value for p in phis[:d]] + [None] * (3 - d)))
    out = (C.c_double * 9)()
    check(load().kp_homogenized_matrix(ctx.handle, coeff.handle, arr, out))
    return np.array(list(out)[:d * d]).reshape(d, d)


def lowrank_factors_2d(N: int, eps: float = 1e-3, rank: int = 0):
    """kp_lowrank_factors_2d (host only): factors (2, R, N) and the report."""
    cap = 2 * 16 * N
    buf = (C.c_double * cap)()
    info = PrecondInfo()
    check(load().kp_lowrank_factors_2d(int(N), float(eps), int(rank), buf, cap, C.byref(info)))
    R = info.rank
    F = np.frombuffer(buf, dtype=np.float64, count=2 * R * N).reshape(2, R, N).copy()
    return F, info.as_dict()


def lowrank_factors(N: int, eps: float = 1e-3, rank: int = 0):
    """kp_lowrank_factors (host only): canonical factors (3, R, N) and the report."""
    cap = 3 * 16 * N
    buf = (C.c_double * cap)()
    info = PrecondInfo()
    check(load().kp_lowrank_factors(int(N), float(eps), int(rank), buf, cap, C.byref(info)))
    R = info.rank
    F = np.frombuffer(buf, dtype=np.float64, count=3 * R * N).reshape(3, R, N).copy()
    return F, info.as_dict()

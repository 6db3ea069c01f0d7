"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
solver's arithmetic (no assembly, no stencil, no preconditioner, no PCG).
Every coefficient realization is a cell array of shape (L, L, L), float64,
C order with the first lattice index slowest (the big-endian convention of
the paper's Section 3.2), one value per unit cell G_s of the checkerboard
(Section 3.1: the coefficient is piecewise constant on the L^3 unit cells).

The named workloads mirror the paper's 3D experiments (Section 5.2, Table 3:
n0 = 4 grid intervals per cell edge, L up to 128) with the value laws of the
benchmark configurations:

  c1  L=4,   n0=4, a in {1, 10} with P(10) = 1/2, seed 1, corrector e_1, R = 4
  c2  L=32,  n0=4, a ~ U[1, 10],                  seed 2, correctors e_1..e_3
  c3  L=64,  n0=4, a in {1, 100} with P(100) = 1/2, seed 3, correctors e_1..e_3
  c4  96 realizations, L cycling over {8, 12, 16, 24}, a = exp(N(0, 1)),
      seeds SeedSequence(4).spawn(96)
  c5  L=128, n0=4, a = exp(N(0, 1.5^2)),           seed 5
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "cells_bernoulli",
    "cells_uniform",
    "cells_lognormal",
    "random_field",
    "CONFIGS",
    "config_cells",
    "batched_realizations",
    "mc_realizations",
    "MC_FIGURE",
]


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.default_rng(seed)
    return np.random.default_rng(np.random.SeedSequence(seed))


def cells_bernoulli(L: int, lo: float, hi: float, p: float, seed) -> np.ndarray:
    """i.i.d. two-valued cells: hi with probability p, lo otherwise."""
    g = _rng(seed)
    u = g.random((L, L, L))
    return np.where(u < p, float(hi), float(lo)).astype(np.float64)


def cells_uniform(L: int, lo: float, hi: float, seed) -> np.ndarray:
    """i.i.d. cells uniform on [lo, hi)."""
    g = _rng(seed)
    return (lo + (hi - lo) * g.random((L, L, L))).astype(np.float64)


def cells_lognormal(L: int, sigma: float, seed, mu: float = 0.0) -> np.ndarray:
    """i.i.d. cells exp(N(mu, sigma^2))."""
    g = _rng(seed)
    return np.exp(mu + sigma * g.standard_normal((L, L, L))).astype(np.float64)


def cells_two_contrast(L: int, lam: float, betas, p: float, seed, layered: bool = False,
                       layer: int = 2, dims: int = 3) -> np.ndarray:
    """Realizations with two contrast parameters (Section 2): a cell holds an
    inclusion with probability p, of value lam + beta; beta is betas[0] or
    betas[1] with equal probability, or, layered, betas[0] on the cells whose
    index along the first axis lies in an even block of `layer` cells and
    betas[1] on the others.  Cells without an inclusion take lam, which with
    sub-cell inclusions is the background."""
    g = _rng(seed)
    shape = (L,) * dims
    occupied = g.random(shape) < p
    if layered:
        even = (np.arange(L) // layer) % 2 == 0
        beta = np.broadcast_to(np.where(even, betas[0], betas[1]).reshape((L,) + (1,) * (dims - 1)), shape)
    else:
        beta = np.where(g.random(shape) < 0.5, betas[0], betas[1])
    return np.where(occupied, lam + beta, lam).astype(np.float64)


def random_field(N: int, seed, dims: int = 3) -> np.ndarray:
    """Standard-normal nodal field of shape (N,)*dims (test vectors)."""
    g = _rng(seed)
    return g.standard_normal((N,) * dims).astype(np.float64)


def even_factors(N: int, R: int, seed, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Random positive vectors u with u[i] = u[N - i], shape (3, R, N).

    Test inputs for the Kronecker-product apply (any even symbol gives a real
    symmetric circulant); the values are uniform on [lo, hi).
    """
    g = _rng(seed)
    half = lo + (hi - lo) * g.random((3, R, N // 2 + 1))
    idx = np.minimum(np.arange(N), N - np.arange(N))
    return half[:, :, idx].astype(np.float64)


CONFIGS = {
    "c1": dict(L=4, n0=4, law="bernoulli", lo=1.0, hi=10.0, p=0.5, seed=1,
               rank=4, eps=1e-3, tol=1e-8, rhs=(1,), precision="fp64"),
    "c2": dict(L=32, n0=4, law="uniform", lo=1.0, hi=10.0, seed=2,
               rank=0, eps=1e-3, tol=1e-8, rhs=(1, 2, 3), precision="fp64"),
    "c3": dict(L=64, n0=4, law="bernoulli", lo=1.0, hi=100.0, p=0.5, seed=3,
               rank=0, eps=1e-3, tol=1e-8, rhs=(1, 2, 3), precision="mixed_bf16"),
    "c5": dict(L=128, n0=4, law="lognormal", sigma=1.5, seed=5,
               rank=0, eps=1e-3, tol=1e-8, rhs=(1, 2, 3), precision="mixed_bf16"),
}


def config_cells(name: str) -> np.ndarray:
    """Cell array of a named single-realization workload."""
    c = CONFIGS[name]
    if c["law"] == "bernoulli":
        return cells_bernoulli(c["L"], c["lo"], c["hi"], c["p"], c["seed"])
    if c["law"] == "uniform":
        return cells_uniform(c["L"], c["lo"], c["hi"], c["seed"])
    if c["law"] == "lognormal":
        return cells_lognormal(c["L"], c["sigma"], c["seed"])
    raise KeyError(c["law"])


def batched_realizations(count: int = 96, sizes=(8, 12, 16, 24), sigma: float = 1.0,
                         seed: int = 4):
    """Realizations with uneven L cycling over `sizes`, log-normal cells."""
    children = np.random.SeedSequence(seed).spawn(count)
    return [cells_lognormal(sizes[m % len(sizes)], sigma, children[m]) for m in range(count)]


def mc_realizations(L: int, M: int, lo: float, hi: float, p: float, seed: int) -> np.ndarray:
    """M i.i.d. two-valued realizations on the L^3 lattice, shape (M, L, L, L).

    Realization m draws from its own child of SeedSequence((seed, L)), so the
    first M realizations do not depend on how many more are drawn.
    """
    children = np.random.SeedSequence((seed, L)).spawn(M)
    return np.stack([cells_bernoulli(L, lo, hi, p, children[m]) for m in range(M)])


# The paper's Monte-Carlo experiment in 3D (Fig. Emp_a12_M20): n0 = 4,
# alpha = 1/4 (sub-cells of 2 voxels per edge), binary {lambda = 0.4, 1} with
# lambda as the background, L = 2^p, M realizations per L.  The probability of
# a perturbed cell is not stated; 1/2 is used.
MC_FIGURE = dict(n0=4, incl=2, background=0.4, lo=0.4, hi=1.0, p=0.5, sizes=(2, 4, 8, 16, 32, 64),
                 M=100, seed=6)

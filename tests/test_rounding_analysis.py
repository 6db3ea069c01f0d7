"""Why the 16-bit circulants are stored as hi + lo (CPU analysis).

Rounding the dense entries of a circulant keeps it circulant, so the symbol
of the rounded preconditioner is computable exactly: rounding once to BF16
makes it indefinite at N = 256 (some G_R * g < 0), the two-term split keeps
the double-precision range.  Uses the library's host factor construction."""

import os

import numpy as np
import pytest

from conftest import ROOT

pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(ROOT, "paper_2007_06524_amd", "libkronpcg.so")),
    reason="library not built")


def _bf16(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rho_range(F, rnd):
    N = F.shape[2]
    H = N // 2 + 1
    mu = 4 * np.sin(np.pi * np.arange(N) / N) ** 2
    g = mu[:H, None, None] + mu[None, :H, None] + mu[None, None, :H]
    cos = np.cos(2 * np.pi * np.outer(np.arange(N), np.arange(N)) / N)
    G = np.zeros((H, H, H))
    for k in range(F.shape[1]):
        us = [(cos @ rnd((cos @ F[l, k]) / N))[:H] for l in range(3)]
        G += us[0][:, None, None] * us[1][None, :, None] * us[2][None, None, :]
    rho = (G * g)[g > 0]
    return rho.min(), rho.max()


def test_single_bf16_rounding_is_indefinite_split_is_not():
    import paper_2007_06524_amd as kp
    F, info = kp.lowrank_factors(256, 1e-3, 7)
    lo, hi = _rho_range(F, lambda c: c)
    assert abs(lo - info["rho_min"]) < 1e-9 and abs(hi - info["rho_max"]) < 1e-9
    lo1, _ = _rho_range(F, _bf16)
    assert lo1 < 0.0
    split = lambda c: _bf16(c) + _bf16(c - _bf16(c))
    lo2, hi2 = _rho_range(F, split)
    assert abs(lo2 - lo) < 1e-3 * lo and abs(hi2 - hi) < 1e-3 * hi

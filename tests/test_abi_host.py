"""CPU tests of the C ABI: the library loads, exports every declared symbol, and
its host-only preconditioner construction matches the oracle's (Section 4.2)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2007_06524_amd", "libkronpcg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kronpcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    import paper_2007_06524_amd._lib as L
    names = declared_functions()
    assert len(names) >= 18
    lib = C.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


@pytest.mark.parametrize("N,eps,rank", [(8, 1e-3, 0), (16, 1e-3, 4), (16, 1e-3, 0), (24, 1e-4, 0),
                                        (32, 1e-3, 0), (48, 1e-3, 6), (64, 1e-3, 0), (15, 1e-3, 3)])
def test_lowrank_factors_match_oracle(N, eps, rank):
    import paper_2007_06524_amd as kp
    from oracle import lowrank as lr
    F, info = kp.lowrank_factors(N, eps, rank)
    Fo, io = lr.canonical_preconditioner(N, eps, rank)
    assert info["rank"] == io["R"] and info["tucker_rank"] == io["rT"]
    assert info["source"] == (0 if io["source"] == "als" else 1)
    GR, GRo = lr.symbol_from_factors(F), lr.symbol_from_factors(Fo)
    # The quadrature refinement is iterative (different linear solvers on the
    # two sides), so the two constructions agree to the refinement's accuracy.
    assert np.abs(GR - GRo).max() <= 1e-6 * np.abs(GRo).max()
    assert abs(info["rho_min"] - io["rho_min"]) < 1e-7
    assert abs(info["rho_max"] - io["rho_max"]) < 1e-7
    assert abs(info["quad_rel_err"] - io["quad_rel_err"]) < 1e-6 * io["quad_rel_err"]
    assert abs(info["cancellation"] - io["cancellation"]) < 1e-6 * io["cancellation"]
    np.testing.assert_allclose(F, F[:, :, (-np.arange(N)) % N], atol=0)   # even factors
    lo, hi = lr.rho_range(F)
    assert abs(lo - info["rho_min"]) < 1e-12 and abs(hi - info["rho_max"]) < 1e-12


def test_lowrank_factors_errors():
    import paper_2007_06524_amd as kp
    from paper_2007_06524_amd._lib import KP_ERR_ARG
    for args in [(1, 1e-3, 0), (16, 0.0, 0), (16, 1.5, 0), (16, 1e-3, 17), (16, 1e-3, -1), (4, 1e-3, 4)]:
        with pytest.raises(kp.KronPCGError) as e:
            kp.lowrank_factors(*args)
        assert e.value.status == KP_ERR_ARG
    lib = kp.load()
    buf = (C.c_double * 4)()
    info = kp._lib.PrecondInfo()
    assert lib.kp_lowrank_factors(16, 1e-3, 4, buf, 4, C.byref(info)) == KP_ERR_ARG
    assert b"capacity" in lib.kp_last_error()


@pytest.mark.parametrize("N", [16, 64, 320, 512])
def test_lowrank_factors_2d_match_oracle(N):
    """The library's 2D factors (host C++: Jacobi for small N, subspace iteration
    above) against the oracle's numpy eigen-truncation: same rank, the same
    G_R to 1e-12 relative, the same rho range and truncation error."""
    import paper_2007_06524_amd as kp
    from oracle import twod as td
    F, info = kp.lowrank_factors_2d(N, 1e-3)
    Fo, io = td.lowrank_factors_2d(N, 1e-3)
    assert info["rank"] == io["R"]
    G = np.einsum("ki,kj->ij", F[0], F[1])
    Go = np.einsum("ki,kj->ij", Fo[0], Fo[1])
    assert np.abs(G - Go).max() <= 1e-12 * np.abs(Go).max()
    assert abs(info["rho_min"] - io["rho_min"]) < 1e-9 and abs(info["rho_max"] - io["rho_max"]) < 1e-9
    assert abs(info["cp_rel_err"] - io["rel_err"]) < 1e-9

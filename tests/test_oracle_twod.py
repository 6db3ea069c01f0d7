"""Pins of the 2D oracle (d = 2): the paper's literal Kronecker assembly,
the Galerkin definition, closed forms (laminates, the constant coefficient,
the Keller-Dykhne value sqrt(alpha beta) of the two-phase checkerboard),
brute force, and the rank-R preconditioner identities."""

import numpy as np
import pytest

from oracle import twod as td
from oracle.pcg import pcg
from workloads import cells_bernoulli, random_field


def cells2(L, lo, hi, seed):
    g = np.random.default_rng(np.random.SeedSequence(seed))
    return lo + (hi - lo) * g.random((L, L))


@pytest.mark.parametrize("L,n0,k", [(2, 2, None), (3, 2, None), (2, 4, None), (2, 4, 2), (3, 6, 4)])
def test_2d_literal_equals_stencil(L, n0, k):
    """eq. As_Kron assembled literally (with the periodic wrap; sub-cells on the
    background Laplacian) equals the two-voxel-mean 5-point stencil."""
    cells = cells2(L, 1.0, 10.0, seed=10 * L + n0)
    bg = 0.4 if k else None
    K = td.kron_stiffness_2d(cells, n0, k, bg)
    w = td.edge_weights_2d(cells, n0, k, bg)
    N = n0 * L
    u = random_field(N, seed=3, dims=2)
    np.testing.assert_allclose(K @ u.reshape(-1), td.stiffness_apply_2d(w, u).reshape(-1),
                               rtol=0, atol=1e-12 * np.abs(K).max() * np.abs(u).max())
    assert abs(K - K.T).max() == 0.0
    np.testing.assert_allclose(K @ np.ones(N * N), 0.0, atol=1e-12)


@pytest.mark.parametrize("k", [None, 2])
def test_2d_rhs_equals_galerkin(k):
    cells = cells2(3, 1.0, 10.0, seed=5)
    w = td.edge_weights_2d(cells, 4, k, 0.4 if k else None)
    for i in (1, 2):
        np.testing.assert_allclose(td.corrector_rhs_2d(w, i),
                                   td.fem_rhs_quadrature_2d(cells, 4, i, k, 0.4 if k else None),
                                   rtol=0, atol=1e-15)


def test_2d_constant_coefficient_one_iteration():
    """a = c: f_i = 0, and for any zero-mean f the exact preconditioner gives the
    solution in one PCG iteration, equal to the Fourier closed form / c."""
    c, N = 2.5, 24
    w = td.edge_weights_2d(np.full((6, 6), c), 4)
    assert np.all(td.corrector_rhs_2d(w, 1) == 0.0)
    f = random_field(N, seed=1, dims=2)
    f -= f.mean()
    res = pcg(lambda u: td.stiffness_apply_2d(w, u), f, td.apply_pinv_laplacian_2d, tol=1e-12)
    assert res["iters"] == 1
    np.testing.assert_allclose(res["x"], td.apply_pinv_laplacian_2d(f) / c, atol=1e-12)


def test_2d_laminate_exact():
    """a(c) = g(c1): flux constant along x1, so a_11 = harmonic mean of g,
    a_22 = arithmetic mean, off-diagonals 0 (discretely exact)."""
    g = np.array([1.0, 7.0, 2.0, 4.0])
    cells = np.repeat(g[:, None], 4, axis=1)
    res = td.solve_correctors_2d(cells, 4, tol=1e-13)
    A = res["ahom"]
    assert A[0, 0] == pytest.approx(1.0 / np.mean(1.0 / g), rel=1e-10)
    assert A[1, 1] == pytest.approx(g.mean(), rel=1e-10)
    assert abs(A[0, 1]) < 1e-10 and abs(A[1, 0]) < 1e-10


def test_2d_checkerboard_keller_dykhne():
    """Two-phase 50/50 periodic checkerboard: a_hom = sqrt(alpha beta) in the
    continuum (Keller-Dykhne duality); the discrete value converges to it at
    first order in h, with a_11 = a_22 and a_12 = 0 by symmetry."""
    for al, be in ((1.0, 4.0), (1.0, 10.0)):
        cells = np.array([[al, be], [be, al]])
        vals = []
        for n0 in (4, 8, 16, 32):
            A = td.solve_correctors_2d(cells, n0, tol=1e-12)["ahom"]
            assert abs(A[0, 0] - A[1, 1]) < 1e-9 * A[0, 0] and abs(A[0, 1]) < 1e-9
            vals.append(A[0, 0])
        errs = [v - np.sqrt(al * be) for v in vals]
        rates = [errs[j] / errs[j + 1] for j in range(3)]
        assert all(e > 0 for e in errs) and all(1.6 < r < 2.4 for r in rates), (errs, rates)
        # first-order Richardson extrapolation from the two finest grids
        assert abs(2 * vals[-1] - vals[-2] - np.sqrt(al * be)) < 0.015 * np.sqrt(al * be)


def test_2d_dense_brute_force_and_bounds():
    cells = cells2(3, 1.0, 10.0, seed=9)
    n0 = 2
    res = td.solve_correctors_2d(cells, n0, tol=1e-13)
    K = td.kron_stiffness_2d(cells, n0).toarray()
    for i in (1, 2):
        f = res["fs"][i - 1]
        u, *_ = np.linalg.lstsq(K, f.reshape(-1), rcond=None)
        np.testing.assert_allclose(res["phis"][i - 1].reshape(-1), u, atol=1e-10 * np.abs(u).max())
    A = res["ahom"]
    np.testing.assert_allclose(A, A.T, atol=1e-10)
    harm, arith = 1.0 / np.mean(1.0 / cells), cells.mean()
    for i in range(2):
        assert harm <= A[i, i] <= arith
        assert td.homogenized_energy_2d(res["w"], res["phis"][i], i + 1) == pytest.approx(A[i, i], rel=1e-9)


@pytest.mark.parametrize("N", [16, 48, 128])
def test_2d_lowrank_factors(N):
    """The rank-R factors: even vectors, the circulant apply equals the FFT apply
    of G_R (eq. Lap2DtimesX), the relative symbol error reported, the rho range
    positive and narrowing as eps decreases."""
    F, info = td.lowrank_factors_2d(N, 1e-3)
    assert F.shape[0] == 2 and F.shape[2] == N
    assert np.allclose(F, F[:, :, (-np.arange(N)) % N])
    x = random_field(N, seed=N, dims=2)
    np.testing.assert_allclose(td.circulant_2d_apply(F, x), td.symbol_apply_2d(F, x),
                               atol=1e-12 * np.abs(td.symbol_apply_2d(F, x)).max())
    assert info["rel_err"] <= 1e-3 and 0.0 < info["rho_min"] <= 1.0 <= info["rho_max"]
    F2, info2 = td.lowrank_factors_2d(N, 1e-6)
    assert info2["R"] > info["R"]
    assert info2["rho_max"] - info2["rho_min"] < info["rho_max"] - info["rho_min"]
    # the rank-R apply preconditions: PCG on a random 2D coefficient converges
    cells = cells2(N // 4, 1.0, 10.0, seed=N)
    w = td.edge_weights_2d(cells, 4)
    f = td.corrector_rhs_2d(w, 1)
    res = pcg(lambda u: td.stiffness_apply_2d(w, u), f, lambda r: td.symbol_apply_2d(F, r), tol=1e-10)
    assert res["converged"]

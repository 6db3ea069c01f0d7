"""Pins of the oracle's Fourier and low-Kronecker-rank pieces (Section 4.2)."""

import numpy as np
import pytest

from oracle import fourier as fo
from oracle import lowrank as lr
from workloads import random_field


@pytest.mark.parametrize("N", [2, 3, 4, 7, 16])
def test_eigenvalues_of_circulant(N):
    """eq. Circ_Fourier: the spectrum of the periodic circulant is 4 sin^2(pi k/N)."""
    ev = np.sort(np.linalg.eigvalsh(fo.periodic_laplacian_1d(N)))
    np.testing.assert_allclose(ev, np.sort(fo.laplacian_eigenvalues(N)), atol=1e-12)
    assert fo.laplacian_eigenvalues(N)[0] == 0.0


@pytest.mark.parametrize("N", [4, 6, 9])
def test_fourier_diagonalizes_kronecker_sum(N):
    """eqs. Lapl_Kron3 / DiagLaplace3D: F* Lambda F equals the 3-term Kronecker sum."""
    u = random_field(N, seed=N)
    A1 = fo.periodic_laplacian_1d(N)
    I = np.eye(N)
    A = np.kron(np.kron(A1, I), I) + np.kron(np.kron(I, A1), I) + np.kron(np.kron(I, I), A1)
    np.testing.assert_allclose(fo.apply_symbol(fo.laplacian_symbol(N), u).reshape(-1),
                               A @ u.reshape(-1), atol=1e-11)
    np.testing.assert_allclose(fo.laplacian_apply(u).reshape(-1), A @ u.reshape(-1), atol=1e-12)


@pytest.mark.parametrize("N", [5, 8])
def test_pseudo_inverse(N):
    """eq. 3a: A A^+ r = r - mean(r); A^+ 1 = 0 (pseudo-inverse on <u,1> = 0)."""
    r = random_field(N, seed=3)
    z = fo.apply_pinv_laplacian(r)
    np.testing.assert_allclose(fo.laplacian_apply(z), r - r.mean(), atol=1e-11)
    np.testing.assert_allclose(fo.apply_pinv_laplacian(np.ones((N, N, N))), 0.0, atol=1e-13)
    assert abs(z.mean()) < 1e-13
    G = fo.pinv_symbol(N)
    assert G[0, 0, 0] == 0.0 and G[1, 0, 0] == 1.0 / fo.laplacian_eigenvalues(N)[1]


def test_laplace_quadrature_converges_geometrically():
    """Lemma RankPinverse: R = O(|log eps|) terms of the Laplace transform quadrature."""
    a, b = fo.laplacian_eigenvalues(16)[1], 12.0
    errs = [lr.laplace_quadrature(R, a, b)[2] for R in (2, 4, 6, 8)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.02
    # the reported error is the true error on an independent dense sample
    t, w, err = lr.laplace_quadrature(6, a, b)
    x = np.linspace(a, b, 20001)
    q = np.exp(-np.outer(x, t)) @ w
    assert abs(np.max(np.abs(x * q - 1)) - err) < 0.05 * err + 1e-12
    assert np.all(q > 0)


@pytest.mark.parametrize("N", [5, 8])
def test_circulant_is_fourier_multiplier(N):
    u = 1.0 + np.cos(2 * np.pi * np.arange(N) / N) ** 2     # even symbol
    C = lr.circulant(u)
    x = np.random.default_rng(1).standard_normal(N)
    np.testing.assert_allclose(C, C.T, atol=1e-14)
    np.testing.assert_allclose(C @ x, np.real(np.fft.ifft(u * np.fft.fft(x))), atol=1e-13)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(C)), np.sort(u), atol=1e-13)
    # the Laplacian circulant is recovered from its own symbol
    np.testing.assert_allclose(lr.circulant(fo.laplacian_eigenvalues(N)), fo.periodic_laplacian_1d(N),
                               atol=1e-13)


def test_kron_apply_mode_order_tiny():
    """eq. Lap3DtimesX with x1 slowest: mode products equal the explicit Kronecker matrix."""
    N, R = 4, 2
    rng = np.random.default_rng(9)
    F = np.empty((3, R, N))
    for l in range(3):
        for k in range(R):
            v = rng.random(N // 2 + 1) + 0.5
            F[l, k] = np.concatenate([v, v[1:N - N // 2][::-1]])  # even
    x = random_field(N, seed=2)
    np.testing.assert_allclose(lr.kron_apply(F, x).reshape(-1), lr.kron_matrix(F) @ x.reshape(-1),
                               atol=1e-12)
    # identity P12: the same operator through the FFT of its symbol
    np.testing.assert_allclose(lr.kron_apply(F, x), fo.apply_symbol(lr.symbol_from_factors(F), x),
                               atol=1e-12)


def test_tucker_full_rank_is_exact_and_error_bound():
    N = 12
    W = fo.pinv_symbol(N)
    W[0, 0, 0] = 5.0
    U = lr.tucker_basis(W, 1e-15, 1)
    B = lr.tucker_core(W, U)
    Wr = np.einsum("abc,ia,jb,kc->ijk", B, U, U, U)
    np.testing.assert_allclose(Wr, W, atol=1e-10 * np.abs(W).max())
    for eps in (1e-2, 1e-4):
        U = lr.tucker_basis(W, eps, 1)
        Wr = np.einsum("abc,ia,jb,kc->ijk", lr.tucker_core(W, U), U, U, U)
        assert np.linalg.norm(W - Wr) <= eps * np.linalg.norm(W) * (1 + 1e-9)
        # even columns (rows i and N-i of the unfolding coincide)
        np.testing.assert_allclose(U, U[(-np.arange(N)) % N], atol=1e-9)


def test_cp_als_recovers_exact_rank():
    rng = np.random.default_rng(4)
    A = [rng.standard_normal((6, 2)) for _ in range(3)]
    B = lr.cp_full(A)
    V0 = [a + 0.01 * rng.standard_normal((6, 2)) for a in A]
    V = lr.cp_als(B, V0, sweeps=200)
    assert np.linalg.norm(B - lr.cp_full(V)) < 1e-8 * np.linalg.norm(B)


@pytest.mark.parametrize("N,rank", [(16, 4), (16, 0), (32, 0)])
def test_canonical_preconditioner_quality(N, rank):
    F, info = lr.canonical_preconditioner(N, 1e-3, rank)
    if rank:
        assert F.shape == (3, rank, N)
    assert info["rho_min"] > 0.5 and info["rho_max"] < 1.5
    assert info["cancellation"] < 10.0
    np.testing.assert_allclose(F, F[:, :, (-np.arange(N)) % N], atol=1e-12)   # even factors
    lo, hi = lr.rho_range(F)
    assert (lo, hi) == (info["rho_min"], info["rho_max"])
    # G_R approximates G+ in relative terms on every nonzero mode
    G = fo.pinv_symbol(N)
    GR = lr.symbol_from_factors(F)
    nz = G > 0
    assert np.max(np.abs(GR[nz] / G[nz] - 1)) <= max(1 - lo, hi - 1) + 1e-12

"""Pins of the oracle's discretization against the paper's worked examples and
the finite-element definition (Sections 3.1-3.3)."""

import os

import numpy as np
import pytest

from conftest import GOLDEN, read_golden_matrices
from oracle import assembly as asm
from oracle import fourier as fo
from workloads import cells_bernoulli, cells_uniform, random_field


def test_worked_matrices_eq_matr_mini():
    """eq. matr_mini: the oracle's Neumann block and periodic circulant for n = 3."""
    g = read_golden_matrices("matr_mini.txt")
    dn = np.array(g["Delta_N"])
    dp = np.array(g["Delta_P"])
    # the oracle uses the positive semidefinite sign (reading of the sign)
    np.testing.assert_array_equal(asm.neumann_block(3), -dn)
    np.testing.assert_array_equal(fo.periodic_laplacian_1d(3), -dp)
    # Delta_P for n=3 has eigenvalues {0, -3, -3}
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(dp)), [-3.0, -3.0, 0.0], atol=1e-13)
    np.testing.assert_allclose(np.sort(fo.laplacian_eigenvalues(3)), [0.0, 3.0, 3.0], atol=1e-13)


def test_first_column_p():
    p = np.loadtxt(os.path.join(GOLDEN, "symbol_p.txt"))
    C = fo.periodic_laplacian_1d(6)
    np.testing.assert_array_equal(C[:, 0], p)
    # the DFT of p gives the eigenvalues (eq. Circ_Fourier), first one zero
    np.testing.assert_allclose(np.real(np.fft.fft(p)), fo.laplacian_eigenvalues(6), atol=1e-13)


@pytest.mark.parametrize("nb", [2, 3, 5])
def test_neumann_and_half_identity_blocks(nb):
    Q = asm.neumann_block(nb)
    I = asm.half_identity(nb)
    assert np.allclose(Q, Q.T)
    np.testing.assert_allclose(Q @ np.ones(nb), 0.0)          # Neumann: constants in the kernel
    np.testing.assert_allclose(np.diag(I)[[0, -1]], [0.5, 0.5])
    assert np.trace(I) == nb - 1                                # lumped 1D mass of nb-1 intervals


@pytest.mark.parametrize("L,n0", [(2, 1), (2, 2), (2, 3), (3, 2), (1, 4)])
def test_kron_literal_equals_stencil(L, n0):
    """eq. As_Kron_d assembled literally equals the edge-average 7-point stencil."""
    cells = cells_uniform(L, 1.0, 10.0, seed=100 + 10 * L + n0)
    N = n0 * L
    K = asm.kron_stiffness(cells, n0)
    w = asm.edge_weights(cells, n0)
    u = random_field(N, seed=7)
    np.testing.assert_allclose(K @ u.reshape(-1), asm.stiffness_apply(w, u).reshape(-1),
                               rtol=0, atol=1e-12 * np.abs(K).max() * np.abs(u).max())
    # symmetric, constants in the kernel
    assert abs(K - K.T).max() == 0.0
    np.testing.assert_allclose(K @ np.ones(N ** 3), 0.0, atol=1e-12)


@pytest.mark.parametrize("L,n0", [(2, 2), (3, 1), (2, 3)])
def test_edge_weight_is_negated_offdiagonal(L, n0):
    cells = cells_uniform(L, 1.0, 10.0, seed=5)
    N = n0 * L
    if N < 3:
        pytest.skip("p+e and p-e coincide")
    K = asm.kron_stiffness(cells, n0).toarray()
    w = asm.edge_weights(cells, n0)
    idx = np.arange(N ** 3).reshape(N, N, N)
    for l in range(3):
        nb = np.roll(idx, -1, axis=l)
        np.testing.assert_allclose(-K[idx.reshape(-1), nb.reshape(-1)], w[l].reshape(-1), atol=1e-13)


@pytest.mark.parametrize("L,n0", [(2, 2), (2, 1), (1, 3)])
def test_rhs_equals_galerkin_definition(L, n0):
    """eq. FEM_discr_RHS by brute-force voxel integration equals h (w_i(p) - w_i(p-e_i))."""
    cells = cells_uniform(L, 1.0, 10.0, seed=11)
    w = asm.edge_weights(cells, n0)
    for i in (1, 2, 3):
        np.testing.assert_allclose(asm.corrector_rhs(w, i), asm.fem_rhs_quadrature(cells, n0, i),
                                   atol=1e-14)
        assert abs(asm.corrector_rhs(w, i).sum()) < 1e-13


def test_nodal_values_fig_check_coef():
    """Fig. Check_coef (2D): 1 interior, 1/2 interface, 1/4 exterior corner.

    A single inclusion cell column (x3-invariant, so the x1-x2 plane is the 2D
    picture) on an L = 2 lattice with n0 = 4.
    """
    vals = {}
    with open(os.path.join(GOLDEN, "nodal_weights_2d.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    cells = np.zeros((2, 2, 2))
    cells[0, 0, :] = 1.0
    nod = asm.nodal_coefficient(cells, 4)[:, :, 0]
    assert nod[2, 2] == vals["interior"]
    assert nod[0, 2] == vals["interface"] and nod[4, 2] == vals["interface"]
    assert nod[2, 0] == vals["interface"]
    for c in [(0, 0), (0, 4), (4, 0), (4, 4)]:
        assert nod[c] == vals["exterior_corner"]
    assert nod[6, 6] == 0.0


def test_lumped_integral_is_mean():
    """The nodal (lumped) quadrature integrates the coefficient exactly: h^3 sum = mean."""
    cells = cells_bernoulli(3, 1.0, 10.0, 0.5, seed=3)
    nod = asm.nodal_coefficient(cells, 2)
    N = nod.shape[0]
    assert abs(nod.sum() / N ** 3 - cells.mean()) < 1e-13
    w = asm.edge_weights(cells, 2)
    for l in range(3):
        assert abs(w[l].mean() - cells.mean()) < 1e-13


def test_constant_coefficient_is_scaled_laplacian():
    cells = np.full((2, 2, 2), 3.5)
    w = asm.edge_weights(cells, 3)
    u = random_field(6, seed=1)
    np.testing.assert_allclose(asm.stiffness_apply(w, u), 3.5 * fo.laplacian_apply(u), atol=1e-12)


# ---- centred sub-cell inclusions (Section 3.1; alpha = k / (2 n0)) ----------

@pytest.mark.parametrize("L,n0,k", [(2, 4, 2), (3, 4, 2), (2, 6, 2), (2, 6, 4)])
def test_inclusion_literal_equals_stencil(L, n0, k):
    """Background periodic Laplacian (eq. Lapl_Kron3) plus the Kronecker sums of
    the (k+1)-node sub-cell blocks (eq. As_Kron_d on S_s) equals the edge-average
    stencil of the voxel field; the off-diagonal entries are the negated weights."""
    b = 0.4
    cells = cells_bernoulli(L, b, 1.0, 0.5, seed=300 + 10 * L + k)
    cells[0, 0, 0], cells[-1, -1, -1] = 1.0, 2.5     # at least one perturbed cell, two values
    N = n0 * L
    K = asm.kron_stiffness_inclusions(cells, n0, k, b)
    w = asm.edge_weights(cells, n0, k, b)
    u = random_field(N, seed=9)
    np.testing.assert_allclose(K @ u.reshape(-1), asm.stiffness_apply(w, u).reshape(-1),
                               rtol=0, atol=1e-12 * np.abs(K).max() * np.abs(u).max())
    idx = lambda p: (p[0] % N) * N * N + (p[1] % N) * N + (p[2] % N)
    g = np.random.default_rng(1)
    for _ in range(20):
        p = tuple(int(v) for v in g.integers(0, N, 3))
        for l in range(3):
            q = list(p)
            q[l] += 1
            assert K[idx(p), idx(q)] == pytest.approx(-w[l][p], abs=1e-14)
    assert abs(K - K.T).max() == 0.0
    np.testing.assert_allclose(K @ np.ones(N ** 3), 0.0, atol=1e-12)


def test_inclusion_full_subcell_is_the_cell():
    """k = n0 (alpha = 1/2): the sub-cell is the cell, whatever the background."""
    cells = cells_uniform(2, 1.0, 10.0, seed=41)
    np.testing.assert_array_equal(asm.voxel_field(cells, 4, 4, 0.3), asm.voxel_field(cells, 4))
    K0 = asm.kron_stiffness(cells, 4)
    for b in (0.3, 7.0):
        Kb = asm.kron_stiffness_inclusions(cells, 4, 4, b)
        assert abs(Kb - K0).max() <= 1e-12 * abs(K0).max()


def test_inclusion_range_and_voxel_mean():
    """The sub-cell is centred (k voxels per edge, (n0 - k)/2 on either side) and the
    voxel mean is b + (k/n0)^3 (mean(a_cell) - b)."""
    assert asm.inclusion_range(4, 2) == (1, 3) and asm.inclusion_range(8, 4) == (2, 6)
    for bad in ((4, 3), (4, 0), (4, 6)):
        with pytest.raises(ValueError):
            asm.inclusion_range(*bad)
    cells = cells_uniform(3, 1.0, 10.0, seed=42)
    for n0, k in ((4, 2), (8, 4), (8, 2), (6, 4)):
        A = asm.voxel_field(cells, n0, k, 0.4)
        assert A.mean() == pytest.approx(0.4 + (k / n0) ** 3 * (cells.mean() - 0.4), rel=1e-13)
        lo, hi = asm.inclusion_range(n0, k)
        # a voxel of cell (1,2,0) at local (lo, hi-1, lo) is inside, at (lo-1, lo, lo) outside
        assert A[n0 + lo, 2 * n0 + hi - 1, lo] == cells[1, 2, 0]
        assert A[n0 + lo - 1, 2 * n0 + lo, lo] == 0.4


def test_inclusion_rhs_equals_galerkin_definition():
    """The corrector right-hand side of the voxel field equals the Galerkin
    integral of eq. FEM_discr_RHS (brute force over voxels) with inclusions."""
    cells = cells_uniform(2, 1.0, 10.0, seed=43)
    w = asm.edge_weights(cells, 4, 2, 0.4)
    for i in (1, 2, 3):
        np.testing.assert_allclose(asm.corrector_rhs(w, i), asm.fem_rhs_quadrature(cells, 4, i, 2, 0.4),
                                   rtol=0, atol=1e-14)


def test_inclusion_nodal_values_fig_check_coef():
    """Fig. Check_coef for a sub-cell inclusion: on the mid-plane of a single
    perturbed sub-cell (k = 2 in n0 = 4) the nodal coefficient in excess of the
    background is 1 inside, 1/2 on the interface, 1/4 at an exterior corner."""
    vals = {}
    with open(os.path.join(GOLDEN, "nodal_weights_2d.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                key, v = line.split()
                vals[key] = float(v)
    b = 0.25
    cells = np.full((2, 2, 2), b)
    cells[0, 0, 0] = b + 1.0
    nod = asm.nodal_coefficient(cells, 4, 2, b)[:, :, 2] - b    # sub-cell voxels 1..2, nodes 1..3
    assert nod[2, 2] == vals["interior"]
    for c in [(1, 2), (3, 2), (2, 1), (2, 3)]:
        assert nod[c] == vals["interface"]
    for c in [(1, 1), (1, 3), (3, 1), (3, 3)]:
        assert nod[c] == vals["exterior_corner"]
    assert nod[0, 0] == 0.0 and nod[5, 5] == 0.0

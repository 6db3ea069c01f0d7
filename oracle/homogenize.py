"""Oracle: corrector solves and the homogenized matrix (Section 3.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For corrector i the discrete solution phi_i of K phi_i = f_i gives
  a_ij = delta_ij * mean(a) - h^(d-2) * sum_p phi_i(p) f_j(p)
which is eq. Ahom3_m_entry_comp written with the same quadrature as the
discretization (lambda + beta int a_hat = mean of the cell values; the
integral of f_j phi_i becomes the lumped sum with the factor h of A = h K).
Two further forms are given for cross-checks: the flux form of the definition
(eq. A_hom_m), a_ij = h^3 sum_p w_j(p)(delta_ij + (phi_i(p+e_j) - phi_i(p))/h),
which equals the linear form identically (summation by parts), and the energy
form a_ii = h^3 sum_p sum_l w_l(p)(delta_il + D_l phi_i(p))^2, which equals it
only at the exact solution.  No symmetrization is applied.
"""

from __future__ import annotations

import numpy as np

from .assembly import corrector_rhs, edge_weights, stiffness_apply, voxel_field
from .fourier import apply_pinv_laplacian
from .pcg import pcg


def homogenized_matrix(a, phis, fs):
    """a: the cell values (full cells) or the voxel field (any coefficient); only
    its mean enters, the exact integral of the coefficient over the cube."""
    N = phis[0].shape[0]
    h = 1.0 / N
    A = np.zeros((3, 3))
    m = float(np.mean(a))
    for i in range(3):
        for j in range(3):
            A[i, j] = (m if i == j else 0.0) - h * float(np.vdot(phis[i], fs[j]))
    return A


def homogenized_flux(w, phis):
    N = phis[0].shape[0]
    h = 1.0 / N
    A = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            D = (np.roll(phis[i], -1, axis=j) - phis[i]) / h
            A[i, j] = h ** 3 * float(np.sum(w[j] * ((1.0 if i == j else 0.0) + D)))
    return A


def homogenized_energy(w, phi, i):
    N = phi.shape[0]
    h = 1.0 / N
    s = 0.0
    for l in range(3):
        D = (np.roll(phi, -1, axis=l) - phi) / h
        s += float(np.sum(w[l] * ((1.0 if l == i - 1 else 0.0) + D) ** 2))
    return h ** 3 * s


def solve_correctors(cells, n0, tol=1e-12, maxit=5000, k=None, background=None):
    """Assemble, solve the three correctors with the exact preconditioner, form a_hom.
    (k, background: centred sub-cell inclusions, see assembly.voxel_field.)"""
    w = edge_weights(cells, n0, k, background)
    K = lambda u: stiffness_apply(w, u)
    fs = [corrector_rhs(w, i) for i in (1, 2, 3)]
    sols = [pcg(K, f, apply_pinv_laplacian, tol=tol, maxit=maxit) for f in fs]
    phis = [s["x"] for s in sols]
    return dict(w=w, fs=fs, phis=phis, solves=sols,
                ahom=homogenized_matrix(voxel_field(cells, n0, k, background), phis, fs))


def empirical_statistics(ahoms):
    """Empirical average and standard deviation over M realizations (Section 5.3).

    eq. A_hom_Empir: the mean of the M matrices; the standard deviation uses the
    M - 1 normalization of the paper's sigma_L^M, entry by entry.
    ahoms: (M, 3, 3).  Returns (mean, std), each 3 x 3.
    """
    A = np.asarray(ahoms, dtype=np.float64)
    M = A.shape[0]
    if M < 2:
        raise ValueError("the standard deviation needs at least two realizations")
    mean = A.sum(axis=0) / M
    std = np.sqrt(((A - mean) ** 2).sum(axis=0) / (M - 1))
    return mean, std

"""Oracle: the two-dimensional problem (d = 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same discretization as the 3D modules with d = 2 (Sections 3.1-3.3): an
L x L lattice of cells, n0 voxels per cell edge, N = n0 L periodic nodes per
axis, h = 1/N, nodes [i1][i2] in C order.  The stiffness is the Kronecker sum
of eq. As_Kron (1D Neumann blocks and half-weight identities per cell, wrapped
modulo N); as a 5-point stencil the weight of the edge (p, p + e_l) is the
mean of the coefficient over the two voxels sharing it.  The FEM matrix is
A = h^(d-2) K = K, so the corrector right-hand side of eq. FEM_discr_RHS is
f_i(p) = h (w_i(p) - w_i(p - e_i)) with no further factor, and
a_ij = delta_ij mean(a) - sum_p phi_i(p) f_j(p) (eq. Ahom3_m_entry_comp with
h^(d-2) = 1).  The preconditioner symbol is 1/(mu_k1 + mu_k2) (eq.
DiagFLaplace2D); its rank-R approximation in 2D is a sum of R outer products
u1 (x) u2 (the 2D decomposition before eq. Lap2DtimesX), applied as
sum_k C1^k X (C2^k)^T with the circulants C = F* diag(u) F.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assembly import embed, half_identity, inclusion_range, neumann_block, periodic_laplacian_block
from .fourier import laplacian_eigenvalues
from .pcg import pcg


def voxel_field_2d(cells: np.ndarray, n0: int, k: int | None = None,
                   background: float | None = None) -> np.ndarray:
    """a_vox(v) = a_cell(floor(v / n0)); with sub-cell inclusions (Section 3.1) the
    cell value only on the centred k x k voxels of each cell, the background elsewhere."""
    a = np.asarray(cells, dtype=np.float64)
    a = np.repeat(np.repeat(a, n0, axis=0), n0, axis=1)
    if k is None or k == n0:
        return a
    if background is None or not background > 0:
        raise ValueError("sub-cell inclusions need a positive background value")
    lo, hi = inclusion_range(n0, k)
    loc = np.arange(a.shape[0]) % n0
    inside = (loc >= lo) & (loc < hi)
    return np.where(inside[:, None] & inside[None, :], a, float(background))


def edge_weights_2d(cells, n0, k=None, background=None) -> np.ndarray:
    """w[l][p], l = 0, 1: the edge (p, p + e_l) lies in voxel layer p_l; the two
    voxels sharing it have transverse coordinate p_t - 1 or p_t (mod N)."""
    A = voxel_field_2d(cells, n0, k, background)
    w = np.empty((2,) + A.shape)
    for l in range(2):
        t = 1 - l
        w[l] = (A + np.roll(A, 1, axis=t)) / 2.0
    return w


def stiffness_apply_2d(w: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(K u)(p) = sum_l w_l(p)(u_p - u_{p+e_l}) + w_l(p - e_l)(u_p - u_{p-e_l})."""
    Ku = np.zeros_like(u, dtype=np.float64)
    for l in range(2):
        up = np.roll(u, -1, axis=l)
        um = np.roll(u, 1, axis=l)
        wm = np.roll(w[l], 1, axis=l)
        Ku += w[l] * (u - up) + wm * (u - um)
    return Ku


def corrector_rhs_2d(w: np.ndarray, i: int) -> np.ndarray:
    """f_i(p) = h (w_i(p) - w_i(p - e_i)) (eq. FEM_discr_RHS; A = K in 2D)."""
    l = i - 1
    h = 1.0 / w.shape[1]
    return h * (w[l] - np.roll(w[l], 1, axis=l))


def fem_rhs_quadrature_2d(cells, n0, i, k=None, background=None) -> np.ndarray:
    """eq. FEM_discr_RHS by brute force: f_mu = -int a dpsi_mu/dx_i with bilinear
    hats; on a voxel the derivative of a corner's hat along x_i is +-1/h times a
    linear transverse factor whose integral over the voxel is h/2, so the voxel
    adds -a_v (+-h/2) to each of its four corners.  Tiny grids only."""
    A = voxel_field_2d(cells, n0, k, background)
    N = A.shape[0]
    h = 1.0 / N
    l = i - 1
    f = np.zeros((N, N))
    for v1 in range(N):
        for v2 in range(N):
            for c in range(4):
                d = ((c >> 1) & 1, c & 1)
                p = ((v1 + d[0]) % N, (v2 + d[1]) % N)
                sign = 1.0 if d[l] == 1 else -1.0
                f[p] += -A[v1, v2] * sign * h / 2.0
    return f


def kron_stiffness_2d(cells, n0, k=None, background=None) -> sp.csr_matrix:
    """Paper-literal stiffness, eq. As_Kron: per cell a_c (Qbar (x) Ibar + Ibar (x) Qbar)
    on the cell's n0 + 1 nodes (mod N); with sub-cell inclusions the background
    times the 2D periodic Laplacian plus (a_c - b) times the blocks of the
    (k+1)-node sub-cells.  Tiny L only."""
    L = cells.shape[0]
    N = n0 * L
    if k is None or k == n0:
        b, lo, nb = 0.0, 0, n0 + 1
        K = sp.csr_matrix((N * N, N * N))
    else:
        b = float(background)
        lo, _ = inclusion_range(n0, k)
        nb = k + 1
        D = periodic_laplacian_block(N)
        E = sp.identity(N, format="csr")
        K = b * (sp.kron(D, E) + sp.kron(E, D))
    Q, I = neumann_block(nb), half_identity(nb)
    for c1 in range(L):
        for c2 in range(L):
            d = float(cells[c1, c2]) - b
            if d == 0.0:
                continue
            Q1, Q2 = embed(Q, c1 * n0 + lo, N), embed(Q, c2 * n0 + lo, N)
            I1, I2 = embed(I, c1 * n0 + lo, N), embed(I, c2 * n0 + lo, N)
            K = K + d * (sp.kron(Q1, I2) + sp.kron(I1, Q2))
    return K.tocsr()


def pinv_symbol_2d(N: int) -> np.ndarray:
    """1 / (mu_k1 + mu_k2), 0 at the zero mode (eq. DiagFLaplace2D)."""
    m = laplacian_eigenvalues(N)
    g = m[:, None] + m[None, :]
    out = np.zeros_like(g)
    out[g > 0] = 1.0 / g[g > 0]
    return out


def apply_pinv_laplacian_2d(r: np.ndarray) -> np.ndarray:
    """The exact preconditioner ("first approach") in 2D, through the 2D FFT."""
    return np.real(np.fft.ifft2(pinv_symbol_2d(r.shape[0]) * np.fft.fft2(r)))


def homogenized_matrix_2d(a, phis, fs) -> np.ndarray:
    """a_ij = delta_ij mean(a) - sum_p phi_i(p) f_j(p) (h^(d-2) = 1)."""
    m = float(np.mean(a))
    A = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            A[i, j] = (m if i == j else 0.0) - float(np.vdot(phis[i], fs[j]))
    return A


def homogenized_energy_2d(w, phi, i) -> float:
    """a_ii = h^2 sum_p sum_l w_l(p) (delta_il + (phi(p + e_l) - phi(p)) / h)^2."""
    h = 1.0 / phi.shape[0]
    s = 0.0
    for l in range(2):
        D = (np.roll(phi, -1, axis=l) - phi) / h
        s += float(np.sum(w[l] * ((1.0 if l == i - 1 else 0.0) + D) ** 2))
    return h * h * s


def solve_correctors_2d(cells, n0, tol=1e-12, maxit=5000, k=None, background=None):
    w = edge_weights_2d(cells, n0, k, background)
    K = lambda u: stiffness_apply_2d(w, u)
    fs = [corrector_rhs_2d(w, i) for i in (1, 2)]
    sols = [pcg(K, f, apply_pinv_laplacian_2d, tol=tol, maxit=maxit) for f in fs]
    phis = [s["x"] for s in sols]
    return dict(w=w, fs=fs, phis=phis, solves=sols,
                ahom=homogenized_matrix_2d(voxel_field_2d(cells, n0, k, background), phis, fs))


def lowrank_factors_2d(N: int, eps: float = 1e-3, rank: int = 0):
    """Rank-R factors (2, R, N) of the 2D preconditioner symbol.

    The symbol is approximated in the relative sense: W = s s^T * G+ with
    s_i = sqrt(mu_i + mu_1) (bounded entries), the zero mode (free: the solver
    projects it out) set to 1/mu_1, the value of its nearest nonzero modes.  W
    is symmetric and even in both indices, so it is reduced to the N/2 + 1
    distinct indices with multiplicities m_i (1 or 2) and M = D^(1/2) W D^(1/2)
    (D = diag m) is diagonalized: its truncated eigen-expansion is the best
    rank-R approximation of W in the Frobenius norm of the full grid.
    rank = 0: the smallest R with ||W - W_R|| <= eps ||W||.  Factors
    u1 = sqrt|lambda| z / s, u2 = sign(lambda) sqrt|lambda| z / s (z expanded
    to the full grid, even).  Returns (F, info) with the rho range
    G_R (mu_k1 + mu_k2) over the nonzero modes.
    """
    mu = laplacian_eigenvalues(N)
    H = N // 2 + 1
    idx = np.minimum(np.arange(N), N - np.arange(N))       # full index -> reduced
    m = np.bincount(idx, minlength=H).astype(np.float64)
    s = np.sqrt(mu[:H] + mu[1])
    g = mu[:H, None] + mu[None, :H]
    G = np.zeros((H, H))
    G[g > 0] = 1.0 / g[g > 0]
    G[0, 0] = 1.0 / mu[1]
    W = s[:, None] * s[None, :] * G
    sq = np.sqrt(m)
    lam, Z = np.linalg.eigh(sq[:, None] * W * sq[None, :])
    order = np.argsort(-np.abs(lam))
    lam, Z = lam[order], Z[:, order]
    total = float(np.sum(lam ** 2))
    if rank > 0:
        R = rank
    else:
        R = H
        for r in range(1, H + 1):
            if float(np.sum(lam[r:] ** 2)) <= eps * eps * total:
                R = r
                break
    z = Z[:, :R] / sq[:, None]                               # reduced, (H, R)
    u = np.sqrt(np.abs(lam[:R]))[None, :] * z / s[:, None]   # (H, R)
    F = np.stack([u.T[:, idx], (np.sign(lam[:R])[:, None] * u.T)[:, idx]])
    GR = np.einsum("ki,kj->ij", F[0], F[1])
    gf = mu[:, None] + mu[None, :]
    rho = (GR * gf)[gf > 0]
    info = dict(R=R, rel_err=float(np.sqrt(np.sum(lam[R:] ** 2) / total)),
                rho_min=float(rho.min()), rho_max=float(rho.max()))
    return F, info


def circulant_2d_apply(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_k C1^k X (C2^k)^T with C = F* diag(u) F built densely (eq. Lap2DtimesX)."""
    from .lowrank import circulant
    z = np.zeros_like(x, dtype=np.float64)
    for k in range(F.shape[1]):
        z += circulant(F[0, k]) @ x @ circulant(F[1, k]).T
    return z


def symbol_apply_2d(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The same operator through the 2D FFT: F* ((sum_k u1 (x) u2) * F x)."""
    GR = np.einsum("ki,kj->ij", F[0], F[1])
    return np.real(np.fft.ifft2(GR * np.fft.fft2(x)))

"""Oracle: discretization of -div(a grad u) on the periodic unit cube.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid (Section 3.1): the cube carries L^3 unit cells, each cell edge holds n0
grid intervals, so there are N = n0*L distinct periodic nodes per axis and
h = 1/N.  (The paper counts n1 = n0*L + 1 nodes; the extra one is the periodic
image of node 0.)  Nodes are flattened big-endian, x1 slowest (Section 3.2),
which is numpy C order for an (N, N, N) array.  Voxel v is the h-cube with
lower corner v*h; it lies in cell floor(v / n0).

Two assembly routes are given and must agree:

* `kron_stiffness` is the paper's Kronecker-sum construction (Section 3.3,
  eqs. As_Kron and As_Kron_d): every cell c contributes
  a_c * sum_l  I_c (x) ... (x) Q_c (x) ... (x) I_c, where Q is the 1D Neumann
  Laplacian block and I = diag(1/2, 1, ..., 1, 1/2) on the n0+1 nodes of the
  cell, embedded at the cell's node indices taken mod N (that wrap is the
  periodization term P^(d)).  The sign is chosen so that K is positive
  semidefinite (the paper's displayed blocks are the negative Laplacian).

* `edge_weights` / `stiffness_apply` is the same matrix written as a 7-point
  stencil: the weight of the edge (p, p + e_l) is the mean of the coefficient
  over the 2^(d-1) voxels that share that edge.

The FEM stiffness of Section 3.1 is A = h^(d-2) K (lumped mass, eq.
Lapl_Kron_D); the solution does not depend on that factor, so the oracle works
with K and scales the right-hand side accordingly.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def inclusion_range(n0: int, k: int) -> tuple[int, int]:
    """Voxel range [lo, lo + k) of the centred sub-cell inside a cell of n0 voxels.

    Section 3.1: the unit cell G_s contains the sub-cell S_s of edge 2 alpha / L
    = k h (k = 2 alpha n0, an even number of grid intervals up to n0) with the
    same centre, so S_s covers the voxels (n0 - k)/2 .. (n0 + k)/2 - 1 of the
    cell along every axis.
    """
    if not (0 < k <= n0) or (n0 - k) % 2:
        raise ValueError(f"sub-cell of {k} voxels does not centre in a cell of {n0}")
    lo = (n0 - k) // 2
    return lo, lo + k


def voxel_field(cells: np.ndarray, n0: int, k: int | None = None,
                background: float | None = None) -> np.ndarray:
    """Coefficient value on every voxel.

    Full cells (k None or n0): a_vox(v) = a_cell(floor(v / n0)).  Sub-cell
    inclusions (Section 3.1, k < n0): a voxel takes its cell's value when it
    lies in the centred sub-cell (every local coordinate v mod n0 in
    inclusion_range) and the background value elsewhere; a cell whose value
    equals the background is an unperturbed cell (the paper's binary model
    a = 1 on the union of the perturbed sub-cells and lambda elsewhere).
    """
    a = np.asarray(cells, dtype=np.float64)
    for ax in range(a.ndim):
        a = np.repeat(a, n0, axis=ax)
    if k is None or k == n0:
        return a
    if background is None or not background > 0:
        raise ValueError("sub-cell inclusions need a positive background value")
    lo, hi = inclusion_range(n0, k)
    loc = np.arange(a.shape[0]) % n0
    inside = (loc >= lo) & (loc < hi)
    mask = inside[:, None, None] & inside[None, :, None] & inside[None, None, :]
    return np.where(mask, a, float(background))


def edge_weights(cells: np.ndarray, n0: int, k: int | None = None,
                 background: float | None = None) -> np.ndarray:
    """Edge weights w[l][p] of the edge (p, p + e_l), shape (3, N, N, N).

    Along axis l the edge lies in voxel layer p_l; on each transverse axis t
    the four voxels sharing it have coordinate p_t - 1 or p_t (mod N).
    (k, background: sub-cell inclusions, see voxel_field.)
    """
    A = voxel_field(cells, n0, k, background)
    w = np.empty((3,) + A.shape)
    for l in range(3):
        t1, t2 = [t for t in range(3) if t != l]
        s = A + np.roll(A, 1, axis=t1) + np.roll(A, 1, axis=t2) \
            + np.roll(np.roll(A, 1, axis=t1), 1, axis=t2)
        w[l] = s / 4.0
    return w


def stiffness_apply(w: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(K u)(p) = sum_l w_l(p)(u_p - u_{p+e_l}) + w_l(p-e_l)(u_p - u_{p-e_l})."""
    Ku = np.zeros_like(u, dtype=np.float64)
    for l in range(3):
        up = np.roll(u, -1, axis=l)          # u_{p+e_l}
        um = np.roll(u, 1, axis=l)           # u_{p-e_l}
        wm = np.roll(w[l], 1, axis=l)        # w_l(p-e_l)
        Ku += w[l] * (u - up) + wm * (u - um)
    return Ku


def corrector_rhs(w: np.ndarray, i: int) -> np.ndarray:
    """Right-hand side of corrector i (1-based), scaled for K = h^(2-d) A.

    eq. FEM_discr_RHS gives f_{mu,i} = -int a dpsi_mu/dx_i; with lumped
    stiffness this is h^2 (w_i(p) - w_i(p - e_i)) in 3D, and dividing by the
    factor h of A = h K leaves f_i(p) = h (w_i(p) - w_i(p - e_i)).
    """
    l = i - 1
    N = w.shape[1]
    h = 1.0 / N
    return h * (w[l] - np.roll(w[l], 1, axis=l))


def fem_rhs_quadrature(cells: np.ndarray, n0: int, i: int, k: int | None = None,
                       background: float | None = None) -> np.ndarray:
    """Corrector right-hand side from the Galerkin definition, by brute force.

    eq. FEM_discr_RHS: f_{mu,i} = -int_Omega a(x) dpsi_mu/dx_i dx with
    trilinear hat functions psi_mu.  On a voxel, the derivative of the hat of
    one of its eight corners along x_i is +-1/h times a bilinear transverse
    factor whose integral over the voxel face is h^2/4, so the voxel adds
    -a_v * (+-h^2/4) to each corner.  Returned divided by h (K = A / h).
    Pure-Python loop: tiny grids only.
    """
    A = voxel_field(cells, n0, k, background)
    N = A.shape[0]
    h = 1.0 / N
    l = i - 1
    f = np.zeros((N, N, N))
    for v1 in range(N):
        for v2 in range(N):
            for v3 in range(N):
                av = A[v1, v2, v3]
                v = (v1, v2, v3)
                for c in range(8):
                    d = ((c >> 2) & 1, (c >> 1) & 1, c & 1)
                    p = tuple((v[k] + d[k]) % N for k in range(3))
                    sign = 1.0 if d[l] == 1 else -1.0    # d psi/dx_l = +-1/h
                    f[p] += -av * sign * h * h / 4.0
    return f / h


def nodal_coefficient(cells: np.ndarray, n0: int, k: int | None = None,
                      background: float | None = None) -> np.ndarray:
    """Mean of the coefficient over the 2^d voxels around each node.

    Section 3.3 (Fig. Check_coef): for a binary inclusion this is 1 inside,
    1/2 on a face, 1/4 on an exterior edge (a corner in 2D), and so on.
    """
    A = voxel_field(cells, n0, k, background)
    s = np.zeros_like(A)
    for c in range(8):
        shifted = A
        for ax in range(3):
            if (c >> ax) & 1:
                shifted = np.roll(shifted, 1, axis=ax)
        s += shifted
    return s / 8.0


def neumann_block(nb: int) -> np.ndarray:
    """-(tridiag{1,-2,1} + diag{1,0,...,0,1}) of size nb (Section 3.3)."""
    Q = np.zeros((nb, nb))
    for k in range(nb):
        Q[k, k] = -2.0
        if k > 0:
            Q[k, k - 1] = 1.0
        if k < nb - 1:
            Q[k, k + 1] = 1.0
    Q[0, 0] += 1.0
    Q[nb - 1, nb - 1] += 1.0
    return -Q


def half_identity(nb: int) -> np.ndarray:
    """diag{1/2, 1, ..., 1, 1/2} of size nb (Section 3.3)."""
    d = np.ones(nb)
    d[0] = 0.5
    d[-1] = 0.5
    return np.diag(d)


def embed(block: np.ndarray, start: int, N: int) -> sp.csr_matrix:
    """Insert a block at node indices start..start+nb-1 taken mod N (adding)."""
    nb = block.shape[0]
    idx = [(start + k) % N for k in range(nb)]
    rows, cols, vals = [], [], []
    for a in range(nb):
        for b in range(nb):
            if block[a, b] != 0.0:
                rows.append(idx[a])
                cols.append(idx[b])
                vals.append(block[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def kron_stiffness(cells: np.ndarray, n0: int) -> sp.csr_matrix:
    """Paper-literal Kronecker-sum stiffness K (eq. As_Kron_d), 3D, sparse.

    Sum over cells of a_c (Qbar x Ibar x Ibar + Ibar x Qbar x Ibar +
    Ibar x Ibar x Qbar), x1 the slowest Kronecker factor.  Tiny L only.
    """
    L = cells.shape[0]
    N = n0 * L
    nb = n0 + 1
    Q = neumann_block(nb)
    I = half_identity(nb)
    K = sp.csr_matrix((N ** 3, N ** 3))
    for c1 in range(L):
        for c2 in range(L):
            for c3 in range(L):
                a = float(cells[c1, c2, c3])
                Q1, Q2, Q3 = (embed(Q, c * n0, N) for c in (c1, c2, c3))
                I1, I2, I3 = (embed(I, c * n0, N) for c in (c1, c2, c3))
                K = K + a * (sp.kron(sp.kron(Q1, I2), I3)
                             + sp.kron(sp.kron(I1, Q2), I3)
                             + sp.kron(sp.kron(I1, I2), Q3))
    return K.tocsr()


def periodic_laplacian_block(N: int) -> sp.csr_matrix:
    """1D periodic Laplacian on N nodes (the positive semidefinite -Delta_{1,P}
    of Section 3.2: 2 on the diagonal, -1 on the two cyclic off-diagonals)."""
    rows, cols, vals = [], [], []
    for a in range(N):
        for b, v in ((a, 2.0), ((a + 1) % N, -1.0), ((a - 1) % N, -1.0)):
            rows.append(a)
            cols.append(b)
            vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def kron_stiffness_inclusions(cells: np.ndarray, n0: int, k: int, background: float) -> sp.csr_matrix:
    """Paper-literal stiffness with centred sub-cell inclusions, 3D, sparse.

    The background value b everywhere is b times the periodic Laplacian as a
    Kronecker sum of 1D periodic Laplacians with identities (eq. Lapl_Kron3);
    every cell c then adds (a_c - b) times the Kronecker sum of the Neumann
    block and the half identity of size k + 1 (eq. As_Kron_d with the sub-cell
    of Section 3.3 in place of the cell), embedded at the sub-cell's node
    indices c n0 + lo .. c n0 + lo + k (mod N).  Tiny L only.
    """
    L = cells.shape[0]
    N = n0 * L
    lo, _ = inclusion_range(n0, k)
    D = periodic_laplacian_block(N)
    E = sp.identity(N, format="csr")
    b = float(background)
    K = b * (sp.kron(sp.kron(D, E), E) + sp.kron(sp.kron(E, D), E) + sp.kron(sp.kron(E, E), D))
    Q = neumann_block(k + 1)
    I = half_identity(k + 1)
    for c1 in range(L):
        for c2 in range(L):
            for c3 in range(L):
                d = float(cells[c1, c2, c3]) - b
                if d == 0.0:
                    continue
                Q1, Q2, Q3 = (embed(Q, c * n0 + lo, N) for c in (c1, c2, c3))
                I1, I2, I3 = (embed(I, c * n0 + lo, N) for c in (c1, c2, c3))
                K = K + d * (sp.kron(sp.kron(Q1, I2), I3)
                             + sp.kron(sp.kron(I1, Q2), I3)
                             + sp.kron(sp.kron(I1, I2), Q3))
    return K.tocsr()

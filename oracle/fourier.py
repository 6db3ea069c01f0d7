"""Oracle: Fourier diagonalization of the periodic Laplacian (Section 4.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The 1D periodic Laplacian is the circulant with first column
p = (2, -1, 0, ..., 0, -1) (eq. Circ_Fourier, sign chosen positive
semidefinite), diagonalized by the DFT with eigenvalues
mu_k = [F p]_k = 4 sin^2(pi k / N), mu_0 = 0.  The 3D operator is the Kronecker
sum (eq. Lapl_Kron3) whose Fourier symbol is g(i,j,k) = mu_i + mu_j + mu_k
(eq. Lamda3D).  Its pseudo-inverse symbol G+ has g+(0,0,0) = 0 and 1/g
elsewhere (eqs. coreTens and 3a).  Applying it through the FFT is the paper's
"first approach".
"""

from __future__ import annotations

import numpy as np


def laplacian_eigenvalues(N: int) -> np.ndarray:
    """mu_k = 4 sin^2(pi k / N), k = 0..N-1 (eq. Circ_Fourier)."""
    k = np.arange(N, dtype=np.float64)
    return 4.0 * np.sin(np.pi * k / N) ** 2


def periodic_laplacian_1d(N: int) -> np.ndarray:
    """Dense circulant with first column (2, -1, 0, ..., 0, -1)."""
    p = np.zeros(N)
    p[0] = 2.0
    p[1 % N] -= 1.0
    p[-1] -= 1.0
    return np.array([[p[(a - b) % N] for b in range(N)] for a in range(N)])


def laplacian_symbol(N: int) -> np.ndarray:
    """g(i,j,k) = mu_i + mu_j + mu_k (eq. Lamda3D), shape (N, N, N)."""
    m = laplacian_eigenvalues(N)
    return m[:, None, None] + m[None, :, None] + m[None, None, :]


def pinv_symbol(N: int) -> np.ndarray:
    """G+ of eq. 3a: 1/g off the zero mode, 0 at (0,0,0)."""
    g = laplacian_symbol(N)
    out = np.zeros_like(g)
    nz = g > 0
    out[nz] = 1.0 / g[nz]
    return out


def apply_symbol(symbol: np.ndarray, r: np.ndarray) -> np.ndarray:
    """F* diag(symbol) F r for a real, even symbol (real result)."""
    return np.real(np.fft.ifftn(symbol * np.fft.fftn(r)))


def apply_pinv_laplacian(r: np.ndarray) -> np.ndarray:
    """Exact preconditioner z = A_Delta^+ r ("first approach", Section 4.2)."""
    return apply_symbol(pinv_symbol(r.shape[0]), r)


def project_zero_mean(u: np.ndarray) -> np.ndarray:
    """Orthogonal projection onto <u, 1> = 0 (the solution subspace of eq. DD_Eqn)."""
    return u - u.mean()


def laplacian_apply(u: np.ndarray) -> np.ndarray:
    """A_Delta u for unit coefficient: sum_l (2u - u_{p+e_l} - u_{p-e_l})."""
    out = np.zeros_like(u, dtype=np.float64)
    for l in range(u.ndim):
        out += 2.0 * u - np.roll(u, -1, axis=l) - np.roll(u, 1, axis=l)
    return out

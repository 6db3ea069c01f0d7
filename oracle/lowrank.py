"""Oracle: low-Kronecker-rank approximation of the Laplacian pseudo-inverse.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.2 reshapes the Fourier-diagonal pseudo-inverse into the tensor G+
(eq. 3a), computes a Tucker decomposition of it and converts the Tucker core to
a canonical (CP) tensor of small rank R ("Tucker-to-canonical"); Lemma
RankPinverse bounds R through a quadrature of the Laplace transform
1/x = int_0^inf exp(-x t) dt.  The canonical factors u_l^(k) then give the
preconditioner as a sum of R Kronecker products of circulants
C_l^(k) = F* diag(u_l^(k)) F (eq. Lap3DtimesX).

The paper fixes neither norms, ranks nor the algorithm.  This oracle takes
the following reading, step by step (all steps are restated by the library's
builder independently):

 1. mu_k = 4 sin^2(pi k/N) and G+ as in eq. 3a.
 2. A Laplace-transform quadrature with R nodes: substituting t = e^s gives
    1/x = int exp(-x e^s + s) ds, and the trapezoidal rule with step eta at
    s_k = -ln(b) - shift + k*eta gives 1/x ~ sum_k w_k exp(-t_k x) with
    t_k = e^{s_k}, w_k = eta*t_k.  (eta, shift) are taken from a fixed grid,
    minimizing the largest relative error on 257 geometric samples of
    [a, b] = [mu_1, 12].  (The paper's 1/pi prefactor is read as a typo.)
    The nodes and weights are then refined towards the best relative
    approximation of 1/x on [a, b] by R exponentials (refined_quadrature);
    "the quadrature" below means the refined one.
 3. The zero mode of G+ is annihilated by the zero-mean projection applied to
    every preconditioned vector, so its value is free; it is set to the
    quadrature's value q(0) = sum_k w_k so that the tensor is smooth there.
 4. Relative weighting: W = (s x s x s) * G~ with s_i = (mu_i + mu_1)^(1/3).
    A rank-one positive weight changes neither Tucker nor canonical ranks; it
    moves the Frobenius fit towards relative accuracy, which is what the
    preconditioner needs (its quality is the spread of G_R / G+).
 5. Tucker: one orthonormal basis U (the tensor is symmetric) from the leading
    eigenvectors of the Gram matrix of the mode-1 unfolding, keeping the
    smallest rank r_T whose discarded eigenvalue tail is <= eps^2 ||W||^2 / 3
    (so the HOSVD error is <= eps ||W||), and at least R.  Core
    B = W x1 U^T x2 U^T x3 U^T.
 6. Tucker-to-canonical: CP-ALS on B with R terms, initialized by the
    quadrature factors projected on U (U^T (s * u_q)), 50 sweeps.  With
    rank = 0, R is the smallest rank >= 2 whose core fit error
    ||B - CP|| / ||B|| is <= eps (else r_T).
 7. The canonical factors are u = U v / s (symmetrized to be even).  Of the
    ALS factors and the plain quadrature factors, the one with the smaller
    spread rho_max / rho_min (rho = G_R * g on the nonzero modes) is kept.
 8. Gate: rho_min must be positive (else the preconditioner is indefinite).
"""

from __future__ import annotations

import numpy as np

from .fourier import laplacian_eigenvalues, laplacian_symbol, pinv_symbol

ALS_SWEEPS = 50
QUAD_SAMPLES = 257
QUAD_STEPS = [0.30 + 0.025 * j for j in range(49)]
QUAD_SHIFTS = [-2.0 + 0.1 * i for i in range(61)]
SPECTRUM_TOP = 12.0     # largest value of g = mu_i + mu_j + mu_k


def laplace_quadrature(R: int, a: float, b: float):
    """Nodes t_k and weights w_k of 1/x ~ sum_k w_k exp(-t_k x) on [a, b]."""
    x = a * (b / a) ** (np.arange(QUAD_SAMPLES) / (QUAD_SAMPLES - 1))
    best = None
    for eta in QUAD_STEPS:
        for shift in QUAD_SHIFTS:
            s = -np.log(b) - shift + eta * np.arange(R)
            t = np.exp(s)
            w = eta * t
            q = np.exp(-np.outer(x, t)) @ w
            err = np.max(np.abs(x * q - 1.0))
            if best is None or err < best[0]:
                best = (err, t, w)
    return best[1], best[2], best[0]


REFINE_SAMPLES = 513
REFINE_OUTER = 20
REFINE_INNER = 50


def refined_quadrature(R: int, a: float, b: float):
    """The quadrature of laplace_quadrature, refined towards the best relative
    (minimax) approximation of 1/x on [a, b] by R exponentials.

    Parameters theta = (ln t_k, ln w_k).  Outer loop (Lawson): weights on 513
    geometric samples, multiplied by sqrt(|e|/max|e| + 1e-3) after each pass
    (e = x q(x) - 1).  Inner loop: damped Gauss-Newton on the weighted
    residual, (J^T J + lam D) d = -J^T r with D = diag(J^T J) + 1e-12 max
    diag(J^T J) and each component of d clipped to [-2, 2]; a step is kept
    only if it lowers the weighted sum of
    squares (then lam /= 10, floor 1e-12), else lam *= 10 (at most 10 tries).
    The iterate with the smallest max |e| is returned.
    """
    t, w, err0 = laplace_quadrature(R, a, b)
    x = a * (b / a) ** (np.arange(REFINE_SAMPLES) / (REFINE_SAMPLES - 1))
    th = np.concatenate([np.log(t), np.log(w)])

    def resid(th, wts):
        tt, ww = np.exp(th[:R]), np.exp(th[R:])
        E = np.exp(-np.outer(x, tt)) * ww[None, :]          # (M, R): w_k exp(-t_k x)
        e = x * E.sum(axis=1) - 1.0
        return e, E, tt

    best = (err0, t, w)
    wts = np.ones_like(x)
    for _ in range(REFINE_OUTER):
        lam = 1e-3
        for _ in range(REFINE_INNER):
            e, E, tt = resid(th, wts)
            r = wts * e
            J = np.concatenate([(wts * x)[:, None] * (-x[:, None] * tt[None, :] * E),
                                (wts * x)[:, None] * E], axis=1)
            A = J.T @ J
            g = J.T @ r
            D = np.diag(A) + 1e-12 * np.diag(A).max()
            f0 = float(r @ r)
            accepted = False
            for _ in range(10):
                d = np.linalg.solve(A + lam * np.diag(D), -g)
                d = np.clip(d, -2.0, 2.0)
                e1, _, _ = resid(th + d, wts)
                r1 = wts * e1
                f1 = float(r1 @ r1)
                if np.isfinite(f1) and f1 < f0:
                    th = th + d
                    lam = max(lam / 10.0, 1e-12)
                    accepted = True
                    break
                lam *= 10.0
            if not accepted or f0 - f1 <= 1e-15 * f0:
                break
        e, _, _ = resid(th, np.ones_like(x))
        m = float(np.abs(e).max())
        if m < best[0]:
            best = (m, np.exp(th[:R]), np.exp(th[R:]))
        wts = wts * np.sqrt(np.abs(e) / m + 1e-3)
        wts = wts / wts.max()
    return best[1], best[2], best[0]


def quadrature_factors(mu: np.ndarray, t: np.ndarray, w: np.ndarray) -> np.ndarray:
    """u^(k)(i) = w_k^(1/3) exp(-t_k mu_i), shape (R, N) (one mode)."""
    return np.cbrt(w)[:, None] * np.exp(-np.outer(t, mu))


def tucker_basis(W: np.ndarray, eps: float, rmin: int):
    """Leading eigenvectors of the mode-1 Gram matrix (HOSVD, symmetric W)."""
    N = W.shape[0]
    W1 = W.reshape(N, N * N)
    M = W1 @ W1.T
    evals, evecs = np.linalg.eigh(M)
    evals = np.clip(evals[::-1], 0.0, None)
    evecs = evecs[:, ::-1]
    total = evals.sum()
    r = N
    for rr in range(1, N + 1):
        if evals[rr:].sum() <= eps * eps * total / 3.0:
            r = rr
            break
    r = min(max(r, rmin), N)
    return evecs[:, :r]


def tucker_core(W: np.ndarray, U: np.ndarray) -> np.ndarray:
    """B = W x1 U^T x2 U^T x3 U^T."""
    return np.einsum("ijk,ia,jb,kc->abc", W, U, U, U, optimize=True)


def cp_full(V) -> np.ndarray:
    """sum_r V0[:, r] (x) V1[:, r] (x) V2[:, r]."""
    return np.einsum("ar,br,cr->abc", V[0], V[1], V[2], optimize=True)


def cp_als(B: np.ndarray, V0, sweeps: int = ALS_SWEEPS):
    """Alternating least squares for B ~ sum_r v1_r (x) v2_r (x) v3_r.

    V0 is one initial factor used for all three modes, or a list of three.
    """
    V = [np.array(v, dtype=np.float64) for v in (V0 if isinstance(V0, (list, tuple)) else (V0, V0, V0))]
    for _ in range(sweeps):
        for m in range(3):
            o = [V[i] for i in range(3) if i != m]
            if m == 0:
                M = np.einsum("abc,br,cr->ar", B, o[0], o[1])
            elif m == 1:
                M = np.einsum("abc,ar,cr->br", B, o[0], o[1])
            else:
                M = np.einsum("abc,ar,br->cr", B, o[0], o[1])
            G = (o[0].T @ o[0]) * (o[1].T @ o[1])
            V[m] = np.linalg.solve(G, M.T).T
    return V


def symbol_from_factors(F: np.ndarray) -> np.ndarray:
    """G_R = sum_k u1^(k) (x) u2^(k) (x) u3^(k); F has shape (3, R, N)."""
    return np.einsum("ri,rj,rk->ijk", F[0], F[1], F[2], optimize=True)


def rho_range(F: np.ndarray):
    """(min, max) of rho = G_R * g over the nonzero modes."""
    N = F.shape[2]
    g = laplacian_symbol(N)
    rho = (symbol_from_factors(F) * g)[g > 0]
    return float(rho.min()), float(rho.max())


def cancellation_ratio(F: np.ndarray) -> float:
    """sum_k ||u1|| ||u2|| ||u3|| / ||G_R||_F (1 means no cancellation)."""
    GR = symbol_from_factors(F)
    terms = sum(np.linalg.norm(F[0, k]) * np.linalg.norm(F[1, k]) * np.linalg.norm(F[2, k])
                for k in range(F.shape[1]))
    return float(terms / np.linalg.norm(GR))


def _even(u: np.ndarray) -> np.ndarray:
    N = u.shape[-1]
    refl = u[..., (-np.arange(N)) % N]
    return 0.5 * (u + refl)


def canonical_preconditioner(N: int, eps: float = 1e-3, rank: int = 0):
    """Canonical factors (3, R, N) of the preconditioner symbol and a report."""
    mu = laplacian_eigenvalues(N)
    a, b = mu[1], SPECTRUM_TOP
    s = np.cbrt(mu + mu[1])
    S = s[:, None, None] * s[None, :, None] * s[None, None, :]

    R_ref = rank if rank > 0 else 12
    t, w, _ = refined_quadrature(R_ref, a, b)
    Gt = pinv_symbol(N)
    Gt[0, 0, 0] = w.sum()
    W = S * Gt
    U = tucker_basis(W, eps, rank if rank > 0 else 1)
    B = tucker_core(W, U)
    nB = np.linalg.norm(B)
    rT = U.shape[1]

    ranks = [rank] if rank > 0 else list(range(2, rT + 1))
    for R in ranks:
        t, w, qerr = refined_quadrature(R, a, b)
        uq = quadrature_factors(mu, t, w)                  # (R, N)
        V0 = U.T @ (s[:, None] * uq.T)                     # (rT, R)
        V = cp_als(B, V0)
        cperr = float(np.linalg.norm(B - cp_full(V)) / nB)
        if rank > 0 or cperr <= eps:
            break

    F_als = np.stack([_even(((U @ V[m]) / s[:, None]).T) for m in range(3)])
    F_q = np.stack([uq, uq, uq])
    lo_a, hi_a = rho_range(F_als)
    lo_q, hi_q = rho_range(F_q)
    spread_a = hi_a / lo_a if lo_a > 0 else np.inf
    spread_q = hi_q / lo_q if lo_q > 0 else np.inf
    if spread_a <= spread_q:
        F, lo, hi, source = F_als, lo_a, hi_a, "als"
    else:
        F, lo, hi, source = F_q, lo_q, hi_q, "quadrature"
    info = dict(R=R, rT=rT, cp_rel_err=cperr, rho_min=lo, rho_max=hi,
                quad_rel_err=float(qerr), source=source,
                cancellation=cancellation_ratio(F))
    if not lo > 0.0:
        raise ValueError("low-rank preconditioner is indefinite (rho_min <= 0)")
    return F, info


def circulant(u: np.ndarray) -> np.ndarray:
    """C = F* diag(u) F for even u: C[a, b] = (1/N) sum_j u_j cos(2 pi j (a-b)/N)."""
    N = u.shape[0]
    j = np.arange(N)
    d = (np.arange(N)[:, None] - np.arange(N)[None, :])
    C = np.zeros((N, N))
    for jj in j:
        C += u[jj] * np.cos(2.0 * np.pi * jj * d / N)
    return C / N


def kron_apply(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_k (C1^(k) (x) C2^(k) (x) C3^(k)) x as three mode products (eq. Lap3DtimesX)."""
    z = np.zeros_like(x, dtype=np.float64)
    for k in range(F.shape[1]):
        C1, C2, C3 = (circulant(F[l, k]) for l in range(3))
        z += np.einsum("ai,bj,ck,ijk->abc", C1, C2, C3, x, optimize=True)
    return z


def kron_matrix(F: np.ndarray) -> np.ndarray:
    """Dense sum_k C1 (x) C2 (x) C3 (tiny N only)."""
    N = F.shape[2]
    M = np.zeros((N ** 3, N ** 3))
    for k in range(F.shape[1]):
        C1, C2, C3 = (circulant(F[l, k]) for l in range(3))
        M += np.kron(np.kron(C1, C2), C3)
    return M

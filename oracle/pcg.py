"""Oracle: textbook preconditioned conjugate gradients (eqs. DD_Eqn, PCG_DD_Eqn).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The system K u = f with <f, 1> = 0 is solved on the subspace <u, 1> = 0
(Section 4.1).  The iteration is the standard Hestenes-Stiefel PCG (as in
Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Algorithm 9.1),
started from x0 = 0.  The paper gives the stopping criterion only as a
tolerance (Sections 5.1, 5.2); it is read as the relative 2-norm of the true
residual ||f - K x|| / ||f|| <= tol: the loop stops on the recursive residual,
then recomputes the true residual and, if it is still above tol, restarts the
recursion from it.  The returned x is projected to zero mean.
"""

from __future__ import annotations

import numpy as np


def pcg(apply_K, f, apply_M, tol=1e-8, maxit=2000, x0=None):
    f = np.asarray(f, dtype=np.float64)
    f = f - f.mean()
    nf = float(np.linalg.norm(f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    hist, alphas, betas = [], [], []
    if nf == 0.0:
        return dict(x=np.zeros_like(f), iters=0, relres=0.0, history=hist,
                    alphas=alphas, betas=betas, converged=True)
    r = f - apply_K(x)
    it = 0
    converged = False
    while it < maxit:
        z = apply_M(r)
        z = z - z.mean()
        p = z.copy()
        rz = float(np.vdot(r, z))
        while it < maxit:
            q = apply_K(p)
            pq = float(np.vdot(p, q))
            alpha = rz / pq
            x += alpha * p
            r -= alpha * q
            it += 1
            alphas.append(alpha)
            rn = float(np.linalg.norm(r))
            hist.append(rn / nf)
            if rn <= tol * nf:
                break
            z = apply_M(r)
            z = z - z.mean()
            rz_new = float(np.vdot(r, z))
            beta = rz_new / rz
            betas.append(beta)
            rz = rz_new
            p = z + beta * p
        r = f - apply_K(x)
        if float(np.linalg.norm(r)) <= tol * nf:
            converged = True
            break
    x = x - x.mean()
    relres = float(np.linalg.norm(f - apply_K(x)) / nf)
    return dict(x=x, iters=it, relres=relres, history=hist, alphas=alphas,
                betas=betas, converged=converged)


def lanczos_ritz_values(alphas, betas, k=None):
    """Eigenvalues of the PCG Lanczos tridiagonal T_k (Ritz values of M K).

    T[j, j] = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T[j, j+1] = sqrt(beta_j)/alpha_j  (Saad, Section 6.7.3).
    """
    k = len(alphas) if k is None else k
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return np.linalg.eigvalsh(T)

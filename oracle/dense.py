"""Oracle: brute-force dense solve for tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

K is singular with null space the constants (periodic problem, eq. DD_Eqn),
so the minimum-norm least-squares solution of K u = f is the zero-mean one.
"""

from __future__ import annotations

import numpy as np

from .assembly import kron_stiffness


def dense_solve(cells, n0, f):
    K = kron_stiffness(cells, n0).toarray()
    u, *_ = np.linalg.lstsq(K, f.reshape(-1), rcond=None)
    return u.reshape(f.shape)

"""Plain FP64 CPU oracle for the periodic 3D checkerboard PCG solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
solver library never calls it, and it shares no code with the HIP path.

Every function follows the paper (Khoromskaia & Khoromskij, "Tensor-based
techniques for fast discretization and solution of 3D elliptic equations with
random coefficients", arXiv:2007.06524) and cites the section or equation it
restates.  The code is deliberately slow and direct: numpy / scipy in float64,
no blocking, fusion or reordering beyond what the cited definition states.

Modules
  assembly   voxel map, paper-literal Kronecker-sum stiffness (eq. As_Kron_d),
             edge-average stencil, corrector right-hand sides (eq. FEM_discr_RHS)
  fourier    periodic Laplacian eigenvalues (eq. Circ_Fourier), the
             pseudo-inverse symbol G+ (eq. 3a), FFT application ("first approach")
  lowrank    Laplace-transform quadrature (Lemma RankPinverse), Tucker basis,
             Tucker-to-canonical ALS, circulant factors, Kronecker apply
             (eq. Lap3DtimesX)
  pcg        textbook preconditioned CG on the zero-mean subspace (eq. DD_Eqn)
  homogenize homogenized matrix (eq. Ahom3_m_entry_comp) and its energy form
  dense      brute-force dense solve for tiny grids
  twod       the same discretization, solve, homogenized matrix and rank-R
             preconditioner with d = 2 (eqs. As_Kron, DiagFLaplace2D,
             Lap2DtimesX)

Parity status: every function is pinned by a test under tests/ against facts
the paper or the mathematics fix (worked matrices, closed forms, invariants,
brute force).  No function is "parity unpinned".
"""

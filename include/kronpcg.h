/*
 * kronpcg.h - C ABI of the MI355X (gfx950) solver for the periodic 3D
 * elliptic problem -div(a grad u) = f with a random checkerboard coefficient,
 * preconditioned by a low-Kronecker-rank approximation of the periodic
 * Laplacian pseudo-inverse.
 *
 * Method: Khoromskaia & Khoromskij, "Tensor-based techniques for fast
 * discretization and solution of 3D elliptic equations with random
 * coefficients" (arXiv:2007.06524).
 *
 * Conventions shared by every entry point
 *  - Every call returns an int status: KP_OK (0), a warning (> 0) or an error
 *    (< 0).  After an error, kp_last_error() returns a message for the calling
 *    thread.
 *  - Grid: the unit cube carries L^3 unit cells with n0 grid intervals per cell
 *    edge, N = n0*L distinct periodic nodes per axis, h = 1/N (Section 3.1; the
 *    paper's n1 = N + 1 counts the periodic image of node 0 as well).
 *  - Layout: every N^3 field is a dense C-order array [i1][i2][i3] with i3
 *    fastest, i.e. the big-endian multi-index map of Section 3.2.  Cell arrays
 *    are [c1][c2][c3] of L^3 doubles in the same order.
 *  - "host" pointers are ordinary CPU memory, copied during the call; the
 *    caller keeps ownership.  "device" pointers are GPU memory on the
 *    context's device, owned by the caller, and must stay valid until the
 *    call's work on the context stream has completed.
 *  - All GPU work is ordered on the context's stream.  Calls that return host
 *    results (stats, info, ahom) synchronize that stream before returning.
 *  - Opaque handles (kp_context, kp_coeff, kp_precond) are owned by the
 *    library and released with the matching kp_*_destroy / kp_free_* call.
 */
#ifndef KRONPCG_H
#define KRONPCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kp_context kp_context;
typedef struct kp_coeff kp_coeff;
typedef struct kp_precond kp_precond;

enum kp_status {
  KP_OK = 0,
  KP_NOT_CONVERGED = 1,        /* maxit reached; x and stats are valid          */
  KP_WARN_RHS_MEAN = 2,        /* f had a nonzero mean, which was projected out */
  KP_ERR_ARG = -1,             /* invalid argument (pointer, size, value)       */
  KP_ERR_HIP = -2,             /* a HIP runtime call failed                     */
  KP_ERR_NOMEM = -3,           /* device allocation failed                      */
  KP_ERR_BREAKDOWN = -4,       /* PCG breakdown: <p,Kp> <= 0, <r,z> <= 0 or NaN */
  KP_ERR_PRECOND_INDEFINITE = -5, /* low-rank symbol not positive on all modes  */
  KP_ERR_STATE = -6            /* handles from different contexts / sizes       */
};

/* Arithmetic of the solve.
 * KP_FP64: stencil, preconditioner (FP64 MFMA) and vectors in double.
 * KP_MIXED_BF16 / KP_MIXED_FP16: stencil and PCG vectors in float, the three
 *   preconditioner mode products on BF16 / FP16 MFMA with float accumulation,
 *   flexible (Polak-Ribiere) PCG; x, all dot products, norms and the zero-mean
 *   projection stay in double, and the residual is periodically replaced by
 *   the true residual f - K x computed in double from double weights.  The
 *   residual is scaled by a power of two before its 16-bit rounding (RMS near
 *   1).  FP16 keeps 11 significant bits in the rounded residual and the
 *   intermediates against BF16's 8 (fewer iterations: 71/71/71 against
 *   84/71/72 on a 256^3 Bernoulli{1,100} checkerboard) at the same MFMA rate;
 *   BF16 has the wider exponent range.  An overflow in FP16 makes the dot
 *   products non-finite and ends the solve with KP_ERR_BREAKDOWN. */
enum kp_precision { KP_FP64 = 0, KP_MIXED_BF16 = 1, KP_MIXED_FP16 = 2 };

typedef struct {
  int rank;              /* canonical rank R actually used                    */
  int tucker_rank;       /* Tucker rank r_T of the weighted symbol            */
  int source;            /* 0: ALS-refined Tucker-to-canonical, 1: Laplace quadrature */
  int pad_;
  double cp_rel_err;     /* ||B - CP|| / ||B|| of the Tucker core fit         */
  double quad_rel_err;   /* max relative error of the Laplace quadrature      */
  double rho_min;        /* min over nonzero modes of G_R / G+                */
  double rho_max;        /* max over nonzero modes of G_R / G+                */
  double cancellation;   /* sum_k |u1||u2||u3| / ||G_R||  (1 = none)          */
  double build_ms;       /* host time of the construction                     */
} kp_precond_info;

typedef struct {
  double tol;            /* stop when ||f - K x||_2 <= tol ||f||_2 (true residual); default 1e-8 */
  int maxit;             /* iteration cap; default 2000                                 */
  int replace_every;     /* mixed precision: true-residual replacement period; 0 = never (default 25 mixed, 0 FP64) */
  int use_x0;            /* 1: start from the contents of x; 0: start from x = 0       */
  int check_every;       /* iterations queued between host convergence checks; 0 = auto */
} kp_solve_opts;

typedef struct {
  int iters;             /* PCG iterations performed                          */
  int replacements;      /* true-residual replacements performed              */
  double relres_true;    /* ||f - K x|| / ||f|| in double at exit             */
  double relres_rec;     /* recursive residual ratio at exit                  */
  double rhs_mean;       /* mean removed from f                               */
  double ms;             /* wall time of the solve on the stream (hipEvents); batched: of the batch */
  int status;            /* kp_status of this solve (batched: of this system)  */
  int pad_;
} kp_solve_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL selects the null stream).  *out receives the handle. */
int kp_context_create(int device, void* hip_stream, kp_context** out);

/* Replace the stream used by later calls. */
int kp_context_set_stream(kp_context* ctx, void* hip_stream);

/* Route the library's device allocations through caller callbacks (for
 * example a caching allocator).  alloc(bytes, user) returns device memory or
 * NULL; release(ptr, user) frees it.  Pass NULL callbacks to go back to
 * hipMalloc / hipFree.  Only affects allocations made after the call. */
int kp_context_set_allocator(kp_context* ctx, void* (*alloc)(size_t bytes, void* user),
                             void (*release)(void* ptr, void* user), void* user);

int kp_context_destroy(kp_context* ctx);

/* Per-kernel-class timing with HIP events recorded on the context stream
 * around every launch of the class (the paper reports matrix generation,
 * right-hand side and solver times, Tables 1-3; this splits the solver).
 * Enabling clears the accumulators; reading synchronizes the stream.
 * ms and launches are host arrays of KP_TIMER_COUNT entries. */
enum kp_timer {
  KP_TIMER_STENCIL = 0,     /* 7-point stencil q = K p inside the iteration      */
  KP_TIMER_GEMM_MODE3 = 1,  /* preconditioner GEMM contracting i3 (first stage)  */
  KP_TIMER_GEMM_MODE2 = 2,  /* preconditioner GEMM contracting i2 (second stage) */
  KP_TIMER_GEMM_MODE1 = 3,  /* preconditioner GEMM contracting (k, i1) (third)   */
  KP_TIMER_VECTOR = 4,      /* vector updates, casts, reductions, finalize       */
  KP_TIMER_ASSEMBLE = 5,    /* assembly of weights and right-hand sides          */
  KP_TIMER_RESIDUAL = 6,    /* true residual f - K x in double                   */
  KP_TIMER_COUNT = 7
};
int kp_context_set_timing(kp_context* ctx, int enable);
int kp_context_read_timing(kp_context* ctx, double* ms, long long* launches);

/* ---- assembly (Sections 3.1-3.3) ---------------------------------------- */

/* Assemble the stiffness and the three corrector right-hand sides of one
 * coefficient realization (the paper's "matr." and "RHS" steps).
 *   a_cell: host, L^3 doubles, [c1][c2][c3]; each value finite and > 0
 *           (the checkerboard coefficient lambda + beta * a_hat of eq.
 *           coef_diag, one value per unit cell).
 *   L >= 1, n0 >= 1, N = n0*L >= 2.
 * The stiffness is the Kronecker sum of eq. As_Kron_d: per cell a_c times the
 * 1D Neumann Laplacian in one direction and the lumped half-weight identity
 * diag(1/2,1,...,1,1/2) in the others, wrapped periodically.  It is stored as
 * the three edge-weight fields w_l(p) = weight of the edge (p, p+e_l) (the
 * mean of the coefficient over the four voxels sharing that edge), in double
 * and, for mixed precision, also in float.  The corrector right-hand sides of
 * eq. FEM_discr_RHS are f_i(p) = h (w_i(p) - w_i(p - e_i)) for the operator
 * K = A / h, in double.  Errors: KP_ERR_ARG on bad sizes or a non-finite or
 * non-positive cell. */
int setup_coeff(kp_context* ctx, int L, int n0, const double* a_cell, int precision,
                kp_coeff** out);

/* Same, with the coefficient perturbed only on the centred sub-cell of every
 * unit cell (Section 3.1: the sub-cell S_s of edge 2 alpha / L = incl * h,
 * i.e. alpha = incl / (2 n0), centred in G_s; Section 3.3 assembles the
 * stiffness from Neumann blocks of incl + 1 nodes on the sub-cells).
 *   incl: voxels per sub-cell edge, 1 <= incl <= n0 with n0 - incl even; the
 *         voxels (n0 - incl)/2 .. (n0 + incl)/2 - 1 of a cell along every axis
 *         form its sub-cell.  incl = n0 is setup_coeff.
 *   background: coefficient everywhere outside the sub-cells (finite, > 0;
 *         ignored when incl = n0).  A cell whose value equals the background
 *         is an unperturbed cell: the paper's binary model is a_cell in
 *         {1, lambda} with background lambda.
 * A voxel inside a sub-cell takes the cell's value, any other the background;
 * the edge weights are the voxel means as above.  The homogenized matrix uses
 * the exact mean of this coefficient, background + (incl/n0)^3 (mean(a_cell)
 * - background).  kp_coeff_update keeps incl and background.  Errors as
 * setup_coeff, and KP_ERR_ARG for a sub-cell that does not centre or a bad
 * background. */
int setup_coeff_inclusions(kp_context* ctx, int L, int n0, int incl, double background,
                           const double* a_cell, int precision, kp_coeff** out);

/* Copy the assembled fields into caller device buffers (either may be NULL):
 *   w_dev: 3*N^3 doubles [l][i1][i2][i3];  f_dev: 3*N^3 doubles [i-1][i1][i2][i3]. */
int kp_coeff_fields(kp_context* ctx, const kp_coeff* coeff, double* w_dev, double* f_dev);

/* Re-assemble an existing coefficient from a new realization whose cells are
 * already in device memory (a_cell_dev: L^3 doubles, same L and n0 as at
 * setup_coeff), as for a long sequence of stochastic realizations.  The cells
 * are validated on the device (finite, > 0; else KP_ERR_ARG, and the
 * coefficient keeps its previous fields).  Synchronizes the stream. */
int kp_coeff_update(kp_context* ctx, kp_coeff* coeff, const double* a_cell_dev);

/* Grid size N of an assembled coefficient (or -1 for NULL). */
int kp_coeff_size(const kp_coeff* coeff);

int kp_free_coeff(kp_coeff* coeff);

/* q = K p for the assembled stiffness (eq. FEM_matrix with the Kronecker-sum
 * stiffness, 7-point form), p and q device arrays of N^3 doubles.  With
 * precision KP_FP64 the operator runs in double; with a mixed precision it
 * runs the float stencil on float weights (inputs rounded to float, output
 * widened to double). */
int kp_stiffness_apply(kp_context* ctx, const kp_coeff* coeff, int precision,
                       const double* p_dev, double* q_dev);

/* ---- preconditioner (Section 4.2) --------------------------------------- */

/* Canonical factors of the low-rank preconditioner symbol, on the host only
 * (no GPU work).  The symbol G+ of eq. 3a (1/(mu_i+mu_j+mu_k),
 * mu_k = 4 sin^2(pi k/N)) is approximated by G_R = sum_k u1^(k) x u2^(k) x u3^(k):
 * Tucker decomposition of the relatively weighted symbol followed by a
 * Tucker-to-canonical ALS of its core, initialized from a quadrature of the
 * Laplace transform 1/x = int exp(-xt) dt (Lemma RankPinverse).
 *   eps:  Tucker truncation tolerance (relative Frobenius); with rank = 0
 *         also the target of the core fit that selects R.
 *   rank: R > 0 fixes the rank (1..16); 0 selects it from eps.
 *   factors_out: host, capacity doubles, receives 3*R*N values [l][k][i].
 * Errors: KP_ERR_ARG (N < 2, eps not in (0,1), rank > 16, capacity too small),
 * KP_ERR_PRECOND_INDEFINITE when min G_R/G+ <= 0. */
int kp_lowrank_factors(int N, double eps, int rank, double* factors_out, size_t capacity,
                       kp_precond_info* info);

/* Build the preconditioner for grid size N: the canonical factors of
 * kp_lowrank_factors, turned into the dense N x N circulants
 * C_l^(k) = F* diag(u_l^(k)) F (real symmetric, eq. Lap3DtimesX) and
 * uploaded in the layout of the mode-product GEMMs.  info may be NULL. */
int build_preconditioner(kp_context* ctx, int N, double eps, int rank, int precision,
                         kp_precond** out, kp_precond_info* info);

/* The paper's first approach (Section 4.2): the exact pseudo-inverse of the
 * periodic Laplacian, diagonal in the Fourier basis (eq. 3a with the constant
 * prefactor dropped), z = F^-1 (g F r) with g(k) = 1 / sum_l 4 sin^2(pi k_l / N)
 * and g(0) = 0, applied by double-precision 3D real-to-complex FFTs (hipFFT)
 * and one symbol-scaling kernel.  FP64 only, one system at a time: usable
 * with pcg_solve (FP64 coefficient) and kp_precond_apply, rejected by
 * pcg_solve_batched (KP_ERR_STATE); rank 0, nothing to autotune.  A
 * comparison point for the low-rank preconditioner.  Errors: KP_ERR_ARG for
 * N outside [2, 2048], KP_ERR_HIP when a plan cannot be made. */
int build_preconditioner_fft(kp_context* ctx, int N, kp_precond** out);

/* Same, from caller-supplied canonical factors: factors is host memory of
 * 3*R*N doubles [l][k][i], each u_l^(k) even (u(i) = u(N-i)), 1 <= R <= 16. */
int kp_precond_from_factors(kp_context* ctx, int N, int R, const double* factors,
                            int precision, kp_precond** out);

/* Autotuner of the three mode-product GEMMs: times each tile configuration of
 * each stage on the context stream (`reps` launches after a warm-up, on
 * scratch operands of the preconditioner's size) and keeps the fastest per
 * stage for later applies.  table (host, may be NULL) receives up to cap
 * entries {stage 0..2 (contracting i3, i2, (k,i1)), tile rows, tile columns,
 * K tile, block order, kernel (0: both operands streamed through LDS;
 * 1: circulant operand built in LDS from the circulants' first columns, only
 * the data operand streamed; 2: as 1, the data operand streamed by each wave
 * straight into registers; a configuration whose kernel cannot run the stage
 * runs as the nearest one that can, and its entry reports the tile, order and
 * kernel that ran), average ms}; *count the number of configurations timed.
 * Block order 0 walks the column tiles of the data operand fastest; order 1
 * gives all row tiles of one column tile to blocks on the same XCD (one L2),
 * so that column tile is read from HBM once.  Each timed launch follows an
 * untimed launch of the previous stage with its chosen tiles, after the
 * intermediates have been overwritten (cache state as in a solve).
 * Synchronizes the stream. */
typedef struct {
  int stage, bm, bn, bk, order, circ;
  double ms;
} kp_tile_timing;
int kp_precond_autotune(kp_context* ctx, kp_precond* pc, int reps, kp_tile_timing* table, int cap,
                        int* count);

/* Pin (set) or read (get) the tile configuration of the three stages, e.g.
 * to reuse an earlier tuning: tiles[s] is the position of the configuration
 * among the ones of stage s in the autotuner's table (0-based), or -1 for the
 * size heuristic.  set: KP_ERR_ARG for an index out of range. */
int kp_precond_set_tiles(kp_precond* pc, const int* tiles);
int kp_precond_get_tiles(const kp_precond* pc, int* tiles);

/* Rank R of a preconditioner (or -1 for NULL). */
int kp_precond_rank(const kp_precond* pc);

/* z = sum_k (C1^(k) x C2^(k) x C3^(k)) r (eq. Lap3DtimesX), as three MFMA
 * mode-product GEMMs, r and z device arrays of N^3 doubles.  No zero-mean
 * projection is applied.  In a mixed precision, r is rounded to BF16/FP16
 * and the result (float accumulation) is widened to double. */
int kp_precond_apply(kp_context* ctx, const kp_precond* pc, const double* r_dev, double* z_dev);

int kp_free_precond(kp_precond* pc);

/* ---- solve (Section 4.1) ------------------------------------------------ */

/* Solve K x = f on the subspace <x,1> = 0 (eq. DD_Eqn) by PCG preconditioned
 * with the low-rank pseudo-inverse (eq. PCG_DD_Eqn).
 *   rhs:   1..3 selects the assembled corrector right-hand side f_rhs;
 *          0 uses f_dev (device, N^3 doubles), projected to zero mean.
 *   x_dev: device, N^3 doubles, caller-owned; read as the initial guess when
 *          opts->use_x0, always overwritten with the zero-mean solution.
 *   opts:  may be NULL for the defaults; stats may be NULL.
 * The precision of the solve is the coefficient's; a mixed coefficient needs a
 * preconditioner of a mixed precision and vice versa (else KP_ERR_STATE).
 * Returns KP_OK, KP_NOT_CONVERGED, KP_WARN_RHS_MEAN (when the removed mean of
 * a user f exceeds 1e-12 ||f|| / sqrt(N^3)), or an error.  ||f|| = 0 gives
 * x = 0 and 0 iterations. */
int pcg_solve(kp_context* ctx, const kp_coeff* coeff, const kp_precond* pc, int rhs,
              const double* f_dev, double* x_dev, const kp_solve_opts* opts,
              kp_solve_stats* stats);

/* Batched corrector solves: the Monte-Carlo setting of Section 5, many
 * realizations of the coefficient (of uneven L) with the three corrector
 * problems of each (eq. DD_Eqn with f = f_1, f_2, f_3).  Instance i is
 * (coeffs[i], preconds[i]) with coeffs[i]->N == preconds[i]->N; all handles
 * belong to ctx and share one precision (mixed or FP64).  System 3 i + j
 * (j = 0..2) solves corrector j+1 of instance i into x_dev[3 i + j] (device,
 * N_i^3 doubles, caller-owned; read as the initial guess when opts->use_x0,
 * always overwritten with the zero-mean solution).
 * Instances that share a preconditioner and the coefficient geometry (n0,
 * sub-cell size, background) form a group; every PCG step of a group runs as
 * one launch over all its systems, the groups run as
 * concurrent branches of one HIP graph that holds opts->check_every
 * iterations (0: 16), and the graph is replayed until every system has
 * stopped.  Convergence is decided per system on the device, by the true
 * residual in double, and a stopped system's share of every launch returns
 * at once (convergence mask).  The GEMM tiles are autotuned for each group's
 * batch size on first use (kept in the preconditioner).
 * stats (host, 3 n_inst, may be NULL) per system, with status KP_OK,
 * KP_NOT_CONVERGED or KP_ERR_BREAKDOWN; ahom (host, 9 n_inst doubles, may be
 * NULL) receives each instance's homogenized matrix (as
 * kp_homogenized_matrix).  Returns KP_OK when every system converged,
 * KP_NOT_CONVERGED when some reached maxit, KP_ERR_BREAKDOWN when some broke
 * down (the other systems are solved and reported), or an error.
 * Synchronizes the stream. */
int pcg_solve_batched(kp_context* ctx, int n_inst, const kp_coeff* const* coeffs,
                      const kp_precond* const* preconds, double* const* x_dev,
                      const kp_solve_opts* opts, kp_solve_stats* stats, double* ahom);

/* ---- the two-dimensional problem (d = 2; Table 2) ------------------------ */

/* The same solver for the periodic 2D problem -div(a grad u) = f on the unit
 * square: an L x L lattice of cells, N = n0 L nodes per axis, fields of N^2
 * doubles [i1][i2].  The stiffness is the Kronecker sum of eq. As_Kron (a
 * 5-point stencil whose edge weight is the mean of the coefficient over the
 * two voxels sharing the edge), the corrector right-hand sides are
 * f_i(p) = h (w_i(p) - w_i(p - e_i)) (A = h^(d-2) K = K), i = 1, 2, and
 * a_hom is 2 x 2: delta_ij mean(a) - sum_p phi_i(p) f_j(p).
 * A 2D coefficient or preconditioner works with pcg_solve (rhs 0..2; with a
 * 2D preconditioner of the same N), kp_stiffness_apply, kp_precond_apply,
 * kp_coeff_fields (2 N^2 doubles each), kp_coeff_update (L^2 cells) and
 * kp_homogenized_matrix (phi_dev[0..1], ahom: 4 doubles row-major); the
 * batched solver, the Monte-Carlo driver and the FFT preconditioner are 3D
 * only (KP_ERR_STATE). */

/* 2D coefficient: a_cell host, L^2 doubles [c1][c2]; incl and background as
 * setup_coeff_inclusions (incl = n0: whole cells). */
int setup_coeff_2d(kp_context* ctx, int L, int n0, int incl, double background, const double* a_cell,
                   int precision, kp_coeff** out);

/* Rank-R factors of the 2D preconditioner symbol 1 / (mu_k1 + mu_k2) (eq.
 * DiagFLaplace2D; the 2D decomposition before eq. Lap2DtimesX), host only.
 * In 2D the Tucker and canonical forms coincide with the truncated
 * eigen-expansion of the symbol matrix: the symbol is weighted to relative
 * form (s s^T * G+, s_i = sqrt(mu_i + mu_1), zero mode set to 1/mu_1), reduced
 * to its N/2 + 1 distinct indices (it is even), and its leading eigenpairs by
 * |lambda| give u1 = sqrt|lambda| z / s and u2 = sign(lambda) u1.  rank = 0
 * selects the smallest R with relative Frobenius error <= eps (at most 16).
 * factors_out: 2 R N doubles [mode][k][i].  info as kp_lowrank_factors
 * (cp_rel_err = the truncation error, tucker_rank = R).  Errors: KP_ERR_ARG,
 * KP_ERR_PRECOND_INDEFINITE if rho_min <= 0. */
int kp_lowrank_factors_2d(int N, double eps, int rank, double* factors_out, size_t capacity,
                          kp_precond_info* info);

/* 2D preconditioner z = sum_k C1^k X (C2^k)^T (eq. Lap2DtimesX with dense
 * circulants), applied as two MFMA GEMM stages (the 3D stages (ii) and (iii)
 * without the third mode).  As build_preconditioner / kp_precond_from_factors
 * (factors: 2 R N doubles, each even). */
int build_preconditioner_2d(kp_context* ctx, int N, double eps, int rank, int precision,
                            kp_precond** out, kp_precond_info* info);
int kp_precond_from_factors_2d(kp_context* ctx, int N, int R, const double* factors, int precision,
                               kp_precond** out);

/* ---- Monte-Carlo statistics (Section 5.3) ------------------------------- */

typedef struct {
  int realizations;        /* M                                                 */
  int batch;               /* realizations per batched solve (B)                */
  int chunks;              /* batched solves run (ceil(M / B))                  */
  int status;              /* worst kp_status over the systems                  */
  long long iters;         /* PCG iterations summed over the 3 M systems        */
  double max_relres_true;  /* largest true relative residual at exit            */
  double ms;               /* wall time of the whole call                       */
} kp_mc_stats;

/* Empirical homogenized matrix of M realizations at one RVE size L: for each
 * realization the three corrector solves and a_hom (eq. Ahom3_m_entry_comp),
 * then entry by entry the empirical average (eq. A_hom_Empir)
 *   mean = (1/M) sum_m A^(m)
 * and the empirical standard deviation sigma_L^M (normalization M - 1)
 *   sd = sqrt( sum_m (A^(m) - mean)^2 / (M - 1) ),
 * both summed on the device in the order m = 0..M-1.
 *   a_cells: host, M * L^3 doubles, realization m at m L^3, [c1][c2][c3],
 *            finite and > 0 (the caller draws them: the random numbers of the
 *            method are an input).
 *   incl, background: the coefficient geometry of setup_coeff_inclusions
 *            (incl = n0: whole cells).
 *   pc: preconditioner of N = n0 L in the precision to solve in (also the
 *            precision of the coefficient objects built here).
 *   opts: as pcg_solve_batched (NULL: defaults).
 *   batch: realizations per batched solve; <= 0 sizes it to about 32 GiB of
 *            solver state.  The realizations stream through B reused
 *            coefficient objects (kp_coeff_update between chunks).
 *   ahom: host, 9 M doubles (may be NULL): every realization's matrix.
 *   mean, sd: host, 9 doubles each, row-major.
 *   stats: host (may be NULL).
 * Returns KP_OK, KP_NOT_CONVERGED or KP_ERR_BREAKDOWN as pcg_solve_batched
 * (worst over the chunks; the statistics are still formed), or an error:
 * KP_ERR_ARG for M < 2, n0 L != pc's N, bad cells or geometry.  Synchronizes
 * the stream. */
int kp_mc_homogenize(kp_context* ctx, int L, int n0, int incl, double background, int M,
                     const double* a_cells, const kp_precond* pc, const kp_solve_opts* opts,
                     int batch, double* ahom, double* mean, double* sd, kp_mc_stats* stats);

/* Homogenized matrix of one realization (eq. Ahom3_m_entry_comp):
 *   ahom[i][j] = delta_ij mean(a) - h sum_p phi_i(p) f_j(p),  i,j = 1..3,
 * where phi_dev[i] (device, N^3 doubles) solves corrector i+1.  ahom is host
 * memory of 9 doubles, row-major.  No symmetrization is applied. */
int kp_homogenized_matrix(kp_context* ctx, const kp_coeff* coeff, const double* const* phi_dev,
                          double* ahom);

/* Message of the last failing call on this thread ("" if none). */
const char* kp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KRONPCG_H */

// Internal declarations of the kronpcg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "kronpcg.h"

namespace kp {

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int fail(int code, const char* fmt, ...);

#define KP_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t kp_e_ = (expr);                                                         \
    if (kp_e_ != hipSuccess)                                                           \
      return ::kp::fail(KP_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(kp_e_), \
                        __FILE__, __LINE__);                                           \
  } while (0)

#define KP_TRY(expr)             \
  do {                           \
    int kp_s_ = (expr);          \
    if (kp_s_ < 0) return kp_s_; \
  } while (0)

using bf16_t = uint16_t;  // storage of bfloat16 / float16 values

// PCG scalars kept on the device so that the iteration needs no host round trip.
struct Scalars {
  double ff;      // ||f||^2 of the projected right-hand side
  double tol2ff;  // tol^2 * ||f||^2
  double rr;      // ||r||^2
  double rho;     // <r, z - mean(z)>
  double pq;      // <p, K p>
  double alpha;
  double beta;
  double mz;      // mean of z
  double x16_scale;       // power of two applied to r before its 16-bit rounding
  double x16_scale_next;  // the scale for the next conversion (from the newest ||r||)
  double sums[8]; // scratch results of the last multi-value reduction
  double rr_rec;  // recursive ||r||^2 when the last true residual was taken
  double rr_ref;  // ||f - K x||^2 at the last true residual (reliable-update reference)
  int done;       // 1: converged (recursive test) or broken down; kernels then no-op
  int breakdown;  // 1: <p,Kp> <= 0, rho <= 0 or non-finite
  int iters;      // iterations completed
  int flexible;   // 1: Polak-Ribiere beta, 0: Fletcher-Reeves beta
  // Device-side control of the batched solver (FIN_RR_CTL / FIN_TRUE_CTL):
  int check;         // 1: take the true residual in this iteration
  int replaced;      // 1: r was replaced by the true residual in this iteration
  int status;        // 0 running, 1 converged, 2 iteration limit, 3 breakdown
  int maxit;         // iteration limit
  int replace_every; // residual replacement period (0: only when the recursion converges)
  int replacements;  // true residuals that replaced r
};

// A batch of `nsys` systems of one grid size.  System b keeps its vectors at
// base + b * vs, reads the coefficient fields of realization b / per at
// base + (b / per) * ws, uses the scalars s[b], and its reduction partials
// occupy partial[b * nvals * nparts ...] (value v at + v * nparts).  The
// default is one system.
struct Batch {
  int nsys = 1;
  int per = 1;
  size_t vs = 0;
  size_t ws = 0;
};

// Grow-only device buffer owned by a context.
struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Workspace slots of a context.
enum Slot {
  WS_R = 0, WS_Z, WS_P, WS_Q,   // PCG vectors (double or float)
  WS_X16,                       // preconditioner input in BF16/FP16
  WS_T, WS_U,                   // mode-product intermediates (R N^3 each)
  WS_PART,                      // reduction partials
  WS_SCAL,                      // Scalars
  WS_TMP64,                     // double scratch field (apply entry points)
  WS_TMP64B,
  WS_FLAG,                      // one int (cell validation)
  WS_X32,                       // float accumulator of x increments (mixed)
  WS_COUNT
};

// Reduction modes of the device finalize kernel.
enum FinMode {
  FIN_SUM = 0,      // sums[v] = total of value v
  FIN_ALPHA = 1,    // pq = sum; alpha = rho / pq
  FIN_RR = 2,       // rr = sum; iteration done; convergence test
  FIN_RR_NOCOUNT = 3,
  FIN_PREC = 4,     // sums of <r,z>, <q,z>, sum z, sum r, sum q -> rho, beta, mz
  FIN_PREC_INIT = 5,// same, beta = 0 (restart)
  FIN_FF = 6,       // ff = second total (sum of squares from k_sum2); tol2ff *= ff
  FIN_PREC_FR = 7,  // as FIN_PREC with the Fletcher-Reeves beta (after a residual replacement)
  FIN_RR_CTL = 8,   // as FIN_RR, but a small recursive residual (or a replacement period, or
                    // the iteration limit) only requests a true residual (check = 1)
  FIN_TRUE_CTL = 9  // after the true residual: converge, stop at the limit, or replace r
};

// Which systems a gated kernel works on.
enum Gate {
  GATE_ACTIVE = 0,   // systems not done
  GATE_CHECK = 1,    // systems with check set
  GATE_REPLACED = 2  // systems with replaced set
};

__device__ __forceinline__ bool gate_open(const Scalars& s, int gate) {
  if (s.done) return false;
  return gate == GATE_ACTIVE || (gate == GATE_CHECK ? s.check != 0 : s.replaced != 0);
}

struct TimerRec {
  int id;
  hipEvent_t a, b;
};

}  // namespace kp

struct kp_context {
  int device = 0;
  hipStream_t stream = nullptr;
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* user = nullptr;
  kp::Buffer ws[kp::WS_COUNT];
  kp::Scalars* host_scal = nullptr;  // pinned mirror of the device scalars
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // per-kernel-class timing (kp_context_set_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<kp::TimerRec> pending;
  double t_ms[KP_TIMER_COUNT] = {};
  long long t_count[KP_TIMER_COUNT] = {};
};

namespace kp {

// Records events around the launches made during its lifetime when timing is on.
class ScopedTimer {
 public:
  ScopedTimer(kp_context* ctx, int id);
  ~ScopedTimer();

 private:
  kp_context* ctx_;
  int id_;
  hipEvent_t a_ = nullptr;
};

// Folds completed event pairs into the accumulators (call after a stream sync).
void resolve_timers(kp_context* ctx);

}  // namespace kp

struct kp_coeff {
  kp_context* ctx = nullptr;
  int dim = 3;       // 3, or 2 for the two-dimensional problem
  int L = 0, n0 = 0, N = 0;
  int incl = 0;      // voxels per edge of the centred sub-cell carrying the cell value (n0: whole cell)
  double bg = 0.0;   // coefficient outside the sub-cells (used when incl < n0)
  int precision = KP_FP64;
  double* cells = nullptr;   // L^3 (the stencils read the coefficient from here)
  float* cells32 = nullptr;  // L^3 float copy (mixed only)
  double* w64 = nullptr;     // 3 N^3 assembled edge weights (kp_coeff_fields)
  double* f = nullptr;       // 3 N^3
};

struct kp_precond {
  kp_context* ctx = nullptr;
  int dim = 3;  // 3, or 2: factors of two modes, stages (ii) and (iii) only (no b3)
  int N = 0, R = 0;
  int precision = KP_FP64;
  // Circulant operands of the three NT GEMMs (see precond.hip for the layouts).
  double* a1_64 = nullptr;  // [j1][(k,i1)]     = C1^k[j1][i1]     N x RN
  double* c2_64 = nullptr;  // [k][j2][i2]      = C2^k[j2][i2]     R x N x N
  double* b3_64 = nullptr;  // [(k,j3)][i3]     = C3^k[j3][i3]     RN x N
  // 16-bit operands: every row holds the rounded value followed by the rounded
  // remainder (hi | lo), so each row is twice as long as in double.
  kp::bf16_t* a1_16 = nullptr;  // N x 2RN
  kp::bf16_t* c2_16 = nullptr;  // R x N x 2N
  kp::bf16_t* b3_16 = nullptr;  // RN x 2N
  // The same 16-bit circulants by their first columns, for GEMM kernels that
  // build the circulant operand in LDS: circ16[l] = [k][plane hi/lo][s][N + 8]
  // with row s holding r(s), r(s+1), ..., r(s+N+7) of the reversed first column
  // r(u) = c((-u) mod N) of C_{l+1}^k (indices mod N), so C[j][i..i+7] =
  // r(u0..u0+7), u0 = (i - j) mod N, is the aligned run at (u0 & ~7) of row u0 & 7.
  kp::bf16_t* circ16[3] = {nullptr, nullptr, nullptr};
  kp_precond_info info{};
  int tile[3] = {-1, -1, -1};   // tile configuration per GEMM stage (-1: size heuristic)
  int tile_batch[3] = {-1, -1, -1};  // the same, tuned for batched solves
  int tuned_nsys = 0;                // batch size tile_batch was tuned for (0: not tuned)
  // FFT-diagonalized exact preconditioner (build_preconditioner_fft; R = 0):
  // hipFFT plans of the N^3 real <-> half-spectrum transforms, the symbol
  // g(k) / N^3 on the half spectrum N x N x (N/2+1), and the complex work array.
  int fft = 0;
  void* fft_fwd = nullptr;   // hipfftHandle, D2Z
  void* fft_inv = nullptr;   // hipfftHandle, Z2D
  double* fft_sym = nullptr;
  void* fft_work = nullptr;
};

namespace kp {

// Device memory through the context's allocator.
int dev_alloc(kp_context* ctx, void** ptr, size_t bytes);
void dev_free(kp_context* ctx, void* ptr);
// Grow-only workspace slot.
int ws_get(kp_context* ctx, int slot, size_t bytes, void** ptr);

// Number of blocks used by the grid-stride reduction kernels.
constexpr int kRedBlocks = 1024;
constexpr int kMaxPartials = 65536;
// Number of GEMM tile configurations (double and 16-bit kernels).
constexpr int kTiles64 = 4;
constexpr int kTiles16 = 18;

// Times every tile configuration for a batch of nsys systems on scratch T, U,
// X, Z (NULL: the context workspace, nsys = 1) and stores the fastest in tiles[3].
int autotune_precond(kp_context* ctx, kp_precond* pc, int nsys, int reps, kp_tile_timing* table,
                     int cap, int* count, int* tiles, void* T = nullptr, void* U = nullptr,
                     void* X = nullptr, void* Z = nullptr);

// ---- launchers (each returns a kp_status) ----------------------------------
int launch_assemble(kp_context* ctx, kp_coeff* c);

// How the stencils read a realization's coefficient: L^3 cell values, n0
// voxels per cell edge; a voxel whose local coordinates (v mod n0 on every
// axis) lie in [lo, hi) takes its cell's value, any other voxel the
// background bg (Section 3.1: the centred sub-cell of edge 2 alpha / L;
// lo = 0, hi = n0 for whole cells).
struct CellGeom {
  int L = 0, n0 = 0, lo = 0, hi = 0;
  double bg = 0.0;
  int dim = 3;
  bool sub() const { return lo > 0 || hi < n0; }
};
inline CellGeom geom_of(const kp_coeff* c) {
  CellGeom g;
  g.dim = c->dim;
  g.L = c->L;
  g.n0 = c->n0;
  g.lo = (c->n0 - c->incl) / 2;
  g.hi = g.lo + c->incl;
  g.bg = c->bg;
  return g;
}
// Sets *bad (device int, zeroed by the caller) when a cell is not finite or <= 0.
int launch_validate_cells(kp_context* ctx, const double* cells, size_t n, int* bad);

// Stencil q = K p (or out = f - K p when f is given) on the coefficient given
// by its L^3 cells (n0 grid intervals per cell), block partials of <p,q> (or
// ||out||^2).  s (nullable) gates the systems (gate: enum Gate); bt.ws strides
// the cells of successive realizations.
int launch_stencil_f64(kp_context* ctx, const double* p, const double* cells, const CellGeom& cg,
                       const double* f, double* out, double* partial, int* nparts, const Scalars* s,
                       int N, const Batch& bt = Batch(), int gate = GATE_ACTIVE);
int launch_stencil_f32(kp_context* ctx, const float* p, const float* cells, const CellGeom& cg, float* out,
                       double* partial, int* nparts, const Scalars* s, int N,
                       const Batch& bt = Batch());
int launch_resid_f64_to_f32(kp_context* ctx, const double* x, const double* cells, const CellGeom& cg,
                            const double* f, float* out, double* partial, int* nparts,
                            const Scalars* s, int N, const Batch& bt = Batch(), int gate = GATE_ACTIVE);

// One block per system: totals of nvals values, then the scalar update `mode`.
int launch_finalize(kp_context* ctx, const double* partial, int nparts, int nvals, int mode,
                    Scalars* s, size_t n3, int nsys = 1);

// z = F^-1 (g F r) with the exact symbol (pc->fft), one system.
int launch_precond_fft(kp_context* ctx, const kp_precond* pc, const double* r, double* z);
// Preconditioner: z = sum_k (C1 x C2 x C3) x for x in the precision's input type
// (FP64: or the FFT preconditioner when pc->fft).
// tiles: the tile configuration per stage (NULL: the preconditioner's own).
int launch_precond_f64(kp_context* ctx, const kp_precond* pc, const double* x, double* z,
                       const Scalars* s, const Batch& bt = Batch(), void* T = nullptr,
                       void* U = nullptr, const int* tiles = nullptr);
// x16 holds c * r rounded to 16 bits, with c = s[b].x16_scale when s is given
// (a power of two; 1 without s); the result z is divided by c again.  With
// dots, the last stage also leaves block partials of <r,z>, <q,z>, sum z,
// sum r, sum q (the k_prec_dots values) in dots->part, laid out as a 5-value
// reduction with *dot_parts blocks per system; *dot_parts = 0 when they did
// not fit in dots->cap doubles per system (then nothing was written).
struct PrecDots {
  const float* r;
  const float* q;  // may be NULL
  double* part;
  size_t cap;      // doubles available per system
};
int launch_precond_16(kp_context* ctx, const kp_precond* pc, const bf16_t* x, float* z,
                      const Scalars* s, const Batch& bt = Batch(), void* T = nullptr,
                      void* U = nullptr, const int* tiles = nullptr, const PrecDots* dots = nullptr,
                      int* dot_parts = nullptr);

// Vector kernels (double vectors: T = double; mixed: T = float).  All take a
// batch: vectors at + b * bt.vs, scalars s + b.
int launch_copy_project_f(kp_context* ctx, const double* f, double mean, double* out, size_t n);
// out = f - s[b].sums[0] / n (the mean from a FIN_SUM / FIN_FF reduction).
int launch_project_s(kp_context* ctx, const double* f, double* out, size_t n, const Scalars* s,
                     const Batch& bt);
int launch_sum2(kp_context* ctx, const double* a, size_t n, double* partial, int* nparts,
                const Batch& bt = Batch());
int launch_cast_f64_f32(kp_context* ctx, const double* a, float* b, size_t n);
int launch_cast_f32_f64(kp_context* ctx, const float* a, double* b, size_t n);
int launch_cast_to16(kp_context* ctx, const double* a, bf16_t* b, size_t n, int fp16);
// b = 16-bit(a * s->x16_scale) (scale 1 when s is NULL); gated by s.
int launch_cast32_to16(kp_context* ctx, const float* a, bf16_t* b, size_t n, int fp16,
                       const Scalars* s, const Batch& bt = Batch(), int gate = GATE_ACTIVE);
int launch_fill_f64(kp_context* ctx, double* a, double v, size_t n);

// x += alpha p into the double x, or into the float x32 when given (then
// launch_fold adds x32 into x); r -= alpha q; r16 = 16-bit(r * scale) when given.
template <typename T>
int launch_update_xr(kp_context* ctx, double* x, float* x32, const T* p, T* r, const T* q,
                     bf16_t* r16, int fp16, const Scalars* s, double* partial, int* nparts,
                     size_t n, const Batch& bt = Batch());
// x += x32, x32 = 0 for the gated systems (s NULL: all).
int launch_fold(kp_context* ctx, double* x, float* x32, size_t n, const Scalars* s,
                const Batch& bt = Batch(), int gate = GATE_ACTIVE);
template <typename T>
int launch_prec_dots(kp_context* ctx, const T* z, const T* r, const T* q, const Scalars* s,
                     double* partial, int* nparts, size_t n, const Batch& bt = Batch());
template <typename T>
int launch_update_p(kp_context* ctx, const T* z, T* p, const Scalars* s, size_t n,
                    const Batch& bt = Batch());
// *out = number of systems of s[0..nsys) that are not done.
int launch_count_active(kp_context* ctx, const Scalars* s, int nsys, int* out);
// Per-system partial counts: the most a stencil launch writes at grid size N,
// and what a reducing vector kernel writes per value for n elements.
int stencil_parts_max(int N);
int vector_parts(size_t n);
// a_hom (9 doubles at out, device) of realization c from its three correctors.
int launch_ahom(kp_context* ctx, const kp_coeff* c, const double* const* phi, double* part,
                double* out);
int launch_multidot9(kp_context* ctx, const double* const* phi, const double* f, size_t n,
                     const double* cells, size_t ncells, double* partial, int* nparts, int d = 3);

}  // namespace kp

namespace kp {
// Unknowns of a coefficient / preconditioner: N^dim.
inline size_t unknowns(int N, int dim) { return dim == 2 ? (size_t)N * N : (size_t)N * N * N; }
}  // namespace kp

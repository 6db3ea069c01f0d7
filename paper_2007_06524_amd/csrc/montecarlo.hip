// Monte-Carlo homogenization statistics (Section 5.3): M realizations of the
// random coefficient at one RVE size L, the three corrector solves and the
// homogenized matrix of each (eq. Ahom3_m_entry_comp), then the empirical
// average (eq. A_hom_Empir) and the empirical standard deviation sigma_L^M
// (normalization M - 1) of every entry.
//
// The realizations stream through the batched solver in chunks of B: B
// coefficient objects are assembled once and re-assembled in place from each
// new chunk of cells (kp_coeff_update), B x 3 solution fields are reused, and
// every chunk's matrices land in one device array, reduced by a single block
// in a fixed order at the end (bitwise repeatable for a given M, whatever B).

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "kp_internal.h"

namespace kp {

namespace {

// Entry e (one thread each) of M row-major 3 x 3 matrices: mean, then the
// standard deviation with the M - 1 normalization, both summed in order m = 0..M-1.
__global__ void k_mc_moments(const double* __restrict__ A, int M, double* __restrict__ out) {
  const int e = threadIdx.x;
  if (e >= 9) return;
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += A[(size_t)m * 9 + e];
  const double mean = s / M;
  double v = 0.0;
  for (int m = 0; m < M; ++m) {
    const double d = A[(size_t)m * 9 + e] - mean;
    v += d * d;
  }
  out[e] = mean;
  out[9 + e] = sqrt(v / (M - 1));
}

// Device bytes of one realization in the batched solver (three systems): the
// double x and right-hand side, four PCG vectors, the float increment and
// 16-bit input, and the two GEMM intermediates of R N^3 elements.
size_t bytes_per_realization(size_t n3, int R, bool mixed) {
  const size_t word = mixed ? 4 : 8, inter = mixed ? 2 : 8;
  return 3 * n3 * (2 * 8 + 4 * word + (mixed ? 4 + 2 : 0) + 2 * (size_t)R * inter) + 6 * n3 * 8;
}

}  // namespace

}  // namespace kp

using namespace kp;

extern "C" int kp_mc_homogenize(kp_context* ctx, int L, int n0, int incl, double background, int M,
                                const double* a_cells, const kp_precond* pc, const kp_solve_opts* opts,
                                int batch, double* ahom, double* mean, double* sd, kp_mc_stats* stats) {
  if (!ctx || !a_cells || !pc || !mean || !sd) return fail(KP_ERR_ARG, "kp_mc_homogenize: NULL argument");
  if (M < 2) return fail(KP_ERR_ARG, "kp_mc_homogenize: need M >= 2 realizations (got %d)", M);
  if (pc->ctx != ctx) return fail(KP_ERR_STATE, "kp_mc_homogenize: preconditioner of another context");
  if ((long long)L * n0 != pc->N)
    return fail(KP_ERR_ARG, "kp_mc_homogenize: n0 * L = %lld but the preconditioner has N = %d",
                (long long)L * n0, pc->N);
  const auto t0 = std::chrono::steady_clock::now();
  const size_t nc = (size_t)L * L * L, n3 = (size_t)pc->N * pc->N * pc->N;
  const bool mixed = pc->precision != KP_FP64;
  int B = batch;
  if (B <= 0) {
    const size_t budget = (size_t)32 << 30;
    B = (int)std::max<size_t>(1, budget / bytes_per_realization(n3, pc->R, mixed));
  }
  B = std::min(B, M);

  std::vector<kp_coeff*> co(B, nullptr);
  void* cells_dev = nullptr;
  void* x = nullptr;
  void* A = nullptr;
  void* mom = nullptr;
  int st = KP_OK, worst = KP_OK;
  long long iters = 0;
  double max_rr = 0.0;
  int chunks = 0;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (kp_coeff* c : co)
      if (c) kp_free_coeff(c);
    dev_free(ctx, cells_dev);
    dev_free(ctx, x);
    dev_free(ctx, A);
    dev_free(ctx, mom);
  };
  for (int j = 0; j < B && st >= 0; ++j)
    st = setup_coeff_inclusions(ctx, L, n0, incl, background, a_cells + (size_t)j * nc, pc->precision, &co[j]);
  if (st >= 0) st = dev_alloc(ctx, &cells_dev, (size_t)B * nc * sizeof(double));
  if (st >= 0) st = dev_alloc(ctx, &x, (size_t)3 * B * n3 * sizeof(double));
  if (st >= 0) st = dev_alloc(ctx, &A, (size_t)9 * M * sizeof(double));
  if (st >= 0) st = dev_alloc(ctx, &mom, 18 * sizeof(double));
  if (st < 0) {
    cleanup();
    return st;
  }
  std::vector<double*> xs(3 * (size_t)B);
  for (size_t j = 0; j < xs.size(); ++j) xs[j] = (double*)x + j * n3;
  std::vector<const kp_precond*> pcs(B, pc);
  std::vector<kp_solve_stats> sst(3 * (size_t)B);
  std::vector<double> ah(9 * (size_t)B);
  for (int m0 = 0; m0 < M; m0 += B) {
    const int nb = std::min(B, M - m0);
    if (m0 > 0) {  // re-assemble the coefficient objects from the next realizations
      hipError_t e = hipMemcpyAsync(cells_dev, a_cells + (size_t)m0 * nc, (size_t)nb * nc * sizeof(double),
                                    hipMemcpyHostToDevice, ctx->stream);
      if (e != hipSuccess) {
        cleanup();
        return fail(KP_ERR_HIP, "kp_mc_homogenize: cell upload: %s", hipGetErrorString(e));
      }
      for (int j = 0; j < nb && st >= 0; ++j) st = kp_coeff_update(ctx, co[j], (const double*)cells_dev + (size_t)j * nc);
      if (st < 0) {
        cleanup();
        return st;
      }
    }
    st = pcg_solve_batched(ctx, nb, co.data(), pcs.data(), xs.data(), opts, sst.data(), ah.data());
    if (st < 0 && st != KP_ERR_BREAKDOWN) {
      cleanup();
      return st;
    }
    if (st == KP_ERR_BREAKDOWN || (st == KP_NOT_CONVERGED && worst == KP_OK)) worst = st;
    for (int j = 0; j < 3 * nb; ++j) {
      iters += sst[j].iters;
      max_rr = std::max(max_rr, sst[j].relres_true);
    }
    hipError_t e = hipMemcpyAsync((double*)A + (size_t)9 * m0, ah.data(), (size_t)9 * nb * sizeof(double),
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);  // ah is reused by the next chunk
    if (e != hipSuccess) {
      cleanup();
      return fail(KP_ERR_HIP, "kp_mc_homogenize: %s", hipGetErrorString(e));
    }
    if (ahom) std::copy(ah.begin(), ah.begin() + 9 * (size_t)nb, ahom + (size_t)9 * m0);
    ++chunks;
  }
  hipLaunchKernelGGL(k_mc_moments, dim3(1), dim3(64), 0, ctx->stream, (const double*)A, M, (double*)mom);
  double hm[18];
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hm, mom, sizeof(hm), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e != hipSuccess) return fail(KP_ERR_HIP, "kp_mc_homogenize: %s", hipGetErrorString(e));
  std::copy(hm, hm + 9, mean);
  std::copy(hm + 9, hm + 18, sd);
  if (stats) {
    stats->realizations = M;
    stats->batch = B;
    stats->chunks = chunks;
    stats->status = worst;
    stats->iters = iters;
    stats->max_relres_true = max_rr;
    stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return worst;
}

// The paper's first approach to the preconditioner (Section 4.2): the
// pseudo-inverse of the periodic Laplacian, diagonal in the Fourier basis,
// applied exactly as z = F^-1 (g F r) with the symbol
//   g(k) = 1 / (mu(k1) + mu(k2) + mu(k3)),  mu(k) = 4 sin^2(pi k / N),
// and g(0) = 0 (eq. 3a; the constant prefactor of the paper's preconditioner
// is dropped, PCG being invariant under positive scaling).  The real input
// goes through a double-precision real-to-half-spectrum 3D FFT (hipFFT), the
// half spectrum is scaled by g / N^3 in one kernel, and the inverse transform
// writes z.  A comparison point for the low-rank mode products: FP64, one
// system at a time.

#include <cmath>

#include <hipfft/hipfft.h>

#include "kp_internal.h"

namespace kp {

namespace {

// Symbol g(k) / N^3 on the half spectrum [k1][k2][k3], k3 <= N/2.
__global__ __launch_bounds__(256) void k_fft_symbol(int N, double* __restrict__ g) {
  const int H = N / 2 + 1;
  const size_t n = (size_t)N * N * H;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int k3 = (int)(i % H), k2 = (int)((i / H) % N), k1 = (int)(i / ((size_t)N * H));
  const double pn = M_PI / N;
  const double s1 = sin(pn * k1), s2 = sin(pn * k2), s3 = sin(pn * k3);
  const double mu = 4.0 * (s1 * s1 + s2 * s2 + s3 * s3);
  const double n3 = (double)N * N * N;
  g[i] = (k1 == 0 && k2 == 0 && k3 == 0) ? 0.0 : 1.0 / (mu * n3);
}

__global__ __launch_bounds__(256) void k_fft_scale(double2* __restrict__ w, const double* __restrict__ g,
                                                   size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double s = g[i];
    double2 v = w[i];
    v.x *= s;
    v.y *= s;
    w[i] = v;
  }
}

int fft_check(hipfftResult r, const char* what) {
  if (r != HIPFFT_SUCCESS) return fail(KP_ERR_HIP, "hipFFT %s failed (%d)", what, (int)r);
  return KP_OK;
}

}  // namespace

int launch_precond_fft(kp_context* ctx, const kp_precond* pc, const double* r, double* z) {
  const int N = pc->N, H = N / 2 + 1;
  const size_t nh = (size_t)N * N * H;
  hipfftHandle fwd = (hipfftHandle)pc->fft_fwd, inv = (hipfftHandle)pc->fft_inv;
  KP_TRY(fft_check(hipfftSetStream(fwd, ctx->stream), "set stream"));
  KP_TRY(fft_check(hipfftSetStream(inv, ctx->stream), "set stream"));
  hipfftDoubleComplex* w = (hipfftDoubleComplex*)pc->fft_work;
  KP_TRY(fft_check(hipfftExecD2Z(fwd, (hipfftDoubleReal*)const_cast<double*>(r), w), "forward transform"));
  const int blocks = (int)std::min<size_t>((nh + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fft_scale, dim3(blocks), dim3(256), 0, ctx->stream, (double2*)w,
                     (const double*)pc->fft_sym, nh);
  KP_HIP(hipGetLastError());
  return fft_check(hipfftExecZ2D(inv, w, (hipfftDoubleReal*)z), "inverse transform");
}

}  // namespace kp

using namespace kp;

extern "C" int build_preconditioner_fft(kp_context* ctx, int N, kp_precond** out) {
  if (!ctx || !out) return fail(KP_ERR_ARG, "build_preconditioner_fft: NULL argument");
  *out = nullptr;
  if (N < 2 || N > 2048) return fail(KP_ERR_ARG, "build_preconditioner_fft: need 2 <= N <= 2048");
  KP_HIP(hipSetDevice(ctx->device));
  kp_precond* pc = new kp_precond();
  pc->ctx = ctx;
  pc->N = N;
  pc->R = 0;
  pc->precision = KP_FP64;
  pc->fft = 1;
  pc->info.rank = 0;
  pc->info.rho_min = pc->info.rho_max = 1.0;
  const int H = N / 2 + 1;
  const size_t nh = (size_t)N * N * H;
  hipfftHandle fwd = nullptr, inv = nullptr;
  int st = KP_OK;
  if ((st = fft_check(hipfftPlan3d(&fwd, N, N, N, HIPFFT_D2Z), "plan")) >= 0) pc->fft_fwd = fwd;
  if (st >= 0 && (st = fft_check(hipfftPlan3d(&inv, N, N, N, HIPFFT_Z2D), "plan")) >= 0) pc->fft_inv = inv;
  if (st >= 0) st = dev_alloc(ctx, (void**)&pc->fft_sym, nh * sizeof(double));
  if (st >= 0) st = dev_alloc(ctx, &pc->fft_work, nh * 2 * sizeof(double));
  if (st >= 0) {
    hipLaunchKernelGGL(k_fft_symbol, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, ctx->stream, N,
                       pc->fft_sym);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = fail(KP_ERR_HIP, "build_preconditioner_fft: %s", hipGetErrorString(e));
  }
  if (st < 0) {
    kp_free_precond(pc);
    return st;
  }
  *out = pc;
  return KP_OK;
}

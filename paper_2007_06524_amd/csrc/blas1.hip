// Vector updates and reductions of the PCG iteration.
//
// Every reduction is deterministic: each block accumulates a fixed grid-stride
// subset in double, reduces it with 64-lane wavefront shuffles and LDS, and
// writes one partial; a one-block finalize kernel adds the partials in a fixed
// order and updates the PCG scalars on the device, so the iteration never
// waits for the host.

#include <cmath>

#include "kp_internal.h"

namespace kp {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of NV values over a 256-thread block, written to out[v * stride].
template <int NV>
__device__ __forceinline__ void block_sums_store(double (&v)[NV], double* out, size_t stride) {
  __shared__ double red[NV][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    out[k * stride] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

__device__ __forceinline__ bf16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

__device__ __forceinline__ bf16_t f32_to_f16_rne(float x) {
  _Float16 hv = (_Float16)x;  // IEEE round to nearest even
  return __builtin_bit_cast(bf16_t, hv);
}

__device__ __forceinline__ bf16_t to16(float x, int fp16) {
  return fp16 ? f32_to_f16_rne(x) : f32_to_bf16_rne(x);
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Power of two bringing the RMS of r near 1 before 16-bit rounding (keeps FP16
// inputs normal as the residual shrinks; exact to undo).
__device__ double x16_scale_for(double rr, double n3) {
  double sc = 1.0;
  if (rr > 0.0 && finite(rr)) {
    double e = rint(-0.5 * log2(rr / n3));
    e = fmin(fmax(e, -120.0), 120.0);
    sc = exp2(e);
  }
  return sc;
}

// Reliable updates in mixed precision: once the recursive ||r|| has fallen by
// 1e4 below the last true residual, the float recursion is near the end of
// its accuracy (float unit roundoff 6e-8 times the larger residual it carries
// errors from), so the residual is replaced by f - K x in double.  With the
// fixed replacement period this only fires for fast convergence.
constexpr double kReliableDrop = 1e-8;  // on ||r||^2

__device__ void stop(Scalars* s, int status) {
  s->done = 1;
  s->status = status;
  if (status == 3) s->breakdown = 1;
}

// One block of 256 threads per system: totals of nvals values, then the PCG
// scalar logic of `mode` for that system.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partial, int nparts,
                                                  int nvals, int mode, Scalars* s, double n3) {
  const int b = blockIdx.x;
  s += b;
  partial += (size_t)b * nvals * nparts;
  if (s->done && mode != FIN_SUM && mode != FIN_FF) return;
  if (mode == FIN_TRUE_CTL && !s->check) return;
  __shared__ double tot[8];
  for (int v = 0; v < nvals; ++v) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += partial[(size_t)v * nparts + i];
    __shared__ double red[4];
    acc = wave_sum(acc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) tot[v] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int v = 0; v < nvals; ++v) s->sums[v] = tot[v];
  switch (mode) {
    case FIN_SUM:
      break;
    case FIN_FF: {  // partials of k_sum2: (sum, sum of squares)
      const double ff = tot[1];
      s->ff = ff;
      s->tol2ff *= ff;  // tol^2 -> tol^2 ||f||^2 (the single solver writes it afterwards)
      if (!(ff > 0.0)) stop(s, 1);  // zero right-hand side: x = 0
      break;
    }
    case FIN_ALPHA: {
      const double pq = tot[0];
      s->pq = pq;
      s->x16_scale = s->x16_scale_next;  // r of this iteration is rounded with this scale
      if (!(pq > 0.0) || !finite(pq)) {
        stop(s, 3);
        s->alpha = 0.0;
      } else {
        s->alpha = s->rho / pq;
      }
      break;
    }
    case FIN_RR:
    case FIN_RR_NOCOUNT: {
      const double rr = tot[0];
      s->rr = rr;
      if (mode == FIN_RR) s->iters += 1;
      const double sc = x16_scale_for(rr, n3);
      s->x16_scale_next = sc;
      if (mode == FIN_RR_NOCOUNT) {
        s->x16_scale = sc;  // followed by a fresh conversion
        s->rr_ref = rr;     // a true residual
      }
      if (!finite(rr)) {
        stop(s, 3);
      } else if (rr <= s->tol2ff) {
        s->done = 1;
        if (mode == FIN_RR_NOCOUNT) s->status = 1;  // a true residual: converged
      } else if (mode == FIN_RR && s->flexible && rr <= kReliableDrop * s->rr_ref) {
        s->done = 1;  // the single solver's host loop takes the true residual and restarts
      }
      break;
    }
    case FIN_RR_CTL: {
      const double rr = tot[0];
      s->rr = rr;
      s->iters += 1;
      s->x16_scale_next = x16_scale_for(rr, n3);
      if (!finite(rr)) {
        stop(s, 3);
        break;
      }
      s->check = rr <= s->tol2ff || s->iters >= s->maxit ||
                 (s->replace_every > 0 && s->iters % s->replace_every == 0) ||
                 (s->flexible && rr <= kReliableDrop * s->rr_ref);
      if (s->check) s->rr_rec = rr;
      break;
    }
    case FIN_TRUE_CTL: {
      // r now holds f - K x in the iterate's precision; tot[0] = ||f - K x||^2 (double).
      const double rr = tot[0];
      s->check = 0;
      if (!finite(rr)) {
        stop(s, 3);
        break;
      }
      s->rr = rr;
      s->rr_ref = rr;
      if (rr <= s->tol2ff) {
        stop(s, 1);
      } else if (s->iters >= s->maxit) {
        stop(s, 2);
      } else {
        s->replaced = 1;
        s->replacements += 1;
        const double sc = x16_scale_for(rr, n3);
        s->x16_scale = sc;
        s->x16_scale_next = sc;
      }
      break;
    }
    case FIN_PREC:
    case FIN_PREC_FR:
    case FIN_PREC_INIT: {
      // tot: <r,z>, <q,z>, sum z, sum r, sum q
      const double mz = tot[2] / n3;
      const double rho_new = tot[0] - mz * tot[3];
      const bool fr = mode == FIN_PREC_FR || s->replaced;
      s->replaced = 0;
      s->mz = mz;
      if (!(rho_new > 0.0) || !finite(rho_new)) {
        stop(s, 3);
        break;
      }
      if (mode == FIN_PREC_INIT) {
        s->beta = 0.0;
      } else if (s->flexible && !fr) {
        // <z - mz, r_new - r_old> = -alpha <z - mz, q>
        s->beta = -s->alpha * (tot[1] - mz * tot[4]) / s->rho;
      } else {
        s->beta = rho_new / s->rho;
      }
      s->rho = rho_new;
      break;
    }
  }
}

// Four consecutive elements per thread and step, moved as one 16-byte (float)
// or two 16-byte (double) accesses; the n % 4 tail is handled element-wise.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float4 type;
};
template <>
struct Vec4<double> {
  typedef double4 type;
};

template <typename T>
__device__ __forceinline__ void ld4(const T* __restrict__ p, size_t i, T (&v)[4]) {
  const typename Vec4<T>::type t = *(const typename Vec4<T>::type*)(p + i);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}

template <typename T>
__device__ __forceinline__ void st4(T* __restrict__ p, size_t i, const T (&v)[4]) {
  typename Vec4<T>::type t;
  t.x = v[0];
  t.y = v[1];
  t.z = v[2];
  t.w = v[3];
  *(typename Vec4<T>::type*)(p + i) = t;
}

// Vector kernels: blockIdx.y is the system of the batch (Batch layout).
// x += alpha p goes to the double x or, with X32, to a float accumulator that
// k_fold adds into the double x before every true residual (reliable
// updates: the float part only ever holds the increments since the last one).
template <typename T, bool X32>
__global__ __launch_bounds__(256) void k_update_xr(double* __restrict__ x, float* __restrict__ x32,
                                                   const T* __restrict__ p, T* __restrict__ r,
                                                   const T* __restrict__ q, bf16_t* __restrict__ r16,
                                                   int fp16, const Scalars* __restrict__ s,
                                                   double* __restrict__ partial, size_t n, size_t vs) {
  const int b = blockIdx.y;
  s += b;
  if (s->done) return;
  const size_t off = b * vs;
  if (X32)
    x32 += off;
  else
    x += off;
  p += off;
  r += off;
  q += off;
  if (r16) r16 += off;
  const double alpha = s->alpha;
  const T ta = (T)alpha;
  const float fa = (float)alpha;
  const float sc = (float)s->x16_scale;
  double acc[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * 256, n4 = n / 4;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n4; c += stride) {
    const size_t i = 4 * c;
    T pv[4], rv[4], qv[4];
    ld4(p, i, pv);
    ld4(r, i, rv);
    ld4(q, i, qv);
    if constexpr (X32) {
      float xv[4];
      ld4(x32, i, xv);
#pragma unroll
      for (int e = 0; e < 4; ++e) xv[e] += fa * (float)pv[e];
      st4(x32, i, xv);
    } else {
      double xv[4];
      ld4(x, i, xv);
#pragma unroll
      for (int e = 0; e < 4; ++e) xv[e] += alpha * (double)pv[e];
      st4(x, i, xv);
    }
    ushort4 h;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      rv[e] = rv[e] - ta * qv[e];
      acc[0] += (double)rv[e] * (double)rv[e];
    }
    st4(r, i, rv);
    if (r16) {
      h.x = to16((float)rv[0] * sc, fp16);
      h.y = to16((float)rv[1] * sc, fp16);
      h.z = to16((float)rv[2] * sc, fp16);
      h.w = to16((float)rv[3] * sc, fp16);
      *(ushort4*)(r16 + i) = h;
    }
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const T pi = p[i];
    if constexpr (X32)
      x32[i] += fa * (float)pi;
    else
      x[i] += alpha * (double)pi;
    const T rn = r[i] - ta * q[i];
    r[i] = rn;
    if (r16) r16[i] = to16((float)rn * sc, fp16);
    acc[0] += (double)rn * (double)rn;
  }
  block_sums_store<1>(acc, partial + (size_t)b * gridDim.x + blockIdx.x, gridDim.x);
}

// <r,z>, <q,z>, sum z, sum r, sum q (q may be null on the first application).
template <typename T>
__global__ __launch_bounds__(256) void k_prec_dots(const T* __restrict__ z, const T* __restrict__ r,
                                                   const T* __restrict__ q,
                                                   const Scalars* __restrict__ s,
                                                   double* __restrict__ partial, size_t n,
                                                   size_t vs) {
  const int b = blockIdx.y;
  if (s[b].done) return;
  const size_t off = b * vs;
  z += off;
  r += off;
  if (q) q += off;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t stride = (size_t)gridDim.x * 256, n4 = n / 4;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n4; c += stride) {
    const size_t i = 4 * c;
    T zv[4], rv[4], qv[4] = {0, 0, 0, 0};
    ld4(z, i, zv);
    ld4(r, i, rv);
    if (q) ld4(q, i, qv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double zi = (double)zv[e], ri = (double)rv[e], qi = (double)qv[e];
      acc[0] += ri * zi;
      acc[1] += qi * zi;
      acc[2] += zi;
      acc[3] += ri;
      acc[4] += qi;
    }
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double zi = (double)z[i], ri = (double)r[i], qi = q ? (double)q[i] : 0.0;
    acc[0] += ri * zi;
    acc[1] += qi * zi;
    acc[2] += zi;
    acc[3] += ri;
    acc[4] += qi;
  }
  block_sums_store<5>(acc, partial + (size_t)b * 5 * gridDim.x + blockIdx.x, gridDim.x);
}

// p = (z - mean(z)) + beta p  (beta = 0: restart, p may hold stale or uninitialized values)
template <typename T>
__global__ __launch_bounds__(256) void k_update_p(const T* __restrict__ z, T* __restrict__ p,
                                                  const Scalars* __restrict__ s, size_t n,
                                                  size_t vs) {
  const int b = blockIdx.y;
  s += b;
  if (s->done) return;
  z += b * vs;
  p += b * vs;
  const T beta = (T)s->beta;
  const T mz = (T)s->mz;
  const bool restart = s->beta == 0.0;
  const size_t stride = (size_t)gridDim.x * 256, n4 = n / 4;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n4; c += stride) {
    const size_t i = 4 * c;
    T zv[4], pv[4] = {0, 0, 0, 0};
    ld4(z, i, zv);
    if (!restart) ld4(p, i, pv);
#pragma unroll
    for (int e = 0; e < 4; ++e) pv[e] = restart ? zv[e] - mz : (zv[e] - mz) + beta * pv[e];
    st4(p, i, pv);
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    p[i] = restart ? z[i] - mz : (z[i] - mz) + beta * p[i];
}

__global__ __launch_bounds__(256) void k_sum2(const double* __restrict__ a, size_t n,
                                              double* __restrict__ partial, size_t vs) {
  const int b = blockIdx.y;
  a += b * vs;
  double acc[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double v = a[i];
    acc[0] += v;
    acc[1] += v * v;
  }
  block_sums_store<2>(acc, partial + (size_t)b * 2 * gridDim.x + blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_copy_project(const double* __restrict__ f, double mean,
                                                      double* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    out[i] = f[i] - mean;
}

__global__ __launch_bounds__(256) void k_project_s(const double* __restrict__ f,
                                                   double* __restrict__ out, size_t n,
                                                   const Scalars* __restrict__ s, size_t vs) {
  const int b = blockIdx.y;
  const double mean = s[b].sums[0] / (double)n;
  f += b * vs;
  out += b * vs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    out[i] = f[i] - mean;
}

__global__ __launch_bounds__(256) void k_cast_f64_f32(const double* __restrict__ a,
                                                      float* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    b[i] = (float)a[i];
}

__global__ __launch_bounds__(256) void k_cast_f32_f64(const float* __restrict__ a,
                                                      double* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    b[i] = (double)a[i];
}

__global__ __launch_bounds__(256) void k_cast_to16(const double* __restrict__ a,
                                                   bf16_t* __restrict__ b, size_t n, int fp16) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    b[i] = to16((float)a[i], fp16);
}

__global__ __launch_bounds__(256) void k_cast32_to16(const float* __restrict__ a,
                                                     bf16_t* __restrict__ b, size_t n, int fp16,
                                                     const Scalars* __restrict__ s, int gate,
                                                     size_t vs) {
  const int bi = blockIdx.y;
  if (s && !gate_open(s[bi], gate)) return;
  const float sc = s ? (float)s[bi].x16_scale : 1.0f;
  a += bi * vs;
  b += bi * vs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    b[i] = to16(a[i] * sc, fp16);
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ a, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    a[i] = v;
}

// x += x32, x32 = 0 (gated systems).
__global__ __launch_bounds__(256) void k_fold(double* __restrict__ x, float* __restrict__ x32, size_t n,
                                              const Scalars* __restrict__ s, int gate, size_t vs) {
  const int b = blockIdx.y;
  if (s && !gate_open(s[b], gate)) return;
  x += b * vs;
  x32 += b * vs;
  const size_t stride = (size_t)gridDim.x * 256, n4 = n / 4;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n4; c += stride) {
    const size_t i = 4 * c;
    double xv[4];
    float av[4];
    ld4(x, i, xv);
    ld4(x32, i, av);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xv[e] += (double)av[e];
      av[e] = 0.0f;
    }
    st4(x, i, xv);
    st4(x32, i, av);
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    x[i] += (double)x32[i];
    x32[i] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_count_active(const Scalars* __restrict__ s, int nsys,
                                                      int* __restrict__ out) {
  int c = 0;
  for (int i = threadIdx.x; i < nsys; i += 256) c += s[i].done ? 0 : 1;
  __shared__ int red[256];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Nine dot products <phi_i, f_j> and the sum of the cell values.
struct PhiPtrs {
  const double* p[3];
};

// <phi_a, f_b> for a, b < D (value 3 a + b; the others stay 0) and the cell sum (value 9).
template <int D>
__global__ __launch_bounds__(256) void k_multidot9(PhiPtrs phi, const double* __restrict__ f,
                                                   size_t n, const double* __restrict__ cells,
                                                   size_t ncells, double* __restrict__ partial) {
  double acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    double fb[D];
#pragma unroll
    for (int b = 0; b < D; ++b) fb[b] = f[b * n + i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double v = phi.p[a][i];
#pragma unroll
      for (int b = 0; b < D; ++b) acc[3 * a + b] += v * fb[b];
    }
  }
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < ncells; i += (size_t)gridDim.x * 256)
    acc[9] += cells[i];
  block_sums_store<10>(acc, partial + blockIdx.x, gridDim.x);
}

int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

// Blocks per system of the reducing vector kernels: about four 4-element
// steps per thread, at most kRedBlocks.
int red_blocks(size_t n) {
  size_t b = (n + 4095) / 4096;
  if (b > (size_t)kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int launch_finalize(kp_context* ctx, const double* partial, int nparts, int nvals, int mode,
                    Scalars* s, size_t n3, int nsys) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_finalize, dim3(nsys), dim3(256), 0, ctx->stream, partial, nparts, nvals, mode,
                     s, (double)n3);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

template <typename T>
int launch_update_xr(kp_context* ctx, double* x, float* x32, const T* p, T* r, const T* q,
                     bf16_t* r16, int fp16, const Scalars* s, double* partial, int* nparts,
                     size_t n, const Batch& bt) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  const int g = red_blocks(n);
  if (x32)
    hipLaunchKernelGGL((k_update_xr<T, true>), dim3(g, bt.nsys), dim3(256), 0, ctx->stream, x, x32, p, r, q,
                       r16, fp16, s, partial, n, bt.vs);
  else
    hipLaunchKernelGGL((k_update_xr<T, false>), dim3(g, bt.nsys), dim3(256), 0, ctx->stream, x, x32, p, r,
                       q, r16, fp16, s, partial, n, bt.vs);
  KP_HIP(hipGetLastError());
  *nparts = g;
  return KP_OK;
}

int launch_fold(kp_context* ctx, double* x, float* x32, size_t n, const Scalars* s, const Batch& bt,
                int gate) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_fold, dim3(red_blocks(n), bt.nsys), dim3(256), 0, ctx->stream, x, x32, n, s, gate,
                     bt.vs);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

template <typename T>
int launch_prec_dots(kp_context* ctx, const T* z, const T* r, const T* q, const Scalars* s,
                     double* partial, int* nparts, size_t n, const Batch& bt) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  const int g = red_blocks(n);
  hipLaunchKernelGGL(k_prec_dots<T>, dim3(g, bt.nsys), dim3(256), 0, ctx->stream, z, r, q, s, partial,
                     n, bt.vs);
  KP_HIP(hipGetLastError());
  *nparts = g;
  return KP_OK;
}

template <typename T>
int launch_update_p(kp_context* ctx, const T* z, T* p, const Scalars* s, size_t n,
                    const Batch& bt) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_update_p<T>, dim3(red_blocks(n), bt.nsys), dim3(256), 0, ctx->stream, z, p, s,
                     n, bt.vs);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

template int launch_update_xr<double>(kp_context*, double*, float*, const double*, double*,
                                      const double*, bf16_t*, int, const Scalars*, double*, int*,
                                      size_t, const Batch&);
template int launch_update_xr<float>(kp_context*, double*, float*, const float*, float*, const float*,
                                     bf16_t*, int, const Scalars*, double*, int*, size_t,
                                     const Batch&);
template int launch_prec_dots<double>(kp_context*, const double*, const double*, const double*,
                                      const Scalars*, double*, int*, size_t, const Batch&);
template int launch_prec_dots<float>(kp_context*, const float*, const float*, const float*,
                                     const Scalars*, double*, int*, size_t, const Batch&);
template int launch_update_p<double>(kp_context*, const double*, double*, const Scalars*, size_t,
                                     const Batch&);
template int launch_update_p<float>(kp_context*, const float*, float*, const Scalars*, size_t,
                                    const Batch&);

int launch_sum2(kp_context* ctx, const double* a, size_t n, double* partial, int* nparts,
                const Batch& bt) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  const int g = red_blocks(n);
  hipLaunchKernelGGL(k_sum2, dim3(g, bt.nsys), dim3(256), 0, ctx->stream, a, n, partial, bt.vs);
  KP_HIP(hipGetLastError());
  *nparts = g;
  return KP_OK;
}

int launch_copy_project_f(kp_context* ctx, const double* f, double mean, double* out, size_t n) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_copy_project, dim3(grid_for(n)), dim3(256), 0, ctx->stream, f, mean, out, n);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_project_s(kp_context* ctx, const double* f, double* out, size_t n, const Scalars* s,
                     const Batch& bt) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_project_s, dim3(red_blocks(n), bt.nsys), dim3(256), 0, ctx->stream, f, out, n,
                     s, bt.vs);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_cast_f64_f32(kp_context* ctx, const double* a, float* b, size_t n) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_cast_f64_f32, dim3(grid_for(n)), dim3(256), 0, ctx->stream, a, b, n);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_cast_f32_f64(kp_context* ctx, const float* a, double* b, size_t n) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_cast_f32_f64, dim3(grid_for(n)), dim3(256), 0, ctx->stream, a, b, n);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_cast_to16(kp_context* ctx, const double* a, bf16_t* b, size_t n, int fp16) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_cast_to16, dim3(grid_for(n)), dim3(256), 0, ctx->stream, a, b, n, fp16);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_cast32_to16(kp_context* ctx, const float* a, bf16_t* b, size_t n, int fp16,
                       const Scalars* s, const Batch& bt, int gate) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_cast32_to16, dim3(red_blocks(n), bt.nsys), dim3(256), 0, ctx->stream, a, b, n,
                     fp16, s, gate, bt.vs);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_fill_f64(kp_context* ctx, double* a, double v, size_t n) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, ctx->stream, a, v, n);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int vector_parts(size_t n) { return red_blocks(n); }

int launch_count_active(kp_context* ctx, const Scalars* s, int nsys, int* out) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, ctx->stream, s, nsys, out);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_multidot9(kp_context* ctx, const double* const* phi, const double* f, size_t n,
                     const double* cells, size_t ncells, double* partial, int* nparts, int d) {
  ScopedTimer tm(ctx, KP_TIMER_VECTOR);
  PhiPtrs pp;
  for (int a = 0; a < 3; ++a) pp.p[a] = a < d ? phi[a] : nullptr;
  const int g = kRedBlocks;
  if (d == 2)
    hipLaunchKernelGGL(k_multidot9<2>, dim3(g), dim3(256), 0, ctx->stream, pp, f, n, cells, ncells, partial);
  else
    hipLaunchKernelGGL(k_multidot9<3>, dim3(g), dim3(256), 0, ctx->stream, pp, f, n, cells, ncells, partial);
  KP_HIP(hipGetLastError());
  *nparts = g;
  return KP_OK;
}

}  // namespace kp

// Low-Kronecker-rank preconditioner: z = sum_k (C1^k x C2^k x C3^k) x
// (eq. Lap3DtimesX with the circulants C_l^k = F* diag(u_l^k) F held as dense
// real symmetric N x N matrices), evaluated as three MFMA GEMMs:
//
//   (i)   T[k][j3][i1][i2]   = sum_i3  X[i1][i2][i3]  C3^k[j3][i3]
//   (ii)  U[(j2,j3)][(k,i1)] = sum_i2  C2^k[j2][i2]   T[k][j3][i1][i2]
//   (iii) Z[j1][(j2,j3)]     = sum_(k,i1) C1^k[j1][i1] U[(j2,j3)][(k,i1)]
//
// Every stage is an "NT" product D = A * Bt^T with both operands contiguous in
// the contraction index, so each MFMA fragment is one contiguous LDS read.
// Stage (iii) contracts over R*N at once, which folds the sum over the R
// Kronecker terms into the GEMM.  The layouts of T and U are chosen by the
// output address maps of stages (i) and (ii) so that they are the contiguous
// operands of the next stage.
//
// FP64: v_mfma_f64_16x16x4_f64.  BF16 / FP16: v_mfma_f32_16x16x32_{bf16,f16}
// with float accumulation; intermediates are rounded to the 16-bit type.  In
// 16 bits every circulant is held as a rounded part plus the rounded remainder
// and both are contracted (the K extent doubles): the symbol of G_R spans about
// N^2 / (4 pi^2) * 12 in magnitude across frequencies, more than one 16-bit
// rounding of the dense circulant entries can resolve.

#include <climits>

#include "kp_internal.h"

namespace kp {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Output address of element (m, n) of batch b:
//   m*sm + (n / nd)*sn1 + (n % nd)*sn2 + b*sb
struct OutMap {
  long long sm, sn1, sn2, sb;
  int nd;
};

struct GemmArgs {
  const void* A;   // M x K, row stride lda
  const void* B;   // Nn x K, row stride ldb  (the transposed right operand)
  void* C;
  int M, Nn, K;
  long long lda, ldb, sAb, sBb;
  OutMap om;
  const int* done;
  int vec;         // 1: 16-byte operand loads are legal (alignment and K)
  int krep_a;      // > 0: A is stored with krep_a columns and read at column k mod krep_a
  int krep_b;      // same for B
  const double* out_div;  // non-null: results are divided by *out_div
};

GemmArgs gemm_args(const void* A, const void* B, void* C, long long M, long long Nn, long long K,
                   long long lda, long long ldb, long long sAb, long long sBb, OutMap om,
                   const int* done, int krep_a = 0, int krep_b = 0,
                   const double* out_div = nullptr) {
  return GemmArgs{A, B, C, (int)M, (int)Nn, (int)K, lda, ldb, sAb, sBb, om, done, 0, krep_a, krep_b,
                  out_div};
}

__device__ __forceinline__ long long out_addr(const OutMap& o, int m, int n, int b) {
  return (long long)m * o.sm + (long long)(n / o.nd) * o.sn1 + (long long)(n % o.nd) * o.sn2 +
         (long long)b * o.sb;
}

__device__ __forceinline__ bf16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

template <typename TO, bool F16>
__device__ __forceinline__ TO cvt_out(float v) {
  if constexpr (sizeof(TO) == 4) {
    return v;
  } else if constexpr (F16) {
    _Float16 h = (_Float16)v;
    return __builtin_bit_cast(bf16_t, h);
  } else {
    return f32_to_bf16_rne(v);
  }
}

// ---------------------------------------------------------------- FP64 MFMA
// 256 threads = 2 x 2 wavefronts, block tile BM x BN, K tile 16, wave tile
// (BM/2) x (BN/2) made of 16 x 16 MFMA tiles.  Global loads for the next K
// tile are issued before the MFMAs of the current one.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  if (g.done && *g.done) return;
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ double As[BM][BK + 1];
  __shared__ double Bs[BN][BK + 1];
  const int bz = blockIdx.z;
  const double* __restrict__ A = (const double*)g.A + (long long)bz * g.sAb;
  const double* __restrict__ B = (const double*)g.B + (long long)bz * g.sBb;
  double* __restrict__ C = (double*)g.C;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  dbl4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  double ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int e = tid + 256 * t, r = e / BK, c = e % BK;
      const int gm = m0 + r, gk = k0 + c;
      ra[t] = (gm < g.M && gk < g.K) ? A[(long long)gm * g.lda + gk] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int e = tid + 256 * t, r = e / BK, c = e % BK;
      const int gn = n0 + r, gk = k0 + c;
      rb[t] = (gn < g.Nn && gk < g.K) ? B[(long long)gn * g.ldb + gk] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int t = 0; t < LA; ++t) {
      const int e = tid + 256 * t;
      As[e / BK][e % BK] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int e = tid + 256 * t;
      Bs[e / BK][e % BK] = rb[t];
    }
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[wm * WM + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = Bs[wn * WN + j * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      // v_mfma_f64_16x16x4_f64 result: item v of lane l is row 4v + l/16, column l%16.
      const int n = n0 + wn * WN + j * 16 + (lane & 15);
      if (n >= g.Nn) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * WM + i * 16 + 4 * v + (lane >> 4);
        if (m < g.M) C[out_addr(g.om, m, n, bz)] = acc[i][j][v];
      }
    }
}

// ---------------------------------------------------- BF16 / FP16 MFMA
// Same structure with K tile 64 (two 16x16x32 MFMA steps); operands are moved
// as 16-byte vectors of eight 16-bit values; rows are padded by 16 bytes.
template <int BM, int BN, bool F16, typename TO>
__global__ __launch_bounds__(256) void k_gemm_16(GemmArgs g) {
  if (g.done && *g.done) return;
  constexpr int BK = 64;
  constexpr int PAD = 8;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int VA = BM * BK / 8 / 256, VB = BN * BK / 8 / 256;  // 16-byte vectors per thread
  __shared__ __attribute__((aligned(16))) bf16_t As[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) bf16_t Bs[BN][BK + PAD];
  const int bz = blockIdx.z;
  const bf16_t* __restrict__ A = (const bf16_t*)g.A + (long long)bz * g.sAb;
  const bf16_t* __restrict__ B = (const bf16_t*)g.B + (long long)bz * g.sBb;
  TO* __restrict__ C = (TO*)g.C;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  flt4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

  u32x4 ra[VA], rb[VB];
  // 8 consecutive contraction indices of one operand row; with krep > 0 the
  // operand is repeated along K (column k is read at k mod krep).
  auto load_vec = [&](const bf16_t* __restrict__ P, long long ld, int rows, int r0, int k0,
                      int krep, int e, u32x4& dst) {
    const int r = e / (BK / 8), c = (e % (BK / 8)) * 8;
    const int gr = r0 + r, gk = k0 + c;
    if (gr < rows && g.vec && gk + 8 <= g.K) {
      const int kc = krep ? gk % krep : gk;
      dst = *(const u32x4*)(P + (long long)gr * ld + kc);
    } else {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
      if (gr < rows) {
        for (int q = 0; q < 8; ++q) {
          const int kq = gk + q;
          const int kc = krep ? kq % krep : kq;
          const uint32_t v = (kq < g.K) ? (uint32_t)P[(long long)gr * ld + kc] : 0u;
          w[q >> 1] |= v << (16 * (q & 1));
        }
      }
      dst = u32x4{w[0], w[1], w[2], w[3]};
    }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < VA; ++t) load_vec(A, g.lda, g.M, m0, k0, g.krep_a, tid + 256 * t, ra[t]);
#pragma unroll
    for (int t = 0; t < VB; ++t) load_vec(B, g.ldb, g.Nn, n0, k0, g.krep_b, tid + 256 * t, rb[t]);
  };
  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int t = 0; t < VA; ++t) {
      const int e = tid + 256 * t;
      *(u32x4*)&As[e / (BK / 8)][(e % (BK / 8)) * 8] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < VB; ++t) {
      const int e = tid + 256 * t;
      *(u32x4*)&Bs[e / (BK / 8)][(e % (BK / 8)) * 8] = rb[t];
    }
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      u32x4 af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        af[i] = *(const u32x4*)&As[wm * WM + i * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bfr[j] = *(const u32x4*)&Bs[wn * WN + j * 16 + (lane & 15)][ks + 8 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (F16)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(f16x8, af[i]), __builtin_bit_cast(f16x8, bfr[j]), acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, af[i]), __builtin_bit_cast(bf16x8, bfr[j]), acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const float oscale = g.out_div ? (float)(1.0 / *g.out_div) : 1.0f;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      // v_mfma_f32_16x16x32_{bf16,f16} result: item v of lane l is row 4(l/16) + v, column l%16.
      const int n = n0 + wn * WN + j * 16 + (lane & 15);
      if (n >= g.Nn) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * WM + i * 16 + 4 * (lane >> 4) + v;
        if (m < g.M) C[out_addr(g.om, m, n, bz)] = cvt_out<TO, F16>(acc[i][j][v] * oscale);
      }
    }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int run_gemm_f64(kp_context* ctx, const GemmArgs& g, int batch) {
  const bool big = (long long)g.M * g.Nn >= 256LL * 128 * 128;
  if (big) {
    dim3 grid((g.Nn + 127) / 128, (g.M + 127) / 128, batch);
    hipLaunchKernelGGL((k_gemm_f64<128, 128>), grid, dim3(256), 0, ctx->stream, g);
  } else {
    dim3 grid((g.Nn + 63) / 64, (g.M + 63) / 64, batch);
    hipLaunchKernelGGL((k_gemm_f64<64, 64>), grid, dim3(256), 0, ctx->stream, g);
  }
  KP_HIP(hipGetLastError());
  return KP_OK;
}

template <typename TO>
int run_gemm_16(kp_context* ctx, GemmArgs g, int batch, bool f16) {
  g.vec = (g.K % 8 == 0) && (g.lda % 8 == 0) && (g.ldb % 8 == 0) && (g.sAb % 8 == 0) &&
          (g.sBb % 8 == 0) && (g.krep_a % 8 == 0) && (g.krep_b % 8 == 0) && aligned16(g.A) &&
          aligned16(g.B);
  const bool big = (long long)g.M * g.Nn >= 256LL * 128 * 128;
  if (big) {
    dim3 grid((g.Nn + 127) / 128, (g.M + 127) / 128, batch);
    if (f16) hipLaunchKernelGGL((k_gemm_16<128, 128, true, TO>), grid, dim3(256), 0, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16<128, 128, false, TO>), grid, dim3(256), 0, ctx->stream, g);
  } else {
    dim3 grid((g.Nn + 63) / 64, (g.M + 63) / 64, batch);
    if (f16) hipLaunchKernelGGL((k_gemm_16<64, 64, true, TO>), grid, dim3(256), 0, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16<64, 64, false, TO>), grid, dim3(256), 0, ctx->stream, g);
  }
  KP_HIP(hipGetLastError());
  return KP_OK;
}

// The three stages.  With split = true the circulant operands carry (hi | lo)
// halves along K, the contraction runs over 2K and the other operand is read
// twice (k mod K), so that C x = C_hi x + C_lo x is accumulated in float.
struct Stages {
  GemmArgs s1, s2, s3;
};

Stages make_stages(int N, int R, const void* x, const void* a1, const void* c2, const void* b3,
                   void* T, void* U, void* z, const int* done, bool split,
                   const double* out_div) {
  const long long n = N, nn = n * n, n3 = nn * n, RN = (long long)R * N;
  const long long f = split ? 2 : 1;
  const int rn = split ? N : 0, rrn = split ? (int)RN : 0;
  Stages s;
  // (i) rows (i1,i2), cols (k,j3), K = i3; store transposed: addr = m + n*M.
  s.s1 = gemm_args(x, b3, T, nn, RN, f * n, n, f * n, 0, 0, OutMap{1, 0, nn, 0, INT_MAX}, done,
                   rn, 0);
  // (ii) batch k: rows j2, cols (j3,i1), K = i2; addr = j2*R*N^2 + j3*R*N + k*N + i1.
  s.s2 = gemm_args(c2, T, U, n, nn, f * n, f * n, n, f * nn, n3, OutMap{RN * n, RN, 1, n, N}, done,
                   0, rn);
  // (iii) rows j1, cols (j2,j3), K = (k,i1); natural row-major output.
  s.s3 = gemm_args(a1, U, z, n, nn, f * RN, f * RN, RN, 0, 0, OutMap{nn, 0, 1, 0, INT_MAX}, done,
                   0, rrn, out_div);
  return s;
}

}  // namespace

int launch_precond_f64(kp_context* ctx, const kp_precond* pc, const double* x, double* z,
                       const int* done) {
  const size_t n3 = (size_t)pc->N * pc->N * pc->N;
  void *T, *U;
  KP_TRY(ws_get(ctx, WS_T, n3 * pc->R * sizeof(double), &T));
  KP_TRY(ws_get(ctx, WS_U, n3 * pc->R * sizeof(double), &U));
  Stages s = make_stages(pc->N, pc->R, x, pc->a1_64, pc->c2_64, pc->b3_64, T, U, z, done, false,
                         nullptr);
  {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE3);
    KP_TRY(run_gemm_f64(ctx, s.s1, 1));
  }
  {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE2);
    KP_TRY(run_gemm_f64(ctx, s.s2, pc->R));
  }
  ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE1);
  KP_TRY(run_gemm_f64(ctx, s.s3, 1));
  return KP_OK;
}

int launch_precond_16(kp_context* ctx, const kp_precond* pc, const bf16_t* x, float* z,
                      const int* done, const double* scale) {
  const size_t n3 = (size_t)pc->N * pc->N * pc->N;
  const bool f16 = pc->precision == KP_MIXED_FP16;
  void *T, *U;
  KP_TRY(ws_get(ctx, WS_T, n3 * pc->R * sizeof(bf16_t), &T));
  KP_TRY(ws_get(ctx, WS_U, n3 * pc->R * sizeof(bf16_t), &U));
  Stages s = make_stages(pc->N, pc->R, x, pc->a1_16, pc->c2_16, pc->b3_16, T, U, z, done, true,
                         scale);
  {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE3);
    KP_TRY(run_gemm_16<bf16_t>(ctx, s.s1, 1, f16));
  }
  {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE2);
    KP_TRY(run_gemm_16<bf16_t>(ctx, s.s2, pc->R, f16));
  }
  ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE1);
  KP_TRY(run_gemm_16<float>(ctx, s.s3, 1, f16));
  return KP_OK;
}

}  // namespace kp

// Low-Kronecker-rank preconditioner: z = sum_k (C1^k x C2^k x C3^k) x
// (eq. Lap3DtimesX with the circulants C_l^k = F* diag(u_l^k) F held as dense
// real symmetric N x N matrices), evaluated as three MFMA GEMMs, each of the
// form D = A * B^T with the circulant operand as A and both operands
// contiguous in the contraction index:
//
//   (i)   T[k][j3][i1][i2]   = sum_i3     C3^k[j3][i3] X[i1][i2][i3]
//   (ii)  U[(j2,j3)][(k,i1)] = sum_i2     C2^k[j2][i2] T[k][j3][i1][i2]
//   (iii) Z[j1][(j2,j3)]     = sum_(k,i1) C1^k[j1][i1] U[(j2,j3)][(k,i1)]
//
// Stage (iii) contracts over R*N at once, which folds the sum over the R
// Kronecker terms into the GEMM.  The layouts of T and U are set by the output
// address maps of stages (i) and (ii) so that each is the contiguous B operand
// of the next stage.
//
// FP64: v_mfma_f64_16x16x4_f64.  BF16 / FP16: v_mfma_f32_16x16x32_{bf16,f16}
// with float accumulation; T and U are rounded to the 16-bit type.  In 16 bits
// each circulant is held as its rounded value plus the rounded remainder
// (hi + lo) and both are multiplied into the same accumulator, reusing every
// fragment of the data operand: the symbol of the low-rank preconditioner
// spans about 12 N^2 / (4 pi^2) in magnitude across frequencies, more than one
// 16-bit rounding of the dense circulant entries resolves.

#include <climits>
#include <type_traits>

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

// Batch index z = blockIdx.z splits as z = bo * bdiv + bi: the A operand is
// A + bi * sAb, the B operand B + z * sBb, the output C + bo * sCb at the
// address map with batch index bi; done[bo * done_stride] != 0 skips the
// block and out_div[bo * div_stride] scales the results.  (bo is the system
// of a batched solve, bi the rank term of stage (ii).)
struct GemmArgs {
  const void* A;   // M x K, row stride lda (16-bit: remainder plane at +a_lo in each row)
  const void* B;   // Nn x K, row stride ldb  (the transposed right operand)
  void* C;
  int M, Nn, K;
  long long lda, ldb, sAb, sBb;
  OutMap om;
  const int* done;
  int vec;                // 1: 16-byte operand loads are legal (alignment and K)
  long long a_lo;         // > 0: A = A[.., k] + A[.., a_lo + k] (hi + lo planes)
  const double* out_div;  // non-null: results are divided by out_div[bo * div_stride]
  int order;              // block-to-tile order (tile_of)
  int bdiv;
  long long sCb;
  int done_stride, div_stride;
  // Circulant operand by its first columns (kp_precond::circ16 layout), for
  // k_gemm_16c: A[m][kk] = C_ci[j][i] with j = m mod cn, i = kk mod cn and
  // ci = m / cn (cmode 0), the batch index bi (cmode 1) or kk / cn (cmode 2).
  const bf16_t* circ;
  int cn, cmode;
  // Optional dot products of the result z with r and q at the same positions
  // (float vectors, stride sCb per system): block partials of <r,z>, <q,z>,
  // sum z, sum r, sum q at dpart[bo * 5 G + v G + block], G = blocks per system.
  const float* dr;
  const float* dq;
  double* dpart;
};

GemmArgs gemm_args(const void* A, const void* B, void* C, long long M, long long Nn, long long K,
                   long long lda, long long ldb, long long sAb, long long sBb, OutMap om,
                   const int* done, long long a_lo, const double* out_div, int bdiv, long long sCb) {
  return GemmArgs{A,  B, C,      (int)M, (int)Nn, (int)K, lda, ldb, sAb, sBb, om, done, 0,
                  a_lo, out_div, 0, bdiv, sCb, (int)(sizeof(Scalars) / sizeof(int)),
                  (int)(sizeof(Scalars) / sizeof(double)), nullptr, 0, 0, nullptr, nullptr, nullptr};
}

__device__ __forceinline__ long long out_addr(const OutMap& o, int m, int n, int b) {
  return (long long)m * o.sm + (long long)(n / o.nd) * o.sn1 + (long long)(n % o.nd) * o.sn2 +
         (long long)b * o.sb;
}

// Block-to-tile map over a 1D grid of Mt x Nt tiles (z = batch).
//  order 0: column tile fastest in launch order; concurrently resident blocks
//           sweep along the data operand and the (small) circulant operand
//           stays in every L2.
//  order 1: the hardware deals the blocks of a launch round-robin to the eight
//           XCDs (block b to XCD b % 8), each with its own L2.  Block b takes
//           tile t = (b % 8) * (G / 8) + b / 8 with tiles numbered row tile
//           fastest, so the Mt blocks that share one column tile of the data
//           operand run on one XCD at about the same time and that tile
//           crosses from HBM into that L2 once.  (G not a multiple of 8: row
//           tile fastest in launch order.)
// The autotuner times both orders.
__device__ __forceinline__ void tile_of(int Mt, int order, int& mt, int& nt) {
  const int G = gridDim.x, b = blockIdx.x;
  if (order == 0) {
    const int Nt = G / Mt;
    nt = b % Nt;
    mt = b / Nt;
  } else {
    const int t = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
    mt = t % Mt;
    nt = t / Mt;
  }
}

// float -> output type; 16-bit results round to nearest even (the
// conversion instructions of gfx950).
template <typename TO, bool F16>
__device__ __forceinline__ TO cvt_out(float v) {
  if constexpr (sizeof(TO) == 4) {
    return v;
  } else if constexpr (F16) {
    return __builtin_bit_cast(bf16_t, (_Float16)v);
  } else {
    return __builtin_bit_cast(bf16_t, (__bf16)v);
  }
}

// ---------------------------------------------------------------- FP64 MFMA
// 256 threads = 2 x 2 wavefronts, block tile BM x BN, K tile 16, wave tile
// (BM/2) x (BN/2) made of 16 x 16 MFMA tiles.  Global loads for the next K
// tile are issued before the MFMAs of the current one.
// STAGE (0..2) only separates the three stages' kernel names in profiles.
template <int STAGE, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  const int bz = blockIdx.z, bo = bz / g.bdiv, bi = bz - bo * g.bdiv;
  if (g.done && g.done[(long long)bo * g.done_stride]) return;
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ double As[BM][BK + 1];
  __shared__ double Bs[BN][BK + 1];
  const double* __restrict__ A = (const double*)g.A + (long long)bi * g.sAb;
  const double* __restrict__ B = (const double*)g.B + (long long)bz * g.sBb;
  double* __restrict__ C = (double*)g.C + (long long)bo * g.sCb;
  int mt, nt;
  tile_of((g.M + BM - 1) / BM, g.order, mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
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
        if (m < g.M) C[out_addr(g.om, m, n, bi)] = acc[i][j][v];
      }
    }
}

// ---------------------------------------------------- BF16 / FP16 MFMA
// LDS barrier that leaves global loads in flight: waits for this wave's LDS
// accesses only (a __syncthreads would also wait for the register prefetch).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// LDS rows hold BK 16-bit values as 16-byte chunks; chunk c of row r sits at
// slot c ^ (r & 7) (BK = 64 or 128: eight or sixteen chunks) or
// c ^ ((r >> 2) & 3) (BK = 32, four chunks), so the rows read by one fragment
// load, or written by one store, fall in different banks.  No padding.
template <int BK>
__device__ __forceinline__ int swz(int row) {
  return BK == 32 ? ((row >> 2) & 3) : (row & 7);
}

// Epilogue of the 16-bit kernels.  Step i stages rows i*16 .. i*16+15 of both
// wave rows (32 block rows x BN columns) in LDS (smem, free again after the K
// loop) and writes them as 16-byte vectors along n, each block row as one
// contiguous run of BN values where the output map allows (sn2 = 1 and the
// block's column range inside one run of nd columns; always for interior
// tiles of the three stages at sizes that are multiples of the tile), which
// writes whole cache lines (partially written lines cost a fetch).  The run's
// start is computed once per block instead of per element.
template <int BM, int BN, bool F16, typename TO>
__device__ __forceinline__ void epilogue16(const GemmArgs& g, const flt4 (&acc)[BM / 32][BN / 32],
                                           unsigned char* smem, TO* __restrict__ C, int m0, int n0,
                                           int bo, int bi, bool interior) {
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int VL = 16 / (int)sizeof(TO);  // output elements per 16-byte vector
  constexpr int LDB = BN + VL;              // padded staging row
  constexpr int VPR = BN / VL;              // vectors per block row
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const float oscale = g.out_div ? (float)(1.0 / g.out_div[(long long)bo * g.div_stride]) : 1.0f;
  TO* stg = reinterpret_cast<TO*>(smem);
  const int run_q = n0 / g.om.nd, run_r = n0 - run_q * g.om.nd;
  const bool fast = interior && g.om.sn2 == 1 && run_r + BN <= g.om.nd;
  const long long col0 = (long long)run_q * g.om.sn1 + run_r + (long long)bi * g.om.sb;
  // Fused dot products (float results only; r, q at the same index as z).
  constexpr bool DOTS = sizeof(TO) == 4;
  double dacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool dots = DOTS && g.dpart;
  const float* dr = dots ? g.dr + (long long)bo * g.sCb : nullptr;
  const float* dq = dots && g.dq ? g.dq + (long long)bo * g.sCb : nullptr;
  auto dot1 = [&](long long idx, float zv) {
    const double z = zv, r = dr[idx], q = dq ? (double)dq[idx] : 0.0;
    dacc[0] += r * z;
    dacc[1] += q * z;
    dacc[2] += z;
    dacc[3] += r;
    dacc[4] += q;
  };
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    // v_mfma_f32_16x16x32_{bf16,f16} result: item v of lane l is row 4(l/16) + v, column l%16.
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stg[(wm * 16 + 4 * (lane >> 4) + v) * LDB + wn * WN + j * 16 + (lane & 15)] =
            cvt_out<TO, F16>(acc[i][j][v] * oscale);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 32 * VPR / 256; ++t) {
      const int e = tid + 256 * t, r = e / VPR, c = (e % VPR) * VL;
      const int m = m0 + (r >> 4) * WM + i * 16 + (r & 15), n = n0 + c;
      const TO* src = stg + r * LDB + c;
      if (fast) {
        const long long idx = (long long)m * g.om.sm + col0 + c;
        TO* dst = C + idx;
        if (((uintptr_t)dst & 15u) == 0) {
          const u32x4 v = *(const u32x4*)src;
          *(u32x4*)dst = v;
          if constexpr (DOTS) {
            if (dots) {
              const flt4 zv = __builtin_bit_cast(flt4, v);
              const flt4 rv = *(const flt4*)(dr + idx);
              const flt4 qv = dq ? *(const flt4*)(dq + idx) : flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const double z = zv[e], r = rv[e], q = qv[e];
                dacc[0] += r * z;
                dacc[1] += q * z;
                dacc[2] += z;
                dacc[3] += r;
                dacc[4] += q;
              }
            }
          }
          continue;
        }
      }
      if (m >= g.M || n >= g.Nn) continue;
      for (int q = 0; q < VL && n + q < g.Nn; ++q) {
        const long long idx = out_addr(g.om, m, n + q, bi);
        C[idx] = src[q];
        if constexpr (DOTS) {
          if (dots) dot1(idx, (float)src[q]);
        }
      }
    }
    __syncthreads();
  }
  if constexpr (DOTS) {
    if (dots) {
      // Block sums in a fixed order: wave shuffles, then the four waves.
      double* red = reinterpret_cast<double*>(smem);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double x = dacc[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[v * 4 + wid] = x;
      }
      __syncthreads();
      if (tid < 5) {
        const int G = gridDim.x;
        g.dpart[((long long)bo * 5 + tid) * G + blockIdx.x] =
            (red[tid * 4 + 0] + red[tid * 4 + 1]) + (red[tid * 4 + 2] + red[tid * 4 + 3]);
      }
    }
  }
}

// 256 threads = 2 x 2 wavefronts, block tile BM x BN, K tile BK (BK/32
// 16x16x32 steps).  Operands move as 16-byte vectors of eight 16-bit values;
// the next K tile is fetched into registers while the current one is
// multiplied.  With SPLIT the A tile is staged twice (hi and lo planes) and
// every B fragment feeds two MFMAs.  Tiles inside the matrices (all but the
// ragged edges) take a lean path: global loads from a uniform base plus 32-bit
// per-thread offsets, no bounds tests, and a division-free epilogue; LDS
// addresses are per-thread constants in both paths.
template <int STAGE, int BM, int BN, int BK, bool F16, bool SPLIT, typename TO>
__global__ __launch_bounds__(256) void k_gemm_16(GemmArgs g) {
  const int bz = blockIdx.z, bo = bz / g.bdiv, bi = bz - bo * g.bdiv;
  if (g.done && g.done[(long long)bo * g.done_stride]) return;
  static_assert(BK == 32 || BK == 64, "K tile");
  constexpr int CH = BK / 8;  // 16-byte chunks per row
  constexpr int NP = SPLIT ? 2 : 1;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int VA = BM * BK / 8 / 256, VB = BN * BK / 8 / 256;  // 16-byte vectors per thread
  constexpr int RS = 256 / CH;  // rows between a thread's successive vectors
  // Operand tiles; after the K loop the same memory stages the output.
  constexpr int VL = 16 / (int)sizeof(TO);  // output elements per 16-byte vector
  constexpr int OP_BYTES = (NP * BM + BN) * BK * 2;
  constexpr int STG_BYTES = 32 * (BN + VL) * (int)sizeof(TO);
  __shared__ __attribute__((aligned(16))) unsigned char smem[OP_BYTES > STG_BYTES ? OP_BYTES : STG_BYTES];
  bf16_t* const sA = reinterpret_cast<bf16_t*>(smem);  // [NP][BM][BK]
  bf16_t* const sB = sA + NP * BM * BK;                 // [BN][BK]
  const bf16_t* __restrict__ A = (const bf16_t*)g.A + (long long)bi * g.sAb;
  const bf16_t* __restrict__ B = (const bf16_t*)g.B + (long long)bz * g.sBb;
  TO* __restrict__ C = (TO*)g.C + (long long)bo * g.sCb;
  int mt, nt;
  tile_of((g.M + BM - 1) / BM, g.order, mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  flt4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

  // Thread t stores vectors e = t + 256 v: row e / CH = t / CH + RS v, chunk
  // t % CH; the swizzle of those rows does not depend on v.
  const int st_row = tid / CH, st_ch = tid % CH;
  const int st_off = st_row * BK + ((st_ch ^ swz<BK>(st_row)) * 8);
  // Fragment reads: row base + (lane & 15), chunk ks / 8 + lane / 16.
  const int rd_sw = swz<BK>(lane & 15);
  int rdA[BK / 32], rdB[BK / 32];
#pragma unroll
  for (int q = 0; q < BK / 32; ++q) {
    const int ch = (4 * q + (lane >> 4)) ^ rd_sw;
    rdA[q] = (wm * WM + (lane & 15)) * BK + ch * 8;
    rdB[q] = (wn * WN + (lane & 15)) * BK + ch * 8;
  }

  u32x4 ra[NP][VA], rb[VB];
  auto store_lds = [&]() {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int t = 0; t < VA; ++t) *(u32x4*)(sA + (p * BM + RS * t) * BK + st_off) = ra[p][t];
#pragma unroll
    for (int t = 0; t < VB; ++t) *(u32x4*)(sB + RS * t * BK + st_off) = rb[t];
  };
  auto mfma = [&](const u32x4& a, const u32x4& b, flt4& c) {
    if constexpr (F16)
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  };
  auto multiply = [&]() {
#pragma unroll
    for (int q = 0; q < BK / 32; ++q) {
      u32x4 bfr[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *(const u32x4*)(sB + rdB[q] + j * 16 * BK);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        u32x4 af[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const u32x4*)(sA + rdA[q] + (p * BM + i * 16) * BK);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) mfma(af[i], bfr[j], acc[i][j]);
      }
    }
  };

  const bool interior = m0 + BM <= g.M && n0 + BN <= g.Nn && g.vec && g.K % BK == 0;
  if (interior) {
    // Uniform tile origins plus 32-bit per-thread offsets (in elements).
    const bf16_t* __restrict__ Ab = A + (long long)m0 * g.lda;
    const bf16_t* __restrict__ Bb = B + (long long)n0 * g.ldb;
    unsigned offA[VA], offB[VB];
#pragma unroll
    for (int t = 0; t < VA; ++t) offA[t] = (unsigned)((st_row + RS * t) * g.lda + st_ch * 8);
#pragma unroll
    for (int t = 0; t < VB; ++t) offB[t] = (unsigned)((st_row + RS * t) * g.ldb + st_ch * 8);
    auto load = [&](int k0) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const bf16_t* __restrict__ Ap = Ab + p * g.a_lo + k0;
#pragma unroll
        for (int t = 0; t < VA; ++t) ra[p][t] = *(const u32x4*)(Ap + offA[t]);
      }
      const bf16_t* __restrict__ Bp = Bb + k0;
#pragma unroll
      for (int t = 0; t < VB; ++t) rb[t] = *(const u32x4*)(Bp + offB[t]);
    };
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
      store_lds();
      lds_barrier();
      if (k0 + BK < g.K) load(k0 + BK);
      multiply();
      lds_barrier();
    }
  } else {
    // Ragged tile: element-wise zero fill outside the matrices.
    auto load_vec = [&](const bf16_t* __restrict__ P, long long ld, int rows, int r, int k0,
                        u32x4& dst) {
      const int gk = k0 + st_ch * 8;
      if (r < rows && g.vec && gk + 8 <= g.K) {
        dst = *(const u32x4*)(P + (long long)r * ld + gk);
      } else {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (r < rows) {
          for (int q = 0; q < 8; ++q) {
            const uint32_t v = (gk + q < g.K) ? (uint32_t)P[(long long)r * ld + gk + q] : 0u;
            w[q >> 1] |= v << (16 * (q & 1));
          }
        }
        dst = u32x4{w[0], w[1], w[2], w[3]};
      }
    };
    auto load = [&](int k0) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int t = 0; t < VA; ++t) load_vec(A + p * g.a_lo, g.lda, g.M, m0 + st_row + RS * t, k0, ra[p][t]);
#pragma unroll
      for (int t = 0; t < VB; ++t) load_vec(B, g.ldb, g.Nn, n0 + st_row + RS * t, k0, rb[t]);
    };
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
      store_lds();
      lds_barrier();
      if (k0 + BK < g.K) load(k0 + BK);
      multiply();
      lds_barrier();
    }
  }
  __syncthreads();

  epilogue16<BM, BN, F16, TO>(g, acc, smem, C, m0, n0, bo, bi, interior);
}

// The same product with the circulant operand built in LDS.  Every A tile is
// a block of one circulant C (the rows of a tile never leave one circulant,
// nor do the K tiles), and C[j][i..i+7] = r((i - j) mod N ..) is an aligned
// 16-byte run of one of eight shifted copies of the reversed first column r
// (kp_precond::circ16), so the block loads those copies (2 planes x 8 x (N+8)
// values, 8.4 KB at N = 256) once per circulant instead of streaming A tiles;
// only the data operand B goes through the K loop.  All tiles must be interior
// (checked by the launcher).  Dynamic LDS: the copies.  Launch bounds for three
// blocks per CU: every tile fits in 168 registers without spilling (the
// accumulators move from AGPRs to VGPRs), and the third block per CU took the
// last stage at N = 256 from 110 to 101 us.
template <int STAGE, int BM, int BN, int BK, bool F16, typename TO>
__global__ __launch_bounds__(256, 3) void k_gemm_16c(GemmArgs g) {
  const int bz = blockIdx.z, bo = bz / g.bdiv, bi = bz - bo * g.bdiv;
  if (g.done && g.done[(long long)bo * g.done_stride]) return;
  static_assert(BK == 32 || BK == 64 || BK == 128, "K tile");
  constexpr int CH = BK / 8;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int VB = BN * BK / 8 / 256;
  constexpr int RS = 256 / CH;
  constexpr int VL = 16 / (int)sizeof(TO);
  constexpr int OP_BYTES = BN * BK * 2;
  constexpr int STG_BYTES = 32 * (BN + VL) * (int)sizeof(TO);
  __shared__ __attribute__((aligned(16))) unsigned char smem[OP_BYTES > STG_BYTES ? OP_BYTES : STG_BYTES];
  extern __shared__ __attribute__((aligned(16))) bf16_t cpy[];  // [2][8][N + 8]
  bf16_t* const sB = reinterpret_cast<bf16_t*>(smem);
  const bf16_t* __restrict__ B = (const bf16_t*)g.B + (long long)bz * g.sBb;
  TO* __restrict__ C = (TO*)g.C + (long long)bo * g.sCb;
  int mt, nt;
  tile_of(g.M / BM, g.order, mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int N = g.cn, NP8 = N + 8;
  flt4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

  // Copies of circulant ci into LDS (16-byte vectors; N + 8 is a multiple of 8).
  auto fill = [&](int ci) {
    const u32x4* __restrict__ src = (const u32x4*)(g.circ + (long long)ci * 16 * NP8);
    u32x4* dst = (u32x4*)cpy;
    for (int v = tid; v < 2 * NP8; v += 256) dst[v] = src[v];
  };
  const int st_row = tid / CH, st_ch = tid % CH;
  const int st_off = st_row * BK + ((st_ch ^ swz<BK>(st_row)) * 8);
  const int rd_sw = swz<BK>(lane & 15);
  int rdB[BK / 32];
#pragma unroll
  for (int q = 0; q < BK / 32; ++q) rdB[q] = (wn * WN + (lane & 15)) * BK + ((4 * q + (lane >> 4)) ^ rd_sw) * 8;
  // Row of fragment i inside its circulant: jr + 16 i; K offset of the lane's run: 8 (lane / 16).
  const int jr = m0 % N + wm * WM + (lane & 15);
  const int kl = 8 * (lane >> 4);

  const bf16_t* __restrict__ Bb = B + (long long)n0 * g.ldb;
  unsigned offB[VB];
#pragma unroll
  for (int t = 0; t < VB; ++t) offB[t] = (unsigned)((st_row + RS * t) * g.ldb + st_ch * 8);
  u32x4 rb[VB];
  auto load = [&](int k0) {
    const bf16_t* __restrict__ Bp = Bb + k0;
#pragma unroll
    for (int t = 0; t < VB; ++t) rb[t] = *(const u32x4*)(Bp + offB[t]);
  };
  auto mfma = [&](const u32x4& a, const u32x4& b, flt4& c) {
    if constexpr (F16)
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  };

  int ci = g.cmode == 0 ? m0 / N : (g.cmode == 1 ? bi : 0);
  fill(ci);
  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    if (g.cmode == 2 && k0 / N != ci) {  // the K tiles enter the next circulant
      ci = k0 / N;
      fill(ci);
    }
#pragma unroll
    for (int t = 0; t < VB; ++t) *(u32x4*)(sB + RS * t * BK + st_off) = rb[t];
    lds_barrier();
    if (k0 + BK < g.K) load(k0 + BK);
    const int kin = k0 - (k0 / N) * N + kl;  // column of the run inside the circulant
#pragma unroll
    for (int q = 0; q < BK / 32; ++q) {
      u32x4 bfr[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *(const u32x4*)(sB + rdB[q] + j * 16 * BK);
      int aoff[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        int u0 = kin + 32 * q - (jr + 16 * i);
        if (u0 < 0) u0 += N;
        aoff[i] = (u0 & 7) * NP8 + (u0 & ~7);
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {  // hi, then lo plane
        u32x4 af[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const u32x4*)(cpy + p * 8 * NP8 + aoff[i]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) mfma(af[i], bfr[j], acc[i][j]);
      }
    }
    lds_barrier();
  }
  __syncthreads();
  epilogue16<BM, BN, F16, TO>(g, acc, smem, C, m0, n0, bo, bi, true);
}

// Wave-streamed product for large circulant stages.  The data operand is the
// first MFMA operand and goes from global memory straight into registers: each
// wave owns 32 columns of the result and keeps the next four 32-wide K steps
// of them in flight (a register ring, no LDS and no barrier in the K loop).
// The circulant is the second MFMA operand, read from the shifted copies in
// LDS.  A wave covers 128 circulant rows as eight 16-row fragments; fragment c
// at K step q (inside one circulant) starts at (32 q - 16 c - row) mod N, which
// depends on 2q - c only (a Toeplitz matrix), so going from step q to q + 1
// keeps six of the eight fragments and reads two new ones (hi and lo planes).
// The MFMA result of a lane is four consecutive data columns of one circulant
// row; the data fragments' rows are assigned to columns so that each lane ends
// with 4 TND consecutive columns: float results go straight to memory as
// 16-byte stores, 16-bit ones through a block staging tile in LDS so that the
// stores cover whole rows of the block tile.  Block: WAVES_M x (4 / WAVES_M) waves.  Stage (iii)
// runs over R circulants along K: two LDS buffers, the next circulant loaded
// while the current one is used, one barrier per circulant.
// Requires: N a multiple of 256, every tile interior (checked by wave_ok).
template <int STAGE, int TMC, int TND, int WAVES_M, bool F16, typename TO>
__global__ __launch_bounds__(256, 2) void k_gemm_16w(GemmArgs g) {
  // (TMC = 4 with TND = 2 or 4 measured slower than 8 x 2 on every stage.)
  static_assert((TMC == 4 || TMC == 8) && TND % 2 == 0, "wave tile");
  constexpr int WM = 16 * TMC, WN = 16 * TND;
  constexpr int WAVES_N = 4 / WAVES_M;
  constexpr int BM = WAVES_M * WM, BN = WAVES_N * WN;
  constexpr int D = 4;  // K steps in flight per wave (a multiple of 4, dividing N / 32)
  const int bz = blockIdx.z, bo = bz / g.bdiv, bi = bz - bo * g.bdiv;
  if (g.done && g.done[(long long)bo * g.done_stride]) return;
  extern __shared__ __attribute__((aligned(16))) bf16_t cpy[];  // [buffer][2][8][N + 8]
  __shared__ double red[20];
  // Output staging tile of 16-bit results, rows padded by 16 bytes.
  constexpr int SLD = BN + 8;
  __shared__ __attribute__((aligned(16))) bf16_t stg[sizeof(TO) == 2 ? BM * SLD : 8];
  const bf16_t* __restrict__ B = (const bf16_t*)g.B + (long long)bz * g.sBb;
  TO* __restrict__ C = (TO*)g.C + (long long)bo * g.sCb;
  int mt, nt;
  tile_of(g.M / BM, g.order, mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WAVES_N, wn = wid - (wid / WAVES_N) * WAVES_N;
  const int l16 = lane & 15, kg = lane >> 4;
  const int N = g.cn, NP8 = N + 8, CPY = 16 * NP8;
  const int QC = N / 32, QT = g.K / 32;  // K steps per circulant / in total

  // Data rows of this lane: fragment j, MFMA row l16 -> column
  // nb + 4 TND (l16 / 4) + 4 j + l16 % 4, K run 8 kg .. 8 kg + 7 of each step.
  const int nb = n0 + wn * WN;
  const bf16_t* __restrict__ bp[TND];
#pragma unroll
  for (int j = 0; j < TND; ++j)
    bp[j] = B + (long long)(nb + 4 * TND * (l16 >> 2) + 4 * j + (l16 & 3)) * g.ldb + 8 * kg;
  u32x4 rb[D][TND];
  auto load = [&](int slot, int q) {
#pragma unroll
    for (int j = 0; j < TND; ++j) rb[slot][j] = *(const u32x4*)(bp[j] + 32 * q);
  };
#pragma unroll
  for (int s = 0; s < D; ++s) load(s, s);  // QT >= 8

  // Copies of circulant ci into LDS buffer b.
  auto fill = [&](int ci, int b) {
    const u32x4* __restrict__ src = (const u32x4*)(g.circ + (long long)ci * CPY);
    u32x4* dst = (u32x4*)(cpy + b * CPY);
    for (int v = tid; v < 2 * NP8; v += 256) dst[v] = src[v];
  };
  const int nc = g.cmode == 2 ? QT / QC : 1;  // circulants along K
  fill(g.cmode == 0 ? m0 / N : (g.cmode == 1 ? bi : 0), 0);
  if (nc > 1) fill(1, 1);
  __syncthreads();

  // Circulant fragment s = 2 q - c (in ring slot s mod TMC): copy offset of
  // u = (16 s + base) mod N, base = (8 kg - row) mod N.
  const int mr = m0 % N + wm * WM + l16;
  int base = 8 * kg - mr;
  base = base < 0 ? base + N : base;
  u32x4 ca[TMC][2];
  const bf16_t* cb = cpy;
  auto frag = [&](int slot, int s) {
    int u = 16 * s + base;
    u = u < 0 ? u + N : (u >= N ? u - N : u);
    const bf16_t* p = cb + (u & 7) * NP8 + (u & ~7);
    ca[slot][0] = *(const u32x4*)p;
    ca[slot][1] = *(const u32x4*)(p + 8 * NP8);
  };
  auto mfma = [&](const u32x4& a, const u32x4& b, flt4& c) {
    if constexpr (F16)
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  };
  flt4 acc[TMC][TND];
#pragma unroll
  for (int c = 0; c < TMC; ++c)
#pragma unroll
    for (int j = 0; j < TND; ++j) acc[c][j] = flt4{0.f, 0.f, 0.f, 0.f};

  for (int q0 = 0; q0 < QT; q0 += D) {
    const int qc = q0 - (q0 / QC) * QC;  // step inside the current circulant
    if (qc == 0) {
      const int cc = q0 / QC;
      if (cc > 0) {
        // Everyone is done with circulant cc - 1 (its buffer is free) and the
        // copies of cc (loaded at the previous boundary) are visible.
        __syncthreads();
        if (cc + 1 < nc) fill(cc + 1, (cc + 1) & 1);
      }
      cb = cpy + (cc & 1) * CPY;
#pragma unroll
      for (int c = 0; c < TMC; ++c) frag((TMC - c) & (TMC - 1), -c);
    }
#pragma unroll
    for (int dq = 0; dq < D; ++dq) {
      const int q = q0 + dq, qp = qc + dq;
      if (dq > 0 || qc > 0) {  // two new fragments: s = 2 qp - 1 and 2 qp
        frag((2 * dq + TMC - 1) & (TMC - 1), 2 * qp - 1);
        frag((2 * dq) & (TMC - 1), 2 * qp);
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int c = 0; c < TMC; ++c)
#pragma unroll
          for (int j = 0; j < TND; ++j) mfma(rb[dq][j], ca[(2 * dq - c + TMC) & (TMC - 1)][p], acc[c][j]);
      if (q + D < QT) load(dq, q + D);
    }
  }

  // Epilogue: lane (l16, kg) holds rows m = m0 + wm WM + 16 c + l16 and the
  // 4 TND columns nb + 4 TND kg .. (acc[c][j][v] at column + 4 j + v).
  const float oscale = g.out_div ? (float)(1.0 / g.out_div[(long long)bo * g.div_stride]) : 1.0f;
  const int ncol = nb + 4 * TND * kg;
  const int run_q = ncol / g.om.nd;
  const long long col = (long long)run_q * g.om.sn1 + (ncol - run_q * g.om.nd) + (long long)bi * g.om.sb;
  constexpr bool DOTS = sizeof(TO) == 4;
  const bool dots = DOTS && g.dpart;
  double dacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < TMC; ++c) {
    const long long idx = (long long)(m0 + wm * WM + 16 * c + l16) * g.om.sm + col;
    if constexpr (DOTS) {
#pragma unroll
      for (int j = 0; j < TND; ++j) {
        const flt4 z = acc[c][j] * oscale;
        *(flt4*)(C + idx + 4 * j) = z;
        if (dots) {
          const flt4 r = *(const flt4*)(g.dr + (long long)bo * g.sCb + idx + 4 * j);
          const flt4 qv = g.dq ? *(const flt4*)(g.dq + (long long)bo * g.sCb + idx + 4 * j)
                               : flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double zd = z[e], rd = r[e], qd = qv[e];
            dacc[0] += rd * zd;
            dacc[1] += qd * zd;
            dacc[2] += zd;
            dacc[3] += rd;
            dacc[4] += qd;
          }
        }
      }
    } else {
      // 16-bit results go through the block's staging tile (below): a wave holds
      // only 32 or 64 bytes of each row, the block a whole run of BN columns.
      const int r = wm * WM + 16 * c + l16;
#pragma unroll
      for (int h = 0; h < TND / 2; ++h) {  // eight columns per 16-byte vector
        u32x4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          w[e] = (uint32_t)cvt_out<TO, F16>(acc[c][2 * h + (e >> 1)][2 * (e & 1)] * oscale) |
                 ((uint32_t)cvt_out<TO, F16>(acc[c][2 * h + (e >> 1)][2 * (e & 1) + 1] * oscale) << 16);
        *(u32x4*)(stg + r * SLD + wn * WN + 4 * TND * kg + 8 * h) = w;
      }
    }
  }
  if constexpr (!DOTS) {
    // Whole rows of the block tile: BN / 8 vectors per row, each a 16-byte
    // store; four or more consecutive lanes cover one row segment of BN
    // columns (whole cache lines).
    __syncthreads();
    constexpr int VPR = BN / 8, ROWS = 256 / VPR;
    const int vr = tid / VPR, vc = (tid - (tid / VPR) * VPR) * 8;
    const long long col_b = (long long)(n0 / g.om.nd) * g.om.sn1 + (n0 - (n0 / g.om.nd) * g.om.nd) +
                            (long long)bi * g.om.sb + vc;
#pragma unroll
    for (int r = vr; r < BM; r += ROWS)
      *(u32x4*)(C + (long long)(m0 + r) * g.om.sm + col_b) = *(const u32x4*)(stg + r * SLD + vc);
  }
  if constexpr (DOTS) {
    if (dots) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double x = dacc[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[v * 4 + wid] = x;
      }
      __syncthreads();
      if (tid < 5) {
        const int G = gridDim.x;
        g.dpart[((long long)bo * 5 + tid) * G + blockIdx.x] =
            (red[tid * 4 + 0] + red[tid * 4 + 1]) + (red[tid * 4 + 2] + red[tid * 4 + 3]);
      }
    }
  }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Tile configurations (block rows x block columns [x K tile for 16-bit]).  The
// autotuner times them per stage; without tuning a size heuristic picks one.
constexpr int kCfg64[kTiles64][2] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}};
// 16-bit: {BM, BN, BK, kernel}: kernel 0 streams both operands (k_gemm_16),
// 1 builds the circulant operand in LDS (k_gemm_16c), 2 streams the data
// operand per wave (k_gemm_16w; BK is the number of 16-row circulant
// fragments per wave, so the block has BM / (16 BK) waves along its rows and
// the rest of its four waves along its columns).
constexpr int kCfg16[kTiles16][4] = {{64, 64, 64, 0},  {128, 64, 64, 0},   {64, 128, 64, 0},
                                     {128, 128, 64, 0}, {128, 128, 32, 0},  {64, 128, 32, 0},
                                     {64, 128, 64, 1},  {128, 128, 64, 1},  {128, 128, 32, 1},
                                     {32, 64, 32, 1},   {128, 128, 8, 2},   {256, 64, 8, 2},
                                     {128, 128, 128, 1}, {64, 128, 128, 1}, {256, 64, 64, 1},
                                     {256, 64, 128, 1},  {96, 64, 32, 1},   {96, 128, 32, 1}};

int heuristic64(const GemmArgs& g) {
  return (long long)g.M * g.Nn >= 256LL * 128 * 128 ? 3 : 0;
}

// Large problems: 256 x 64 x 128 with the circulant operand in LDS (else
// 128 x 128 x 64, else that tile streamed) in the XCD-grouped order, the
// fastest on the N = 256 stages when measured; small ones: 64 x 64.
int heuristic16(const GemmArgs& g, int batch) {
  if ((long long)g.M * g.Nn * batch >= 128LL * 128 * 256) return 15 + kTiles16;
  return 0;
}

template <int BM, int BN>
void launch64(kp_context* ctx, const GemmArgs& g, int batch, int stage) {
  dim3 grid(((g.Nn + BN - 1) / BN) * ((g.M + BM - 1) / BM), 1, batch);
  if (stage == 0) hipLaunchKernelGGL((k_gemm_f64<0, BM, BN>), grid, dim3(256), 0, ctx->stream, g);
  else if (stage == 1) hipLaunchKernelGGL((k_gemm_f64<1, BM, BN>), grid, dim3(256), 0, ctx->stream, g);
  else hipLaunchKernelGGL((k_gemm_f64<2, BM, BN>), grid, dim3(256), 0, ctx->stream, g);
}

// cfg = tile + kTiles64 * order; out of range: size heuristic, order 0.
int run_gemm_f64(kp_context* ctx, GemmArgs g, int batch, int cfg, int stage) {
  if (cfg < 0 || cfg >= 2 * kTiles64) cfg = heuristic64(g);
  g.order = cfg / kTiles64;
  switch (cfg % kTiles64) {
    case 0: launch64<64, 64>(ctx, g, batch, stage); break;
    case 1: launch64<128, 64>(ctx, g, batch, stage); break;
    case 2: launch64<64, 128>(ctx, g, batch, stage); break;
    default: launch64<128, 128>(ctx, g, batch, stage); break;
  }
  KP_HIP(hipGetLastError());
  return KP_OK;
}

// KIND: both operands streamed (k_gemm_16), the circulant operand built in
// LDS (k_gemm_16c) or the data operand streamed per wave (k_gemm_16w).
template <int STAGE, int BM, int BN, int BK, int KIND, typename TO>
void launch16(kp_context* ctx, const GemmArgs& g, int batch, bool f16) {
  dim3 grid(((g.Nn + BN - 1) / BN) * ((g.M + BM - 1) / BM), 1, batch);
  if constexpr (KIND == 2) {  // BK: circulant fragments per wave (TMC); wave tile 16 TMC x (1024 / TMC / 4 waves)
    constexpr int TMC = BK, WM = 16 * TMC, WAVES_M = BM / WM, TND = BN * WAVES_M / 64;
    static_assert(WAVES_M >= 1 && 4 % WAVES_M == 0 && TND >= 2, "wave tile");
    const int nbuf = (g.cmode == 2 && g.K > g.cn) ? 2 : 1;
    const size_t shm = (size_t)nbuf * 16 * (g.cn + 8) * sizeof(bf16_t);
    if (f16) hipLaunchKernelGGL((k_gemm_16w<STAGE, TMC, TND, WAVES_M, true, TO>), grid, dim3(256), shm, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16w<STAGE, TMC, TND, WAVES_M, false, TO>), grid, dim3(256), shm, ctx->stream, g);
  } else if constexpr (KIND == 1) {
    const size_t shm = (size_t)16 * (g.cn + 8) * sizeof(bf16_t);
    if (f16) hipLaunchKernelGGL((k_gemm_16c<STAGE, BM, BN, BK, true, TO>), grid, dim3(256), shm, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16c<STAGE, BM, BN, BK, false, TO>), grid, dim3(256), shm, ctx->stream, g);
  } else if (g.a_lo) {
    if (f16) hipLaunchKernelGGL((k_gemm_16<STAGE, BM, BN, BK, true, true, TO>), grid, dim3(256), 0, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16<STAGE, BM, BN, BK, false, true, TO>), grid, dim3(256), 0, ctx->stream, g);
  } else {
    if (f16) hipLaunchKernelGGL((k_gemm_16<STAGE, BM, BN, BK, true, false, TO>), grid, dim3(256), 0, ctx->stream, g);
    else hipLaunchKernelGGL((k_gemm_16<STAGE, BM, BN, BK, false, false, TO>), grid, dim3(256), 0, ctx->stream, g);
  }
}

// 16-byte operand loads are legal: K, strides and planes in multiples of 8
// elements, 16-byte aligned bases.
int vec_ok(const GemmArgs& g) {
  return (g.K % 8 == 0) && (g.lda % 8 == 0) && (g.ldb % 8 == 0) && (g.sAb % 8 == 0) && (g.sBb % 8 == 0) &&
         (g.a_lo % 8 == 0) && aligned16(g.A) && aligned16(g.B);
}

// Can k_gemm_16c run this product with tile BM x BN x BK?  Every tile
// interior, the circulant operand available (hi + lo), N a multiple of 8 and
// of BK, and for row-indexed circulants (cmode 0) the row tiles inside one.
bool circ_ok(const GemmArgs& g, int BM, int BN, int BK) {
  return g.circ && g.a_lo && vec_ok(g) && g.cn % 8 == 0 && g.cn % BK == 0 && g.M % BM == 0 &&
         g.Nn % BN == 0 && g.K % BK == 0 && (g.cmode != 0 || g.cn % BM == 0) &&
         (g.cmode == 0 || g.M == g.cn);
}
// Can k_gemm_16w run it with block tile BM x BN?  As circ_ok, plus N a
// multiple of 256 (eight K steps per ring turn inside one circulant), K whole
// circulants, every block's BN columns inside one contiguous output run, and
// 16-byte aligned runs of eight columns in the output (and in r, q for the
// fused dot products).
bool wave_ok(const GemmArgs& g, int BM, int BN) {
  const bool out = g.om.sn2 == 1 && (g.om.nd == INT_MAX || g.om.nd % BN == 0) && g.om.sm % 8 == 0 && g.om.sn1 % 8 == 0 &&
                   g.om.sb % 8 == 0 && g.sCb % 8 == 0 && aligned16(g.C);
  const bool dots = !g.dpart || (aligned16(g.dr) && (!g.dq || aligned16(g.dq)));
  return g.circ && g.a_lo && vec_ok(g) && g.cn % 256 == 0 && g.M % BM == 0 && g.Nn % BN == 0 &&
         g.K % g.cn == 0 && (g.cmode != 0 || g.cn % BM == 0) && (g.cmode == 0 || g.M == g.cn) &&
         (g.cmode == 2 || g.K == g.cn) && out && dots;
}
bool tile_ok(const GemmArgs& g, int t) {
  if (kCfg16[t][3] == 2) return wave_ok(g, kCfg16[t][0], kCfg16[t][1]);
  if (kCfg16[t][3] == 1) return circ_ok(g, kCfg16[t][0], kCfg16[t][1], kCfg16[t][2]);
  return true;
}
// The tile configuration a 16-bit launch uses: cfg = tile + kTiles16 * order
// (out of range: the size heuristic); a tile whose kernel cannot run this
// product becomes the nearest one that can (circulant in LDS, else streamed).
int resolve16(const GemmArgs& g, int batch, int cfg, int* order) {
  if (cfg < 0 || cfg >= 2 * kTiles16) cfg = heuristic16(g, batch);
  *order = cfg / kTiles16;
  int t = cfg % kTiles16;
  if (!tile_ok(g, t) && kCfg16[t][3] == 2) t = 7;
  if (!tile_ok(g, t) && t >= 12) t = t == 13 ? 6 : 7;
  if (!tile_ok(g, t)) t = t == 9 ? 0 : (t == 8 ? 4 : (t == 7 ? 3 : 2));
  return t;
}

// Blocks per system of a 16-bit launch.
int blocks16(const GemmArgs& g, int batch, int cfg) {
  int order;
  const int t = resolve16(g, batch, cfg, &order);
  return ((g.Nn + kCfg16[t][1] - 1) / kCfg16[t][1]) * ((g.M + kCfg16[t][0] - 1) / kCfg16[t][0]);
}

// cfg = tile + kTiles16 * order; out of range: size heuristic, order 0.
// Stages 0 and 1 write 16-bit intermediates, stage 2 the float result.
template <int STAGE, typename TO>
int run_gemm_16(kp_context* ctx, GemmArgs g, int batch, bool f16, int cfg) {
  g.vec = vec_ok(g);
  const int t = resolve16(g, batch, cfg, &g.order);
  switch (t) {
    case 0: launch16<STAGE, 64, 64, 64, 0, TO>(ctx, g, batch, f16); break;
    case 1: launch16<STAGE, 128, 64, 64, 0, TO>(ctx, g, batch, f16); break;
    case 2: launch16<STAGE, 64, 128, 64, 0, TO>(ctx, g, batch, f16); break;
    case 3: launch16<STAGE, 128, 128, 64, 0, TO>(ctx, g, batch, f16); break;
    case 4: launch16<STAGE, 128, 128, 32, 0, TO>(ctx, g, batch, f16); break;
    case 5: launch16<STAGE, 64, 128, 32, 0, TO>(ctx, g, batch, f16); break;
    case 6: launch16<STAGE, 64, 128, 64, 1, TO>(ctx, g, batch, f16); break;
    case 7: launch16<STAGE, 128, 128, 64, 1, TO>(ctx, g, batch, f16); break;
    case 8: launch16<STAGE, 128, 128, 32, 1, TO>(ctx, g, batch, f16); break;
    case 9: launch16<STAGE, 32, 64, 32, 1, TO>(ctx, g, batch, f16); break;
    case 10: launch16<STAGE, 128, 128, 8, 2, TO>(ctx, g, batch, f16); break;
    case 11: launch16<STAGE, 256, 64, 8, 2, TO>(ctx, g, batch, f16); break;
    case 12: launch16<STAGE, 128, 128, 128, 1, TO>(ctx, g, batch, f16); break;
    case 13: launch16<STAGE, 64, 128, 128, 1, TO>(ctx, g, batch, f16); break;
    case 14: launch16<STAGE, 256, 64, 64, 1, TO>(ctx, g, batch, f16); break;
    case 15: launch16<STAGE, 256, 64, 128, 1, TO>(ctx, g, batch, f16); break;
    case 16: launch16<STAGE, 96, 64, 32, 1, TO>(ctx, g, batch, f16); break;
    default: launch16<STAGE, 96, 128, 32, 1, TO>(ctx, g, batch, f16); break;
  }
  KP_HIP(hipGetLastError());
  return KP_OK;
}

// The three stages for a batch of nsys systems.  `planes` = 2 when each
// circulant row holds (hi | lo).  x: nsys inputs (stride N^3), T and U: nsys
// intermediates (stride R N^3), z: nsys outputs (stride N^3); s (nullable):
// per-system done flags and, with `scaled`, the divisors x16_scale.
struct Stages {
  GemmArgs s1, s2, s3;
  int nsys, R;
  int dim = 3;  // 2: no stage (i)
};

Stages make_stages(int N, int R, const void* x, const void* a1, const void* c2, const void* b3,
                   void* T, void* U, void* z, int planes, const Scalars* s, bool scaled, int nsys,
                   const bf16_t* const* circ = nullptr) {
  const long long n = N, nn = n * n, n3 = nn * n, RN = (long long)R * N;
  const long long p = planes;
  const long long lo_n = planes == 2 ? n : 0, lo_rn = planes == 2 ? RN : 0;
  const int* done = s ? &s->done : nullptr;
  const double* div = (s && scaled) ? &s->x16_scale : nullptr;
  Stages st;
  st.nsys = nsys;
  st.R = R;
  // (i) rows (k,j3), cols (i1,i2), K = i3; addr = m*N^2 + n = T[k][j3][i1][i2].
  st.s1 = gemm_args(b3, x, T, RN, nn, n, p * n, n, 0, n3, OutMap{nn, 0, 1, 0, INT_MAX}, done, lo_n,
                    nullptr, 1, R * n3);
  // (ii) batch (system, k): rows j2, cols (j3,i1), K = i2; addr = j2*R*N^2 + j3*R*N + k*N + i1.
  st.s2 = gemm_args(c2, T, U, n, nn, n, p * n, n, p * nn, n3, OutMap{RN * n, RN, 1, n, N}, done, lo_n,
                    nullptr, R, R * n3);
  // (iii) rows j1, cols (j2,j3), K = (k,i1); natural row-major output.
  st.s3 = gemm_args(a1, U, z, n, nn, RN, p * RN, RN, 0, R * n3, OutMap{nn, 0, 1, 0, INT_MAX}, done,
                    lo_rn, div, 1, n3);
  if (circ) {  // the same operands by their first columns: C3 (rows), C2 (batch), C1 (K)
    st.s1.circ = circ[2];
    st.s1.cmode = 0;
    st.s2.circ = circ[1];
    st.s2.cmode = 1;
    st.s3.circ = circ[0];
    st.s3.cmode = 2;
    st.s1.cn = st.s2.cn = st.s3.cn = N;
  }
  return st;
}

// d = 2 (eq. Lap2DtimesX): Z = sum_k C1^k X (C2^k)^T as stages (ii) and (iii)
// of the 3D product without the i3 mode, one system:
//   (ii)  T[j2][(k,i1)] = sum_i2     C2^k[j2][i2] X[i1][i2]   (batch k, X shared)
//   (iii) Z[j1][j2]     = sum_(k,i1) C1^k[j1][i1] T[j2][(k,i1)]
Stages make_stages_2d(int N, int R, const void* x, const void* a1, const void* c2, void* T, void* z,
                      int planes, const Scalars* s, bool scaled, const bf16_t* const* circ = nullptr) {
  const long long n = N, nn = n * n, RN = (long long)R * N;
  const long long p = planes;
  const long long lo_n = planes == 2 ? n : 0, lo_rn = planes == 2 ? RN : 0;
  const int* done = s ? &s->done : nullptr;
  const double* div = (s && scaled) ? &s->x16_scale : nullptr;
  Stages st;
  st.nsys = 1;
  st.R = R;
  st.dim = 2;
  st.s2 = gemm_args(c2, x, T, n, n, n, p * n, n, p * nn, 0, OutMap{RN, 0, 1, n, INT_MAX}, done, lo_n,
                    nullptr, R, R * nn);
  st.s3 = gemm_args(a1, T, z, n, n, RN, p * RN, RN, 0, R * nn, OutMap{n, 0, 1, 0, INT_MAX}, done,
                    lo_rn, div, 1, nn);
  if (circ) {
    st.s2.circ = circ[1];
    st.s2.cmode = 1;
    st.s3.circ = circ[0];
    st.s3.cmode = 2;
    st.s2.cn = st.s3.cn = N;
  }
  return st;
}

template <typename F>
int run_stages(kp_context* ctx, const Stages& st, const int* tiles, F&& run) {
  if (st.dim == 3) {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE3);
    KP_TRY(run(0, st.s1, st.nsys, tiles[0]));
  }
  {
    ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE2);
    KP_TRY(run(1, st.s2, st.nsys * st.R, tiles[1]));
  }
  ScopedTimer tm(ctx, KP_TIMER_GEMM_MODE1);
  return run(2, st.s3, st.nsys, tiles[2]);
}

}  // namespace

int launch_precond_f64(kp_context* ctx, const kp_precond* pc, const double* x, double* z,
                       const Scalars* s, const Batch& bt, void* T, void* U, const int* tiles) {
  if (pc->fft) {
    if (bt.nsys != 1) return fail(KP_ERR_STATE, "the FFT preconditioner applies to one system at a time");
    return launch_precond_fft(ctx, pc, x, z);
  }
  const size_t n3 = unknowns(pc->N, pc->dim);
  if (!T) KP_TRY(ws_get(ctx, WS_T, n3 * pc->R * sizeof(double), &T));
  if (!U && pc->dim == 3) KP_TRY(ws_get(ctx, WS_U, n3 * pc->R * sizeof(double), &U));
  if (pc->dim == 2 && bt.nsys != 1) return fail(KP_ERR_STATE, "2D preconditioner: one system at a time");
  Stages st = pc->dim == 2 ? make_stages_2d(pc->N, pc->R, x, pc->a1_64, pc->c2_64, T, z, 1, s, false)
                           : make_stages(pc->N, pc->R, x, pc->a1_64, pc->c2_64, pc->b3_64, T, U, z, 1, s,
                                         false, bt.nsys);
  return run_stages(ctx, st, tiles ? tiles : pc->tile,
                    [&](int stage, const GemmArgs& g, int batch, int cfg) {
                      return run_gemm_f64(ctx, g, batch, cfg, stage);
                    });
}

int launch_precond_16(kp_context* ctx, const kp_precond* pc, const bf16_t* x, float* z,
                      const Scalars* s, const Batch& bt, void* T, void* U, const int* tiles,
                      const PrecDots* dots, int* dot_parts) {
  const size_t n3 = unknowns(pc->N, pc->dim);
  const bool f16 = pc->precision == KP_MIXED_FP16;
  if (!T) KP_TRY(ws_get(ctx, WS_T, n3 * pc->R * sizeof(bf16_t), &T));
  if (!U && pc->dim == 3) KP_TRY(ws_get(ctx, WS_U, n3 * pc->R * sizeof(bf16_t), &U));
  if (pc->dim == 2 && bt.nsys != 1) return fail(KP_ERR_STATE, "2D preconditioner: one system at a time");
  Stages st = pc->dim == 2 ? make_stages_2d(pc->N, pc->R, x, pc->a1_16, pc->c2_16, T, z, 2, s, true, pc->circ16)
                           : make_stages(pc->N, pc->R, x, pc->a1_16, pc->c2_16, pc->b3_16, T, U, z, 2, s,
                                         true, bt.nsys, pc->circ16);
  if (!tiles) tiles = pc->tile;
  if (dot_parts) *dot_parts = 0;
  if (dots) {
    st.s3.vec = vec_ok(st.s3);
    const int G = blocks16(st.s3, bt.nsys, tiles[2]);
    if ((size_t)5 * G <= dots->cap) {  // else the caller reduces z itself
      st.s3.dr = dots->r;
      st.s3.dq = dots->q;
      st.s3.dpart = dots->part;
      *dot_parts = G;
    }
  }
  return run_stages(ctx, st, tiles, [&](int stage, const GemmArgs& g, int batch, int cfg) {
    if (stage == 0) return run_gemm_16<0, bf16_t>(ctx, g, batch, f16, cfg);
    if (stage == 1) return run_gemm_16<1, bf16_t>(ctx, g, batch, f16, cfg);
    return run_gemm_16<2, float>(ctx, g, batch, f16, cfg);
  });
}

// Times every tile configuration of every stage (`reps` launches each, after
// one warm-up launch) for a batch of nsys systems and keeps the fastest per
// stage in tiles[].  The stages are tuned in order and every timed launch of
// stage s > first follows an untimed launch of stage s - 1 with its chosen
// tiles, as in an apply: the candidate then finds its input operand where the
// previous stage left it in the caches.  Before that, the intermediates T and
// U (2 R N^3 values, more than the 256 MB last-level cache at N = 256) are
// overwritten with zeros, so that the rest of the candidate's operands are no
// warmer than in a solve, where about a gigabyte of vector traffic separates
// two applies (the values do not matter: the scratch is zero-filled).  Scratch: T, U (nsys R N^3 elements each), X (nsys N^3
// inputs), Z (nsys N^3 outputs); all NULL: the context workspace (nsys = 1).
// T, U and X are zero-filled first.
int autotune_precond(kp_context* ctx, kp_precond* pc, int nsys, int reps, kp_tile_timing* table,
                     int cap, int* count, int* tiles, void* T, void* U, void* X, void* Z) {
  if (pc->fft) {  // no GEMM tiles to choose
    if (count) *count = 0;
    return KP_OK;
  }
  const size_t n3 = unknowns(pc->N, pc->dim);
  const bool sixteen = pc->precision != KP_FP64;
  const size_t el = sixteen ? sizeof(bf16_t) : sizeof(double);
  if (nsys < 1 || ((!T || !U || !X || !Z) && nsys != 1)) return fail(KP_ERR_ARG, "autotune: bad batch");
  if (pc->dim == 2 && nsys != 1) return fail(KP_ERR_STATE, "autotune: 2D preconditioners tune one system");
  if (!T) KP_TRY(ws_get(ctx, WS_T, n3 * pc->R * el, &T));
  if (!U) KP_TRY(ws_get(ctx, WS_U, n3 * pc->R * el, &U));
  if (!X) KP_TRY(ws_get(ctx, sixteen ? WS_X16 : WS_TMP64, n3 * el, &X));
  if (!Z) KP_TRY(ws_get(ctx, WS_TMP64B, n3 * sizeof(double), &Z));
  KP_HIP(hipMemsetAsync(T, 0, nsys * n3 * pc->R * el, ctx->stream));
  KP_HIP(hipMemsetAsync(U, 0, nsys * n3 * pc->R * el, ctx->stream));
  KP_HIP(hipMemsetAsync(X, 0, nsys * n3 * el, ctx->stream));
  Stages st;
  if (pc->dim == 2)
    st = sixteen ? make_stages_2d(pc->N, pc->R, X, pc->a1_16, pc->c2_16, T, Z, 2, nullptr, false, pc->circ16)
                 : make_stages_2d(pc->N, pc->R, X, pc->a1_64, pc->c2_64, T, Z, 1, nullptr, false);
  else
    st = sixteen ? make_stages(pc->N, pc->R, X, pc->a1_16, pc->c2_16, pc->b3_16, T, U, Z, 2, nullptr,
                               false, nsys, pc->circ16)
                 : make_stages(pc->N, pc->R, X, pc->a1_64, pc->c2_64, pc->b3_64, T, U, Z, 1, nullptr,
                               false, nsys);
  const bool f16 = pc->precision == KP_MIXED_FP16;
  const int ntile = sixteen ? kTiles16 : kTiles64, ncfg = 2 * ntile;
  // 16-bit: stage (iii) is timed with the fused dot products it carries in the
  // solvers (scratch r, q of zeros and a partials buffer), so the choice
  // includes the cost of its epilogue.
  void *dr = nullptr, *dq = nullptr, *dpart = nullptr;
  const size_t dcap = (size_t)5 * nsys * 65536;
  struct Scratch {
    kp_context* ctx;
    void** p[3];
    ~Scratch() {
      for (void** q : p)
        if (*q) dev_free(ctx, *q);
    }
  } scratch{ctx, {&dr, &dq, &dpart}};
  if (sixteen) {
    KP_TRY(dev_alloc(ctx, &dr, nsys * n3 * sizeof(float)));
    KP_TRY(dev_alloc(ctx, &dq, nsys * n3 * sizeof(float)));
    KP_TRY(dev_alloc(ctx, &dpart, dcap * sizeof(double)));
    KP_HIP(hipMemsetAsync(dr, 0, nsys * n3 * sizeof(float), ctx->stream));
    KP_HIP(hipMemsetAsync(dq, 0, nsys * n3 * sizeof(float), ctx->stream));
  }
  struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } evs;
  evs.ev.reserve(2 * (size_t)reps);
  for (int r = 0; r < 2 * reps; ++r) {
    hipEvent_t e;
    KP_HIP(hipEventCreate(&e));
    evs.ev.push_back(e);
  }
  const int first = pc->dim == 2 ? 1 : 0;
  int n = 0;
  for (int stg = first; stg < 3; ++stg) {
    const GemmArgs& g = stg == 0 ? st.s1 : (stg == 1 ? st.s2 : st.s3);
    const int batch = stg == 1 ? nsys * pc->R : nsys;
    auto run_prev = [&]() -> int {
      if (stg == first) return KP_OK;
      const GemmArgs& gp = stg == 1 ? st.s1 : st.s2;
      const int bp = stg == 2 ? nsys * pc->R : nsys;
      if (!sixteen) return run_gemm_f64(ctx, gp, bp, tiles[stg - 1], stg - 1);
      if (stg == 1) return run_gemm_16<0, bf16_t>(ctx, gp, bp, f16, tiles[0]);
      return run_gemm_16<1, bf16_t>(ctx, gp, bp, f16, tiles[1]);
    };
    double best = 1e300;
    int best_cfg = -1;
    std::vector<double> times(ncfg, 1e300);
    for (int c = 0; c < ncfg; ++c) {
      GemmArgs gd = g;
      if (sixteen && stg == 2) {
        gd.vec = vec_ok(gd);
        if ((size_t)5 * nsys * blocks16(gd, batch, c) <= dcap) {
          gd.dr = (const float*)dr;
          gd.dq = (const float*)dq;
          gd.dpart = (double*)dpart;
        }
      }
      auto run = [&]() -> int {
        if (!sixteen) return run_gemm_f64(ctx, g, batch, c, stg);
        if (stg == 0) return run_gemm_16<0, bf16_t>(ctx, g, batch, f16, c);
        if (stg == 1) return run_gemm_16<1, bf16_t>(ctx, g, batch, f16, c);
        return run_gemm_16<2, float>(ctx, gd, batch, f16, c);
      };
      const size_t inter = nsys * n3 * pc->R * el;
      KP_TRY(run_prev());
      KP_TRY(run());
      for (int r = 0; r < reps; ++r) {
        KP_HIP(hipMemsetAsync(T, 0, inter, ctx->stream));
        if (pc->dim == 3) KP_HIP(hipMemsetAsync(U, 0, inter, ctx->stream));
        KP_TRY(run_prev());
        KP_HIP(hipEventRecord(evs.ev[2 * r], ctx->stream));
        KP_TRY(run());
        KP_HIP(hipEventRecord(evs.ev[2 * r + 1], ctx->stream));
      }
      KP_HIP(hipEventSynchronize(evs.ev[2 * reps - 1]));
      double tot = 0.0;
      for (int r = 0; r < reps; ++r) {
        float ms = 0.f;
        KP_HIP(hipEventElapsedTime(&ms, evs.ev[2 * r], evs.ev[2 * r + 1]));
        tot += ms;
      }
      const double avg = tot / reps;
      if (table && n < cap) {
        kp_tile_timing& e = table[n];
        e.stage = stg;
        // the tile that ran: a configuration whose kernel cannot run this
        // product falls back to another (resolve16)
        int ord = c / ntile;
        const int t = sixteen ? resolve16(g, batch, c, &ord) : c % ntile;
        e.bm = sixteen ? kCfg16[t][0] : kCfg64[t][0];
        e.bn = sixteen ? kCfg16[t][1] : kCfg64[t][1];
        e.bk = sixteen ? kCfg16[t][2] : 16;
        e.circ = sixteen ? kCfg16[t][3] : 0;
        e.order = ord;
        e.ms = avg;
      }
      ++n;
      times[c] = avg;
      if (avg < best) {
        best = avg;
        best_cfg = c;
      }
    }
    // The two block orders of one tile shape within 3 % of each other (about
    // the spread of repeated tunings): take the XCD-grouped one, which reads
    // each column tile of the data operand from HBM once instead of once per
    // row tile.
    if (best_cfg >= 0 && best_cfg < ntile && times[best_cfg + ntile] <= 1.03 * best) best_cfg += ntile;
    tiles[stg] = best_cfg;
  }
  if (count) *count = n;
  return KP_OK;
}

}  // namespace kp

// Assembly of the Kronecker-sum stiffness and the 7-point stencil matvec.
//
// Stiffness (Section 3.3, eq. As_Kron_d): each unit cell c contributes a_c times
// the 1D Neumann Laplacian of its n0+1 nodes in one direction and the lumped
// half-weight identity diag(1/2,1,...,1,1/2) in the two others, wrapped modulo N
// (the periodization term).  Summed over cells, the weight of the grid edge
// (p, p+e_l) is the mean of the coefficient over the four voxels that share the
// edge, and the matrix acts as the 7-point stencil
//   (K u)(p) = sum_l w_l(p) (u_p - u_{p+e_l}) + w_l(p-e_l) (u_p - u_{p-e_l}).
// The corrector right-hand sides (eq. FEM_discr_RHS, integrated by parts) are
// f_l(p) = h (w_l(p) - w_l(p-e_l)) for K = A / h.
//
// Both kernels read the C-order [i1][i2][i3] layout with i3 fastest.

#include <cmath>

#include "kp_internal.h"

namespace kp {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block of 256 threads: deterministic sum written by thread 0 into *out.
__device__ __forceinline__ void block_sum_store(double v, double* out) {
  __shared__ double red[4];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// One thread per node; the eight voxels around node p are v = p - 1 + d, d in {0,1}^3.
// A voxel takes its cell's value when its local coordinates v mod n0 all lie in
// [lo, hi) (the centred sub-cell; lo = 0, hi = n0 for whole cells), else bg.
__global__ __launch_bounds__(256) void k_assemble(const double* __restrict__ cells, int L, int n0,
                                                  int lo, int hi, double bg, int N, double h,
                                                  double* __restrict__ w64, double* __restrict__ f) {
  const size_t n3 = (size_t)N * N * N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n3) return;
  const int p3 = (int)(idx % N);
  const int p2 = (int)((idx / N) % N);
  const int p1 = (int)(idx / ((size_t)N * N));
  int c1[2], c2[2], c3[2];
  bool in1[2], in2[2], in3[2];
  const int v1[2] = {(p1 + N - 1) % N, p1}, v2[2] = {(p2 + N - 1) % N, p2}, v3[2] = {(p3 + N - 1) % N, p3};
  for (int d = 0; d < 2; ++d) {
    c1[d] = v1[d] / n0;
    c2[d] = v2[d] / n0;
    c3[d] = v3[d] / n0;
    const int l1 = v1[d] - c1[d] * n0, l2 = v2[d] - c2[d] * n0, l3 = v3[d] - c3[d] * n0;
    in1[d] = l1 >= lo && l1 < hi;
    in2[d] = l2 >= lo && l2 < hi;
    in3[d] = l3 >= lo && l3 < hi;
  }
  double a[2][2][2];
  for (int d1 = 0; d1 < 2; ++d1)
    for (int d2 = 0; d2 < 2; ++d2)
      for (int d3 = 0; d3 < 2; ++d3)
        a[d1][d2][d3] = (in1[d1] && in2[d2] && in3[d3]) ? cells[((size_t)c1[d1] * L + c2[d2]) * L + c3[d3]] : bg;
  // Edge (p, p+e_l): voxel layer p_l along l, p_t - 1 or p_t across.
  const double w0 = (((a[1][1][1] + a[1][0][1]) + a[1][1][0]) + a[1][0][0]) / 4.0;
  const double w0m = (((a[0][1][1] + a[0][0][1]) + a[0][1][0]) + a[0][0][0]) / 4.0;
  const double w1 = (((a[1][1][1] + a[0][1][1]) + a[1][1][0]) + a[0][1][0]) / 4.0;
  const double w1m = (((a[1][0][1] + a[0][0][1]) + a[1][0][0]) + a[0][0][0]) / 4.0;
  const double w2 = (((a[1][1][1] + a[0][1][1]) + a[1][0][1]) + a[0][0][1]) / 4.0;
  const double w2m = (((a[1][1][0] + a[0][1][0]) + a[1][0][0]) + a[0][0][0]) / 4.0;
  w64[idx] = w0;
  w64[n3 + idx] = w1;
  w64[2 * n3 + idx] = w2;
  f[idx] = h * (w0 - w0m);
  f[n3 + idx] = h * (w1 - w1m);
  f[2 * n3 + idx] = h * (w2 - w2m);
}

// d = 2: one thread per node [i1][i2]; the four voxels around p are
// v = p - 1 + d, d in {0,1}^2, and the weight of the edge (p, p + e_l) is the
// mean of the two voxels in layer p_l along l (transverse p_t - 1 or p_t).
__global__ __launch_bounds__(256) void k_assemble2d(const double* __restrict__ cells, int L, int n0,
                                                    int lo, int hi, double bg, int N, double h,
                                                    double* __restrict__ w64, double* __restrict__ f) {
  const size_t n2 = (size_t)N * N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n2) return;
  const int p2 = (int)(idx % N), p1 = (int)(idx / N);
  const int v1[2] = {(p1 + N - 1) % N, p1}, v2[2] = {(p2 + N - 1) % N, p2};
  double a[2][2];
  for (int d1 = 0; d1 < 2; ++d1)
    for (int d2 = 0; d2 < 2; ++d2) {
      const int c1 = v1[d1] / n0, c2 = v2[d2] / n0;
      const int l1 = v1[d1] - c1 * n0, l2 = v2[d2] - c2 * n0;
      const bool in = l1 >= lo && l1 < hi && l2 >= lo && l2 < hi;
      a[d1][d2] = in ? cells[(size_t)c1 * L + c2] : bg;
    }
  const double w0 = (a[1][0] + a[1][1]) / 2.0, w0m = (a[0][0] + a[0][1]) / 2.0;
  const double w1 = (a[0][1] + a[1][1]) / 2.0, w1m = (a[0][0] + a[1][0]) / 2.0;
  w64[idx] = w0;
  w64[n2 + idx] = w1;
  f[idx] = h * (w0 - w0m);
  f[n2 + idx] = h * (w1 - w1m);
}

constexpr int kTX = 64;  // i3 extent of a tile (one wavefront)
constexpr int kTY = 4;   // i2 extent of a tile (four wavefronts)

// Coefficient of one realization as the stencil reads it: the L^3 cell values
// [c1][c2][c3] (cell of voxel v: v / n0 per axis) and, for sub-cell
// inclusions, the voxel range [lo, hi) of the sub-cell and the background.
template <typename TC>
struct Cells {
  const TC* a;
  int L, n0, lo, hi;
  TC bg;
  int dim;
};

// 2.5D tiled stencil on the cell values.  The edge weights are not read from
// memory: around node p the eight voxels v = p - 1 + d, d in {0,1}^3, belong to
// cells a[d1][d2][d3], and each of the six weights of p is the mean of the four
// voxels on one side (w_1(p) = mean of a[1][.][.], w_1(p - e_1) of a[0][.][.],
// and so on), summed in the order of the assembly kernel, so that in double
// the weights are those of k_assemble bit for bit.  Along i1 the layer
// a[1][.][.] of plane z is the layer a[0][.][.] of plane z + 1 and changes only
// when z crosses a cell boundary, so a thread loads four cell values once per
// n0 planes (cache hits: the L^3 cells are 64 times smaller than a field).
// Traffic: the field u (with its halo) and the output, two words per node.
//
// A 64 x 4 block of columns (i2, i3) marches along i1 over TZ planes; the i1
// neighbours of u ride in registers, the current plane of u is staged in LDS
// for the in-plane neighbours, and neighbours outside the tile (halo,
// periodic wrap, ragged edges) come from global memory.  MODE 0: out = K u
// and dot = <u, K u>.  MODE 1: out = f - K u and dot = ||f - K u||^2 (true
// residual).  Cell type TC, accumulation type C, output type TO.
// blockIdx.z = system * gz + plane chunk (Batch layout; bt.ws strides the
// cells of successive realizations).  INCL: sub-cell inclusions; the voxel
// values are the cell values where the voxel's plane, row and column all lie
// inside the sub-cell range and the background elsewhere (three per-thread
// masks and one per plane), again summed in the assembly kernel's order.
template <typename TU, typename TC, typename TO, typename C, int MODE, bool INCL>
__global__ __launch_bounds__(256) void k_stencil(const TU* __restrict__ u, Cells<TC> cc,
                                                 const double* __restrict__ f,
                                                 TO* __restrict__ out,
                                                 double* __restrict__ partial,
                                                 const Scalars* __restrict__ s, int gate, int N,
                                                 int TZ, int gz, Batch bt) {
  const int b = blockIdx.z / gz, zc = blockIdx.z - b * gz;
  if (s && !gate_open(s[b], gate)) return;
  u += b * bt.vs;
  out += b * bt.vs;
  if (MODE == 1) f += b * bt.vs;
  const TC* __restrict__ cells = cc.a + (size_t)(b / bt.per) * bt.ws;
  const int L = cc.L, n0 = cc.n0;
  __shared__ TU su[kTY][kTX];
  const int tx = threadIdx.x & (kTX - 1);
  const int ty = threadIdx.x / kTX;
  const int i3 = blockIdx.x * kTX + tx;
  const int i2 = blockIdx.y * kTY + ty;
  const int z0 = zc * TZ;
  const int z1 = min(z0 + TZ, N);
  const bool act = (i3 < N) && (i2 < N);
  const size_t NN = (size_t)N * N;
  const int i2m = (i2 == 0) ? N - 1 : i2 - 1;
  const int i2p = (i2 + 1 >= N) ? 0 : i2 + 1;
  const int i3m = (i3 == 0) ? N - 1 : i3 - 1;
  const int i3p = (i3 + 1 >= N) ? 0 : i3 + 1;
  const size_t col = (size_t)i2 * N + i3;
  // Transverse cell offsets: [d2][d3] -> c2 * L + c3 for d = 0 (p - 1) and 1 (p);
  // with inclusions, whether voxel column [d2][d3] lies in the sub-cell's range.
  int toff[2][2] = {{0, 0}, {0, 0}};
  bool tin[2][2] = {{true, true}, {true, true}};
  if (act) {
    const int c2[2] = {i2m / n0, i2 / n0}, c3[2] = {i3m / n0, i3 / n0};
    const int l2[2] = {i2m - c2[0] * n0, i2 - c2[1] * n0}, l3[2] = {i3m - c3[0] * n0, i3 - c3[1] * n0};
    for (int d2 = 0; d2 < 2; ++d2)
      for (int d3 = 0; d3 < 2; ++d3) {
        toff[d2][d3] = c2[d2] * L + c3[d3];
        tin[d2][d3] = l2[d2] >= cc.lo && l2[d2] < cc.hi && l3[d3] >= cc.lo && l3[d3] < cc.hi;
      }
  }
  auto layer = [&](int c1, C (&a)[2][2]) {
    const size_t base = (size_t)c1 * L * L;
#pragma unroll
    for (int d2 = 0; d2 < 2; ++d2)
#pragma unroll
      for (int d3 = 0; d3 < 2; ++d3) a[d2][d3] = (C)cells[base + toff[d2][d3]];
  };
  double dot = 0.0;
  C um = 0, uc = 0, un = 0;
  C a0[2][2] = {{0, 0}, {0, 0}}, a1[2][2] = {{0, 0}, {0, 0}};
  int cz = z0 / n0, rz = z0 - cz * n0;  // cell layer of plane z and position inside it
  if (act) {
    const int zm = (z0 == 0) ? N - 1 : z0 - 1;
    um = (C)u[zm * NN + col];
    uc = (C)u[z0 * NN + col];
    layer(zm / n0, a0);
    layer(cz, a1);
  }
  for (int z = z0; z < z1; ++z) {
    const size_t base = (size_t)z * NN;
    if (act) {
      const int zp = (z + 1 >= N) ? 0 : z + 1;
      un = (C)u[zp * NN + col];
      su[ty][tx] = (TU)uc;
    }
    __syncthreads();
    if (act) {
      const C u2m = (ty > 0) ? (C)su[ty - 1][tx] : (C)u[base + (size_t)i2m * N + i3];
      const C u2p = (ty + 1 < kTY && i2 + 1 < N) ? (C)su[ty + 1][tx] : (C)u[base + (size_t)i2p * N + i3];
      const C u3m = (tx > 0) ? (C)su[ty][tx - 1] : (C)u[base + (size_t)i2 * N + i3m];
      const C u3p = (tx + 1 < kTX && i3 + 1 < N) ? (C)su[ty][tx + 1] : (C)u[base + (size_t)i2 * N + i3p];
      const C q = (C)0.25;
      C e0[2][2], e1[2][2];  // voxel values of layers z - 1 and z
      if constexpr (INCL) {
        const int r0 = rz == 0 ? n0 - 1 : rz - 1;
        const bool in0 = r0 >= cc.lo && r0 < cc.hi, in1 = rz >= cc.lo && rz < cc.hi;
        const C bg = (C)cc.bg;
#pragma unroll
        for (int d2 = 0; d2 < 2; ++d2)
#pragma unroll
          for (int d3 = 0; d3 < 2; ++d3) {
            e0[d2][d3] = (in0 && tin[d2][d3]) ? a0[d2][d3] : bg;
            e1[d2][d3] = (in1 && tin[d2][d3]) ? a1[d2][d3] : bg;
          }
      } else {
#pragma unroll
        for (int d2 = 0; d2 < 2; ++d2)
#pragma unroll
          for (int d3 = 0; d3 < 2; ++d3) {
            e0[d2][d3] = a0[d2][d3];
            e1[d2][d3] = a1[d2][d3];
          }
      }
      const C w0c = (((e1[1][1] + e1[0][1]) + e1[1][0]) + e1[0][0]) * q;
      const C w0m = (((e0[1][1] + e0[0][1]) + e0[1][0]) + e0[0][0]) * q;
      const C w1c = (((e1[1][1] + e0[1][1]) + e1[1][0]) + e0[1][0]) * q;
      const C w1m = (((e1[0][1] + e0[0][1]) + e1[0][0]) + e0[0][0]) * q;
      const C w2c = (((e1[1][1] + e0[1][1]) + e1[0][1]) + e0[0][1]) * q;
      const C w2m = (((e1[1][0] + e0[1][0]) + e1[0][0]) + e0[0][0]) * q;
      C ku = w0c * (uc - un) + w0m * (uc - um);
      ku += w1c * (uc - u2p) + w1m * (uc - u2m);
      ku += w2c * (uc - u3p) + w2m * (uc - u3m);
      if (MODE == 0) {
        const TO o = (TO)ku;
        out[base + col] = o;
        dot += (double)uc * (double)o;
      } else {
        const double res = f[base + col] - (double)ku;
        out[base + col] = (TO)res;
        dot += res * res;
      }
      // next plane: layer a1 becomes a0; a new layer when z + 1 starts a cell
#pragma unroll
      for (int d2 = 0; d2 < 2; ++d2)
#pragma unroll
        for (int d3 = 0; d3 < 2; ++d3) a0[d2][d3] = a1[d2][d3];
      if (++rz == n0) {
        rz = 0;
        ++cz;
        if (z + 1 < z1) layer(cz, a1);
      }
    }
    __syncthreads();
    um = uc;
    uc = un;
  }
  const size_t nparts = (size_t)gridDim.x * gridDim.y * gz;
  block_sum_store(dot, partial + b * nparts +
                           (blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * zc)));
}

// d = 2: the 5-point stencil on the cell values, one thread per node (the
// neighbours come from L2; the field is N^2, at most 4M nodes), weights as
// in k_assemble2d (bit for bit in double).  blockIdx.y = system.
template <typename TU, typename TC, typename TO, typename C, int MODE, bool INCL>
__global__ __launch_bounds__(256) void k_stencil2d(const TU* __restrict__ u, Cells<TC> cc,
                                                   const double* __restrict__ f, TO* __restrict__ out,
                                                   double* __restrict__ partial, const Scalars* __restrict__ s,
                                                   int gate, int N, Batch bt) {
  const int b = blockIdx.y;
  if (s && !gate_open(s[b], gate)) return;
  u += b * bt.vs;
  out += b * bt.vs;
  if (MODE == 1) f += b * bt.vs;
  const TC* __restrict__ cells = cc.a + (size_t)(b / bt.per) * bt.ws;
  const size_t n2 = (size_t)N * N;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  double dot = 0.0;
  if (idx < n2) {
    const int p2 = (int)(idx % N), p1 = (int)(idx / N);
    const int p1m = p1 == 0 ? N - 1 : p1 - 1, p1p = p1 + 1 == N ? 0 : p1 + 1;
    const int p2m = p2 == 0 ? N - 1 : p2 - 1, p2p = p2 + 1 == N ? 0 : p2 + 1;
    const int n0 = cc.n0;
    const int v1[2] = {p1m, p1}, v2[2] = {p2m, p2};
    C a[2][2];
#pragma unroll
    for (int d1 = 0; d1 < 2; ++d1)
#pragma unroll
      for (int d2 = 0; d2 < 2; ++d2) {
        const int c1 = v1[d1] / n0, c2 = v2[d2] / n0;
        C v = (C)cells[(size_t)c1 * cc.L + c2];
        if constexpr (INCL) {
          const int l1 = v1[d1] - c1 * n0, l2 = v2[d2] - c2 * n0;
          if (!(l1 >= cc.lo && l1 < cc.hi && l2 >= cc.lo && l2 < cc.hi)) v = (C)cc.bg;
        }
        a[d1][d2] = v;
      }
    const C hf = (C)0.5;
    const C w0c = (a[1][0] + a[1][1]) * hf, w0m = (a[0][0] + a[0][1]) * hf;
    const C w1c = (a[0][1] + a[1][1]) * hf, w1m = (a[0][0] + a[1][0]) * hf;
    const C uc = (C)u[idx];
    C ku = w0c * (uc - (C)u[(size_t)p1p * N + p2]) + w0m * (uc - (C)u[(size_t)p1m * N + p2]);
    ku += w1c * (uc - (C)u[(size_t)p1 * N + p2p]) + w1m * (uc - (C)u[(size_t)p1 * N + p2m]);
    if (MODE == 0) {
      const TO o = (TO)ku;
      out[idx] = o;
      dot = (double)uc * (double)o;
    } else {
      const double res = f[idx] - (double)ku;
      out[idx] = (TO)res;
      dot = res * res;
    }
  }
  block_sum_store(dot, partial + (size_t)b * gridDim.x + blockIdx.x);
}

// Row-segment variant for N a multiple of 256 and n0 = 4 (the paper's cell
// size and the benchmark's): a block of 256 threads owns a 256-wide segment of
// i3 and RY consecutive i2 rows (8 for float fields, two cells; 4 for double
// ones, one cell) and marches along i1 over TZ planes; every thread carries one
// i3 position of all RY rows (register queues along i1 as above).  The in-row
// neighbours of plane z come from a double-buffered LDS copy of the block's
// rows (one barrier per plane); only the two segment-edge threads read a
// neighbour from global memory (N > 256), and the only halo rows are the two
// i2 neighbours of the row group, so the field is read about
// (1 + 2/RY + 1/TZ) times, against the 64 x 4 tile's i2 and i3 halos (whose
// single-float column reads fetch whole lines of other tiles).  With n0 = 4
// the RY rows touch RY/4 + 1 cell rows, so a layer of cell values is
// (RY/4 + 1) x 2 registers and a row's voxel rows map to them statically.
// Weights as in k_stencil (bit for bit in double).
constexpr int kRY = 8;

// RY rows per thread: 8 for float fields, 4 for double ones (half the row
// registers, so the double residual keeps more waves per SIMD).
template <typename TU>
constexpr int rows_per_thread() {
  return sizeof(TU) == 8 ? 4 : kRY;
}

// The float kernel without sub-cell masks fits five waves per SIMD in 96
// registers without spilling (30.8 against 31.6 us at N = 256); the other
// variants spill at that bound and keep the default.
template <typename TU, typename TC, typename TO, typename C, int MODE, bool INCL>
__global__ __launch_bounds__(256, (sizeof(TU) == 4 && !INCL) ? 5 : 1) void k_stencil_rows(const TU* __restrict__ u, Cells<TC> cc,
                                                      const double* __restrict__ f,
                                                      TO* __restrict__ out, double* __restrict__ partial,
                                                      const Scalars* __restrict__ s, int gate, int N,
                                                      int TZ, int gz, Batch bt) {
  constexpr int N0 = 4;
  constexpr int RY = rows_per_thread<TU>();
  constexpr int SL = RY / N0 + 1;  // cell rows a layer needs (the row above and RY / 4 own)
  // XCD-aware block order: consecutive hardware blocks go to the eight XCDs in
  // turn, so hardware block h takes logical block (h mod 8) * (nb / 8) + h / 8
  // (nb a multiple of 8): each XCD then works through a contiguous run of row
  // groups and plane chunks, and the halo rows and planes that neighbouring
  // blocks share are fetched once into that XCD's L2.
  const unsigned gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
  unsigned lb = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((nb & 7u) == 0) lb = (lb & 7u) * (nb >> 3) + (lb >> 3);
  const int bx = (int)(lb % gx), by = (int)((lb / gx) % gy), bz = (int)(lb / (gx * gy));
  const int b = bz / gz, zc = bz - b * gz;
  if (s && !gate_open(s[b], gate)) return;
  u += b * bt.vs;
  out += b * bt.vs;
  if (MODE == 1) f += b * bt.vs;
  const TC* __restrict__ cells = cc.a + (size_t)(b / bt.per) * bt.ws;
  const int L = cc.L;
  __shared__ TU su[2][RY][256];
  const int tx = threadIdx.x;
  const int i3 = bx * 256 + tx;
  const int r0 = by * RY;  // first i2 row of the group (a multiple of 4: cell row r0 / 4)
  const int z0 = zc * TZ, z1 = min(z0 + TZ, N);
  const size_t NN = (size_t)N * N;
  const int i3m = i3 == 0 ? N - 1 : i3 - 1, i3p = i3 + 1 == N ? 0 : i3 + 1;
  const int rm = r0 == 0 ? N - 1 : r0 - 1, rp = r0 + RY == N ? 0 : r0 + RY;  // halo rows
  // Cell rows of the group: slot 0 = the cell row above (voxel row r0 - 1), 1.. its own.
  const int cr = r0 / N0;
  int c2L[SL];
  c2L[0] = (cr == 0 ? L - 1 : cr - 1) * L;
#pragma unroll
  for (int k = 1; k < SL; ++k) c2L[k] = (cr + k - 1) * L;
  const int c3[2] = {i3m / N0, i3 / N0};
  const int l3[2] = {i3m - c3[0] * N0, i3 - c3[1] * N0};
  bool in3[2] = {true, true};
  if constexpr (INCL) {
    in3[0] = l3[0] >= cc.lo && l3[0] < cc.hi;
    in3[1] = l3[1] >= cc.lo && l3[1] < cc.hi;
  }
  auto layer = [&](int c1, C (&a)[SL][2]) {
    const size_t base = (size_t)c1 * L * L;
#pragma unroll
    for (int k = 0; k < SL; ++k)
#pragma unroll
      for (int d3 = 0; d3 < 2; ++d3) a[k][d3] = (C)cells[base + c2L[k] + c3[d3]];
  };
  C um[RY], uc[RY], un[RY];
  C a0[SL][2], a1[SL][2];
  int cz = z0 / N0, rz = z0 - cz * N0;
  {
    const int zm = z0 == 0 ? N - 1 : z0 - 1;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      um[r] = (C)u[zm * NN + (size_t)(r0 + r) * N + i3];
      uc[r] = (C)u[z0 * NN + (size_t)(r0 + r) * N + i3];
    }
    layer(zm / N0, a0);
    layer(cz, a1);
  }
  double dot = 0.0;
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    const size_t base = (size_t)z * NN;
    const int zp = z + 1 >= N ? 0 : z + 1;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      un[r] = (C)u[zp * NN + (size_t)(r0 + r) * N + i3];
      su[buf][r][tx] = (TU)uc[r];
    }
    const C hm = (C)u[base + (size_t)rm * N + i3], hp = (C)u[base + (size_t)rp * N + i3];
    __syncthreads();
    const C q = (C)0.25;
    const int rzm = rz == 0 ? N0 - 1 : rz - 1;
    const bool in0 = !INCL || (rzm >= cc.lo && rzm < cc.hi), in1 = !INCL || (rz >= cc.lo && rz < cc.hi);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const C u2m = r > 0 ? uc[r - 1] : hm;
      const C u2p = r + 1 < RY ? uc[r + 1] : hp;
      const C u3m = tx > 0 ? (C)su[buf][r][tx - 1]
                           : (N == 256 ? (C)su[buf][r][255] : (C)u[base + (size_t)(r0 + r) * N + i3m]);
      const C u3p = tx < 255 ? (C)su[buf][r][tx + 1]
                             : (N == 256 ? (C)su[buf][r][0] : (C)u[base + (size_t)(r0 + r) * N + i3p]);
      C e0[2][2], e1[2][2];
#pragma unroll
      for (int d2 = 0; d2 < 2; ++d2) {
        const int vr = r - 1 + d2;                           // voxel row r0 + vr
        const int k = vr < 0 ? 0 : 1 + vr / N0;              // its cell slot
        const int l2 = vr < 0 ? N0 - 1 : vr % N0;            // its row inside the cell
#pragma unroll
        for (int d3 = 0; d3 < 2; ++d3) {
          if constexpr (INCL) {
            const bool t = l2 >= cc.lo && l2 < cc.hi && in3[d3];
            e0[d2][d3] = (in0 && t) ? a0[k][d3] : (C)cc.bg;
            e1[d2][d3] = (in1 && t) ? a1[k][d3] : (C)cc.bg;
          } else {
            e0[d2][d3] = a0[k][d3];
            e1[d2][d3] = a1[k][d3];
          }
        }
      }
      const C w0c = (((e1[1][1] + e1[0][1]) + e1[1][0]) + e1[0][0]) * q;
      const C w0m = (((e0[1][1] + e0[0][1]) + e0[1][0]) + e0[0][0]) * q;
      const C w1c = (((e1[1][1] + e0[1][1]) + e1[1][0]) + e0[1][0]) * q;
      const C w1m = (((e1[0][1] + e0[0][1]) + e1[0][0]) + e0[0][0]) * q;
      const C w2c = (((e1[1][1] + e0[1][1]) + e1[0][1]) + e0[0][1]) * q;
      const C w2m = (((e1[1][0] + e0[1][0]) + e1[0][0]) + e0[0][0]) * q;
      const C c = uc[r];
      C ku = w0c * (c - un[r]) + w0m * (c - um[r]);
      ku += w1c * (c - u2p) + w1m * (c - u2m);
      ku += w2c * (c - u3p) + w2m * (c - u3m);
      const size_t idx = base + (size_t)(r0 + r) * N + i3;
      if (MODE == 0) {
        const TO o = (TO)ku;
        out[idx] = o;
        dot += (double)c * (double)o;
      } else {
        const double res = f[idx] - (double)ku;
        out[idx] = (TO)res;
        dot += res * res;
      }
    }
    // next plane: layer a1 becomes a0; a new layer when z + 1 starts a cell
#pragma unroll
    for (int k = 0; k < SL; ++k)
#pragma unroll
      for (int d3 = 0; d3 < 2; ++d3) a0[k][d3] = a1[k][d3];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      um[r] = uc[r];
      uc[r] = un[r];
    }
    if (++rz == N0) {
      rz = 0;
      ++cz;
      if (z + 1 < z1) layer(cz, a1);
    }
    buf ^= 1;  // the other LDS buffer next plane: one barrier per plane suffices
  }
  const size_t nparts = (size_t)gridDim.x * gridDim.y * gz;
  block_sum_store(dot, partial + b * nparts + (bx + (size_t)gx * (by + (size_t)gy * zc)));
}

template <typename TU, typename TC, typename TO, typename C, int MODE>
int run_stencil(kp_context* ctx, const TU* u, Cells<TC> cc, const double* f, TO* out,
                double* partial, int* nparts, const Scalars* s, int gate, int N, const Batch& bt) {
  ScopedTimer tm(ctx, MODE == 1 ? KP_TIMER_RESIDUAL : KP_TIMER_STENCIL);
  if (cc.dim == 2) {
    const int g2 = (int)(((size_t)N * N + 255) / 256);
    if (g2 > kMaxPartials || bt.nsys > 65535) return fail(KP_ERR_ARG, "stencil: 2D grid of N=%d too large", N);
    const dim3 grid(g2, bt.nsys);
    if (cc.lo > 0 || cc.hi < cc.n0)
      hipLaunchKernelGGL((k_stencil2d<TU, TC, TO, C, MODE, true>), grid, dim3(256), 0, ctx->stream, u, cc, f,
                         out, partial, s, gate, N, bt);
    else
      hipLaunchKernelGGL((k_stencil2d<TU, TC, TO, C, MODE, false>), grid, dim3(256), 0, ctx->stream, u, cc,
                         f, out, partial, s, gate, N, bt);
    KP_HIP(hipGetLastError());
    *nparts = g2;
    return KP_OK;
  }
  if (N % 256 == 0 && cc.n0 == 4) {
    // Row-segment kernel: enough blocks to fill 256 CUs with 8-plane chunks.
    constexpr int RY = rows_per_thread<TU>();
    int TZ = 32;
    const size_t rows = (size_t)(N / 256) * (N / RY);
    while (TZ > 8 && rows * ((N + TZ - 1) / TZ) * bt.nsys < 1024) TZ /= 2;
    const int gz = (N + TZ - 1) / TZ;
    if (rows * gz <= (size_t)kMaxPartials && (size_t)gz * bt.nsys <= 65535) {
      const dim3 grid(N / 256, N / RY, gz * bt.nsys);
      if (cc.lo > 0 || cc.hi < cc.n0)
        hipLaunchKernelGGL((k_stencil_rows<TU, TC, TO, C, MODE, true>), grid, dim3(256), 0, ctx->stream, u,
                           cc, f, out, partial, s, gate, N, TZ, gz, bt);
      else
        hipLaunchKernelGGL((k_stencil_rows<TU, TC, TO, C, MODE, false>), grid, dim3(256), 0, ctx->stream, u,
                           cc, f, out, partial, s, gate, N, TZ, gz, bt);
      KP_HIP(hipGetLastError());
      *nparts = (int)(rows * gz);
      return KP_OK;
    }
  }
  const int gx = (N + kTX - 1) / kTX;
  const int gy = (N + kTY - 1) / kTY;
  // Enough planes per block to amortize the register queue, enough blocks to fill 256 CUs.
  int TZ = 32;
  while (TZ > 4 && (size_t)gx * gy * ((N + TZ - 1) / TZ) * bt.nsys < 2048) TZ /= 2;
  int gz = (N + TZ - 1) / TZ;
  while ((size_t)gx * gy * gz > (size_t)kMaxPartials || (size_t)gz * bt.nsys > 65535) {
    if (TZ >= N) return fail(KP_ERR_ARG, "stencil: batch of %d systems of N=%d too large", bt.nsys, N);
    TZ *= 2;
    gz = (N + TZ - 1) / TZ;
  }
  const dim3 grid(gx, gy, gz * bt.nsys);
  if (cc.lo > 0 || cc.hi < cc.n0)
    hipLaunchKernelGGL((k_stencil<TU, TC, TO, C, MODE, true>), grid, dim3(256), 0, ctx->stream, u, cc, f,
                       out, partial, s, gate, N, TZ, gz, bt);
  else
    hipLaunchKernelGGL((k_stencil<TU, TC, TO, C, MODE, false>), grid, dim3(256), 0, ctx->stream, u, cc,
                       f, out, partial, s, gate, N, TZ, gz, bt);
  KP_HIP(hipGetLastError());
  *nparts = gx * gy * gz;
  return KP_OK;
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void k_validate(const double* __restrict__ cells, size_t n,
                                                  int* __restrict__ bad) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double v = cells[i];
    if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
  }
}
}  // namespace

int launch_validate_cells(kp_context* ctx, const double* cells, size_t n, int* bad) {
  size_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_validate, dim3((int)b), dim3(256), 0, ctx->stream, cells, n, bad);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

int launch_assemble(kp_context* ctx, kp_coeff* c) {
  ScopedTimer tm(ctx, KP_TIMER_ASSEMBLE);
  const size_t n3 = (size_t)c->N * c->N * c->N;
  const int blocks = (int)((n3 + 255) / 256);
  const CellGeom cg = geom_of(c);
  if (c->dim == 2) {
    const size_t n2 = (size_t)c->N * c->N;
    hipLaunchKernelGGL(k_assemble2d, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, ctx->stream, c->cells,
                       c->L, c->n0, cg.lo, cg.hi, cg.bg, c->N, 1.0 / c->N, c->w64, c->f);
    KP_HIP(hipGetLastError());
    if (c->cells32) return launch_cast_f64_f32(ctx, c->cells, c->cells32, (size_t)c->L * c->L);
    return KP_OK;
  }
  hipLaunchKernelGGL(k_assemble, dim3(blocks), dim3(256), 0, ctx->stream, c->cells, c->L, c->n0, cg.lo,
                     cg.hi, cg.bg, c->N, 1.0 / c->N, c->w64, c->f);
  KP_HIP(hipGetLastError());
  if (c->cells32) return launch_cast_f64_f32(ctx, c->cells, c->cells32, (size_t)c->L * c->L * c->L);
  return KP_OK;
}


int stencil_parts_max(int N) {
  return ((N + kTX - 1) / kTX) * ((N + kTY - 1) / kTY) * ((N + 3) / 4);
}

template <typename TC>
Cells<TC> cells_of(const TC* a, const CellGeom& cg) {
  return Cells<TC>{a, cg.L, cg.n0, cg.lo, cg.hi, (TC)cg.bg, cg.dim};
}

int launch_stencil_f64(kp_context* ctx, const double* p, const double* cells, const CellGeom& cg,
                       const double* f, double* out, double* partial, int* nparts, const Scalars* s,
                       int N, const Batch& bt, int gate) {
  const Cells<double> cc = cells_of(cells, cg);
  if (f)
    return run_stencil<double, double, double, double, 1>(ctx, p, cc, f, out, partial, nparts, s, gate,
                                                          N, bt);
  return run_stencil<double, double, double, double, 0>(ctx, p, cc, nullptr, out, partial, nparts, s,
                                                        gate, N, bt);
}

int launch_stencil_f32(kp_context* ctx, const float* p, const float* cells, const CellGeom& cg, float* out,
                       double* partial, int* nparts, const Scalars* s, int N, const Batch& bt) {
  return run_stencil<float, float, float, float, 0>(ctx, p, cells_of(cells, cg), nullptr, out, partial,
                                                    nparts, s, GATE_ACTIVE, N, bt);
}

int launch_resid_f64_to_f32(kp_context* ctx, const double* x, const double* cells, const CellGeom& cg,
                            const double* f, float* out, double* partial, int* nparts,
                            const Scalars* s, int N, const Batch& bt, int gate) {
  return run_stencil<double, double, float, double, 1>(ctx, x, cells_of(cells, cg), f, out, partial,
                                                       nparts, s, gate, N, bt);
}

}  // namespace kp

// Context, memory, assembly, preconditioner set-up and the operator entry
// points of the C ABI (see include/kronpcg.h for the contracts).

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <hipfft/hipfft.h>

#include "kp_internal.h"

namespace kp {

namespace {
thread_local std::string g_last_error;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// a_hom = delta_ij mean(a) - h <phi_i, f_j> from the partials of the nine dot
// products and of the cell sum (eq. Ahom3_m_entry_comp).  mean(a) is the
// integral of the coefficient over the cube: the mean cell value, or with
// sub-cell inclusions (frac = (k / n0)^3 of every cell carries its value)
// bg + frac (mean cell value - bg).
__global__ __launch_bounds__(256) void k_ahom_final(const double* __restrict__ partial, int nparts,
                                                    double ncells, double h, int sub, double frac,
                                                    double bg, int d, double* __restrict__ out) {
  __shared__ double tot[10];
  __shared__ double red[4];
  for (int v = 0; v < 10; ++v) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += partial[(size_t)v * nparts + i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) tot[v] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
  // d x d entries, row-major; the lumped integral carries h^(d-2).
  if (threadIdx.x < d * d) {
    const int i = threadIdx.x / d, j = threadIdx.x % d;
    const double mc = tot[9] / ncells;
    const double mean = sub ? bg + frac * (mc - bg) : mc;
    out[threadIdx.x] = (i == j ? mean : 0.0) - h * tot[3 * i + j];
  }
}

uint16_t host_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

uint16_t host_f16(double v) {
  _Float16 h = (_Float16)(float)v;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

bool valid_precision(int p) { return p == KP_FP64 || p == KP_MIXED_BF16 || p == KP_MIXED_FP16; }

}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int dev_alloc(kp_context* ctx, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 256;
  if (ctx->alloc) {
    *ptr = ctx->alloc(bytes, ctx->user);
    if (!*ptr) return fail(KP_ERR_NOMEM, "allocator callback returned NULL for %zu bytes", bytes);
    return KP_OK;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(e == hipErrorOutOfMemory ? KP_ERR_NOMEM : KP_ERR_HIP, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  }
  return KP_OK;
}

void dev_free(kp_context* ctx, void* ptr) {
  if (!ptr) return;
  if (ctx->release) {
    ctx->release(ptr, ctx->user);
  } else {
    (void)hipFree(ptr);
  }
}

ScopedTimer::ScopedTimer(kp_context* ctx, int id) : ctx_(ctx), id_(id) {
  if (!ctx_->timing) return;
  if (ctx_->ev_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx_->ev_pool.push_back(e);
  }
  a_ = ctx_->ev_pool.back();
  ctx_->ev_pool.pop_back();
  if (hipEventRecord(a_, ctx_->stream) != hipSuccess) {
    ctx_->ev_pool.push_back(a_);
    a_ = nullptr;
  }
}

ScopedTimer::~ScopedTimer() {
  if (!a_) return;
  hipEvent_t b;
  if (!ctx_->ev_pool.empty()) {
    b = ctx_->ev_pool.back();
    ctx_->ev_pool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    ctx_->ev_pool.push_back(a_);
    return;
  }
  if (hipEventRecord(b, ctx_->stream) != hipSuccess) {
    ctx_->ev_pool.push_back(a_);
    ctx_->ev_pool.push_back(b);
    return;
  }
  ctx_->pending.push_back(TimerRec{id_, a_, b});
}

void resolve_timers(kp_context* ctx) {
  for (const TimerRec& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      ctx->t_ms[t.id] += ms;
      ctx->t_count[t.id] += 1;
    }
    ctx->ev_pool.push_back(t.a);
    ctx->ev_pool.push_back(t.b);
  }
  ctx->pending.clear();
}

int ws_get(kp_context* ctx, int slot, size_t bytes, void** ptr) {
  Buffer& b = ctx->ws[slot];
  if (b.bytes < bytes) {
    if (b.ptr) {
      KP_HIP(hipStreamSynchronize(ctx->stream));
      dev_free(ctx, b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
    }
    KP_TRY(dev_alloc(ctx, &b.ptr, bytes));
    b.bytes = bytes;
  }
  *ptr = b.ptr;
  return KP_OK;
}

// Canonical factors [l][k][i] -> dense circulant operands of the three GEMMs.
// modes = 3, or 2 for the 2D preconditioner (factors of C1 and C2 only; no b3).
static int upload_precond(kp_context* ctx, int N, int R, const double* factors, int precision,
                          kp_precond** out, int modes = 3) {
  const size_t n = N, RN = (size_t)R * N;
  // First column of each circulant: c[d] = (1/N) sum_j u(j) cos(2 pi j d / N).
  std::vector<double> col((size_t)3 * R * N);
  for (int l = 0; l < modes; ++l)
    for (int k = 0; k < R; ++k) {
      const double* u = factors + ((size_t)l * R + k) * n;
      double* c = col.data() + ((size_t)l * R + k) * n;
      for (int d = 0; d < N; ++d) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) {
          const long long jd = ((long long)j * d) % N;
          s += u[j] * std::cos(2.0 * M_PI * (double)jd / (double)N);
        }
        c[d] = s / (double)N;
      }
    }
  auto C = [&](int l, int k, int a, int b) {
    return col[((size_t)l * R + k) * n + (size_t)((a - b + N) % N)];
  };
  std::vector<double> a1(n * RN), c2(RN * n), b3(modes == 3 ? RN * n : 0);
  for (int j1 = 0; j1 < N; ++j1)
    for (int k = 0; k < R; ++k)
      for (int i1 = 0; i1 < N; ++i1) a1[(size_t)j1 * RN + (size_t)k * n + i1] = C(0, k, j1, i1);
  for (int k = 0; k < R; ++k)
    for (int j2 = 0; j2 < N; ++j2)
      for (int i2 = 0; i2 < N; ++i2) c2[((size_t)k * n + j2) * n + i2] = C(1, k, j2, i2);
  if (modes == 3)
    for (int k = 0; k < R; ++k)
      for (int j3 = 0; j3 < N; ++j3)
        for (int i3 = 0; i3 < N; ++i3) b3[((size_t)k * n + j3) * n + i3] = C(2, k, j3, i3);

  kp_precond* pc = new kp_precond();
  pc->ctx = ctx;
  pc->dim = modes;
  pc->N = N;
  pc->R = R;
  pc->precision = precision;
  const size_t bytes = n * RN * sizeof(double);
  int st = KP_OK;
  if ((st = dev_alloc(ctx, (void**)&pc->a1_64, bytes)) < 0 ||
      (st = dev_alloc(ctx, (void**)&pc->c2_64, bytes)) < 0 ||
      (modes == 3 && (st = dev_alloc(ctx, (void**)&pc->b3_64, bytes)) < 0)) {
    kp_free_precond(pc);
    return st;
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpyAsync(pc->a1_64, a1.data(), bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(pc->c2_64, c2.data(), bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && modes == 3)
    e = hipMemcpyAsync(pc->b3_64, b3.data(), bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && precision != KP_FP64) {
    // Each 16-bit row is (hi | lo): hi = round(c), lo = round(c - hi).  A single
    // rounding perturbs the symbol of every circulant by ~2^-9 max|u| at all
    // frequencies, which exceeds the small high-frequency values of the
    // preconditioner symbol and can make it indefinite; hi + lo does not.
    const bool f16 = precision == KP_MIXED_FP16;
    auto r16 = [&](double v) { return f16 ? host_f16(v) : host_bf16(v); };
    auto back = [&](uint16_t h) {
      if (f16) {
        _Float16 x;
        std::memcpy(&x, &h, 2);
        return (double)(float)x;
      }
      uint32_t u = (uint32_t)h << 16;
      float x;
      std::memcpy(&x, &u, 4);
      return (double)x;
    };
    auto split_rows = [&](const std::vector<double>& src, size_t rows, size_t cols,
                          std::vector<uint16_t>& dst) {
      dst.resize(rows * cols * 2);
      for (size_t r = 0; r < rows; ++r)
        for (size_t c = 0; c < cols; ++c) {
          const double v = src[r * cols + c];
          const uint16_t hi = r16(v);
          dst[r * 2 * cols + c] = hi;
          dst[r * 2 * cols + cols + c] = r16(v - back(hi));
        }
    };
    std::vector<uint16_t> h1, h2, h3;
    split_rows(a1, n, RN, h1);
    split_rows(c2, RN, n, h2);
    if (modes == 3) split_rows(b3, RN, n, h3);
    const size_t b16 = 2 * n * RN * sizeof(uint16_t);
    // Shifted reversed first columns (see kp_precond::circ16), same hi / lo values.
    const size_t np8 = n + 8, per_k = 2 * 8 * np8;
    std::vector<uint16_t> hc[3];
    for (int l = 0; l < modes; ++l) {
      hc[l].assign((size_t)R * per_k, 0);
      for (int k = 0; k < R; ++k)
        for (int sft = 0; sft < 8; ++sft)
          for (size_t v = 0; v < np8; ++v) {
            const size_t u = (v + sft) % n;                 // r(u) = c((-u) mod N) = C[0][u]
            const double x = C(l, k, 0, (int)u);
            const uint16_t hi = r16(x);
            hc[l][(size_t)k * per_k + (0 * 8 + sft) * np8 + v] = hi;
            hc[l][(size_t)k * per_k + (1 * 8 + sft) * np8 + v] = r16(x - back(hi));
          }
    }
    const size_t bc = (size_t)R * per_k * sizeof(uint16_t);
    if ((st = dev_alloc(ctx, (void**)&pc->a1_16, b16)) < 0 ||
        (st = dev_alloc(ctx, (void**)&pc->c2_16, b16)) < 0 ||
        (modes == 3 && (st = dev_alloc(ctx, (void**)&pc->b3_16, b16)) < 0) ||
        (st = dev_alloc(ctx, (void**)&pc->circ16[0], bc)) < 0 ||
        (st = dev_alloc(ctx, (void**)&pc->circ16[1], bc)) < 0 ||
        (modes == 3 && (st = dev_alloc(ctx, (void**)&pc->circ16[2], bc)) < 0)) {
      kp_free_precond(pc);
      return st;
    }
    e = hipMemcpyAsync(pc->a1_16, h1.data(), b16, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pc->c2_16, h2.data(), b16, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && modes == 3)
      e = hipMemcpyAsync(pc->b3_16, h3.data(), b16, hipMemcpyHostToDevice, ctx->stream);
    for (int l = 0; l < modes && e == hipSuccess; ++l)
      e = hipMemcpyAsync(pc->circ16[l], hc[l].data(), bc, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);  // host staging goes out of scope
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    kp_free_precond(pc);
    return fail(KP_ERR_HIP, "preconditioner upload: %s", hipGetErrorString(e));
  }
  *out = pc;
  return KP_OK;
}

int launch_ahom(kp_context* ctx, const kp_coeff* c, const double* const* phi, double* part,
                double* out) {
  const size_t n3 = unknowns(c->N, c->dim);
  const size_t nc = unknowns(c->L, c->dim);
  int np = 0;
  KP_TRY(launch_multidot9(ctx, phi, c->f, n3, c->cells, nc, part, &np, c->dim));
  const CellGeom cg = geom_of(c);
  const double fr = (double)c->incl / c->n0;
  const double frac = c->dim == 2 ? fr * fr : fr * fr * fr;
  const double hfac = c->dim == 2 ? 1.0 : 1.0 / c->N;  // h^(d-2)
  hipLaunchKernelGGL(k_ahom_final, dim3(1), dim3(256), 0, ctx->stream, (const double*)part, np,
                     (double)nc, hfac, (int)cg.sub(), frac, c->bg, c->dim, out);
  KP_HIP(hipGetLastError());
  return KP_OK;
}

}  // namespace kp

using namespace kp;

extern "C" {

const char* kp_last_error(void) { return g_last_error.c_str(); }

int kp_context_create(int device, void* hip_stream, kp_context** out) {
  if (!out) return fail(KP_ERR_ARG, "kp_context_create: out is NULL");
  *out = nullptr;
  int count = 0;
  KP_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return fail(KP_ERR_ARG, "kp_context_create: device %d not in [0,%d)", device, count);
  KP_HIP(hipSetDevice(device));
  kp_context* c = new kp_context();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipHostMalloc((void**)&c->host_scal, sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    kp_context_destroy(c);
    return fail(KP_ERR_HIP, "kp_context_create: host buffer or event creation failed");
  }
  *out = c;
  return KP_OK;
}

int kp_context_set_stream(kp_context* ctx, void* hip_stream) {
  if (!ctx) return fail(KP_ERR_ARG, "kp_context_set_stream: NULL context");
  ctx->stream = (hipStream_t)hip_stream;
  return KP_OK;
}

int kp_context_set_allocator(kp_context* ctx, void* (*alloc)(size_t, void*),
                             void (*release)(void*, void*), void* user) {
  if (!ctx) return fail(KP_ERR_ARG, "kp_context_set_allocator: NULL context");
  if ((alloc == nullptr) != (release == nullptr))
    return fail(KP_ERR_ARG, "kp_context_set_allocator: give both callbacks or neither");
  // Workspace made by the previous allocator is released by it.
  (void)hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < WS_COUNT; ++i) {
    dev_free(ctx, ctx->ws[i].ptr);
    ctx->ws[i] = Buffer{};
  }
  ctx->alloc = alloc;
  ctx->release = release;
  ctx->user = user;
  return KP_OK;
}

int kp_context_destroy(kp_context* ctx) {
  if (!ctx) return KP_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < WS_COUNT; ++i) dev_free(ctx, ctx->ws[i].ptr);
  if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  resolve_timers(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return KP_OK;
}

int kp_context_set_timing(kp_context* ctx, int enable) {
  if (!ctx) return fail(KP_ERR_ARG, "kp_context_set_timing: NULL context");
  KP_HIP(hipStreamSynchronize(ctx->stream));
  resolve_timers(ctx);
  for (int i = 0; i < KP_TIMER_COUNT; ++i) {
    ctx->t_ms[i] = 0.0;
    ctx->t_count[i] = 0;
  }
  ctx->timing = enable != 0;
  return KP_OK;
}

int kp_context_read_timing(kp_context* ctx, double* ms, long long* launches) {
  if (!ctx) return fail(KP_ERR_ARG, "kp_context_read_timing: NULL context");
  KP_HIP(hipStreamSynchronize(ctx->stream));
  resolve_timers(ctx);
  for (int i = 0; i < KP_TIMER_COUNT; ++i) {
    if (ms) ms[i] = ctx->t_ms[i];
    if (launches) launches[i] = ctx->t_count[i];
  }
  return KP_OK;
}

int kp_coeff_update(kp_context* ctx, kp_coeff* c, const double* a_cell_dev) {
  if (!ctx || !c || !a_cell_dev) return fail(KP_ERR_ARG, "kp_coeff_update: NULL argument");
  if (c->ctx != ctx) return fail(KP_ERR_STATE, "kp_coeff_update: coefficient of another context");
  const size_t nc = unknowns(c->L, c->dim);
  void* flag;
  KP_TRY(ws_get(ctx, WS_FLAG, sizeof(int), &flag));
  KP_HIP(hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
  KP_TRY(launch_validate_cells(ctx, a_cell_dev, nc, (int*)flag));
  int bad = 0;
  KP_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  KP_HIP(hipStreamSynchronize(ctx->stream));
  if (bad) return fail(KP_ERR_ARG, "kp_coeff_update: a cell is not finite or not > 0");
  KP_HIP(hipMemcpyAsync(c->cells, a_cell_dev, nc * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return launch_assemble(ctx, c);
}

namespace {
int setup_coeff_dim(kp_context* ctx, int dim, int L, int n0, int incl, double background,
                    const double* a_cell, int precision, kp_coeff** out) {
  if (!ctx || !a_cell || !out) return fail(KP_ERR_ARG, "setup_coeff: NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "setup_coeff: bad precision %d", precision);
  if (L < 1 || n0 < 1 || (long long)L * n0 < 2 || (long long)L * n0 > 2048)
    return fail(KP_ERR_ARG, "setup_coeff: need L >= 1, n0 >= 1, 2 <= N = n0*L <= 2048");
  if (incl < 1 || incl > n0 || (n0 - incl) % 2 != 0)
    return fail(KP_ERR_ARG, "setup_coeff: a sub-cell of %d voxels does not centre in a cell of %d", incl, n0);
  if (incl < n0 && (!std::isfinite(background) || !(background > 0.0)))
    return fail(KP_ERR_ARG, "setup_coeff: background %g must be finite and > 0", background);
  const int N = L * n0;
  const size_t nc = unknowns(L, dim);
  for (size_t i = 0; i < nc; ++i) {
    if (!std::isfinite(a_cell[i]) || !(a_cell[i] > 0.0))
      return fail(KP_ERR_ARG, "setup_coeff: cell %zu has value %g (must be finite and > 0)", i, a_cell[i]);
  }
  KP_HIP(hipSetDevice(ctx->device));
  kp_coeff* c = new kp_coeff();
  c->ctx = ctx;
  c->dim = dim;
  c->L = L;
  c->n0 = n0;
  c->N = N;
  c->incl = incl;
  c->bg = incl < n0 ? background : 0.0;
  c->precision = precision;
  const size_t n3 = unknowns(N, dim);
  int st;
  if ((st = dev_alloc(ctx, (void**)&c->cells, nc * sizeof(double))) < 0 ||
      (st = dev_alloc(ctx, (void**)&c->w64, dim * n3 * sizeof(double))) < 0 ||
      (st = dev_alloc(ctx, (void**)&c->f, dim * n3 * sizeof(double))) < 0 ||
      (precision != KP_FP64 && (st = dev_alloc(ctx, (void**)&c->cells32, nc * sizeof(float))) < 0)) {
    kp_free_coeff(c);
    return st;
  }
  hipError_t e = hipMemcpyAsync(c->cells, a_cell, nc * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    kp_free_coeff(c);
    return fail(KP_ERR_HIP, "setup_coeff upload: %s", hipGetErrorString(e));
  }
  if ((st = launch_assemble(ctx, c)) < 0) {
    kp_free_coeff(c);
    return st;
  }
  *out = c;
  return KP_OK;
}
}  // namespace

int setup_coeff_inclusions(kp_context* ctx, int L, int n0, int incl, double background,
                           const double* a_cell, int precision, kp_coeff** out) {
  return setup_coeff_dim(ctx, 3, L, n0, incl, background, a_cell, precision, out);
}

int setup_coeff(kp_context* ctx, int L, int n0, const double* a_cell, int precision,
                kp_coeff** out) {
  return setup_coeff_dim(ctx, 3, L, n0, n0, 0.0, a_cell, precision, out);
}

int setup_coeff_2d(kp_context* ctx, int L, int n0, int incl, double background, const double* a_cell,
                   int precision, kp_coeff** out) {
  return setup_coeff_dim(ctx, 2, L, n0, incl, background, a_cell, precision, out);
}

int kp_coeff_size(const kp_coeff* c) { return c ? c->N : -1; }

int kp_coeff_fields(kp_context* ctx, const kp_coeff* c, double* w_dev, double* f_dev) {
  if (!ctx || !c) return fail(KP_ERR_ARG, "kp_coeff_fields: NULL argument");
  const size_t bytes = c->dim * unknowns(c->N, c->dim) * sizeof(double);
  if (w_dev) KP_HIP(hipMemcpyAsync(w_dev, c->w64, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (f_dev) KP_HIP(hipMemcpyAsync(f_dev, c->f, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return KP_OK;
}

int kp_free_coeff(kp_coeff* c) {
  if (!c) return KP_OK;
  kp_context* ctx = c->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, c->cells);
  dev_free(ctx, c->w64);
  dev_free(ctx, c->cells32);
  dev_free(ctx, c->f);
  delete c;
  return KP_OK;
}

int kp_stiffness_apply(kp_context* ctx, const kp_coeff* c, int precision, const double* p_dev,
                       double* q_dev) {
  if (!ctx || !c || !p_dev || !q_dev) return fail(KP_ERR_ARG, "kp_stiffness_apply: NULL argument");
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "kp_stiffness_apply: bad precision");
  if (precision != KP_FP64 && !c->cells32)
    return fail(KP_ERR_STATE, "kp_stiffness_apply: coefficient was set up without float cells");
  const int N = c->N;
  const size_t n3 = unknowns(N, c->dim);
  void* part;
  KP_TRY(ws_get(ctx, WS_PART, (size_t)kMaxPartials * 8 * sizeof(double), &part));
  int np = 0;
  if (precision == KP_FP64)
    return launch_stencil_f64(ctx, p_dev, c->cells, geom_of(c), nullptr, q_dev, (double*)part, &np,
                              nullptr, N);
  void *p32, *q32;
  KP_TRY(ws_get(ctx, WS_R, n3 * sizeof(float), &p32));
  KP_TRY(ws_get(ctx, WS_Q, n3 * sizeof(float), &q32));
  KP_TRY(launch_cast_f64_f32(ctx, p_dev, (float*)p32, n3));
  KP_TRY(launch_stencil_f32(ctx, (const float*)p32, c->cells32, geom_of(c), (float*)q32, (double*)part,
                            &np, nullptr, N));
  return launch_cast_f32_f64(ctx, (const float*)q32, q_dev, n3);
}

int build_preconditioner(kp_context* ctx, int N, double eps, int rank, int precision,
                         kp_precond** out, kp_precond_info* info) {
  if (!ctx || !out) return fail(KP_ERR_ARG, "build_preconditioner: NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "build_preconditioner: bad precision");
  if (N < 2 || N > 2048) return fail(KP_ERR_ARG, "build_preconditioner: N = %d out of range", N);
  KP_HIP(hipSetDevice(ctx->device));
  std::vector<double> fac((size_t)3 * 16 * N);
  kp_precond_info inf{};
  KP_TRY(kp_lowrank_factors(N, eps, rank, fac.data(), fac.size(), &inf));
  kp_precond* pc = nullptr;
  KP_TRY(upload_precond(ctx, N, inf.rank, fac.data(), precision, &pc));
  pc->info = inf;
  if (info) *info = inf;
  *out = pc;
  return KP_OK;
}

int kp_precond_from_factors(kp_context* ctx, int N, int R, const double* factors, int precision,
                            kp_precond** out) {
  if (!ctx || !factors || !out) return fail(KP_ERR_ARG, "kp_precond_from_factors: NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "kp_precond_from_factors: bad precision");
  if (N < 2 || N > 2048 || R < 1 || R > 16)
    return fail(KP_ERR_ARG, "kp_precond_from_factors: need 2 <= N <= 2048 and 1 <= R <= 16");
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < N; ++i) {
        const double* u = factors + ((size_t)l * R + k) * N;
        if (!std::isfinite(u[i])) return fail(KP_ERR_ARG, "kp_precond_from_factors: non-finite factor");
        const double d = std::fabs(u[i] - u[(N - i) % N]);
        if (d > 1e-12 * (std::fabs(u[i]) + 1e-300) && d > 0.0)
          return fail(KP_ERR_ARG, "kp_precond_from_factors: factor (%d,%d) is not even", l, k);
      }
  KP_HIP(hipSetDevice(ctx->device));
  kp_precond* pc = nullptr;
  KP_TRY(upload_precond(ctx, N, R, factors, precision, &pc));
  pc->info.rank = R;
  *out = pc;
  return KP_OK;
}

int build_preconditioner_2d(kp_context* ctx, int N, double eps, int rank, int precision,
                            kp_precond** out, kp_precond_info* info) {
  if (!ctx || !out) return fail(KP_ERR_ARG, "build_preconditioner_2d: NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "build_preconditioner_2d: bad precision");
  if (N < 2 || N > 2048) return fail(KP_ERR_ARG, "build_preconditioner_2d: N = %d out of range", N);
  KP_HIP(hipSetDevice(ctx->device));
  std::vector<double> fac((size_t)2 * 16 * N);
  kp_precond_info inf{};
  KP_TRY(kp_lowrank_factors_2d(N, eps, rank, fac.data(), fac.size(), &inf));
  kp_precond* pc = nullptr;
  KP_TRY(upload_precond(ctx, N, inf.rank, fac.data(), precision, &pc, 2));
  pc->info = inf;
  if (info) *info = inf;
  *out = pc;
  return KP_OK;
}

int kp_precond_from_factors_2d(kp_context* ctx, int N, int R, const double* factors, int precision,
                               kp_precond** out) {
  if (!ctx || !factors || !out) return fail(KP_ERR_ARG, "kp_precond_from_factors_2d: NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(KP_ERR_ARG, "kp_precond_from_factors_2d: bad precision");
  if (N < 2 || N > 2048 || R < 1 || R > 16)
    return fail(KP_ERR_ARG, "kp_precond_from_factors_2d: need 2 <= N <= 2048 and 1 <= R <= 16");
  for (int l = 0; l < 2; ++l)
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < N; ++i) {
        const double* u = factors + ((size_t)l * R + k) * N;
        if (!std::isfinite(u[i])) return fail(KP_ERR_ARG, "kp_precond_from_factors_2d: non-finite factor");
        const double d = std::fabs(u[i] - u[(N - i) % N]);
        if (d > 1e-12 * (std::fabs(u[i]) + 1e-300) && d > 0.0)
          return fail(KP_ERR_ARG, "kp_precond_from_factors_2d: factor (%d,%d) is not even", l, k);
      }
  KP_HIP(hipSetDevice(ctx->device));
  kp_precond* pc = nullptr;
  KP_TRY(upload_precond(ctx, N, R, factors, precision, &pc, 2));
  pc->info.rank = R;
  *out = pc;
  return KP_OK;
}

int kp_precond_rank(const kp_precond* pc) { return pc ? pc->R : -1; }

int kp_precond_set_tiles(kp_precond* pc, const int* tiles) {
  if (!pc || !tiles) return fail(KP_ERR_ARG, "kp_precond_set_tiles: NULL argument");
  const int n = 2 * (pc->precision == KP_FP64 ? kTiles64 : kTiles16);  // tiles x block orders
  for (int s = 0; s < 3; ++s)
    if (tiles[s] < -1 || tiles[s] >= n)
      return fail(KP_ERR_ARG, "kp_precond_set_tiles: tile index %d of stage %d not in [-1,%d)", tiles[s], s, n);
  for (int s = 0; s < 3; ++s) pc->tile[s] = tiles[s];
  return KP_OK;
}

int kp_precond_get_tiles(const kp_precond* pc, int* tiles) {
  if (!pc || !tiles) return fail(KP_ERR_ARG, "kp_precond_get_tiles: NULL argument");
  for (int s = 0; s < 3; ++s) tiles[s] = pc->tile[s];
  return KP_OK;
}

int kp_precond_autotune(kp_context* ctx, kp_precond* pc, int reps, kp_tile_timing* table, int cap,
                        int* count) {
  if (!ctx || !pc) return fail(KP_ERR_ARG, "kp_precond_autotune: NULL argument");
  if (pc->ctx != ctx) return fail(KP_ERR_STATE, "kp_precond_autotune: preconditioner of another context");
  if (reps < 1 || reps > 1000) return fail(KP_ERR_ARG, "kp_precond_autotune: reps must be 1..1000");
  KP_HIP(hipSetDevice(ctx->device));
  KP_TRY(autotune_precond(ctx, pc, 1, reps, table, table ? cap : 0, count, pc->tile));
  KP_HIP(hipStreamSynchronize(ctx->stream));
  return KP_OK;
}

int kp_free_precond(kp_precond* pc) {
  if (!pc) return KP_OK;
  kp_context* ctx = pc->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, pc->a1_64);
  dev_free(ctx, pc->c2_64);
  dev_free(ctx, pc->b3_64);
  dev_free(ctx, pc->a1_16);
  dev_free(ctx, pc->c2_16);
  dev_free(ctx, pc->b3_16);
  for (int l = 0; l < 3; ++l) dev_free(ctx, pc->circ16[l]);
  if (pc->fft_fwd) hipfftDestroy((hipfftHandle)pc->fft_fwd);
  if (pc->fft_inv) hipfftDestroy((hipfftHandle)pc->fft_inv);
  dev_free(ctx, pc->fft_sym);
  dev_free(ctx, pc->fft_work);
  delete pc;
  return KP_OK;
}

int kp_precond_apply(kp_context* ctx, const kp_precond* pc, const double* r_dev, double* z_dev) {
  if (!ctx || !pc || !r_dev || !z_dev) return fail(KP_ERR_ARG, "kp_precond_apply: NULL argument");
  const size_t n3 = unknowns(pc->N, pc->dim);
  if (pc->precision == KP_FP64) return launch_precond_f64(ctx, pc, r_dev, z_dev, nullptr);
  void *x16, *z32;
  KP_TRY(ws_get(ctx, WS_X16, n3 * sizeof(bf16_t), &x16));
  KP_TRY(ws_get(ctx, WS_Z, n3 * sizeof(float), &z32));
  KP_TRY(launch_cast_to16(ctx, r_dev, (bf16_t*)x16, n3, pc->precision == KP_MIXED_FP16));
  KP_TRY(launch_precond_16(ctx, pc, (const bf16_t*)x16, (float*)z32, nullptr));
  return launch_cast_f32_f64(ctx, (const float*)z32, z_dev, n3);
}

int kp_homogenized_matrix(kp_context* ctx, const kp_coeff* c, const double* const* phi_dev,
                          double* ahom) {
  if (!ctx || !c || !phi_dev || !ahom) return fail(KP_ERR_ARG, "kp_homogenized_matrix: NULL argument");
  for (int i = 0; i < c->dim; ++i)
    if (!phi_dev[i]) return fail(KP_ERR_ARG, "kp_homogenized_matrix: phi[%d] is NULL", i);
  void *part, *res;
  KP_TRY(ws_get(ctx, WS_PART, (size_t)kMaxPartials * 8 * sizeof(double), &part));
  KP_TRY(ws_get(ctx, WS_SCAL, sizeof(Scalars), &res));
  KP_TRY(launch_ahom(ctx, c, phi_dev, (double*)part, (double*)res));
  KP_HIP(hipMemcpyAsync(ahom, res, (size_t)c->dim * c->dim * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  KP_HIP(hipStreamSynchronize(ctx->stream));
  return KP_OK;
}

}  // extern "C"

// Preconditioned conjugate gradients on the zero-mean subspace (Section 4.1,
// eqs. DD_Eqn and PCG_DD_Eqn), driven from the host in chunks of iterations
// whose scalars (alpha, beta, rho, norms, convergence flag) never leave the
// device.  The host looks at the device scalars once per chunk; kernels queued
// after convergence see the flag and return immediately.
//
// Plain FP64: standard PCG, beta = rho_new / rho.
// Mixed: float vectors, float stencil on float cell values, BF16/FP16 MFMA
// preconditioner, flexible PCG (Polak-Ribiere beta, which tolerates a
// preconditioner that is only approximately linear and symmetric because of
// rounding); dot products, norms and the zero-mean projection in double; x in
// double, its increments accumulated in float and added into it before every
// true residual;
// every `replace_every` iterations the recursive residual is replaced by the
// true residual f - K x computed in double from the double cell values.
//
// The preconditioned vector is projected to zero mean inside the p update,
// p = (z - mean z) + beta p, and rho = <r, z - mean z>, so the iterates stay
// in the subspace <u, 1> = 0 although the low-rank symbol is not zero at the
// zero mode.  Stopping: the true relative residual ||f - K x|| / ||f|| in
// double (the recursive residual only decides when to look).

#include <cmath>
#include <cstring>

#include "kp_internal.h"

namespace kp {

namespace {

struct Solver {
  kp_context* ctx;
  const kp_coeff* c;
  const kp_precond* pc;
  bool mixed;
  bool fp16;
  int N;
  size_t n3;
  Scalars* s;        // device
  double* part;
  double* fp;        // projected right-hand side (double)
  double* x;
  float* x32;        // mixed: increments of x since the last true residual
  void *r, *z, *p, *q;
  bf16_t* x16;
  int np = 0;
};

int fin(Solver& S, int nvals, int mode) {
  return launch_finalize(S.ctx, S.part, S.np, nvals, mode, S.s, S.n3);
}

// r = f - K x (double), ||r||^2 -> s->rr (no iteration counted); convergence flag.
int true_residual(Solver& S, bool into_r) {
  if (S.mixed) {
    KP_TRY(launch_fold(S.ctx, S.x, S.x32, S.n3, nullptr));
    // double residual into the double scratch, then (optionally) into the float r.
    void* r64;
    KP_TRY(ws_get(S.ctx, WS_TMP64B, S.n3 * sizeof(double), &r64));
    KP_TRY(launch_stencil_f64(S.ctx, S.x, S.c->cells, geom_of(S.c), S.fp, (double*)r64, S.part, &S.np, nullptr, S.N));
    KP_TRY(fin(S, 1, FIN_RR_NOCOUNT));
    if (into_r) {
      KP_TRY(launch_cast_f64_f32(S.ctx, (const double*)r64, (float*)S.r, S.n3));
      KP_TRY(launch_cast32_to16(S.ctx, (const float*)S.r, S.x16, S.n3, S.fp16, S.s));
    }
    return KP_OK;
  }
  if (into_r) {
    KP_TRY(launch_stencil_f64(S.ctx, S.x, S.c->cells, geom_of(S.c), S.fp, (double*)S.r, S.part, &S.np, nullptr, S.N));
  } else {
    void* r64;
    KP_TRY(ws_get(S.ctx, WS_TMP64B, S.n3 * sizeof(double), &r64));
    KP_TRY(launch_stencil_f64(S.ctx, S.x, S.c->cells, geom_of(S.c), S.fp, (double*)r64, S.part, &S.np, nullptr, S.N));
  }
  return fin(S, 1, FIN_RR_NOCOUNT);
}

// z = M r; rho, mean(z), beta from the dot products; p = (z - mz) + beta p.
int precondition_and_update(Solver& S, int fin_mode, bool have_q) {
  if (S.mixed) {
    // The last GEMM stage computes the dot products of z as it writes z.
    const PrecDots dots{(const float*)S.r, have_q ? (const float*)S.q : nullptr, S.part,
                        (size_t)kMaxPartials * 8};
    KP_TRY(launch_precond_16(S.ctx, S.pc, S.x16, (float*)S.z, S.s, Batch(), nullptr, nullptr, nullptr,
                             &dots, &S.np));
    if (S.np == 0)
      KP_TRY(launch_prec_dots<float>(S.ctx, (const float*)S.z, (const float*)S.r,
                                     have_q ? (const float*)S.q : nullptr, S.s, S.part, &S.np, S.n3));
    KP_TRY(fin(S, 5, fin_mode));
    return launch_update_p<float>(S.ctx, (const float*)S.z, (float*)S.p, S.s, S.n3);
  }
  KP_TRY(launch_precond_f64(S.ctx, S.pc, (const double*)S.r, (double*)S.z, S.s));
  KP_TRY(launch_prec_dots<double>(S.ctx, (const double*)S.z, (const double*)S.r,
                                  have_q ? (const double*)S.q : nullptr, S.s, S.part, &S.np, S.n3));
  KP_TRY(fin(S, 5, fin_mode));
  return launch_update_p<double>(S.ctx, (const double*)S.z, (double*)S.p, S.s, S.n3);
}

int iteration(Solver& S, bool replace) {
  if (S.mixed) {
    KP_TRY(launch_stencil_f32(S.ctx, (const float*)S.p, S.c->cells32, geom_of(S.c), (float*)S.q, S.part, &S.np, S.s, S.N));
    KP_TRY(fin(S, 1, FIN_ALPHA));
    KP_TRY(launch_update_xr<float>(S.ctx, S.x, S.x32, (const float*)S.p, (float*)S.r, (const float*)S.q,
                                   S.x16, S.fp16, S.s, S.part, &S.np, S.n3));
    KP_TRY(fin(S, 1, FIN_RR));
    if (replace) {
      void* r64;
      KP_TRY(ws_get(S.ctx, WS_TMP64B, S.n3 * sizeof(double), &r64));
      KP_TRY(launch_fold(S.ctx, S.x, S.x32, S.n3, S.s));
      KP_TRY(launch_resid_f64_to_f32(S.ctx, S.x, S.c->cells, geom_of(S.c), S.fp, (float*)S.r, S.part, &S.np, S.s, S.N));
      KP_TRY(fin(S, 1, FIN_RR_NOCOUNT));
      KP_TRY(launch_cast32_to16(S.ctx, (const float*)S.r, S.x16, S.n3, S.fp16, S.s));
    }
    return precondition_and_update(S, replace ? FIN_PREC_FR : FIN_PREC, true);
  }
  KP_TRY(launch_stencil_f64(S.ctx, (const double*)S.p, S.c->cells, geom_of(S.c), nullptr, (double*)S.q, S.part, &S.np, S.s, S.N));
  KP_TRY(fin(S, 1, FIN_ALPHA));
  KP_TRY(launch_update_xr<double>(S.ctx, S.x, nullptr, (const double*)S.p, (double*)S.r, (const double*)S.q,
                                  nullptr, 0, S.s, S.part, &S.np, S.n3));
  KP_TRY(fin(S, 1, FIN_RR));
  return precondition_and_update(S, FIN_PREC, true);
}

int read_scalars(Solver& S, Scalars* h) {
  KP_HIP(hipMemcpyAsync(S.ctx->host_scal, S.s, sizeof(Scalars), hipMemcpyDeviceToHost, S.ctx->stream));
  KP_HIP(hipStreamSynchronize(S.ctx->stream));
  resolve_timers(S.ctx);
  std::memcpy(h, S.ctx->host_scal, sizeof(Scalars));
  return KP_OK;
}

int write_scalars(Solver& S, const Scalars& h) {
  std::memcpy(S.ctx->host_scal, &h, sizeof(Scalars));
  KP_HIP(hipMemcpyAsync(S.s, S.ctx->host_scal, sizeof(Scalars), hipMemcpyHostToDevice, S.ctx->stream));
  KP_HIP(hipStreamSynchronize(S.ctx->stream));
  return KP_OK;
}

}  // namespace

}  // namespace kp

using namespace kp;

extern "C" int pcg_solve(kp_context* ctx, const kp_coeff* c, const kp_precond* pc, int rhs,
                         const double* f_dev, double* x_dev, const kp_solve_opts* opts,
                         kp_solve_stats* stats) {
  if (!ctx || !c || !pc || !x_dev) return fail(KP_ERR_ARG, "pcg_solve: NULL argument");
  if (rhs < 0 || rhs > 3) return fail(KP_ERR_ARG, "pcg_solve: rhs must be 0..3");
  if (rhs == 0 && !f_dev) return fail(KP_ERR_ARG, "pcg_solve: rhs = 0 needs f_dev");
  if (c->ctx != ctx || pc->ctx != ctx) return fail(KP_ERR_STATE, "pcg_solve: handles of another context");
  if (c->N != pc->N) return fail(KP_ERR_STATE, "pcg_solve: coefficient N=%d, preconditioner N=%d", c->N, pc->N);
  if (c->dim != pc->dim && !pc->fft)
    return fail(KP_ERR_STATE, "pcg_solve: %dD coefficient with a %dD preconditioner", c->dim, pc->dim);
  if (pc->fft && c->dim != 3) return fail(KP_ERR_STATE, "pcg_solve: the FFT preconditioner is 3D");
  if (rhs > c->dim) return fail(KP_ERR_ARG, "pcg_solve: rhs %d of a %dD problem", rhs, c->dim);
  const bool mixed = c->precision != KP_FP64;
  if (mixed != (pc->precision != KP_FP64))
    return fail(KP_ERR_STATE, "pcg_solve: coefficient and preconditioner precisions differ");
  kp_solve_opts o{1e-8, 2000, mixed ? 25 : 0, 0, 0};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.maxit < 0 || o.replace_every < 0)
    return fail(KP_ERR_ARG, "pcg_solve: need tol > 0, maxit >= 0, replace_every >= 0");
  if (!mixed) o.replace_every = 0;
  const int chunk = o.check_every > 0 ? o.check_every : (mixed ? 8 : 4);
  KP_HIP(hipSetDevice(ctx->device));

  Solver S;
  S.ctx = ctx;
  S.c = c;
  S.pc = pc;
  S.mixed = mixed;
  S.fp16 = pc->precision == KP_MIXED_FP16;
  S.N = c->N;
  S.n3 = unknowns(c->N, c->dim);
  const size_t vb = S.n3 * (mixed ? sizeof(float) : sizeof(double));
  void *sv, *pv, *fpv;
  KP_TRY(ws_get(ctx, WS_SCAL, sizeof(Scalars), &sv));
  KP_TRY(ws_get(ctx, WS_PART, (size_t)kMaxPartials * 8 * sizeof(double), &pv));
  KP_TRY(ws_get(ctx, WS_TMP64, S.n3 * sizeof(double), &fpv));
  KP_TRY(ws_get(ctx, WS_R, vb, &S.r));
  KP_TRY(ws_get(ctx, WS_Z, vb, &S.z));
  KP_TRY(ws_get(ctx, WS_P, vb, &S.p));
  KP_TRY(ws_get(ctx, WS_Q, vb, &S.q));
  S.x16 = nullptr;
  S.x32 = nullptr;
  if (mixed) {
    void* xv;
    KP_TRY(ws_get(ctx, WS_X16, S.n3 * sizeof(bf16_t), &xv));
    S.x16 = (bf16_t*)xv;
    KP_TRY(ws_get(ctx, WS_X32, S.n3 * sizeof(float), &xv));
    S.x32 = (float*)xv;
    KP_HIP(hipMemsetAsync(S.x32, 0, S.n3 * sizeof(float), ctx->stream));
  }
  S.s = (Scalars*)sv;
  S.part = (double*)pv;
  S.fp = (double*)fpv;
  S.x = x_dev;

  KP_HIP(hipEventRecord(ctx->ev0, ctx->stream));
  Scalars h{};
  KP_TRY(write_scalars(S, h));

  // Right-hand side: mean and norm, projection to zero mean.
  const double* f = rhs ? c->f + (size_t)(rhs - 1) * S.n3 : f_dev;
  KP_TRY(launch_sum2(ctx, f, S.n3, S.part, &S.np));
  KP_TRY(fin(S, 2, FIN_SUM));
  KP_TRY(read_scalars(S, &h));
  const double fmean = h.sums[0] / (double)S.n3;
  const double fnorm_raw = std::sqrt(std::fmax(h.sums[1], 0.0));
  KP_TRY(launch_copy_project_f(ctx, f, fmean, S.fp, S.n3));
  KP_TRY(launch_sum2(ctx, S.fp, S.n3, S.part, &S.np));
  KP_TRY(fin(S, 2, FIN_FF));
  KP_TRY(read_scalars(S, &h));
  int warn = KP_OK;
  if (rhs == 0 && std::fabs(fmean) > 1e-12 * fnorm_raw / std::sqrt((double)S.n3)) warn = KP_WARN_RHS_MEAN;
  const double ff = h.ff;
  kp_solve_stats st{};
  st.rhs_mean = fmean;
  if (!(ff > 0.0)) {
    KP_TRY(launch_fill_f64(ctx, x_dev, 0.0, S.n3));
    KP_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    KP_HIP(hipStreamSynchronize(ctx->stream));
    st.status = warn;
    if (stats) *stats = st;
    return warn;
  }
  h = Scalars{};
  h.ff = ff;
  h.tol2ff = o.tol * o.tol * ff;
  h.flexible = mixed ? 1 : 0;
  h.x16_scale = h.x16_scale_next = 1.0;
  KP_TRY(write_scalars(S, h));
  if (!o.use_x0) KP_TRY(launch_fill_f64(ctx, x_dev, 0.0, S.n3));

  // r0 = f - K x0, z0 = M r0, p0 = z0 - mean(z0).
  KP_TRY(true_residual(S, true));
  KP_TRY(precondition_and_update(S, FIN_PREC_INIT, false));

  int queued = 0;
  int status = KP_NOT_CONVERGED;
  double rr_true = 0.0;
  // Chunk length: at most `chunk`, shortened to the number of iterations the
  // recent convergence rate predicts are left, so that few launches are queued
  // after convergence (they would see the flag and return at once).
  int prev_it = -1;
  double prev_rr = 0.0;
  int predicted = chunk;
  while (true) {
    const int todo = std::min(std::min(chunk, predicted), o.maxit - queued);
    for (int i = 0; i < todo; ++i) {
      const bool replace = o.replace_every > 0 && ((queued + 1) % o.replace_every) == 0;
      KP_TRY(iteration(S, replace));
      ++queued;
    }
    KP_TRY(read_scalars(S, &h));
    predicted = chunk;
    if (prev_it >= 0 && h.iters > prev_it && h.rr > 0.0 && prev_rr > h.rr && h.rr > h.tol2ff) {
      const double rate = std::log(h.rr / prev_rr) / (double)(h.iters - prev_it);  // < 0
      const double left = std::log(h.tol2ff / h.rr) / rate;
      if (std::isfinite(left)) predicted = std::max(1, (int)std::ceil(left));
    }
    prev_it = h.iters;
    prev_rr = h.rr;
    if (h.breakdown) {
      st.iters = h.iters;
      st.status = KP_ERR_BREAKDOWN;
      if (stats) *stats = st;
      return fail(KP_ERR_BREAKDOWN, "pcg_solve: breakdown after %d iterations (pq=%g rho=%g rr=%g)",
                  h.iters, h.pq, h.rho, h.rr);
    }
    if (h.done) {
      // Recursive residual below tol: confirm with the true residual in double.
      const double rr_rec = h.rr;
      h.done = 0;
      KP_TRY(write_scalars(S, h));
      KP_TRY(true_residual(S, false));
      Scalars t;
      KP_TRY(read_scalars(S, &t));
      rr_true = t.rr;
      if (rr_true <= h.tol2ff) {
        status = KP_OK;
        st.relres_rec = std::sqrt(rr_rec / ff);
        break;
      }
      // Drifted: restart the recursion from the true residual.
      t.done = 0;
      KP_TRY(write_scalars(S, t));
      KP_TRY(true_residual(S, true));
      KP_TRY(precondition_and_update(S, FIN_PREC_INIT, false));
      st.replacements += 1;
      KP_TRY(read_scalars(S, &h));
      if (h.breakdown) return fail(KP_ERR_BREAKDOWN, "pcg_solve: breakdown at a restart");
    }
    if (queued >= o.maxit) {
      KP_TRY(true_residual(S, false));
      Scalars t;
      KP_TRY(read_scalars(S, &t));
      rr_true = t.rr;
      st.relres_rec = std::sqrt(h.rr / ff);
      if (rr_true <= h.tol2ff) status = KP_OK;
      break;
    }
  }
  KP_TRY(read_scalars(S, &h));
  st.iters = h.iters;
  if (mixed && o.replace_every > 0) st.replacements += h.iters / o.replace_every;
  st.relres_true = std::sqrt(rr_true / ff);

  // x <- x - mean(x)
  if (mixed) KP_TRY(launch_fold(ctx, S.x, S.x32, S.n3, nullptr));
  KP_TRY(launch_sum2(ctx, x_dev, S.n3, S.part, &S.np));
  KP_TRY(fin(S, 2, FIN_SUM));
  KP_TRY(read_scalars(S, &h));
  KP_TRY(launch_copy_project_f(ctx, x_dev, h.sums[0] / (double)S.n3, x_dev, S.n3));
  KP_HIP(hipEventRecord(ctx->ev1, ctx->stream));
  KP_HIP(hipStreamSynchronize(ctx->stream));
  float ms = 0.f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  st.ms = ms;
  if (status == KP_OK) status = warn;
  st.status = status;
  if (stats) *stats = st;
  return status;
}

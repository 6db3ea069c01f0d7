// Batched corrector solves: many coefficient realizations of uneven size, the
// three corrector problems of each (eq. DD_Eqn with the right-hand sides of
// eq. FEM_discr_RHS), as in the Monte-Carlo averages of Section 5.
//
// Instances that share a preconditioner (hence one grid size N) and the cell
// size n0 form a group.  A group's vectors are stored system after system
// (stride N^3) and its realizations' cell values realization after
// realization (stride L^3), so every PCG step of the group is one launch over
// all its systems (Batch layout).  The PCG control of each system lives in its own device scalars:
// the recursive residual only requests a true residual (in double, from the
// double cell values), which then decides convergence, the iteration limit, or a
// residual replacement (FIN_RR_CTL, FIN_TRUE_CTL).  Stopped systems are masked:
// every block of theirs returns at once.
//
// `check_every` iterations of all groups are captured in one HIP graph, each
// group as its own branch (forked and joined through events, so the branches
// may run concurrently), followed by a count of the systems still running;
// the host replays the graph until the count is zero.  The graph holds no
// memset nodes.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "kp_internal.h"

namespace kp {

namespace {

struct Group {
  const kp_precond* pc = nullptr;
  int N = 0, L = 0, n0 = 0;
  CellGeom cg;  // the coefficient geometry shared by the group's realizations
  size_t n3 = 0;
  std::vector<int> inst;  // instance indices
  int nsys = 0;
  Batch bt;
  // device buffers (context allocator)
  double* x = nullptr;    // nsys N^3
  float* x32 = nullptr;   // nsys N^3 (mixed): increments since the last true residual
  double* fp = nullptr;   // nsys N^3, projected right-hand sides
  double* c64 = nullptr;  // ninst L^3 cell values
  float* c32 = nullptr;   // ninst L^3 (mixed)
  void *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  bf16_t* x16 = nullptr;
  void *T = nullptr, *U = nullptr;
  double* part = nullptr;
  size_t part_cap = 0;  // doubles of part per system
  Scalars* s = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t joined = nullptr;
};

struct BatchState {
  kp_context* ctx;
  bool mixed, fp16;
  std::vector<Group> groups;
  int* active = nullptr;  // one count per group (device)
  hipStream_t cap = nullptr;  // capture stream (the context stream may be the null stream)
  hipEvent_t fork = nullptr;
  std::vector<void*> owned;

  int alloc(void** p, size_t bytes) {
    KP_TRY(dev_alloc(ctx, p, bytes));
    owned.push_back(*p);
    return KP_OK;
  }
  ~BatchState() {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : owned) dev_free(ctx, p);
    for (Group& g : groups) {
      if (g.stream) (void)hipStreamDestroy(g.stream);
      if (g.joined) (void)hipEventDestroy(g.joined);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

int fin(kp_context* ctx, Group& g, int np, int nvals, int mode) {
  return launch_finalize(ctx, g.part, np, nvals, mode, g.s, g.n3, g.nsys);
}

// z = M r, the preconditioner dot products and p = (z - mz) + beta p.
int precondition_and_update(kp_context* ctx, BatchState& B, Group& g, int fin_mode, bool have_q) {
  int np = 0;
  if (B.mixed) {
    const PrecDots dots{(const float*)g.r, have_q ? (const float*)g.q : nullptr, g.part, g.part_cap};
    KP_TRY(launch_precond_16(ctx, g.pc, g.x16, (float*)g.z, g.s, g.bt, g.T, g.U, g.pc->tile_batch, &dots,
                             &np));
    if (np == 0)
      KP_TRY(launch_prec_dots<float>(ctx, (const float*)g.z, (const float*)g.r,
                                     have_q ? (const float*)g.q : nullptr, g.s, g.part, &np, g.n3, g.bt));
    KP_TRY(fin(ctx, g, np, 5, fin_mode));
    return launch_update_p<float>(ctx, (const float*)g.z, (float*)g.p, g.s, g.n3, g.bt);
  }
  KP_TRY(launch_precond_f64(ctx, g.pc, (const double*)g.r, (double*)g.z, g.s, g.bt, g.T, g.U,
                            g.pc->tile_batch));
  KP_TRY(launch_prec_dots<double>(ctx, (const double*)g.z, (const double*)g.r,
                                  have_q ? (const double*)g.q : nullptr, g.s, g.part, &np, g.n3, g.bt));
  KP_TRY(fin(ctx, g, np, 5, fin_mode));
  return launch_update_p<double>(ctx, (const double*)g.z, (double*)g.p, g.s, g.n3, g.bt);
}

// r = f - K x in double (into the iterate's precision), ||r||^2; gated systems only.
int true_residual(kp_context* ctx, BatchState& B, Group& g, int gate, int fin_mode) {
  int np = 0;
  if (B.mixed) KP_TRY(launch_fold(ctx, g.x, g.x32, g.n3, g.s, g.bt, gate));
  if (B.mixed)
    KP_TRY(launch_resid_f64_to_f32(ctx, g.x, g.c64, g.cg, g.fp, (float*)g.r, g.part, &np, g.s, g.N,
                                   g.bt, gate));
  else
    KP_TRY(launch_stencil_f64(ctx, g.x, g.c64, g.cg, g.fp, (double*)g.r, g.part, &np, g.s, g.N, g.bt,
                              gate));
  return fin(ctx, g, np, 1, fin_mode);
}

int iteration(kp_context* ctx, BatchState& B, Group& g) {
  int np = 0;
  if (B.mixed) {
    KP_TRY(launch_stencil_f32(ctx, (const float*)g.p, g.c32, g.cg, (float*)g.q, g.part, &np, g.s, g.N,
                              g.bt));
    KP_TRY(fin(ctx, g, np, 1, FIN_ALPHA));
    KP_TRY(launch_update_xr<float>(ctx, g.x, g.x32, (const float*)g.p, (float*)g.r, (const float*)g.q, g.x16,
                                   B.fp16, g.s, g.part, &np, g.n3, g.bt));
  } else {
    KP_TRY(launch_stencil_f64(ctx, (const double*)g.p, g.c64, g.cg, nullptr, (double*)g.q, g.part, &np,
                              g.s, g.N, g.bt));
    KP_TRY(fin(ctx, g, np, 1, FIN_ALPHA));
    KP_TRY(launch_update_xr<double>(ctx, g.x, nullptr, (const double*)g.p, (double*)g.r, (const double*)g.q,
                                    nullptr, 0, g.s, g.part, &np, g.n3, g.bt));
  }
  KP_TRY(fin(ctx, g, np, 1, FIN_RR_CTL));
  KP_TRY(true_residual(ctx, B, g, GATE_CHECK, FIN_TRUE_CTL));
  if (B.mixed)
    KP_TRY(launch_cast32_to16(ctx, (const float*)g.r, g.x16, g.n3, B.fp16, g.s, g.bt, GATE_REPLACED));
  return precondition_and_update(ctx, B, g, FIN_PREC, true);
}

// Enqueues `iters` iterations of every group, each group on its own stream
// between a fork and a join event of the context stream, then the counts of
// running systems.
int enqueue_chunk(kp_context* ctx, BatchState& B, int iters, bool concurrent) {
  hipStream_t main = ctx->stream;
  if (concurrent) KP_HIP(hipEventRecord(B.fork, main));
  int st = KP_OK;
  for (Group& g : B.groups) {
    if (concurrent) {
      KP_HIP(hipStreamWaitEvent(g.stream, B.fork, 0));
      ctx->stream = g.stream;
    }
    for (int i = 0; i < iters && st >= 0; ++i) st = iteration(ctx, B, g);
    ctx->stream = main;
    if (st < 0) return st;
    if (concurrent) {
      KP_HIP(hipEventRecord(g.joined, g.stream));
      KP_HIP(hipStreamWaitEvent(main, g.joined, 0));
    }
  }
  for (size_t k = 0; k < B.groups.size(); ++k)
    KP_TRY(launch_count_active(ctx, B.groups[k].s, B.groups[k].nsys, B.active + k));
  return KP_OK;
}

// Projects every system's x to zero mean (x <- x - mean x).
int project_x(kp_context* ctx, Group& g) {
  int np = 0;
  if (g.x32) KP_TRY(launch_fold(ctx, g.x, g.x32, g.n3, nullptr, g.bt));
  KP_TRY(launch_sum2(ctx, g.x, g.n3, g.part, &np, g.bt));
  KP_TRY(fin(ctx, g, np, 2, FIN_SUM));
  return launch_project_s(ctx, g.x, g.x, g.n3, g.s, g.bt);
}

}  // namespace

}  // namespace kp

using namespace kp;

extern "C" int pcg_solve_batched(kp_context* ctx, int n_inst, const kp_coeff* const* coeffs,
                                 const kp_precond* const* preconds, double* const* x_dev,
                                 const kp_solve_opts* opts, kp_solve_stats* stats, double* ahom) {
  if (!ctx || !coeffs || !preconds || !x_dev) return fail(KP_ERR_ARG, "pcg_solve_batched: NULL argument");
  if (n_inst < 1) return fail(KP_ERR_ARG, "pcg_solve_batched: n_inst must be >= 1");
  bool mixed = false;
  for (int i = 0; i < n_inst; ++i) {
    const kp_coeff* c = coeffs[i];
    const kp_precond* pc = preconds[i];
    if (!c || !pc) return fail(KP_ERR_ARG, "pcg_solve_batched: instance %d has a NULL handle", i);
    for (int j = 0; j < 3; ++j)
      if (!x_dev[3 * i + j]) return fail(KP_ERR_ARG, "pcg_solve_batched: x_dev[%d] is NULL", 3 * i + j);
    if (c->ctx != ctx || pc->ctx != ctx)
      return fail(KP_ERR_STATE, "pcg_solve_batched: instance %d: handles of another context", i);
    if (c->N != pc->N)
      return fail(KP_ERR_STATE, "pcg_solve_batched: instance %d: coefficient N=%d, preconditioner N=%d", i,
                  c->N, pc->N);
    const bool m = c->precision != KP_FP64;
    if (m != (pc->precision != KP_FP64))
      return fail(KP_ERR_STATE, "pcg_solve_batched: instance %d: coefficient and preconditioner precisions differ", i);
    if (i == 0) mixed = m;
    if (m != mixed) return fail(KP_ERR_STATE, "pcg_solve_batched: instances of different precisions");
  }
  kp_solve_opts o{1e-8, 2000, mixed ? 25 : 0, 0, 0};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.maxit < 0 || o.replace_every < 0 || o.check_every < 0)
    return fail(KP_ERR_ARG, "pcg_solve_batched: need tol > 0, maxit >= 0, replace_every >= 0, check_every >= 0");
  if (!mixed) o.replace_every = 0;
  const int chunk = o.check_every > 0 ? o.check_every : 16;
  KP_HIP(hipSetDevice(ctx->device));
  // The graph replays need the per-kernel timers off (no event nodes).
  const bool timing = ctx->timing;
  ctx->timing = false;
  struct Restore {
    kp_context* c;
    bool t;
    ~Restore() { c->timing = t; }
  } restore{ctx, timing};

  BatchState B;
  B.ctx = ctx;
  B.mixed = mixed;
  B.fp16 = preconds[0]->precision == KP_MIXED_FP16;
  {
    // Group key: preconditioner, cell size and sub-cell geometry (incl, background).
    std::map<std::tuple<const kp_precond*, int, int, double>, int> gid;
    for (int i = 0; i < n_inst; ++i) {
      const kp_coeff* c = coeffs[i];
      const auto key = std::make_tuple(preconds[i], c->n0, c->incl, c->incl < c->n0 ? c->bg : 0.0);
      auto it = gid.find(key);
      if (it == gid.end()) {
        it = gid.emplace(key, (int)B.groups.size()).first;
        B.groups.emplace_back();
        B.groups.back().pc = preconds[i];
        B.groups.back().n0 = c->n0;
        B.groups.back().L = c->L;
        B.groups.back().cg = geom_of(c);
      }
      B.groups[it->second].inst.push_back(i);
    }
  }
  const size_t word = mixed ? sizeof(float) : sizeof(double);
  size_t total_sys = 0;
  for (Group& g : B.groups) {
    if ((preconds[g.inst[0]]->precision == KP_MIXED_FP16) != B.fp16)
      return fail(KP_ERR_STATE, "pcg_solve_batched: BF16 and FP16 preconditioners in one batch");
    if (g.pc->fft)
      return fail(KP_ERR_STATE, "pcg_solve_batched: the FFT preconditioner is for single solves");
    if (g.pc->dim != 3 || coeffs[g.inst[0]]->dim != 3)
      return fail(KP_ERR_STATE, "pcg_solve_batched: 2D problems are solved one at a time (pcg_solve)");
    g.N = g.pc->N;
    g.n3 = (size_t)g.N * g.N * g.N;
    g.nsys = 3 * (int)g.inst.size();
    g.bt.nsys = g.nsys;
    g.bt.per = 3;
    g.bt.vs = g.n3;
    const size_t nc = (size_t)g.L * g.L * g.L;
    g.bt.ws = nc;
    total_sys += g.nsys;
    const size_t ns = g.nsys, ni = g.inst.size(), R = g.pc->R;
    const size_t parts = (size_t)8 * std::max(stencil_parts_max(g.N), vector_parts(g.n3));
    void* v;
    KP_TRY(B.alloc(&v, ns * g.n3 * sizeof(double))); g.x = (double*)v;
    KP_TRY(B.alloc(&v, ns * g.n3 * sizeof(double))); g.fp = (double*)v;
    KP_TRY(B.alloc(&v, ni * nc * sizeof(double))); g.c64 = (double*)v;
    if (mixed) {
      KP_TRY(B.alloc(&v, ni * nc * sizeof(float))); g.c32 = (float*)v;
      KP_TRY(B.alloc(&v, ns * g.n3 * sizeof(bf16_t))); g.x16 = (bf16_t*)v;
      KP_TRY(B.alloc(&v, ns * g.n3 * sizeof(float))); g.x32 = (float*)v;
      KP_HIP(hipMemsetAsync(g.x32, 0, ns * g.n3 * sizeof(float), ctx->stream));
    }
    KP_TRY(B.alloc(&g.r, ns * g.n3 * word));
    KP_TRY(B.alloc(&g.z, ns * g.n3 * word));
    KP_TRY(B.alloc(&g.p, ns * g.n3 * word));
    KP_TRY(B.alloc(&g.q, ns * g.n3 * word));
    const size_t el = mixed ? sizeof(bf16_t) : sizeof(double);
    KP_TRY(B.alloc(&g.T, ns * R * g.n3 * el));
    KP_TRY(B.alloc(&g.U, ns * R * g.n3 * el));
    KP_TRY(B.alloc(&v, ns * parts * sizeof(double))); g.part = (double*)v;
    g.part_cap = parts;
    KP_TRY(B.alloc(&v, ns * sizeof(Scalars))); g.s = (Scalars*)v;
  }
  {
    void* v;
    KP_TRY(B.alloc(&v, B.groups.size() * sizeof(int)));
    B.active = (int*)v;
  }
  const bool concurrent = B.groups.size() > 1;
  if (concurrent) {
    KP_HIP(hipEventCreateWithFlags(&B.fork, hipEventDisableTiming));
    for (Group& g : B.groups) {
      KP_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
      KP_HIP(hipEventCreateWithFlags(&g.joined, hipEventDisableTiming));
    }
  }

  // Tiles for each group, tuned once per preconditioner on a batch of about
  // 2^24 unknowns (every stage then has blocks enough to fill the chip; at most
  // the group's systems, a prefix of its buffers), so that the cost of tuning
  // does not grow with the batch and chunks of different sizes share one result.
  for (Group& g : B.groups) {
    const int nt = (int)std::min<size_t>((size_t)g.nsys, std::max<size_t>(1, ((size_t)1 << 24) / g.n3));
    if (g.pc->tuned_nsys == nt) continue;
    kp_precond* pcm = const_cast<kp_precond*>(g.pc);  // the tile cache only
    KP_TRY(autotune_precond(ctx, pcm, nt, 2, nullptr, 0, nullptr, pcm->tile_batch, g.T, g.U,
                            mixed ? (void*)g.x16 : g.r, g.z));
    pcm->tuned_nsys = nt;
  }

  KP_HIP(hipEventRecord(ctx->ev0, ctx->stream));
  // Gather the fields, the right-hand sides and the initial guesses.
  for (Group& g : B.groups) {
    for (size_t j = 0; j < g.inst.size(); ++j) {
      const kp_coeff* c = coeffs[g.inst[j]];
      const size_t nc = (size_t)g.L * g.L * g.L;
      KP_HIP(hipMemcpyAsync(g.c64 + j * nc, c->cells, nc * sizeof(double), hipMemcpyDeviceToDevice,
                            ctx->stream));
      if (mixed)
        KP_HIP(hipMemcpyAsync(g.c32 + j * nc, c->cells32, nc * sizeof(float), hipMemcpyDeviceToDevice,
                              ctx->stream));
      KP_HIP(hipMemcpyAsync(g.fp + j * 3 * g.n3, c->f, 3 * g.n3 * sizeof(double), hipMemcpyDeviceToDevice,
                            ctx->stream));
      for (int k = 0; k < 3; ++k) {
        double* xs = g.x + (3 * j + k) * g.n3;
        if (o.use_x0)
          KP_HIP(hipMemcpyAsync(xs, x_dev[3 * g.inst[j] + k], g.n3 * sizeof(double), hipMemcpyDeviceToDevice,
                                ctx->stream));
        else
          KP_TRY(launch_fill_f64(ctx, xs, 0.0, g.n3));
      }
    }
    std::vector<Scalars> h(g.nsys);
    for (Scalars& e : h) {
      std::memset(&e, 0, sizeof(Scalars));
      e.tol2ff = o.tol * o.tol;  // times ||f||^2 in FIN_FF
      e.flexible = mixed ? 1 : 0;
      e.x16_scale = e.x16_scale_next = 1.0;
      e.maxit = o.maxit;
      e.replace_every = o.replace_every;
    }
    KP_HIP(hipMemcpyAsync(g.s, h.data(), g.nsys * sizeof(Scalars), hipMemcpyHostToDevice, ctx->stream));
    KP_HIP(hipStreamSynchronize(ctx->stream));  // h goes out of scope
  }
  // f <- f - mean f, ||f||^2; r0 = f - K x0; z0 = M r0; p0 = z0 - mean z0.
  std::vector<std::vector<double>> rhs_mean(B.groups.size());
  for (size_t k = 0; k < B.groups.size(); ++k) {
    Group& g = B.groups[k];
    int np = 0;
    KP_TRY(launch_sum2(ctx, g.fp, g.n3, g.part, &np, g.bt));
    KP_TRY(fin(ctx, g, np, 2, FIN_SUM));
    KP_TRY(launch_project_s(ctx, g.fp, g.fp, g.n3, g.s, g.bt));
    std::vector<Scalars> h(g.nsys);
    KP_HIP(hipMemcpyAsync(h.data(), g.s, g.nsys * sizeof(Scalars), hipMemcpyDeviceToHost, ctx->stream));
    KP_HIP(hipStreamSynchronize(ctx->stream));
    for (const Scalars& e : h) rhs_mean[k].push_back(e.sums[0] / (double)g.n3);
    KP_TRY(launch_sum2(ctx, g.fp, g.n3, g.part, &np, g.bt));
    KP_TRY(fin(ctx, g, np, 2, FIN_FF));
    KP_TRY(true_residual(ctx, B, g, GATE_ACTIVE, FIN_RR_NOCOUNT));
    if (mixed)
      KP_TRY(launch_cast32_to16(ctx, (const float*)g.r, g.x16, g.n3, B.fp16, g.s, g.bt, GATE_ACTIVE));
    KP_TRY(precondition_and_update(ctx, B, g, FIN_PREC_INIT, false));
  }

  // Capture `chunk` iterations of every group in one graph and replay it.
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphGuard {
    hipGraph_t* g;
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } guard{&graph, &exec};
  if (o.maxit > 0) {
    KP_HIP(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
    hipStream_t main = ctx->stream;
    ctx->stream = B.cap;
    hipError_t ce = hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal);
    int cst = ce == hipSuccess ? enqueue_chunk(ctx, B, chunk, concurrent) : KP_OK;
    if (ce == hipSuccess) ce = hipStreamEndCapture(B.cap, &graph);
    ctx->stream = main;
    KP_TRY(cst);
    KP_HIP(ce);
    KP_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  std::vector<int> active(B.groups.size());
  const int max_launches = o.maxit > 0 ? o.maxit / chunk + 2 : 0;  // every system stops by maxit
  for (int l = 0; l < max_launches; ++l) {
    KP_HIP(hipGraphLaunch(exec, ctx->stream));
    KP_HIP(hipMemcpyAsync(active.data(), B.active, active.size() * sizeof(int), hipMemcpyDeviceToHost,
                          ctx->stream));
    KP_HIP(hipStreamSynchronize(ctx->stream));
    int left = 0;
    for (int a : active) left += a;
    if (left == 0) break;
  }

  // Zero-mean x, results back to the caller, a_hom per instance.
  for (Group& g : B.groups) KP_TRY(project_x(ctx, g));
  for (Group& g : B.groups)
    for (size_t j = 0; j < g.inst.size(); ++j)
      for (int k = 0; k < 3; ++k)
        KP_HIP(hipMemcpyAsync(x_dev[3 * g.inst[j] + k], g.x + (3 * j + k) * g.n3, g.n3 * sizeof(double),
                              hipMemcpyDeviceToDevice, ctx->stream));
  KP_HIP(hipEventRecord(ctx->ev1, ctx->stream));
  std::vector<double> ah;
  if (ahom) {
    void* res;
    KP_TRY(B.alloc(&res, (size_t)n_inst * 9 * sizeof(double)));
    size_t parts = 0;
    for (Group& g : B.groups) parts = std::max(parts, (size_t)g.nsys * 8 * vector_parts(g.n3));
    void* part;
    KP_TRY(ws_get(ctx, WS_PART, std::max(parts, (size_t)kMaxPartials * 8) * sizeof(double), &part));
    for (int i = 0; i < n_inst; ++i) {
      const double* phi[3] = {x_dev[3 * i], x_dev[3 * i + 1], x_dev[3 * i + 2]};
      KP_TRY(launch_ahom(ctx, coeffs[i], phi, (double*)part, (double*)res + 9 * i));
    }
    ah.resize((size_t)n_inst * 9);
    KP_HIP(hipMemcpyAsync(ah.data(), res, ah.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  KP_HIP(hipStreamSynchronize(ctx->stream));
  float ms = 0.f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  if (ahom) std::memcpy(ahom, ah.data(), ah.size() * sizeof(double));

  int n_fail = 0, n_break = 0;
  for (size_t k = 0; k < B.groups.size(); ++k) {
    Group& g = B.groups[k];
    std::vector<Scalars> h(g.nsys);
    KP_HIP(hipMemcpy(h.data(), g.s, g.nsys * sizeof(Scalars), hipMemcpyDeviceToHost));
    for (int b = 0; b < g.nsys; ++b) {
      const Scalars& e = h[b];
      int status = KP_OK;
      if (e.status == 3 || e.breakdown) {
        status = KP_ERR_BREAKDOWN;
        ++n_break;
      } else if (e.status != 1) {
        status = KP_NOT_CONVERGED;
        ++n_fail;
      }
      if (stats) {
        kp_solve_stats& st = stats[3 * g.inst[b / 3] + b % 3];
        std::memset(&st, 0, sizeof(st));
        st.iters = e.iters;
        st.replacements = e.replacements;
        st.relres_true = e.ff > 0.0 ? std::sqrt(e.rr / e.ff) : 0.0;
        st.relres_rec = e.ff > 0.0 ? std::sqrt(e.rr_rec / e.ff) : 0.0;
        st.rhs_mean = rhs_mean[k][b];
        st.ms = ms;
        st.status = status;
      }
    }
  }
  if (n_break) return fail(KP_ERR_BREAKDOWN, "pcg_solve_batched: %d of %zu systems broke down", n_break, total_sys);
  return n_fail ? KP_NOT_CONVERGED : KP_OK;
}

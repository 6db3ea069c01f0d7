// Host construction of the canonical factors of the low-rank preconditioner
// symbol (Section 4.2: Tucker decomposition of the reshaped Fourier-diagonal
// pseudo-inverse G+ of eq. 3a followed by the Tucker-to-canonical transform;
// Lemma RankPinverse for the Laplace-transform quadrature).
//
// The paper leaves norms, ranks and the algorithm open.  The construction used
// here, step by step:
//  1. mu_k = 4 sin^2(pi k / N); g = mu_i + mu_j + mu_k; G+ = 1/g, 0 at (0,0,0).
//  2. Laplace quadrature: with t = e^s, 1/x = int exp(-x e^s + s) ds; the
//     trapezoidal rule with step eta on s_k = -ln(12) - shift + k eta gives
//     1/x ~ sum_k w_k exp(-t_k x), t_k = e^{s_k}, w_k = eta t_k.  (eta, shift)
//     come from the grid eta = 0.30 + 0.025 j (j < 49), shift = -2 + 0.1 i
//     (i < 61), minimizing max |x q(x) - 1| on 257 geometric samples of
//     [mu_1, 12] (the first strict minimum in that scan order), then refined
//     towards the best relative approximation of 1/x by R exponentials
//     (refined_quadrature below).
//  3. The zero mode is removed by the zero-mean projection of the solver, so
//     its value is free: it is set to the quadrature value sum_k w_k (rank 12,
//     or the requested rank) to keep the tensor smooth.
//  4. Relative weighting by the rank-one tensor s x s x s, s_i = (mu_i+mu_1)^(1/3).
//  5. Tucker: the mode-1 Gram matrix of the weighted tensor; its leading
//     eigenvectors U (r_T of them: the smallest count whose discarded tail is
//     <= eps^2 ||W||^2 / 3, and at least R); core B = W x1 U^T x2 U^T x3 U^T.
//  6. Tucker-to-canonical: CP-ALS on B, rank R, started from the quadrature
//     factors projected on U, 50 sweeps.  rank = 0 selects the smallest R >= 2
//     with ||B - CP|| <= eps ||B|| (else r_T).
//  7. Factors u = U v / s.  Whichever of the ALS factors and the quadrature
//     factors has the smaller spread rho_max / rho_min (rho = G_R g on the
//     nonzero modes) is returned; rho_min <= 0 is an error.
//
// Every factor is even in its index (mu_k = mu_{N-k}), so all tensors are
// handled on the H+1 = N/2+1 distinct indices with multiplicities 1 or 2,
// which is exact and about 8x cheaper than the full grid.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "kronpcg.h"

namespace kp {
int fail(int code, const char* fmt, ...);
}

namespace {

constexpr int kSamples = 257;
constexpr int kSweeps = 50;
constexpr double kTop = 12.0;
constexpr int kMaxRank = 16;

struct Quadrature {
  std::vector<double> t, w;
  double err = 0.0;
};

Quadrature laplace_quadrature(int R, double a, double b) {
  std::vector<double> x(kSamples);
  for (int m = 0; m < kSamples; ++m) x[m] = a * std::pow(b / a, (double)m / (double)(kSamples - 1));
  Quadrature best;
  bool have = false;
  std::vector<double> t(R), w(R);
  for (int j = 0; j < 49; ++j) {
    const double eta = 0.30 + 0.025 * j;
    for (int i = 0; i < 61; ++i) {
      const double shift = -2.0 + 0.1 * i;
      for (int k = 0; k < R; ++k) {
        const double s = -std::log(b) - shift + eta * k;
        t[k] = std::exp(s);
        w[k] = eta * t[k];
      }
      double err = 0.0;
      for (int m = 0; m < kSamples; ++m) {
        double q = 0.0;
        for (int k = 0; k < R; ++k) q += std::exp(-x[m] * t[k]) * w[k];
        err = std::max(err, std::fabs(x[m] * q - 1.0));
      }
      if (!have || err < best.err) {
        best.t = t;
        best.w = w;
        best.err = err;
        have = true;
      }
    }
  }
  return best;
}

// Solve G x = b for an R x R system (partial pivoting); G and b are copied.
void solve_small(std::vector<double> G, std::vector<double>& b, int R);

// The quadrature refined towards the best relative (minimax) approximation of
// 1/x on [a, b] by R exponentials: parameters (ln t_k, ln w_k); Lawson
// reweighting (20 passes) of damped Gauss-Newton steps (at most 50 per pass,
// 10 damping tries per step, steps clipped to [-2, 2] per component) on 513
// geometric samples; the iterate with the smallest max relative error wins.
Quadrature refined_quadrature(int R, double a, double b) {
  Quadrature best = laplace_quadrature(R, a, b);
  constexpr int M = 513;
  std::vector<double> x(M), wts(M, 1.0);
  for (int m = 0; m < M; ++m) x[m] = a * std::pow(b / a, (double)m / (double)(M - 1));
  const int P = 2 * R;
  std::vector<double> th(P), E((size_t)M * R), e(M), tt(R);
  for (int k = 0; k < R; ++k) {
    th[k] = std::log(best.t[k]);
    th[R + k] = std::log(best.w[k]);
  }
  // e = x q(x) - 1 at parameters p; also E[m][k] = w_k exp(-t_k x_m) and tt = t.
  auto resid = [&](const std::vector<double>& p, std::vector<double>& ee) {
    for (int k = 0; k < R; ++k) tt[k] = std::exp(p[k]);
    for (int m = 0; m < M; ++m) {
      double q = 0.0;
      for (int k = 0; k < R; ++k) {
        const double v = std::exp(-x[m] * tt[k]) * std::exp(p[R + k]);
        E[(size_t)m * R + k] = v;
        q += v;
      }
      ee[m] = x[m] * q - 1.0;
    }
  };
  auto wsum2 = [&](const std::vector<double>& ee) {
    double f = 0.0;
    for (int m = 0; m < M; ++m) f += (wts[m] * ee[m]) * (wts[m] * ee[m]);
    return f;
  };
  std::vector<double> J((size_t)M * P), A((size_t)P * P), g(P), D(P), d(P), th1(P), e1(M);
  for (int outer = 0; outer < 20; ++outer) {
    double lam = 1e-3;
    for (int inner = 0; inner < 50; ++inner) {
      resid(th, e);
      for (int m = 0; m < M; ++m) {
        const double s = wts[m] * x[m];
        for (int k = 0; k < R; ++k) {
          const double v = E[(size_t)m * R + k];
          J[(size_t)m * P + k] = s * (-x[m] * tt[k] * v);
          J[(size_t)m * P + R + k] = s * v;
        }
      }
      double dmax = 0.0;
      for (int i = 0; i < P; ++i) {
        for (int j = 0; j < P; ++j) {
          double acc = 0.0;
          for (int m = 0; m < M; ++m) acc += J[(size_t)m * P + i] * J[(size_t)m * P + j];
          A[(size_t)i * P + j] = acc;
        }
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += J[(size_t)m * P + i] * (wts[m] * e[m]);
        g[i] = acc;
        dmax = std::max(dmax, A[(size_t)i * P + i]);
      }
      for (int i = 0; i < P; ++i) D[i] = A[(size_t)i * P + i] + 1e-12 * dmax;
      const double f0 = wsum2(e);
      double f1 = f0;
      bool accepted = false;
      for (int tries = 0; tries < 10; ++tries) {
        std::vector<double> Gm(A);
        for (int i = 0; i < P; ++i) {
          Gm[(size_t)i * P + i] += lam * D[i];
          d[i] = -g[i];
        }
        solve_small(Gm, d, P);
        for (int i = 0; i < P; ++i) th1[i] = th[i] + std::min(2.0, std::max(-2.0, d[i]));
        resid(th1, e1);
        f1 = wsum2(e1);
        if (std::isfinite(f1) && f1 < f0) {
          th = th1;
          lam = std::max(lam / 10.0, 1e-12);
          accepted = true;
          break;
        }
        lam *= 10.0;
      }
      if (!accepted || f0 - f1 <= 1e-15 * f0) break;
    }
    resid(th, e);
    double mx = 0.0;
    for (int m = 0; m < M; ++m) mx = std::max(mx, std::fabs(e[m]));
    if (mx < best.err) {
      best.err = mx;
      for (int k = 0; k < R; ++k) {
        best.t[k] = std::exp(th[k]);
        best.w[k] = std::exp(th[R + k]);
      }
    }
    double wmax = 0.0;
    for (int m = 0; m < M; ++m) {
      wts[m] *= std::sqrt(std::fabs(e[m]) / mx + 1e-3);
      wmax = std::max(wmax, wts[m]);
    }
    for (int m = 0; m < M; ++m) wts[m] /= wmax;
  }
  return best;
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major).
// On return A holds the eigenvalues on its diagonal and V the eigenvectors as columns.
void jacobi_eigen(std::vector<double>& A, std::vector<double>& V, int n) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// Solve G x = b for an R x R system (partial pivoting); G and b are copied.
void solve_small(std::vector<double> G, std::vector<double>& b, int R) {
  for (int c = 0; c < R; ++c) {
    int piv = c;
    for (int r = c + 1; r < R; ++r)
      if (std::fabs(G[(size_t)r * R + c]) > std::fabs(G[(size_t)piv * R + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < R; ++k) std::swap(G[(size_t)c * R + k], G[(size_t)piv * R + k]);
      std::swap(b[c], b[piv]);
    }
    const double d = G[(size_t)c * R + c];
    for (int r = c + 1; r < R; ++r) {
      const double f = G[(size_t)r * R + c] / d;
      for (int k = c; k < R; ++k) G[(size_t)r * R + k] -= f * G[(size_t)c * R + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = R - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < R; ++k) s -= G[(size_t)r * R + k] * b[k];
    b[r] = s / G[(size_t)r * R + r];
  }
}

void parallel_for(int n, const std::function<void(int)>& body) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hw ? hw : 1u, 16u);
  nt = std::max(1, std::min(nt, n));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int i = t; i < n; i += nt) body(i);
    });
  for (auto& x : th) x.join();
}

struct Even {
  int N, H, nr;
  std::vector<double> m;  // multiplicity of reduced index i in 0..H
  explicit Even(int N_) : N(N_), H(N_ / 2), nr(N_ / 2 + 1), m(N_ / 2 + 1, 2.0) {
    m[0] = 1.0;
    if (N % 2 == 0) m[H] = 1.0;
    if (N == 1) m[0] = 1.0;
  }
};

// rho = G_R * g over the nonzero modes (reduced indices cover all by evenness).
void rho_range(const std::vector<double>& F, int R, const Even& E, const std::vector<double>& mu,
               double* lo, double* hi) {
  const int nr = E.nr;
  std::vector<double> plo(nr, 1e300), phi(nr, -1e300);
  parallel_for(nr, [&](int i) {
    double l = 1e300, h = -1e300;
    for (int j = 0; j < nr; ++j)
      for (int k = 0; k < nr; ++k) {
        if (i == 0 && j == 0 && k == 0) continue;
        double g = 0.0;
        for (int r = 0; r < R; ++r)
          g += F[(size_t)(0 * R + r) * nr + i] * F[(size_t)(1 * R + r) * nr + j] * F[(size_t)(2 * R + r) * nr + k];
        const double rho = g * (mu[i] + mu[j] + mu[k]);
        l = std::min(l, rho);
        h = std::max(h, rho);
      }
    plo[i] = l;
    phi[i] = h;
  });
  *lo = *std::min_element(plo.begin(), plo.end());
  *hi = *std::max_element(phi.begin(), phi.end());
}

double cancellation(const std::vector<double>& F, int R, const Even& E) {
  const int nr = E.nr;
  auto nrm = [&](int l, int r) {
    double s = 0.0;
    for (int i = 0; i < nr; ++i) s += E.m[i] * F[(size_t)(l * R + r) * nr + i] * F[(size_t)(l * R + r) * nr + i];
    return std::sqrt(s);
  };
  double terms = 0.0;
  for (int r = 0; r < R; ++r) terms += nrm(0, r) * nrm(1, r) * nrm(2, r);
  // ||G_R||_F^2 = sum_{r,s} prod_l <u_l^r, u_l^s>
  double g2 = 0.0;
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < R; ++s) {
      double p = 1.0;
      for (int l = 0; l < 3; ++l) {
        double d = 0.0;
        for (int i = 0; i < nr; ++i)
          d += E.m[i] * F[(size_t)(l * R + r) * nr + i] * F[(size_t)(l * R + s) * nr + i];
        p *= d;
      }
      g2 += p;
    }
  return terms / std::sqrt(std::max(g2, 1e-300));
}

}  // namespace

extern "C" int kp_lowrank_factors(int N, double eps, int rank, double* out, size_t capacity,
                                  kp_precond_info* info) {
  using kp::fail;
  const auto t0 = std::chrono::steady_clock::now();
  if (N < 2 || N > 1024) return fail(KP_ERR_ARG, "kp_lowrank_factors: N = %d not in [2, 1024]", N);
  if (!(eps > 0.0 && eps < 1.0)) return fail(KP_ERR_ARG, "kp_lowrank_factors: eps must be in (0,1)");
  if (rank < 0 || rank > kMaxRank) return fail(KP_ERR_ARG, "kp_lowrank_factors: rank must be 0..16");
  if (!out) return fail(KP_ERR_ARG, "kp_lowrank_factors: NULL output");
  const Even E(N);
  const int nr = E.nr;
  if (rank > nr) return fail(KP_ERR_ARG, "kp_lowrank_factors: rank %d exceeds N/2+1 = %d", rank, nr);

  std::vector<double> mu(N);
  for (int k = 0; k < N; ++k) {
    const double sn = std::sin(M_PI * (double)k / (double)N);
    mu[k] = 4.0 * sn * sn;
  }
  const double a = mu[1], b = kTop;
  std::vector<double> s(nr);
  for (int i = 0; i < nr; ++i) s[i] = std::cbrt(mu[i] + mu[1]);

  // 1-4: weighted symbol on the reduced grid.
  const Quadrature qref = refined_quadrature(rank > 0 ? rank : 12, a, b);
  double fill = 0.0;
  for (double w : qref.w) fill += w;
  const size_t nr2 = (size_t)nr * nr, nr3 = nr2 * nr;
  std::vector<double> W(nr3);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nr; ++j)
      for (int k = 0; k < nr; ++k) {
        const double g = mu[i] + mu[j] + mu[k];
        const double gp = (i == 0 && j == 0 && k == 0) ? fill : 1.0 / g;
        W[((size_t)i * nr + j) * nr + k] = s[i] * s[j] * s[k] * gp;
      }

  // 5: Gram matrix of the mode-1 unfolding (full grid) in symmetrized reduced form
  //    S[i][i'] = sqrt(m_i m_i') sum_{j,k} m_j m_k W[i][j][k] W[i'][j][k].
  std::vector<double> mjk(nr2);
  for (int j = 0; j < nr; ++j)
    for (int k = 0; k < nr; ++k) mjk[(size_t)j * nr + k] = E.m[j] * E.m[k];
  std::vector<double> S(nr2);
  parallel_for(nr, [&](int i) {
    const double* wi = &W[(size_t)i * nr2];
    for (int i2 = 0; i2 <= i; ++i2) {
      const double* wj = &W[(size_t)i2 * nr2];
      double acc = 0.0;
      for (size_t t = 0; t < nr2; ++t) acc += mjk[t] * wi[t] * wj[t];
      acc *= std::sqrt(E.m[i] * E.m[i2]);
      S[(size_t)i * nr + i2] = acc;
      S[(size_t)i2 * nr + i] = acc;
    }
  });
  std::vector<double> V;
  jacobi_eigen(S, V, nr);
  std::vector<int> order(nr);
  for (int i = 0; i < nr; ++i) order[i] = i;
  std::vector<double> ev(nr);
  for (int i = 0; i < nr; ++i) ev[i] = S[(size_t)i * nr + i];
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ev[x] > ev[y]; });
  std::vector<double> evs(nr);
  double total = 0.0;
  for (int i = 0; i < nr; ++i) {
    evs[i] = std::max(ev[order[i]], 0.0);
    total += evs[i];
  }
  int rT = nr;
  for (int rr = 1; rr <= nr; ++rr) {
    double tail = 0.0;
    for (int i = rr; i < nr; ++i) tail += evs[i];
    if (tail <= eps * eps * total / 3.0) {
      rT = rr;
      break;
    }
  }
  rT = std::min(std::max(rT, std::max(rank, 1)), nr);
  // U (reduced rows, full-space orthonormal): U[i][c] = z_c[i] / sqrt(m_i)
  std::vector<double> U((size_t)nr * rT);
  for (int i = 0; i < nr; ++i)
    for (int c = 0; c < rT; ++c) U[(size_t)i * rT + c] = V[(size_t)i * nr + order[c]] / std::sqrt(E.m[i]);

  // Core B[a][b][c] = sum_{ijk} m_i m_j m_k W[i][j][k] U[i][a] U[j][b] U[k][c].
  std::vector<double> T1((size_t)rT * nr2, 0.0);
  parallel_for(rT, [&](int a2) {
    for (int i = 0; i < nr; ++i) {
      const double f = E.m[i] * U[(size_t)i * rT + a2];
      const double* wi = &W[(size_t)i * nr2];
      double* t = &T1[(size_t)a2 * nr2];
      for (size_t q = 0; q < nr2; ++q) t[q] += f * wi[q];
    }
  });
  std::vector<double> T2((size_t)rT * rT * nr, 0.0);  // [a][b][k]
  for (int a2 = 0; a2 < rT; ++a2)
    for (int j = 0; j < nr; ++j)
      for (int b2 = 0; b2 < rT; ++b2) {
        const double f = E.m[j] * U[(size_t)j * rT + b2];
        const double* t1 = &T1[((size_t)a2 * nr + j) * nr];
        double* t2 = &T2[((size_t)a2 * rT + b2) * nr];
        for (int k = 0; k < nr; ++k) t2[k] += f * t1[k];
      }
  const size_t rT3 = (size_t)rT * rT * rT;
  std::vector<double> B(rT3, 0.0);
  for (int a2 = 0; a2 < rT; ++a2)
    for (int b2 = 0; b2 < rT; ++b2)
      for (int c2 = 0; c2 < rT; ++c2) {
        double acc = 0.0;
        const double* t2 = &T2[((size_t)a2 * rT + b2) * nr];
        for (int k = 0; k < nr; ++k) acc += E.m[k] * U[(size_t)k * rT + c2] * t2[k];
        B[((size_t)a2 * rT + b2) * rT + c2] = acc;
      }
  double nB = 0.0;
  for (double v : B) nB += v * v;
  nB = std::sqrt(nB);

  // 6: Tucker-to-canonical by ALS.
  std::vector<int> ranks;
  if (rank > 0) ranks.push_back(rank);
  else
    for (int r = 2; r <= rT; ++r) ranks.push_back(r);
  int R = 0;
  double cperr = 0.0;
  Quadrature q;
  std::vector<double> Vf[3];
  std::vector<double> uq;
  for (int Rc : ranks) {
    R = Rc;
    q = refined_quadrature(R, a, b);
    uq.assign((size_t)R * nr, 0.0);  // [k][i] reduced
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < nr; ++i) uq[(size_t)k * nr + i] = std::cbrt(q.w[k]) * std::exp(-q.t[k] * mu[i]);
    std::vector<double> V0((size_t)rT * R, 0.0);  // [a][k] = sum_i (full) U[i][a] s_i uq[k][i]
    for (int a2 = 0; a2 < rT; ++a2)
      for (int k = 0; k < R; ++k) {
        double acc = 0.0;
        for (int i = 0; i < nr; ++i) acc += E.m[i] * U[(size_t)i * rT + a2] * s[i] * uq[(size_t)k * nr + i];
        V0[(size_t)a2 * R + k] = acc;
      }
    for (int m = 0; m < 3; ++m) Vf[m] = V0;
    std::vector<double> M((size_t)rT * R), G((size_t)R * R), rhs(R);
    for (int sweep = 0; sweep < kSweeps; ++sweep) {
      for (int m = 0; m < 3; ++m) {
        const std::vector<double>& P = Vf[m == 0 ? 1 : 0];
        const std::vector<double>& Q = Vf[m == 2 ? 1 : 2];
        // MTTKRP
        for (int x = 0; x < rT; ++x)
          for (int r = 0; r < R; ++r) {
            double acc = 0.0;
            for (int y = 0; y < rT; ++y)
              for (int z = 0; z < rT; ++z) {
                double bv;
                if (m == 0) bv = B[((size_t)x * rT + y) * rT + z];
                else if (m == 1) bv = B[((size_t)y * rT + x) * rT + z];
                else bv = B[((size_t)y * rT + z) * rT + x];
                acc += bv * P[(size_t)y * R + r] * Q[(size_t)z * R + r];
              }
            M[(size_t)x * R + r] = acc;
          }
        for (int r = 0; r < R; ++r)
          for (int t = 0; t < R; ++t) {
            double gp = 0.0, gq = 0.0;
            for (int y = 0; y < rT; ++y) {
              gp += P[(size_t)y * R + r] * P[(size_t)y * R + t];
              gq += Q[(size_t)y * R + r] * Q[(size_t)y * R + t];
            }
            G[(size_t)r * R + t] = gp * gq;
          }
        for (int x = 0; x < rT; ++x) {
          for (int r = 0; r < R; ++r) rhs[r] = M[(size_t)x * R + r];
          solve_small(G, rhs, R);
          for (int r = 0; r < R; ++r) Vf[m][(size_t)x * R + r] = rhs[r];
        }
      }
    }
    double e2 = 0.0;
    for (int x = 0; x < rT; ++x)
      for (int y = 0; y < rT; ++y)
        for (int z = 0; z < rT; ++z) {
          double cp = 0.0;
          for (int r = 0; r < R; ++r)
            cp += Vf[0][(size_t)x * R + r] * Vf[1][(size_t)y * R + r] * Vf[2][(size_t)z * R + r];
          const double d = B[((size_t)x * rT + y) * rT + z] - cp;
          e2 += d * d;
        }
    cperr = std::sqrt(e2) / nB;
    if (rank > 0 || cperr <= eps) break;
  }

  // 7: candidates on the reduced grid, [l][k][i].
  std::vector<double> Fa((size_t)3 * R * nr), Fq((size_t)3 * R * nr);
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < nr; ++i) {
        double acc = 0.0;
        for (int a2 = 0; a2 < rT; ++a2) acc += U[(size_t)i * rT + a2] * Vf[l][(size_t)a2 * R + k];
        Fa[((size_t)l * R + k) * nr + i] = acc / s[i];
        Fq[((size_t)l * R + k) * nr + i] = uq[(size_t)k * nr + i];
      }
  double loA, hiA, loQ, hiQ;
  rho_range(Fa, R, E, mu, &loA, &hiA);
  rho_range(Fq, R, E, mu, &loQ, &hiQ);
  const double sprA = loA > 0 ? hiA / loA : INFINITY;
  const double sprQ = loQ > 0 ? hiQ / loQ : INFINITY;
  const bool useA = sprA <= sprQ;
  const std::vector<double>& F = useA ? Fa : Fq;

  kp_precond_info inf{};
  inf.rank = R;
  inf.tucker_rank = rT;
  inf.source = useA ? 0 : 1;
  inf.cp_rel_err = cperr;
  inf.quad_rel_err = q.err;
  inf.rho_min = useA ? loA : loQ;
  inf.rho_max = useA ? hiA : hiQ;
  inf.cancellation = cancellation(F, R, E);
  inf.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (!(inf.rho_min > 0.0))
    return fail(KP_ERR_PRECOND_INDEFINITE, "kp_lowrank_factors: rho_min = %g <= 0", inf.rho_min);
  if (capacity < (size_t)3 * R * N)
    return fail(KP_ERR_ARG, "kp_lowrank_factors: capacity %zu < 3*R*N = %zu", capacity, (size_t)3 * R * N);
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < N; ++i) {
        const int ri = std::min(i, N - i);
        out[((size_t)l * R + k) * N + i] = F[((size_t)l * R + k) * nr + ri];
      }
  return KP_OK;
}

// ---------------------------------------------------------------- d = 2
// Rank-R factors of the 2D preconditioner symbol 1 / (mu_k1 + mu_k2) (eq.
// DiagFLaplace2D; the 2D decomposition before eq. Lap2DtimesX).  In two
// dimensions the Tucker and canonical forms coincide with the truncated
// eigen-expansion of the (symmetric) symbol matrix, which is the best rank-R
// approximation in the Frobenius norm.  Construction:
//  1. Relative weighting W = s s^T * G+ with s_i = sqrt(mu_i + mu_1), so the
//     approximation error is relative to the symbol; the zero mode (free: the
//     solver projects it out) is set to 1/mu_1, its nearest nonzero modes' value.
//  2. Even indices: the reduced nr x nr matrix M = D^(1/2) W D^(1/2) with the
//     multiplicities D has the full grid's Frobenius geometry.
//  3. Its leading eigenpairs by |lambda|: cyclic Jacobi for nr <= 160, else
//     subspace iteration on 64 vectors (10 multiplications, each followed by
//     two modified Gram-Schmidt passes, then Rayleigh-Ritz with Jacobi).
//  4. rank = 0: the smallest R with ||M - M_R||_F <= eps ||M||_F.
//  5. u1 = sqrt|lambda| z / (s sqrt m), u2 = sign(lambda) u1; rho = G_R g on the
//     nonzero modes must be positive.
extern "C" int kp_lowrank_factors_2d(int N, double eps, int rank, double* out, size_t capacity,
                                     kp_precond_info* info) {
  using kp::fail;
  const auto t0 = std::chrono::steady_clock::now();
  if (N < 2 || N > 2048) return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: N = %d not in [2, 2048]", N);
  if (!(eps > 0.0 && eps < 1.0)) return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: eps must be in (0,1)");
  if (rank < 0 || rank > kMaxRank) return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: rank must be 0..16");
  if (!out) return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: NULL output");
  const Even E(N);
  const int nr = E.nr;
  std::vector<double> mu(N);
  for (int k = 0; k < N; ++k) {
    const double sn = std::sin(M_PI * (double)k / (double)N);
    mu[k] = 4.0 * sn * sn;
  }
  std::vector<double> s(nr), sq(nr);
  for (int i = 0; i < nr; ++i) {
    s[i] = std::sqrt(mu[i] + mu[1 % N]);
    sq[i] = std::sqrt(E.m[i]);
  }
  std::vector<double> M((size_t)nr * nr);
  double total = 0.0;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nr; ++j) {
      const double g = mu[i] + mu[j];
      const double gp = (i == 0 && j == 0) ? 1.0 / mu[1 % N] : 1.0 / g;
      const double v = sq[i] * sq[j] * s[i] * s[j] * gp;
      M[(size_t)i * nr + j] = v;
      total += v * v;
    }
  // Leading eigenpairs (lam, Z columns over the reduced index).
  std::vector<double> lam, Z;
  int p;
  if (nr <= 160) {
    std::vector<double> A = M, V;
    jacobi_eigen(A, V, nr);
    p = nr;
    lam.resize(p);
    for (int c = 0; c < p; ++c) lam[c] = A[(size_t)c * nr + c];
    Z = V;  // [i][c]
  } else {
    p = 64;
    std::vector<double> Q((size_t)nr * p), Y((size_t)nr * p);
    for (int i = 0; i < nr; ++i)  // deterministic start: cosines of increasing frequency
      for (int c = 0; c < p; ++c) Q[(size_t)i * p + c] = std::cos(M_PI * (double)c * (i + 0.5) / nr);
    auto orth = [&](std::vector<double>& X) {  // modified Gram-Schmidt on columns
      for (int c = 0; c < p; ++c) {
        for (int d = 0; d < c; ++d) {
          double dot = 0.0;
          for (int i = 0; i < nr; ++i) dot += X[(size_t)i * p + c] * X[(size_t)i * p + d];
          for (int i = 0; i < nr; ++i) X[(size_t)i * p + c] -= dot * X[(size_t)i * p + d];
        }
        double nrm = 0.0;
        for (int i = 0; i < nr; ++i) nrm += X[(size_t)i * p + c] * X[(size_t)i * p + c];
        nrm = std::sqrt(std::max(nrm, 1e-300));
        for (int i = 0; i < nr; ++i) X[(size_t)i * p + c] /= nrm;
      }
    };
    auto mult = [&](const std::vector<double>& X, std::vector<double>& out_) {
      parallel_for(nr, [&](int i) {
        double* o = &out_[(size_t)i * p];
        for (int c = 0; c < p; ++c) o[c] = 0.0;
        for (int j = 0; j < nr; ++j) {
          const double mij = M[(size_t)i * nr + j];
          const double* x = &X[(size_t)j * p];
          for (int c = 0; c < p; ++c) o[c] += mij * x[c];
        }
      });
    };
    orth(Q);
    for (int it = 0; it < 10; ++it) {
      mult(Q, Y);
      Q.swap(Y);
      orth(Q);  // twice: one Gram-Schmidt pass loses orthogonality on the
      orth(Q);  // nearly parallel columns of M Q
    }
    mult(Q, Y);  // B = Q^T M Q
    std::vector<double> B((size_t)p * p), V;
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double acc = 0.0;
        for (int i = 0; i < nr; ++i) acc += Q[(size_t)i * p + a] * Y[(size_t)i * p + b];
        B[(size_t)a * p + b] = acc;
      }
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < a; ++b) B[(size_t)a * p + b] = B[(size_t)b * p + a] = 0.5 * (B[(size_t)a * p + b] + B[(size_t)b * p + a]);
    jacobi_eigen(B, V, p);
    lam.resize(p);
    for (int c = 0; c < p; ++c) lam[c] = B[(size_t)c * p + c];
    Z.assign((size_t)nr * p, 0.0);
    for (int i = 0; i < nr; ++i)
      for (int c = 0; c < p; ++c) {
        double acc = 0.0;
        for (int a = 0; a < p; ++a) acc += Q[(size_t)i * p + a] * V[(size_t)a * p + c];
        Z[(size_t)i * p + c] = acc;
      }
  }
  std::vector<int> order(p);
  for (int c = 0; c < p; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return std::fabs(lam[x]) > std::fabs(lam[y]); });
  int R = rank;
  double kept = 0.0;
  if (R == 0) {
    R = std::min(p, kMaxRank);
    for (int r = 1; r <= std::min(p, kMaxRank); ++r) {
      kept += lam[order[r - 1]] * lam[order[r - 1]];
      if (total - kept <= eps * eps * total) {
        R = r;
        break;
      }
    }
  }
  if (R > p) return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: rank %d exceeds %d", R, p);
  kept = 0.0;
  for (int r = 0; r < R; ++r) kept += lam[order[r]] * lam[order[r]];
  // Factors on the reduced grid: [mode][k][i].
  std::vector<double> F((size_t)2 * R * nr);
  for (int k = 0; k < R; ++k) {
    const int c = order[k];
    const double a = std::sqrt(std::fabs(lam[c])), sg = lam[c] >= 0 ? 1.0 : -1.0;
    for (int i = 0; i < nr; ++i) {
      const double u = a * Z[(size_t)i * p + c] / (s[i] * sq[i]);
      F[(size_t)k * nr + i] = u;
      F[((size_t)R + k) * nr + i] = sg * u;
    }
  }
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nr; ++j) {
      if (i == 0 && j == 0) continue;
      double gr = 0.0;
      for (int k = 0; k < R; ++k) gr += F[(size_t)k * nr + i] * F[((size_t)R + k) * nr + j];
      const double rho = gr * (mu[i] + mu[j]);
      lo = std::min(lo, rho);
      hi = std::max(hi, rho);
    }
  kp_precond_info inf{};
  inf.rank = R;
  inf.tucker_rank = R;
  inf.source = 0;
  inf.cp_rel_err = std::sqrt(std::max(total - kept, 0.0) / total);
  inf.rho_min = lo;
  inf.rho_max = hi;
  inf.cancellation = 1.0;
  inf.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (!(lo > 0.0)) return fail(KP_ERR_PRECOND_INDEFINITE, "kp_lowrank_factors_2d: rho_min = %g <= 0", lo);
  if (capacity < (size_t)2 * R * N)
    return fail(KP_ERR_ARG, "kp_lowrank_factors_2d: capacity %zu < 2*R*N = %zu", capacity, (size_t)2 * R * N);
  for (int l = 0; l < 2; ++l)
    for (int k = 0; k < R; ++k)
      for (int i = 0; i < N; ++i) out[((size_t)l * R + k) * N + i] = F[((size_t)l * R + k) * nr + std::min(i, N - i)];
  return KP_OK;
}

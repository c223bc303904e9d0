// Host unit test of the reverse-communication quasi-Newton minimiser
// (bx_fitcore.hpp): quadratics, Rosenbrock, box bounds (minima on a bound
// and just inside it, a Poisson fit of overlapping templates), fixed
// parameters, single evaluations and a domain wall.  Built with g++ by test_host.py.
#include <cmath>
#include <cstdio>
#include <string>

#include "../../paper_1805_11125_amd/csrc/bx_fitcore.hpp"

namespace bx {
void set_error(const std::string&) {}
}
using namespace bx;

static int fails = 0;
#define CHECK(c, msg)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      std::printf("FAIL %s (%s:%d)\n", msg, __FILE__, __LINE__); \
      ++fails;                                          \
    }                                                   \
  } while (0)

template <class F>
static bx_fit_result run(int P, int S, const double* x0, F fg, const uint8_t* mask = nullptr,
                         const double* lo = nullptr, const double* hi = nullptr, int kind = BX_FIT,
                         double tol = 1e-14, int max_eval = 0, double f_noise = 0.0) {
  bx_fit_opts o{};
  o.kind = kind;
  o.x0 = x0;
  o.float_mask = mask;
  o.lo = lo;
  o.hi = hi;
  o.edm_tol = tol;
  o.max_iter = 2000;
  o.max_eval = max_eval;
  FitProblem pb;
  fit_problem(P, S, &o, &pb);
  pb.f_noise = f_noise;
  Bfgs opt(pb);
  double x[32], g[32];
  while (opt.next(x)) {
    double f = fg(x, g);
    opt.feed(f, g);
  }
  bx_fit_result r{};
  opt.result(&r);
  return r;
}

int main() {
  // ill-conditioned quadratic in 6 parameters with rate-like scales
  {
    const int P = 6;
    const double c[P] = {4e4, 3e4, 2e4, 1e4, 0.05, 0.001};
    const double s[P] = {200, 170, 140, 100, 0.002, 0.0001};
    auto fg = [&](const double* x, double* g) {
      double f = 0;
      for (int i = 0; i < P; ++i) {
        double z = (x[i] - c[i]) / s[i], zn = (i + 1 < P) ? (x[i + 1] - c[i + 1]) / s[i + 1] : 0;
        f += 0.5 * z * z + (i + 1 < P ? 0.3 * z * zn : 0);
      }
      for (int i = 0; i < P; ++i) {
        double z = (x[i] - c[i]) / s[i];
        double gi = z;
        if (i + 1 < P) gi += 0.3 * (x[i + 1] - c[i + 1]) / s[i + 1];
        if (i > 0) gi += 0.3 * (x[i - 1] - c[i - 1]) / s[i - 1];
        g[i] = gi / s[i];
      }
      return f;
    };
    double x0[P] = {4.4e4, 2.7e4, 2.1e4, 0.9e4, 0.06, 0.0008};
    bx_fit_result r = run(P, 4, x0, fg);
    CHECK(r.status == BX_CONVERGED, "quadratic converged");
    for (int i = 0; i < P; ++i) CHECK(std::fabs(r.x[i] - c[i]) < 1e-6 * s[i], "quadratic minimum");
    CHECK(r.edm < 1e-14, "quadratic edm");
  }
  // Rosenbrock (no bounds)
  {
    auto fg = [](const double* x, double* g) {
      const double a = 1 - x[0], b = x[1] - x[0] * x[0];
      g[0] = -2 * a - 400 * x[0] * b;
      g[1] = 200 * b;
      return a * a + 100 * b * b;
    };
    double x0[2] = {-1.2, 1.0};
    double lo[2] = {-INFINITY, -INFINITY};
    bx_fit_result r = run(2, 0, x0, fg, nullptr, lo, nullptr, BX_FIT, 1e-20);
    CHECK(std::fabs(r.x[0] - 1) < 1e-6 && std::fabs(r.x[1] - 1) < 1e-6, "rosenbrock minimum");
    // an evaluation budget ends the fit at the last accepted point
    bx_fit_result rb = run(2, 0, x0, fg, nullptr, lo, nullptr, BX_FIT, 1e-20, 12);
    double gb[2];
    CHECK(rb.status == BX_MAXITER && rb.n_eval == 12, "evaluation budget");
    CHECK(rb.nll == fg(rb.x, gb) && rb.nll < fg(x0, gb), "budget keeps an accepted, lower point");
  }
  // minimum outside the box: rate held at its lower bound 0
  {
    auto fg = [](const double* x, double* g) {
      g[0] = x[0] + 5;  // f = (x0 + 5)^2/2 + (x1 - 3)^2/2
      g[1] = x[1] - 3;
      return 0.5 * (x[0] + 5) * (x[0] + 5) + 0.5 * (x[1] - 3) * (x[1] - 3);
    };
    double x0[2] = {2.0, 1.0};
    bx_fit_result r = run(2, 1, x0, fg);
    CHECK(r.x[0] == 0.0, "bounded rate at zero");
    CHECK(std::fabs(r.x[1] - 3) < 1e-6, "free parameter minimum");
    CHECK(r.status == BX_CONVERGED, "bounded converged");
  }
  // correlated valley (rho = 0.99) whose minimum leaves the box: the rate
  // ends on its bound exactly and the other parameter at its conditional
  // minimum y = 3 + rho (0 - x0*) = 3.99; and the same valley moved so that the
  // rate's minimum sits just inside the box (x0 = 1e-4, 5e-5 of its start
  // value): the bound margin must not hold it on the bound
  for (int inside = 0; inside < 2; ++inside) {
    const double rho = 0.99, c0 = inside ? 1e-4 : -1.0, c1 = 3.0;
    auto fg = [&](const double* x, double* g) {
      const double u = x[0] - c0, w = x[1] - c1, k = 1.0 / (1 - rho * rho);
      g[0] = k * (u - rho * w);
      g[1] = k * (w - rho * u);
      return 0.5 * k * (u * u - 2 * rho * u * w + w * w);
    };
    double x0[2] = {2.0, 1.0};
    bx_fit_result r = run(2, 1, x0, fg);
    CHECK(r.status == BX_CONVERGED, "correlated bounded converged");
    if (inside) {
      CHECK(std::fabs(r.x[0] - c0) < 1e-9 && std::fabs(r.x[1] - c1) < 1e-8, "minimum just inside the box");
    } else {
      CHECK(r.x[0] == 0.0, "correlated rate on its bound");
      CHECK(std::fabs(r.x[1] - (c1 + rho * (0.0 - c0))) < 1e-8, "conditional minimum on the bound");
    }
    CHECK(r.n_eval < 60, "correlated bounded evaluations");
    if (r.n_eval >= 60 || r.status != BX_CONVERGED) std::printf("  inside=%d evals %d edm %g\n", inside, r.n_eval, r.edm);
  }
  // fixed parameter stays put; single evaluation request
  {
    auto fg = [](const double* x, double* g) {
      g[0] = x[0] - 1;
      g[1] = x[1] - 2;
      return 0.5 * ((x[0] - 1) * (x[0] - 1) + (x[1] - 2) * (x[1] - 2));
    };
    double x0[2] = {5.0, 7.0};
    uint8_t mask[2] = {1, 0};
    bx_fit_result r = run(2, 0, x0, fg, mask, nullptr, nullptr);
    CHECK(r.x[1] == 7.0 && std::fabs(r.x[0] - 1) < 1e-6, "masked parameter fixed");
    bx_fit_result e = run(2, 0, x0, fg, nullptr, nullptr, nullptr, BX_EVAL_GRAD);
    CHECK(e.n_eval == 1 && e.nll == 0.5 * (16 + 25) && e.grad[0] == 4.0, "eval-grad request");
  }
  // a domain wall (f = +inf for x < 0.5): the line search backs off
  {
    auto fg = [](const double* x, double* g) {
      if (x[0] < 0.5) return (double)INFINITY;
      g[0] = x[0] - 1;
      return 0.5 * (x[0] - 1) * (x[0] - 1);
    };
    double x0[1] = {40.0};
    double lo[1] = {-INFINITY};
    bx_fit_result r = run(1, 0, x0, fg, nullptr, lo, nullptr);
    CHECK(std::fabs(r.x[0] - 1) < 1e-6, "domain wall");
  }
  // binned Poisson fit of overlapping templates, some of whose rates are zero
  // in the counts: the fit ends on the bound conditions (each rate on its
  // bound with a gradient pushing outward, or free with the gradient ~0)
  // (seeds whose iterates creep toward a bound; 3025 evaluations in all when
  // a parameter is held only exactly on its bound, 1340 when a parameter
  // whose Newton component crosses its bound is held there)
  int pois_evals = 0;
  for (int seed : {9, 20, 37}) {
    const int S = 8, N = 240, P = S + 2;
    double cen[S], wid[S], rt[S];
    unsigned long long st = 0x9e3779b97f4a7c15ull * (seed + 1);
    auto uni = [&]() {  // 53-bit uniform in [0, 1) from a 64-bit LCG
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      return (double)(st >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int s = 0; s < S; ++s) {
      cen[s] = 30 + 180 * uni();
      wid[s] = 20 + 50 * uni();
      rt[s] = (s % 3 == 1) ? 0.0 : 2e4 * uni();
    }
    auto mu_of = [&](const double* x, double* mu, double (*d)[N]) {
      for (int b = 0; b < N; ++b) mu[b] = 1e-3;
      if (d) for (int q = 0; q < P; ++q) for (int b = 0; b < N; ++b) d[q][b] = 0;
      for (int s = 0; s < S; ++s)
        for (int b = 0; b < N; ++b) {
          const double w = wid[s] * x[S + 1], z = (b + 0.5 - cen[s] * x[S]) / w;
          const double t = std::exp(-0.5 * z * z) / (2.5066282746310002 * w);
          mu[b] += x[s] * t;
          if (d) {
            d[s][b] += t;
            d[S][b] += x[s] * t * z * cen[s] / w;
            d[S + 1][b] += x[s] * t * (z * z - 1) / x[S + 1];
          }
        }
    };
    double truth[P], mu[N], cnt[N];
    for (int s = 0; s < S; ++s) truth[s] = rt[s];
    truth[S] = truth[S + 1] = 1.0;
    mu_of(truth, mu, nullptr);
    for (int b = 0; b < N; ++b)  // counts: mu plus a deterministic fluctuation of ~1 sigma
      cnt[b] = std::max(0.0, std::floor(mu[b] + 1.7 * (uni() - 0.5) * std::sqrt(12.0 * mu[b]) * 0.5 + 0.5));
    static double dmu[P][N];
    auto fg = [&](const double* x, double* g) {
      double m[N];
      mu_of(x, m, dmu);
      double f = 0;
      for (int q = 0; q < P; ++q) g[q] = 0;
      for (int b = 0; b < N; ++b) {
        if (!(m[b] > 0)) return (double)INFINITY;
        f += m[b] - cnt[b] * std::log(m[b]);
        for (int q = 0; q < P; ++q) g[q] += (1 - cnt[b] / m[b]) * dmu[q][b];
      }
      return f;
    };
    double x0[P];
    for (int s = 0; s < S; ++s) x0[s] = 1e4;
    x0[S] = 1.01;
    x0[S + 1] = 0.98;
    bx_fit_result r = run(P, S, x0, fg, nullptr, nullptr, nullptr, BX_FIT, 1e-12, 0, 1e-13);
    pois_evals += r.n_eval;
    CHECK(r.status == BX_CONVERGED, "poisson templates converged");
    for (int s = 0; s < S; ++s) CHECK(r.x[s] > 0.0 || r.grad[s] >= 0.0, "rate on its bound pushed outward");
    if (r.status != BX_CONVERGED) std::printf("  seed %d status %d evals %d edm %g\n", seed, r.status, r.n_eval, r.edm);
  }
  CHECK(pois_evals < 1800, "poisson templates evaluations");
  if (pois_evals >= 1800) std::printf("  poisson evaluations %d\n", pois_evals);
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
  return fails ? 1 : 0;
}

// Host unit test of the reverse-communication quasi-Newton minimiser
// (bx_fitcore.hpp): quadratics, Rosenbrock, box bounds, fixed parameters,
// single evaluations and a domain wall.  Built with g++ by test_host.py.
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
                         double tol = 1e-14, int max_eval = 0) {
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
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
  return fails ? 1 : 0;
}

// Bounded quasi-Newton minimiser written in reverse communication: next(x)
// names the point to evaluate, feed(f, g) hands back the NLL and gradient
// there.  The plain path drives one instance from the calling thread; the fit
// server drives thousands, one per resident fit, and evaluates all their
// points in one batched launch per step.  It plays the role of the paper's
// minimiser, which varies the parameters and asks for likelihood values until
// it finds the optimum (Sec. 4, steps 5-7).
//
// Method: the Hessian approximation B (in parameters scaled by their start
// values) starts from forward differences of the analytic gradient, one free
// parameter per evaluation, and is refined by BFGS updates.  Each step solves
// B_FF d_F = -g_F on the free set F (parameters not held at a bound by the
// gradient) by Cholesky with a diagonal shift when B_FF is not positive
// definite; parameters whose Newton component would cross their bound are
// held on it and the rest solve again with that coupling.  The step is
// truncated at the box and backtracks (Armijo, quadratic interpolation).
// EDM, the decrease the quadratic model predicts for the step
// (g_F^T B_FF^-1 g_F / 2 when nothing crosses), ends the fit when it falls
// below the tolerance.
//
// The minimiser is compiled for the host (plain path, fit server) and for the
// device (the batched fits' minimiser steps, k_fit_step): one code, with
// floating-point contraction off, so that both give the same bits.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/bx.h"

// HIP in the library (host and device); plain C++ in the minimiser's CPU
// unit test.
#ifdef __HIP__
#include <hip/hip_runtime.h>
#define BX_FHD __host__ __device__
#else
#define BX_FHD
#endif

#ifdef __clang__
#pragma float_control(push)
#pragma clang fp contract(off)
#endif

// Loops over independent elements.  On the device the fit's whole wave runs
// the minimiser (every lane the same serial code on the state in LDS, so the
// control flow stays uniform), each lane takes every 64th element of such a
// loop, and the wave (the whole workgroup) then waits at a barrier; the host
// runs the elements in order.  An element's arithmetic is the same either
// way, and ordered sums stay serial, so host and device give the same bits.
#if defined(__HIP_DEVICE_COMPILE__)
#define BX_PFOR(i, n) for (int i = (int)threadIdx.x; i < (n); i += 64)
#define BX_PSYNC() __syncthreads()
#else
#define BX_PFOR(i, n) for (int i = 0; i < (n); ++i)
#define BX_PSYNC() ((void)0)
#endif

namespace bx {

void set_error(const std::string& msg);

struct FitProblem {
  int P = 0, S = 0, nf = 0, kind = BX_FIT, max_iter = 500, max_eval = 0;
  int idx[32];                       // free parameters
  double x0[32], lo[32], hi[32], scale[32];
  double edm_tol = 1e-9;
  double f_noise = 0.0;              // relative rounding noise of the NLL values
  double final_tol = 1e-9;           // mixed precision: the polishing model's tolerance
};

// unit: index of a parameter with default bounds [0, 1] (a floated pile-up
// fraction), or -1.
inline bx_status fit_problem(int P, int S, const bx_fit_opts* o, FitProblem* pb, int unit = -1) {
  if (P > 32 || P < 1) {
    set_error("parameter count out of range");
    return BX_E_INVAL;
  }
  pb->P = P;
  pb->S = S;
  pb->kind = o->kind == BX_EVAL_GRAD ? BX_EVAL_GRAD : BX_FIT;
  pb->edm_tol = o->edm_tol > 0 ? o->edm_tol : 1e-9;
  pb->final_tol = pb->edm_tol;
  // mixed precision: the first model stops at the switch tolerance
  if (o->polish) pb->edm_tol = std::max(pb->edm_tol, o->polish_edm > 0 ? o->polish_edm : 1e-8);
  pb->max_iter = o->max_iter > 0 ? o->max_iter : 500;
  pb->nf = 0;
  for (int q = 0; q < P; ++q) {
    pb->x0[q] = o->x0[q];
    if (!std::isfinite(o->x0[q])) {
      set_error("x0 must be finite");
      return BX_E_INVAL;
    }
    pb->lo[q] = o->lo ? o->lo[q] : (q < S || q == unit ? 0.0 : -INFINITY);
    pb->hi[q] = o->hi ? o->hi[q] : (q == unit ? 1.0 : INFINITY);
    if (!(pb->lo[q] <= pb->hi[q])) {
      set_error("lower bound above upper bound");
      return BX_E_INVAL;
    }
    pb->x0[q] = std::min(std::max(pb->x0[q], pb->lo[q]), pb->hi[q]);
    pb->scale[q] = std::fabs(pb->x0[q]) > 0 ? std::fabs(pb->x0[q]) : 1.0;
    if (!o->float_mask || o->float_mask[q]) pb->idx[pb->nf++] = q;
  }
  const int n = pb->nf;
  pb->max_eval = o->max_eval > 0 ? o->max_eval : 200 + 100 * n + 5 * n * n;
  return BX_OK;
}

// element copy (host and device)
BX_FHD inline void fcopy(double* d, const double* s, int n) {
  for (int i = 0; i < n; ++i) d[i] = s[i];
}

class Bfgs {
 public:
  BX_FHD Bfgs() = default;
  BX_FHD explicit Bfgs(const FitProblem& pb) : pb_(pb) {
    fcopy(x_, pb.x0, 32);
    const int n = pb.nf;
    for (int a = 0; a < n * n; ++a) B_[a] = 0.0;
    for (int a = 0; a < n; ++a) B_[a * n + a] = 1.0;
  }

  // Point to evaluate next; false when finished.
  BX_FHD bool next(double* x) {
    if (state_ == kDone) return false;
    fcopy(x, state_ == kInit || state_ == kReeval ? x_ : xt_, pb_.P);
    return true;
  }

  // Go on from the accepted point with evaluations of another model (the
  // FP64 model of a mixed-precision fit): the point is evaluated again, then
  // the iterations continue with the same Hessian approximation until
  // EDM < edm_tol.  Only after a finished fit that did not run out of budget.
  BX_FHD bool polish(double edm_tol, double f_noise) {
    if (!can_polish()) return false;
    pb_.edm_tol = edm_tol;
    pb_.f_noise = f_noise;
    state_ = kReeval;
    status_ = BX_FAILED;
    restarted_ = false;
    refresh_iter_ = iter_;
    edm_refresh_ = INFINITY;
    return true;
  }
  BX_FHD int status() const { return status_; }
  // polish() would go on (a finished fit that can move to another model)
  BX_FHD bool can_polish() const {
    return state_ == kDone && pb_.kind == BX_FIT && status_ != BX_MAXITER && std::isfinite(f_);
  }

  BX_FHD void feed(double f, const double* g) {
    ++n_eval_;
    const int n = pb_.nf;
    if (state_ != kInit && n_eval_ >= pb_.max_eval) {  // budget spent: keep the accepted point
      finish(BX_MAXITER);
      return;
    }
    if (state_ == kReeval) {  // the accepted point, by the polishing model
      f_ = f;
      fcopy(g_, g, pb_.P);
      if (!std::isfinite(f)) {
        finish(BX_FAILED);
        return;
      }
      start_iteration();
      return;
    }
    if (state_ == kInit) {
      f_ = f;
      fcopy(g_, g, pb_.P);
      if (!std::isfinite(f) || pb_.kind == BX_EVAL_GRAD || n == 0) {
        edm_ = std::isfinite(f) && n > 0 ? newton_dir(g_, x_, nullptr) : 0.0;
        finish(std::isfinite(f) ? BX_CONVERGED : BX_FAILED);
        return;
      }
      state_ = kHess;
      hq_ = 0;
      hsign_ = 1.0;
      set_probe();
      return;
    }
    if (state_ == kHess) {
      if (!std::isfinite(f) && hsign_ > 0) {  // probe outside the domain: other side
        hsign_ = -1.0;
        set_probe();
        return;
      }
      const double h = hsign_ * kProbe;
      BX_PFOR(b, n) {
        const int qb = pb_.idx[b];
        Hs_[b * n + hq_] = std::isfinite(f) ? (g[qb] - g_[qb]) * pb_.scale[qb] / h : 0.0;
      }
      BX_PSYNC();
      if (++hq_ < n) {
        hsign_ = 1.0;
        set_probe();
        return;
      }
      BX_PFOR(e, n * n) {
        const int a = e / n, b = e - a * n;
        B_[e] = 0.5 * (Hs_[a * n + b] + Hs_[b * n + a]);
      }
      BX_PSYNC();
      refresh_iter_ = iter_;
      edm_refresh_ = INFINITY;
      start_iteration();
      return;
    }
    // line-search trial at xt_ = clip(x + alpha d): projected Armijo rule on
    // the actual displacement
    double gdx = 0.0;
    for (int a = 0; a < n; ++a) gdx += g_[pb_.idx[a]] * (xt_[pb_.idx[a]] - x_[pb_.idx[a]]);
    if (std::isfinite(f) && f <= f_ + 1e-4 * std::min(gdx, 0.0)) {
      accept(f, g);
      return;
    }
    // Near the minimum the expected decrease can fall below the rounding
    // noise of the NLL values; the gradient still resolves progress there:
    // accept a step whose NLL change is within the noise if it lowers EDM.
    if (std::isfinite(f) && f - f_ <= pb_.f_noise * std::fabs(f_) && newton_dir(g, xt_, nullptr) < 0.9 * edm_) {
      accept(f, g);
      return;
    }
    double an = 0.5 * alpha_;  // safeguarded quadratic interpolation
    if (std::isfinite(f)) {
      const double den = 2.0 * (f - f_ - slope_ * alpha_);
      if (den > 0) an = std::min(0.5 * alpha_, std::max(0.1 * alpha_, -slope_ * alpha_ * alpha_ / den));
    }
    alpha_ = an;
    if (++ls_ > 40 || alpha_ < 1e-20) {
      // no decrease along the direction: restart once from the diagonal of B,
      // then stop (the NLL is flat to rounding here)
      if (!restarted_) {
        restarted_ = true;
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b)
            if (a != b) B_[a * n + b] = 0.0;
        start_iteration();
        return;
      }
      finish(edm_ < pb_.edm_tol ? BX_CONVERGED : BX_FAILED);
      return;
    }
    set_trial();
  }

  BX_FHD void result(bx_fit_result* r) const {
    r->status = status_;
    r->nll = f_;
    for (int q = 0; q < pb_.P; ++q) {
      r->x[q] = x_[q];
      r->grad[q] = g_[q];
    }
    r->edm = edm_;
    r->n_iter = iter_;
    r->n_eval = n_eval_;
  }
  BX_FHD bool done() const { return state_ == kDone; }

 private:
  enum { kInit, kHess, kSearch, kDone, kReeval };
  static constexpr double kProbe = 1e-4;  // Hessian probe step (scaled units)
  static constexpr int kHoldPasses = 4;  // newton_dir: rounds of holding crossing parameters

  BX_FHD double lo_u(int a) const { return pb_.lo[pb_.idx[a]] / pb_.scale[pb_.idx[a]]; }
  BX_FHD double hi_u(int a) const { return pb_.hi[pb_.idx[a]] / pb_.scale[pb_.idx[a]]; }

  BX_FHD void set_probe() {
    fcopy(xt_, x_, 32);
    const int q = pb_.idx[hq_];
    double v = x_[q] / pb_.scale[q] + hsign_ * kProbe;
    if (v > hi_u(hq_) || v < lo_u(hq_)) {  // stay inside the box
      hsign_ = -hsign_;
      v = x_[q] / pb_.scale[q] + hsign_ * kProbe;
    }
    xt_[q] = v * pb_.scale[q];
  }

  // Cholesky solve of B_FF z = r on the free set fr[0..m) (a diagonal shift
  // when B_FF is not positive definite); z may alias nothing else.
  BX_FHD void solve_free(const int* fr, int m, const double* r, double* z) const {
    const int n = pb_.nf;
    double dmax = 0.0;
    for (int i = 0; i < m; ++i) dmax = std::max(dmax, std::fabs(B_[fr[i] * n + fr[i]]));
    if (!(dmax > 0)) dmax = 1.0;
    double* const L = L_;  // the factor (a member: no 8 KB array on a device thread's stack)
    double shift = 0.0;
    for (int attempt = 0; attempt < 40; ++attempt) {
      bool ok = true;
      for (int j = 0; j < m && ok; ++j) {
        double s = B_[fr[j] * n + fr[j]] + shift;
        for (int k = 0; k < j; ++k) s -= L[j * m + k] * L[j * m + k];
        if (!(s > 0)) {
          ok = false;
          break;
        }
        L[j * m + j] = std::sqrt(s);
        BX_PFOR(ii, m - j - 1) {  // the rows below: column j of the factor
          const int i = j + 1 + ii;
          double t = B_[fr[i] * n + fr[j]];
          for (int k = 0; k < j; ++k) t -= L[i * m + k] * L[j * m + k];
          L[i * m + j] = t / L[j * m + j];
        }
        BX_PSYNC();
      }
      if (ok) break;
      shift = shift > 0 ? 4.0 * shift : 1e-10 * dmax;
    }
    double* const y = wb_;
    for (int i = 0; i < m; ++i) {  // L y = r
      double t = r[i];
      for (int k = 0; k < i; ++k) t -= L[i * m + k] * y[k];
      y[i] = t / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {  // L^T z = y
      double t = y[i];
      for (int k = i + 1; k < m; ++k) t -= L[k * m + i] * z[k];
      z[i] = t / L[i * m + i];
    }
  }

  // Step at point x with gradient g.  The free set F holds the parameters
  // that the gradient does not push out of the box from a bound they sit on;
  // the Newton step solves B_FF d_F = -g_F.  A free parameter whose Newton
  // component would cross its bound is then held on that bound (it moves
  // there), and the others solve again with that move's coupling,
  // B_F'F' d_F' = -(g_F' + B_F'H m_H), up to kHoldPasses times.  Clipping
  // the first step at the box instead ignores the coupling, and the clipped
  // step of a correlated fit can fail to descend, so that a parameter a hair
  // above its bound stalls the fit.  When no component crosses, or the held
  // step predicts no decrease, the step is the plain Newton step on F.
  // Returns EDM, the decrease the quadratic model predicts for the step
  // (g_F^T B_FF^-1 g_F / 2 for the plain step), and writes d (scaled units)
  // when d != nullptr.
  BX_FHD double newton_dir(const double* g, const double* x, double* d) const {
    const int n = pb_.nf;
    int* const fr = wi_;  // work arrays are members: on the device they live with the state in LDS
    double* const gu = wa_;
    double* const dd = wc_;
    double* const r = wd_;
    double* const dh = we_;  // the held step: moves of the held parameters, then d_F'
    int m = 0;
    for (int a = 0; a < n; ++a) {
      const int q = pb_.idx[a];
      gu[a] = g[q] * pb_.scale[q];
      const double v = x[q] / pb_.scale[q];
      const bool held = (v <= lo_u(a) && gu[a] > 0) || (v >= hi_u(a) && gu[a] < 0);
      if (d) d[a] = 0.0;
      dh[a] = 0.0;
      if (!held) fr[m++] = a;
    }
    if (m == 0) return 0.0;
    for (int i = 0; i < m; ++i) r[i] = -gu[fr[i]];
    solve_free(fr, m, r, dd);
    double gd = 0.0;
    for (int i = 0; i < m; ++i) {
      gd += gu[fr[i]] * dd[i];
      if (d) d[fr[i]] = dd[i];
    }
    const double edm0 = -0.5 * gd;
    // free parameters whose Newton component crosses their bound
    bool crossed = false;
    for (int pass = 0; pass < kHoldPasses; ++pass) {
      int k = 0;
      bool more = false;
      for (int i = 0; i < m; ++i) {
        const int a = fr[i];
        const double v = x[pb_.idx[a]] / pb_.scale[pb_.idx[a]];
        if (v + dd[i] < lo_u(a)) {
          dh[a] = lo_u(a) - v;
          more = true;
        } else if (v + dd[i] > hi_u(a)) {
          dh[a] = hi_u(a) - v;
          more = true;
        } else {
          fr[k++] = a;
        }
      }
      if (!more) break;
      crossed = true;
      m = k;
      if (m == 0) break;
      BX_PFOR(i, m) {
        double t = -gu[fr[i]];
        for (int b = 0; b < n; ++b) t -= B_[fr[i] * n + b] * dh[b];
        r[i] = t;
      }
      BX_PSYNC();
      solve_free(fr, m, r, dd);
    }
    if (!crossed) return edm0;
    for (int i = 0; i < m; ++i) dh[fr[i]] = dd[i];
    // predicted decrease of the held step: -(g.d + d^T B d / 2), the terms
    // per parameter, then summed in order
    double* const qt = wb_;
    BX_PFOR(a, n) {
      double bd = 0.0;
      for (int b = 0; b < n; ++b) bd += B_[a * n + b] * dh[b];
      qt[a] = dh[a] * (gu[a] + 0.5 * bd);
    }
    BX_PSYNC();
    double q = 0.0;
    for (int a = 0; a < n; ++a) q += qt[a];
    if (!(-q > 0)) return edm0;  // no decrease predicted: the plain step
    if (d)
      for (int a = 0; a < n; ++a) d[a] = dh[a];
    return -q;
  }

  BX_FHD void start_iteration() {
    const int n = pb_.nf;
    edm_ = newton_dir(g_, x_, d_);
    if (!(edm_ == edm_)) edm_ = INFINITY;
    if (edm_ < pb_.edm_tol) {
      finish(BX_CONVERGED);
      return;
    }
    if (iter_ >= pb_.max_iter) {
      finish(BX_MAXITER);
      return;
    }
    // slow progress means the updated Hessian is poor (curved valleys of
    // correlated parameters): probe it again at the current point
    if (!std::isfinite(edm_refresh_)) edm_refresh_ = edm_;
    if (iter_ - refresh_iter_ >= 8) {
      if (edm_ > 0.05 * edm_refresh_) {
        state_ = kHess;
        hq_ = 0;
        hsign_ = 1.0;
        set_probe();
        return;
      }
      refresh_iter_ = iter_;  // enough progress: new reference point
      edm_refresh_ = edm_;
    }
    double gd = 0.0;
    for (int a = 0; a < n; ++a) gd += g_[pb_.idx[a]] * pb_.scale[pb_.idx[a]] * d_[a];
    slope_ = gd;
    alpha_ = 1.0;  // the trial point is projected onto the box (set_trial)
    ls_ = 0;
    state_ = kSearch;
    set_trial();
  }

  BX_FHD void set_trial() {
    fcopy(xt_, x_, 32);
    for (int a = 0; a < pb_.nf; ++a) {
      const int q = pb_.idx[a];
      double v = x_[q] / pb_.scale[q] + alpha_ * d_[a];
      v = std::min(std::max(v, lo_u(a)), hi_u(a));
      xt_[q] = v * pb_.scale[q];
    }
  }

  BX_FHD void accept(double f, const double* g) {
    const int n = pb_.nf;
    double* const s = wa_;
    double* const y = wb_;
    double* const Bs = wc_;
    double sy = 0.0, sBs = 0.0;
    for (int a = 0; a < n; ++a) {
      const int q = pb_.idx[a];
      s[a] = (xt_[q] - x_[q]) / pb_.scale[q];
      y[a] = (g[q] - g_[q]) * pb_.scale[q];
      sy += s[a] * y[a];
    }
    BX_PFOR(a, n) {
      double t = 0.0;
      for (int b = 0; b < n; ++b) t += B_[a * n + b] * s[b];
      Bs[a] = t;
    }
    BX_PSYNC();
    for (int a = 0; a < n; ++a) sBs += s[a] * Bs[a];
    fcopy(x_, xt_, 32);
    fcopy(g_, g, pb_.P);
    f_ = f;
    ++iter_;
    restarted_ = false;
    // BFGS update of the Hessian, skipped when the curvature condition fails
    if (sy > 1e-12 * std::sqrt(sBs > 0 ? sBs : 0.0) * 0 + 1e-300 && sBs > 1e-300) {
      BX_PFOR(e, n * n) {
        const int a = e / n, b = e - a * n;
        B_[e] += y[a] * y[b] / sy - Bs[a] * Bs[b] / sBs;
      }
      BX_PSYNC();
    }
    start_iteration();
  }

  BX_FHD void finish(int st) {
    status_ = st;
    state_ = kDone;
  }

  FitProblem pb_;
  int state_ = kInit, status_ = BX_FAILED, iter_ = 0, n_eval_ = 0, ls_ = 0, hq_ = 0, refresh_iter_ = 0;
  double edm_refresh_ = INFINITY;  // EDM right after the last Hessian probe
  bool restarted_ = false;
  double hsign_ = 1.0;
  double x_[32], xt_[32], g_[32], d_[32], B_[32 * 32], Hs_[32 * 32];
  mutable double L_[32 * 32];  // Cholesky factor of the free block of B
  mutable double wa_[32], wb_[32], wc_[32], wd_[32], we_[32];  // work vectors of newton_dir and accept
  mutable int wi_[32];
  double f_ = INFINITY, alpha_ = 1.0, slope_ = 0.0, edm_ = INFINITY;
};

}  // namespace bx

#ifdef __clang__
#pragma float_control(pop)
#endif

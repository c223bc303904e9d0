// Bounded quasi-Newton minimiser (BFGS on the inverse Hessian, projected
// onto box bounds, backtracking Armijo line search), written in reverse
// communication: next(x) names the point to evaluate, feed(f, g) hands back
// the NLL and gradient there.  The plain path drives one instance from the
// calling thread; the fit server drives thousands, one per resident fit, and
// evaluates all their points in one batched launch per step.  It plays the
// role of the paper's minimiser, which varies the parameters and asks for
// likelihood values until it finds the optimum (Sec. 4, steps 5-7).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/bx.h"

namespace bx {

void set_error(const std::string& msg);

struct FitProblem {
  int P = 0, S = 0, nf = 0, kind = BX_FIT, max_iter = 500;
  int idx[32];                       // free parameters
  double x0[32], lo[32], hi[32], scale[32];
  double edm_tol = 1e-9;
};

inline bx_status fit_problem(int P, int S, const bx_fit_opts* o, FitProblem* pb) {
  if (P > 32 || P < 1) {
    set_error("parameter count out of range");
    return BX_E_INVAL;
  }
  pb->P = P;
  pb->S = S;
  pb->kind = o->kind == BX_EVAL_GRAD ? BX_EVAL_GRAD : BX_FIT;
  pb->edm_tol = o->edm_tol > 0 ? o->edm_tol : 1e-9;
  pb->max_iter = o->max_iter > 0 ? o->max_iter : 500;
  pb->nf = 0;
  for (int q = 0; q < P; ++q) {
    pb->x0[q] = o->x0[q];
    if (!std::isfinite(o->x0[q])) {
      set_error("x0 must be finite");
      return BX_E_INVAL;
    }
    pb->lo[q] = o->lo ? o->lo[q] : (q < S ? 0.0 : -INFINITY);
    pb->hi[q] = o->hi ? o->hi[q] : INFINITY;
    if (!(pb->lo[q] <= pb->hi[q])) {
      set_error("lower bound above upper bound");
      return BX_E_INVAL;
    }
    pb->x0[q] = std::min(std::max(pb->x0[q], pb->lo[q]), pb->hi[q]);
    pb->scale[q] = std::fabs(pb->x0[q]) > 0 ? std::fabs(pb->x0[q]) : 1.0;
    if (!o->float_mask || o->float_mask[q]) pb->idx[pb->nf++] = q;
  }
  return BX_OK;
}

class Bfgs {
 public:
  explicit Bfgs(const FitProblem& pb) : pb_(pb) {
    memcpy(x_, pb.x0, sizeof x_);
    const int n = pb.nf;
    for (int a = 0; a < n * n; ++a) H_[a] = 0.0;
    for (int a = 0; a < n; ++a) H_[a * n + a] = 1.0;
  }

  // Point to evaluate next; false when finished.
  bool next(double* x) {
    if (state_ == kDone) return false;
    memcpy(x, state_ == kInit ? x_ : xt_, sizeof(double) * pb_.P);
    return true;
  }

  void feed(double f, const double* g) {
    ++n_eval_;
    if (state_ == kInit) {
      f_ = f;
      memcpy(g_, g, sizeof(double) * pb_.P);
      if (!std::isfinite(f) || pb_.kind == BX_EVAL_GRAD || pb_.nf == 0) {
        status_ = std::isfinite(f) ? BX_CONVERGED : BX_FAILED;
        edm_ = edm();
        state_ = kDone;
        return;
      }
      start_iteration(true);
      return;
    }
    // line-search trial at xt_
    const double gd = slope_;
    if (std::isfinite(f) && f <= f_ + 1e-4 * alpha_ * gd) {
      accept(f, g);
      return;
    }
    // backtrack: safeguarded quadratic interpolation
    double an = 0.5 * alpha_;
    if (std::isfinite(f)) {
      const double den = 2.0 * (f - f_ - gd * alpha_);
      if (den > 0) an = std::min(0.5 * alpha_, std::max(0.1 * alpha_, -gd * alpha_ * alpha_ / den));
    }
    alpha_ = an;
    if (++ls_ > 40 || alpha_ < 1e-20) {
      // no decrease along the direction: restart once from steepest descent,
      // then stop (the NLL is flat to rounding here)
      if (!restarted_) {
        restarted_ = true;
        reset_h();
        start_iteration(false);
        return;
      }
      finish(edm_ < pb_.edm_tol ? BX_CONVERGED : BX_FAILED);
      return;
    }
    set_trial();
  }

  void result(bx_fit_result* r) const {
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
  bool done() const { return state_ == kDone; }

 private:
  enum { kInit, kSearch, kDone };

  double gu(int a) const { return g_[pb_.idx[a]] * pb_.scale[pb_.idx[a]]; }
  double u(int a) const { return x_[pb_.idx[a]] / pb_.scale[pb_.idx[a]]; }
  double ulo(int a) const { return pb_.lo[pb_.idx[a]] / pb_.scale[pb_.idx[a]]; }
  double uhi(int a) const { return pb_.hi[pb_.idx[a]] / pb_.scale[pb_.idx[a]]; }

  // variables held at a bound by the gradient
  bool pinned(int a) const {
    const double v = u(a), gv = gu(a);
    return (v <= ulo(a) && gv > 0) || (v >= uhi(a) && gv < 0);
  }

  double edm() const {
    const int n = pb_.nf;
    double e = 0.0;
    for (int a = 0; a < n; ++a) {
      if (pinned(a)) continue;
      double hg = 0.0;
      for (int b = 0; b < n; ++b)
        if (!pinned(b)) hg += H_[a * n + b] * gu(b);
      e += gu(a) * hg;
    }
    return 0.5 * e;
  }

  void reset_h() {
    const int n = pb_.nf;
    double gmax = 0.0;
    for (int a = 0; a < n; ++a) gmax = std::max(gmax, std::fabs(gu(a)));
    const double h0 = gmax > 0 ? 0.05 / gmax : 1.0;
    for (int a = 0; a < n * n; ++a) H_[a] = 0.0;
    for (int a = 0; a < n; ++a) H_[a * n + a] = h0;
    fresh_h_ = true;
  }

  void start_iteration(bool first) {
    if (first) reset_h();
    edm_ = edm();
    if (edm_ < pb_.edm_tol) {
      finish(BX_CONVERGED);
      return;
    }
    if (iter_ >= pb_.max_iter) {
      finish(BX_MAXITER);
      return;
    }
    const int n = pb_.nf;
    double gd = 0.0;
    for (int a = 0; a < n; ++a) {
      d_[a] = 0.0;
      if (pinned(a)) continue;
      for (int b = 0; b < n; ++b)
        if (!pinned(b)) d_[a] -= H_[a * n + b] * gu(b);
      gd += gu(a) * d_[a];
    }
    if (!(gd < 0)) {  // not a descent direction: steepest descent
      reset_h();
      gd = 0.0;
      for (int a = 0; a < n; ++a) {
        d_[a] = pinned(a) ? 0.0 : -H_[a * n + a] * gu(a);
        gd += gu(a) * d_[a];
      }
    }
    slope_ = gd;
    // longest step inside the box
    double amax = 1.0;
    for (int a = 0; a < n; ++a) {
      if (d_[a] < 0 && std::isfinite(ulo(a))) amax = std::min(amax, (ulo(a) - u(a)) / d_[a]);
      if (d_[a] > 0 && std::isfinite(uhi(a))) amax = std::min(amax, (uhi(a) - u(a)) / d_[a]);
    }
    alpha_ = std::max(amax, 0.0);
    ls_ = 0;
    if (!(alpha_ > 0)) {  // blocked by a bound: drop the blocking components
      for (int a = 0; a < n; ++a)
        if ((d_[a] < 0 && u(a) <= ulo(a)) || (d_[a] > 0 && u(a) >= uhi(a))) d_[a] = 0.0;
      alpha_ = 1.0;
    }
    state_ = kSearch;
    set_trial();
  }

  void set_trial() {
    memcpy(xt_, x_, sizeof xt_);
    for (int a = 0; a < pb_.nf; ++a) {
      const int q = pb_.idx[a];
      double v = u(a) + alpha_ * d_[a];
      v = std::min(std::max(v, ulo(a)), uhi(a));
      xt_[q] = v * pb_.scale[q];
    }
  }

  void accept(double f, const double* g) {
    const int n = pb_.nf;
    double s[32], y[32], sy = 0.0, yy = 0.0;
    for (int a = 0; a < n; ++a) {
      const int q = pb_.idx[a];
      s[a] = (xt_[q] - x_[q]) / pb_.scale[q];
      y[a] = (g[q] - g_[q]) * pb_.scale[q];
      sy += s[a] * y[a];
      yy += y[a] * y[a];
    }
    memcpy(x_, xt_, sizeof x_);
    memcpy(g_, g, sizeof(double) * pb_.P);
    f_ = f;
    ++iter_;
    restarted_ = false;
    if (sy > 1e-300 && yy > 0) {
      if (fresh_h_) {  // scale the initial inverse Hessian (Nocedal & Wright 6.20)
        const double h0 = sy / yy;
        for (int a = 0; a < n * n; ++a) H_[a] = 0.0;
        for (int a = 0; a < n; ++a) H_[a * n + a] = h0;
        fresh_h_ = false;
      }
      // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T
      const double rho = 1.0 / sy;
      double Hy[32], yHy = 0.0;
      for (int a = 0; a < n; ++a) {
        Hy[a] = 0.0;
        for (int b = 0; b < n; ++b) Hy[a] += H_[a * n + b] * y[b];
        yHy += y[a] * Hy[a];
      }
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
          H_[a * n + b] += -rho * (s[a] * Hy[b] + Hy[a] * s[b]) + (rho * rho * yHy + rho) * s[a] * s[b];
    }
    start_iteration(false);
  }

  void finish(int st) {
    status_ = st;
    edm_ = edm();
    state_ = kDone;
  }

  FitProblem pb_;
  int state_ = kInit, status_ = BX_FAILED, iter_ = 0, n_eval_ = 0, ls_ = 0;
  bool fresh_h_ = true, restarted_ = false;
  double x_[32], xt_[32], g_[32], d_[32], H_[32 * 32];
  double f_ = INFINITY, alpha_ = 1.0, slope_ = 0.0, edm_ = INFINITY;
};

}  // namespace bx

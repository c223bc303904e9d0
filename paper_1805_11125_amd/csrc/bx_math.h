// Special functions of the detector response, for gfx950 (and the host, for
// unit tests of the arithmetic).  Everything here is per column (FP64) or per
// reco edge (FP32 or FP64).
//
//  * Gaussian response: the bin-integrated normal law, written with the
//    smaller tail (erfc) at every reco edge.
//  * Generalized-gamma (Stacy) response with exponent p: F(x) = P(k, (x/a)^p)
//    with P, Q the regularized incomplete gamma ratios.  Large k: Temme's
//    uniform asymptotic expansion in eta, eta^2/2 = lambda - 1 - ln(lambda),
//    lambda = y/k (coefficients from gen_temme.py).  Small k: the power series
//    of P and the Legendre continued fraction of Q (modified Lentz), carried
//    with a forward-mode derivative in k.
//  * Column constants (FP64): ln Gamma differences by the Stirling series with
//    Bernoulli-polynomial coefficients after an upward shift, digamma, and
//    Gamma*(k) = Gamma(k) / (sqrt(2 pi / k) k^k e^-k).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "temme_coef.h"

#define BX_HD __host__ __device__ __forceinline__

namespace bx {

// ---------------------------------------------------------------------------
// Constants shared by host set-up and kernels.
// ---------------------------------------------------------------------------
constexpr int kSeriesTerms = 16;   // Stirling-type series length
constexpr double kShift = 10.0;    // argument shift before the series
constexpr double kSupportB = 75.0;   // FP64 cells: tails beyond k*phi = B (or z^2/2 = B) are < 1e-32
constexpr double kSupportB32 = 32.0; // FP32 cells: tails beyond B are < 1e-14 of the column
constexpr float kTemmeMinK = 12.f;   // FP32: uniform expansion from this shape on
constexpr float kTemmeTailCut = 40.f;  // FP32 uniform expansion: tails beyond k*phi = 40 are set to 0
// FP32 uniform expansion: |t| >= 1.25 lies beyond the tail cut from this shape
// on (k phi(-1.25) = 0.5365 k > 40), so the series of phi below 1.25 suffices
constexpr float kTemmeFarK = 75.f;
// FP32 uniform expansion: shapes from which |eta| <= 0.5 inside the tail cut,
// where h_0..h_3 of low degree keep the truncation below 1e-7 of the tail
constexpr float kTemmeLowDegK = 320.f;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kLnSqrtTwoPi = 0.91893853320467274178032973640562;

// Per-model constants of the generalized gamma with exponent p.
constexpr int kKTab = 512;             // start table of the shape solve
constexpr double kKTabLo = -14.0;      // ln tau range of the table
constexpr double kKTabHi = 4.0;
constexpr int kSupTab = 512;           // support-root table
constexpr double kSupLo = -9.0;        // ln k range of the table
constexpr double kSupHi = 16.0;
struct GGConst {
  double p, ip;                 // p, 1/p
  double cG[kSeriesTerms + 1];  // G(x) = ln Gamma(x) + ln Gamma(x+2/p) - 2 ln Gamma(x+1/p) = sum cG[n] x^-n
  double cD[kSeriesTerms + 1];  // D(x) = ln Gamma(x+1/p) - ln Gamma(x) - ln(x)/p = sum cD[n] x^-n
  double lnk_tab[kKTab];        // ln k at ln tau = kKTabLo + i (kKTabHi - kKTabLo)/(kKTab - 1)
  // roots t- < 0 < t+ of e^t - 1 - t = Bs / k (the support bounds in
  // t = ln(y/k)) at ln k = kSupLo + i (kSupHi - kSupLo)/(kSupTab - 1),
  // rounded outward; Bs is the support cut of the model's precision
  float sup_lo[kSupTab], sup_hi[kSupTab];
  int has_tab;
};

// ---------------------------------------------------------------------------
// FP64 column helpers.
// ---------------------------------------------------------------------------
BX_HD double series_inv(const double* c, int n, double x) {  // sum_{i=1..n} c[i] x^-i
  const double ix = 1.0 / x;
  double s = 0.0;
  for (int i = n; i >= 1; --i) s = (s + c[i]) * ix;
  return s;
}
BX_HD double dseries_inv(const double* c, int n, double x) {  // d/dx of the above
  const double ix = 1.0 / x;
  double s = 0.0;
  for (int i = n; i >= 1; --i) s = s * ix - i * c[i];
  return s * ix * ix;
}

// Stirling remainder ln Gamma*(x) for x >= kShift: sum B_2n / (2n (2n-1) x^(2n-1)).
BX_HD double lngamstar_big(double x) {
  const double ix = 1.0 / x, ix2 = ix * ix;
  // B2/2, B4/12, B6/30, B8/56, B10/90, B12/132, B14/182, B16/240
  const double c[8] = {1.0 / 12, -1.0 / 360, 1.0 / 1260, -1.0 / 1680, 1.0 / 1188,
                       -691.0 / 360360, 1.0 / 156, -3617.0 / 122400};
  double s = 0.0;
  for (int i = 7; i >= 0; --i) s = s * ix2 + c[i];
  return s * ix;
}
// digamma for x >= kShift: ln x - 1/(2x) - sum B_2n / (2n x^2n)
BX_HD double digamma_big(double x) {
  const double ix = 1.0 / x, ix2 = ix * ix;
  const double c[8] = {1.0 / 12, -1.0 / 120, 1.0 / 252, -1.0 / 240, 1.0 / 132,
                       -691.0 / 32760, 1.0 / 12, -3617.0 / 8160};
  double s = 0.0;
  for (int i = 7; i >= 0; --i) s = s * ix2 + c[i];
  return log(x) - 0.5 * ix - s * ix2;
}

// digamma for x > 0: the recurrence psi(x) = psi(x + 1) - 1/x up to x >= 10,
// then the asymptotic series.
BX_HD double digamma_pos(double x) {
  double acc = 0.0;
  while (x < 10.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  return acc + digamma_big(x);
}

// Column quantities of the GG shape k (all FP64).
struct GGShape {
  double G, dG;      // G(k), G'(k)
  double D1, dD1;    // ln Gamma(k+1/p) - ln Gamma(k), derivative
  double lngs;       // ln Gamma*(k)
  double dlngs;      // d ln Gamma*(k)/dk = psi(k) - ln k + 1/(2k)
  double psi;        // psi(k)
};

BX_HD GGShape gg_shape(const GGConst& c, double k, bool full) {
  GGShape o;
  const double a1 = c.ip, a2 = 2.0 * c.ip;
  double x = k, lnprod = 0.0, dsum = 0.0, lnprodD = 0.0, dsumD = 0.0, lnprodG = 0.0, psum = 0.0;
  if (k < kShift) {
    // products over m < shift of (k+m), (k+m+1/p), (k+m+2/p) and their k
    // derivatives (product rule), so the logarithmic derivatives need one
    // division each: ln Gamma(k + a) = ln Gamma(k + shift + a) - sum_m ln(k + m + a)
    double P0 = 1.0, P1 = 1.0, P2 = 1.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int m = 0; m < (int)kShift; ++m) {
      const double km = k + m;
      d0 = d0 * km + P0;
      P0 *= km;
      d1 = d1 * (km + a1) + P1;
      P1 *= km + a1;
      d2 = d2 * (km + a2) + P2;
      P2 *= km + a2;
    }
    const double l0 = log(P0), l1 = log(P1), l2 = log(P2);
    const double q0 = d0 / P0, q1 = d1 / P1, q2 = d2 / P2;
    lnprod = l2 + l0 - 2.0 * l1;
    dsum = q2 + q0 - 2.0 * q1;
    lnprodD = l1 - l0;
    dsumD = q1 - q0;
    lnprodG = l0;
    psum = q0;
    x = k + kShift;
  }
  o.G = series_inv(c.cG, kSeriesTerms, x) - lnprod;
  o.dG = dseries_inv(c.cG, kSeriesTerms, x) - dsum;
  o.D1 = c.ip * log(x) + series_inv(c.cD, kSeriesTerms, x) - lnprodD;
  o.dD1 = c.ip / x + dseries_inv(c.cD, kSeriesTerms, x) - dsumD;
  if (full) {
    // ln Gamma(k) = ln Gamma(x) - ln prod, ln Gamma(x) = (x - 1/2) ln x - x + ln sqrt(2 pi) + lngs(x)
    if (k < kShift) {
      const double lgx = (x - 0.5) * log(x) - x + kLnSqrtTwoPi + lngamstar_big(x);
      const double lgk = lgx - lnprodG;
      o.lngs = lgk - ((k - 0.5) * log(k) - k + kLnSqrtTwoPi);
      o.psi = digamma_big(x) - psum;
    } else {
      o.lngs = lngamstar_big(k);
      o.psi = digamma_big(k);
    }
    o.dlngs = o.psi - log(k) + 0.5 / k;
  }
  return o;
}

// Shape k of the GG with ln(1 + Var/Mean^2) = tau: Newton in u = ln k.
// Newton steps stop once a step is below tol (the error left is then of
// order tol^2).
BX_HD double gg_solve_k(const GGConst& c, double tau, int* iters, double tol = 1e-9) {
  // start: cubic interpolation in the table (~1e-7 relative), else
  // G ~ cG1/k + cG2/k^2 for large k (solve the quadratic), G ~ -ln k for
  // small k
  double u;
  const double lt = log(tau);
  const double pos = (lt - kKTabLo) * ((kKTab - 1) / (kKTabHi - kKTabLo));
  if (c.has_tab && pos >= 1.0 && pos < kKTab - 2) {
    const int i0 = (int)pos;
    const double w = pos - i0;
    const double ym = c.lnk_tab[i0 - 1], y0 = c.lnk_tab[i0], y1 = c.lnk_tab[i0 + 1], y2 = c.lnk_tab[i0 + 2];
    // Lagrange cubic through the four neighbours (unit spacing)
    u = -w * (w - 1.0) * (w - 2.0) * (1.0 / 6.0) * ym + (w + 1.0) * (w - 1.0) * (w - 2.0) * 0.5 * y0 -
        (w + 1.0) * w * (w - 2.0) * 0.5 * y1 + (w + 1.0) * w * (w - 1.0) * (1.0 / 6.0) * y2;
  } else if (tau < 0.1) {
    const double a1 = c.cG[1], a2 = c.cG[2];
    u = log((a1 + sqrt(fmax(a1 * a1 + 4.0 * tau * a2, 0.0))) / (2.0 * tau));
  } else {
    u = tau > 1.0 ? -tau : -log(c.p * c.p * tau);
  }
  int it = 0;
  for (; it < 40; ++it) {
    const double k = exp(u);
    const GGShape s = gg_shape(c, k, false);
    double du = (s.G - tau) / (k * s.dG);
    du = fmax(-2.0, fmin(2.0, du));
    u -= du;
    if (fabs(du) < tol) break;
  }
  if (iters) *iters = it;
  return exp(u);
}

// Reciprocal: the FP32 hardware reciprocal (1 ulp) on the GPU, exact division
// otherwise.
BX_HD float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
BX_HD double rcp(double x) { return 1.0 / x; }

// Square root: the FP32 hardware square root (1 ulp) on the GPU.
BX_HD float sqrt_hw(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
BX_HD double sqrt_hw(double x) { return sqrt(x); }

// phi(t) = e^t - 1 - t from t^2 (1/2! + t/3! + ... + t^10/12!): relative
// truncation error below 4e-9 for |t| < 1.25.
template <class R>
BX_HD R phi_series(R t) {
  R s = (R)(1.0 / 479001600.0);
  const R c[10] = {(R)(1.0 / 39916800.0), (R)(1.0 / 3628800.0), (R)(1.0 / 362880.0),
                   (R)(1.0 / 40320.0),    (R)(1.0 / 5040.0),    (R)(1.0 / 720.0),
                   (R)(1.0 / 120.0),      (R)(1.0 / 24.0),      (R)(1.0 / 6.0),
                   (R)(0.5)};
  for (int i = 0; i < 10; ++i) s = s * t + c[i];
  return s * t * t;
}

// phi(t) = e^t - 1 - t (accurate for small t); also returns e^t - 1.
template <class R>
BX_HD R phi_t(R t, R* um1) {
  if (fabs(t) < (R)0.5) {
    const R ph = phi_series(t);
    *um1 = ph + t;
    return ph;
  }
  const R u = expm1(t);
  *um1 = u;
  return u - t;
}

// ---------------------------------------------------------------------------
// Per-edge evaluation.  Result: v = signed smaller tail (v >= 0: F(x) = v on
// the lower side; v <= 0 with the sign bit set: 1 - F(x) = -v on the upper
// side), and dF/dc1, dF/dc2 for the column parameters (Gauss: m, sigma; GG:
// k, ln a).
// ---------------------------------------------------------------------------
template <class R>
struct EdgeVal {
  R v, d1, d2;
};

// Gaussian.  zd = (x - m)/sigma formed in FP64 by the caller.
template <class R, bool D>
BX_HD EdgeVal<R> gauss_edge(double x, double m, double inv_sigma) {
  EdgeVal<R> o;
  if (inv_sigma > 0.0) {
    const R z = (R)((x - m) * inv_sigma);
    const R tail = (R)0.5 * erfc(fabs(z) * (R)0.70710678118654752440);
    o.v = z > (R)0 ? -tail : tail;
    if (D) {
      const R ph = exp((R)-0.5 * z * z) * (R)0.39894228040143267794;
      o.d1 = -ph * (R)inv_sigma;
      o.d2 = -z * ph * (R)inv_sigma;
    }
  } else {  // zero width: all mass in the bin [x_j, x_j+1) holding m
    o.v = x > m ? -(R)0 : (R)0;
    o.d1 = o.d2 = (R)0;
  }
  return o;
}

// Column constants of the GG edge routine (FP32 or FP64 copies).
template <class R>
struct GGCol {
  double ct;     // p ln a + ln k   (t = p ln x - ct)
  R k, ik;       // k, 1/k
  R skh;         // sqrt(k/2)
  R cR;          // 1 / (sqrt(2 pi k) Gamma*(k))
  R ce;          // 1 / (2 sqrt(2 pi k))
  R dlngs;       // d ln Gamma*/dk
  R lnk_psi;     // ln k - psi(k)
  R p;           // exponent
};

// Uniform expansion (large k): functions h_n(eta).
template <class R>
BX_HD R horner(const double* c, int deg, R x) {
  R s = (R)c[deg];
  for (int i = deg - 1; i >= 0; --i) s = s * x + (R)c[i];
  return s;
}

// Truncated sum h0 + ik (h1 + ik (h2 + ik h3)) and its k-part
// ik^2 (h1 + ik (2 h2 + 3 ik h3)) at |eta| < 1, h_n of degrees N0..N3.
template <int N0, int N1, int N2, int N3, class R>
BX_HD void temme_h(R eta, R ik, R* Hs, R* dH) {
  const R h0 = horner<R>(bx_temme_h0, N0, eta);
  const R h1 = horner<R>(bx_temme_h1, N1, eta);
  const R h2 = horner<R>(bx_temme_h2, N2, eta);
  const R h3 = horner<R>(bx_temme_h3, N3, eta);
  *Hs = h0 + ik * (h1 + ik * (h2 + ik * h3));
  *dH = ik * ik * (h1 + ik * ((R)2 * h2 + (R)3 * ik * h3));
}

// FP32 only (shapes k >= kTemmeMinK).
template <class R, bool D>
BX_HD EdgeVal<R> gg_edge_temme(R t, const GGCol<R>& c) {
  const bool up = t > (R)0;
  EdgeVal<R> o;
  o.v = up ? (R)-0.0 : (R)0.0;  // beyond the tail cut: the side's zero
  o.d1 = o.d2 = (R)0;
  // phi and u = e^t - 1; |t| >= 1.25 is beyond the cut for k >= kTemmeFarK
  R ph, u;
  if (fabs(t) < (R)1.25) {
    ph = phi_series(t);
    u = ph + t;
  } else {
    if (c.k >= (R)kTemmeFarK) return o;
    u = expm1(t);
    ph = u - t;
  }
  const R eta = up ? sqrt_hw((R)2 * ph) : -sqrt_hw((R)2 * ph);
  const R kph = c.k * ph;
  // The two terms of the tail cancel far out, and beyond k*phi ~ 87 both are
  // FP32 subnormals, so their sum can even come out negative (which would put
  // the edge on the wrong side of the median).  Past kTemmeTailCut, beyond the
  // support cut of every column, the tail (< e^-40) is taken as the side's
  // zero and nothing else is evaluated; for k >= 2 kTemmeTailCut this also
  // leaves |eta| < 1 as the only branch inside the cut.
  if (kph > (R)kTemmeTailCut) return o;
  const R E = exp(-kph);
  const R w = fabs(eta) * c.skh;
  const R ik = c.ik;
  R Hs, dH;
  if (fabs(eta) < (R)1) {
    if (c.k >= (R)kTemmeLowDegK) temme_h<6, 3, 0, 0>(eta, ik, &Hs, &dH);
    else temme_h<10, 8, 5, 3>(eta, ik, &Hs, &dH);
  } else {
    const R ie = rcp(eta), ie2 = ie * ie, iu = rcp(u), iu2 = iu * iu;
    const R mu = (R)1 + u;
    const R h0 = iu - ie;
    const R h1 = ie2 * ie - mu * iu2 * iu - (R)(1.0 / 12) * ie;
    const R h2 = (R)-3 * ie2 * ie2 * ie + mu * ((R)2 * mu + (R)1) * iu2 * iu2 * iu +
                 (R)(1.0 / 12) * ie2 * ie - (R)bx_temme_dh1_0 * ie;
    const R h3 = (R)15 * ie2 * ie2 * ie2 * ie - mu * ((R)6 * mu * mu + (R)8 * mu + (R)1) * iu2 * iu2 * iu2 * iu -
                 (R)0.25 * ie2 * ie2 * ie + (R)bx_temme_dh1_0 * ie2 * ie - (R)bx_temme_dh2_0 * ie;
    Hs = h0 + ik * (h1 + ik * (h2 + ik * h3));
    dH = ik * ik * (h1 + ik * ((R)2 * h2 + (R)3 * ik * h3));
  }
  const R Rt = E * c.cR * Hs;
  R T = (R)0.5 * erfc(w) + (up ? Rt : -Rt);
  if (!(T > (R)0)) T = (R)0;  // rounding below zero: the side's zero
  o.v = up ? -T : T;
  if (D) {
    const R g = c.k * c.cR * E;  // y^k e^-y / Gamma(k)
    const R dQk_eta = E * (-eta * c.ce + c.cR * Hs * ((R)-0.5 * eta * eta - (R)0.5 * ik - c.dlngs) -
                           c.cR * dH);
    o.d1 = -(dQk_eta + g * ik);  // dF/dk at fixed y
    o.d2 = -c.p * g;             // dF/d ln a at fixed k
  }
  return o;
}

// Small k: power series of P (y < k + 1) or continued fraction of Q, each
// with d/dk carried alongside (forward mode).
template <class R, bool D>
BX_HD EdgeVal<R> gg_edge_small(R t, const GGCol<R>& c) {
  constexpr bool f32 = sizeof(R) == 4;
  const R eps = f32 ? (R)3e-8 : (R)1e-17;
  const int itmax = f32 ? 200 : 4000;
  R u;
  const R ph = phi_t(t, &u);
  const R k = c.k;
  const R y = k * ((R)1 + u);
  const R g = k * c.cR * exp(-k * ph);  // y^k e^-y / Gamma(k)
  const R lny_psi = t + c.lnk_psi;      // ln y - psi(k)
  EdgeVal<R> o;
  if (y < k + (R)1) {
    R a = (R)1, da = (R)0, S = (R)1, dS = (R)0;
    for (int n = 1; n < itmax; ++n) {
      const R inv = rcp(k + (R)n);
      const R an = a * y * inv;
      da = (da * y - an) * inv;
      a = an;
      S += a;
      dS += da;
      if (a < eps * S) break;
    }
    const R P = g * c.ik * S;
    const R dP = g * c.ik * (S * (lny_psi - c.ik) + dS);  // psi(k+1) = psi(k) + 1/k
    o.v = P <= (R)0.5 ? P : -((R)1 - P);
    o.d1 = dP;
  } else {
    // Q = g * 1/(y+1-k- 1(1-k)/(y+3-k- 2(2-k)/(y+5-k- ...))), modified Lentz
    const R tiny = f32 ? (R)1e-30 : (R)1e-300;
    R b = y + (R)1 - k, db = (R)-1;
    R cc = (R)1 / tiny, dcc = (R)0;
    R d = rcp(b), dd = -db * d * d;
    R h = d, dh = dd;
    for (int i = 1; i < itmax; ++i) {
      const R an = -(R)i * ((R)i - k), dan = (R)i;
      b += (R)2;
      R dn = an * d + b;
      R ddn = dan * d + an * dd + db;
      if (fabs(dn) < tiny) dn = tiny;
      const R icc = rcp(cc);
      R cn = b + an * icc;
      R dcn = db + (dan * cc - an * dcc) * icc * icc;
      if (fabs(cn) < tiny) cn = tiny;
      d = rcp(dn);
      dd = -ddn * d * d;
      cc = cn;
      dcc = dcn;
      const R del = d * cc, ddel = dd * cc + d * dcc;
      dh = dh * del + h * ddel;
      h *= del;
      if (fabs(del - (R)1) < eps) break;
    }
    const R Q = g * h;
    o.v = -Q;
    o.d1 = -(g * lny_psi * h + g * dh);
  }
  if (D) o.d2 = -c.p * g;
  return o;
}

template <class R, bool D>
BX_HD EdgeVal<R> gg_edge(double lnx, const GGCol<R>& c) {
  if (!(lnx > -1e300)) {  // x <= 0: F = 0
    EdgeVal<R> o;
    o.v = (R)0;
    o.d1 = o.d2 = (R)0;
    return o;
  }
  const R t = (R)((double)c.p * lnx - c.ct);
  constexpr bool f32 = sizeof(R) == 4;
  if (f32 && c.k >= (R)kTemmeMinK) return gg_edge_temme<R, D>(t, c);
  return gg_edge_small<R, D>(t, c);
}

// Count estimator (FP64): reco bin j holds the single count n; negative
// binomial P(n) = Gamma(n + r) / (Gamma(r) n!) (r/(r+m))^r (m/(r+m))^n with
// mean m and shape r.  c = {m, r, ln Gamma(r), ln(r/(r+m)), ln(m/(r+m)),
// psi(r), 1/(r+m), 1/m} (per column); lnf = ln n! (a property of the row,
// formed once per lane).
// v = P(n), d1 = dP/dm, d2 = dP/dr.
template <bool D>
BX_HD EdgeVal<double> count_cell(double n, double lnf, const double* c) {
  EdgeVal<double> o;
  o.v = o.d1 = o.d2 = 0.0;
  const double m = c[0], r = c[1];
  if (!(n >= 0.0) || !(m > 0.0)) return o;
  const double P = exp(lgamma(n + r) - c[2] - lnf + r * c[3] + n * c[4]);
  o.v = P;
  if (D) {
    const double irm = c[6];
    o.d1 = P * (n * c[7] - (n + r) * irm);
    o.d2 = P * (digamma_pos(n + r) - c[5] + c[3] + (m - n) * irm);
  }
  return o;
}

// ---------------------------------------------------------------------------
// Cells as bin integrals of the response density (Eq. 1 integrated over one
// reco bin), by Gauss-Legendre quadrature on the bin.  For a bin narrow
// against the column's width this is cancellation-free: the CDF difference
// F(x_j+1) - F(x_j) loses about F/R of its digits, and the difference of the
// two edges' derivatives loses as much again.  The derivatives with respect
// to the column parameters are integrals of the density's derivatives over
// the same nodes, so they carry no difference at all.
//
// Truncation (relative to the bin's value, measured against exact CDF
// differences on the 3000 x 900 generalized-gamma grid and the 400 x 200
// Gaussian grid): with the half-width h of the bin in the column's natural
// variable and the column's width w, h/w <= 0.25 keeps it below 1e-10 with
// four nodes and below 1e-13 with five (relative to the column's sum).
// Wider bins use the CDF differences of the edge routines.
// ---------------------------------------------------------------------------
template <int NQ> struct GaussLegendre;
template <> struct GaussLegendre<4> {
  static constexpr double x[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                                  0.86113631159405257522};
  static constexpr double w[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                                  0.34785484513745385737};
};
template <> struct GaussLegendre<5> {
  static constexpr double x[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                                  0.53846931010568309104, 0.90617984593866399280};
  static constexpr double w[5] = {0.23692688505618908751, 0.47862867049936646804, 0.56888888888888888889,
                                  0.47862867049936646804, 0.23692688505618908751};
};
// 2 / (sum of the weights as R holds them): the scale that makes the rule
// with rounded weights integrate a constant exactly.  A rounded constant that
// multiplies every cell would bias every expected count by the same relative
// amount, and the gradient of the NLL amplifies such a bias by 1/|1 - n/mu|,
// which is ~50 at these counts.
template <class R, int NQ>
constexpr double gl_norm() {
  double s = 0.0;
  for (int q = 0; q < NQ; ++q) s += (double)(R)GaussLegendre<NQ>::w[q];
  return 2.0 / s;
}
constexpr int kNQ32 = 4;         // nodes per cell, FP32 cells
constexpr int kNQ64 = 5;         // nodes per cell, FP64 cells
constexpr double kQuadMax = 0.25;  // largest half-width / column width of one quadrature interval
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;

// e^x: the hardware base-2 exponential (1 ulp) on the GPU for FP32.
BX_HD float exp_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x * (float)kLog2e);
#else
  return expf(x);
#endif
}
BX_HD double exp_fast(double x) { return exp(x); }

// phi(t) = e^t - 1 - t and u = e^t - 1 for any t, accurate near 0: the power
// series inside |t| < 1.25 (FP32, relative error < 4e-9) or |t| < 0.5 (FP64,
// terms to t^17/17!, < 1e-18), expm1 outside, where u - t loses at most a
// few bits.
BX_HD float phi_full(float t, float* u) {
  if (fabsf(t) < 1.25f) {
    const float ph = phi_series(t);
    *u = ph + t;
    return ph;
  }
  const float e = expm1f(t);
  *u = e;
  return e - t;
}
BX_HD double phi_full(double t, double* u) {
  if (fabs(t) < 0.5) {
    double s = 1.0 / 355687428096000.0;  // 1/17!
    const double c[15] = {1.0 / 20922789888000.0, 1.0 / 1307674368000.0, 1.0 / 87178291200.0,
                          1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
                          1.0 / 362880.0, 1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0,
                          1.0 / 24.0, 1.0 / 6.0, 0.5};
    for (int i = 0; i < 15; ++i) s = s * t + c[i];
    const double ph = s * t * t;
    *u = ph + t;
    return ph;
  }
  const double e = expm1(t);
  *u = e;
  return e - t;
}

// A cell from quadrature: the value in FP64 (its scale factors applied in
// FP64, so that no rounded constant is common to many cells) and the two
// derivatives in the cell precision.
template <class R>
struct CellVal {
  double v;
  R d1, d2;
};

// Per reco bin constants of the generalized-gamma quadrature (they depend on
// the reco edges and the exponent p only).  In t = ln(y/k) = p ln x - ct the
// bin is [tm - h, tm + h] with tm = pum - ct, pum = p (ln x_j + ln x_j+1)/2,
// h = p (ln x_j+1 - ln x_j)/2.  Node q sits at tm + d_q, d_q = h xi_q, with
// phi(d_q) and e^d_q - 1.
template <class R, int NQ>
struct QRowGG {
  R d[NQ], fd[NQ], ed[NQ];
};

template <class R, int NQ>
BX_HD QRowGG<R, NQ> qrow_gg(double lnx0, double lnx1, double p) {
  QRowGG<R, NQ> r;
  const double h = 0.5 * p * (lnx1 - lnx0);
  for (int q = 0; q < NQ; ++q) {
    const double d = h * GaussLegendre<NQ>::x[q];
    double u;
    const double f = phi_full(d, &u);
    r.d[q] = (R)d;
    r.fd[q] = (R)f;
    r.ed[q] = (R)u;
  }
  return r;
}

// Sums over the nodes of one interval of the generalized-gamma quadrature
// centred at tc, with phi(tc) = phc, e^tc - 1 = uc and node offsets rw:
// s0 += sum w_q E_q, s1 += sum w_q E_q t_q, s2 += sum w_q E_q (e^t_q - 1),
// E_q = e^{-k phi(t_q)}; phi at the nodes from the centre:
// phi(tc + d) = phi(tc) + (e^tc - 1) d + e^tc phi(d).
template <class R, int NQ, bool D>
BX_HD void gg_nodes(R tc, R phc, R uc, const QRowGG<R, NQ>& rw, R k, R& s0, R& s1, R& s2) {
  const R epc = (R)1 + uc;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const R ph = fma(epc, rw.fd[q], fma(uc, rw.d[q], phc));
    const R wE = (R)GaussLegendre<NQ>::w[q] * exp_fast(-k * ph);
    s0 += wE;
    if (D) {
      s1 = fma(wE, tc + rw.d[q], s1);
      s2 = fma(wE, fma(epc, rw.ed[q], uc), s2);
    }
  }
}

// Generalized-gamma cell R = int g d(ln y) over the bin, g = y^k e^-y /
// Gamma(k) = k cR e^{-k phi(t)} with cR = 1/(sqrt(2 pi k) Gamma*(k)), and its
// derivatives at fixed x:
//   dR/dk    = int g (ln y - psi(k)) d(ln y) = int g (t + ln k - psi(k)),
//   dR/dln a = int g p (y - k) d(ln y)      = int g p k (e^t - 1).
// The bin is [tm - h, tm + h] in t, tm = pum - ct formed in FP64 and rounded
// once.  nsub = 1: one interval with the row's node constants rw; nsub > 1:
// the bin is cut into nsub equal intervals (composite rule), whose node
// constants are formed here.  kcr = k cR (FP64), lnk_psi = ln k - psi(k),
// pk = p k.
template <class R, int NQ, bool D>
BX_HD CellVal<R> gg_cell_quad(double pum, double h, double ct, const QRowGG<R, NQ>& rw, R k, double kcr,
                              R lnk_psi, R pk, int nsub = 1) {
  const R t = (R)(pum - ct);
  R um;
  const R phm = phi_full(t, &um);
  R s0 = (R)0, s1 = (R)0, s2 = (R)0;
  double hs = h;
  if (nsub <= 1) {
    gg_nodes<R, NQ, D>(t, phm, um, rw, k, s0, s1, s2);
  } else {
    hs = h / nsub;
    QRowGG<R, NQ> rs;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const R d = (R)(hs * GaussLegendre<NQ>::x[q]);
      R e;
      rs.fd[q] = phi_full(d, &e);
      rs.d[q] = d;
      rs.ed[q] = e;
    }
    for (int sb = 0; sb < nsub; ++sb) {
      const R c = (R)(h * ((double)(2 * sb + 1) / nsub - 1.0));  // sub-interval centre - tm
      R ec;
      const R fc = phi_full(c, &ec);
      const R epm = (R)1 + um;
      const R phc = fma(epm, fc, fma(um, c, phm));
      const R uc = fma(epm, ec, um);
      gg_nodes<R, NQ, D>(t + c, phc, uc, rs, k, s0, s1, s2);
    }
  }
  const double sc = hs * kcr * gl_norm<R, NQ>();
  CellVal<R> o;
  o.v = sc * (double)s0;
  o.d1 = o.d2 = (R)0;
  if (D) {
    const R c = (R)sc;
    o.d1 = c * fma(lnk_psi, s0, s1);
    o.d2 = c * pk * s2;
  }
  return o;
}

// The common case of gg_cell_quad, written for speed: one interval, the node
// exponentials e^{-k phi} as 2^{-kl phi} with kl = k log2(e), and the FP64
// scale sc = h kcr_n (kcr_n = k cR times the weight normalisation, a column
// constant).  FP32: phi(t) from its series for |t| < 1.25, else as
// (e^t - 1) - t with e^t = 2^{t log2(e)}, which loses nothing there (e^t - 1
// and phi are both bounded away from zero) beyond what the FP32 rounding of t
// itself already costs.  Same quantities as gg_cell_quad.
template <class R>
BX_HD R exp2_fast(R x);
template <>
BX_HD float exp2_fast<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x);
#else
  return exp2f(x);
#endif
}
template <>
BX_HD double exp2_fast<double>(double x) { return exp2(x); }

template <class R, int NQ, bool D>
BX_HD CellVal<R> gg_cell_lean(R t, double sc, const QRowGG<R, NQ>& rw, R kl, R lnk_psi, R pk) {
  R um;
  R phm;
  if constexpr (sizeof(R) == 4) {
    if (fabsf(t) < 1.25f) {
      phm = phi_series(t);
      um = phm + t;
    } else {
      um = exp2_fast<float>(t * (float)kLog2e) - 1.0f;
      phm = um - t;
    }
  } else {
    phm = phi_full(t, &um);
  }
  const R epm = (R)1 + um;
  R s0 = (R)0, s1 = (R)0, s2 = (R)0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const R ph = fma(epm, rw.fd[q], fma(um, rw.d[q], phm));
    const R wE = (R)GaussLegendre<NQ>::w[q] * exp2_fast<R>(-kl * ph);
    s0 += wE;
    if (D) {
      s1 = fma(wE, t + rw.d[q], s1);
      s2 = fma(wE, fma(epm, rw.ed[q], um), s2);
    }
  }
  CellVal<R> o;
  o.v = sc * (double)s0;
  o.d1 = o.d2 = (R)0;
  if (D) {
    const R c = (R)sc;
    o.d1 = c * fma(lnk_psi, s0, s1);
    o.d2 = c * pk * s2;
  }
  return o;
}

// Gaussian cell R = int phi(z) dz over [zm - hs, zm + hs], zm = (x_mid - m)/sigma,
// hs = (half bin width)/sigma, and its derivatives
//   dR/dm     = int phi(z) z dz / sigma,
//   dR/dsigma = int phi(z) (z^2 - 1) dz / sigma;
// nsub > 1: composite rule over nsub equal intervals.
template <class R, int NQ, bool D>
BX_HD CellVal<R> gauss_cell_quad(double xm, double hx, double m, double inv_sigma, int nsub = 1) {
  const R zm = (R)((xm - m) * inv_sigma);
  const int ns = nsub > 1 ? nsub : 1;
  const double hsd = hx * inv_sigma / ns;
  const R hs = (R)hsd;
  R s0 = (R)0, s1 = (R)0, s2 = (R)0;
  for (int sb = 0; sb < ns; ++sb) {
    const R zc = ns == 1 ? zm : (R)((xm - m) * inv_sigma + hsd * (2 * sb + 1 - ns));
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const R z = fma(hs, (R)GaussLegendre<NQ>::x[q], zc);
      const R wE = (R)GaussLegendre<NQ>::w[q] * exp_fast((R)-0.5 * z * z);
      s0 += wE;
      if (D) {
        s1 = fma(wE, z, s1);
        s2 = fma(wE, fma(z, z, (R)-1), s2);  // z^2 - 1 rounded once
      }
    }
  }
  const double sc = hsd * (kInvSqrt2Pi * gl_norm<R, NQ>());
  CellVal<R> o;
  o.v = sc * (double)s0;
  o.d1 = o.d2 = (R)0;
  if (D) {
    const R ci = (R)(sc * inv_sigma);
    o.d1 = ci * s1;
    o.d2 = ci * s2;
  }
  return o;
}

// Intervals of the composite rule for a bin of half-width h (in the column's
// quadrature variable) against the column's inverse width iw: 1 while
// h iw <= kQuadMax, up to kMaxSub intervals of half-width <= kQuadMax / iw,
// 0 beyond (the bin is then taken as a CDF difference).
constexpr int kMaxSub = 16;
BX_HD int quad_intervals(double h, double iw) {
  const double c = h * iw;
  if (!(c <= kQuadMax * kMaxSub)) return 0;  // also h = +inf (a GG bin from x <= 0) or NaN
  return c <= kQuadMax ? 1 : (int)ceil(c * (1.0 / kQuadMax));
}

// Cell from two neighbouring encoded edge values (lower edge lo, upper hi).
template <class R>
BX_HD R cell_from(R lo, R hi) {
  const bool straddle = signbit(hi) && !signbit(lo);
  return (hi - lo) + (straddle ? (R)1 : (R)0);
}

}  // namespace bx

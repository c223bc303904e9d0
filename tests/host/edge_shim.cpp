// Host build of the per-edge response arithmetic (the same header the kernels
// use), for unit tests against library incomplete-gamma ratios.  The column
// constants are passed in, computed by the test from their definitions.
#include "bx_math.h"

using namespace bx;

template <class R>
static void run(int n, const double* ct, const double* k, const double* cR, const double* dlngs,
                const double* lnk_psi, double p, const double* lnx, R* v, R* d1, R* d2) {
  for (int i = 0; i < n; ++i) {
    GGCol<R> c;
    c.ct = ct[i];
    c.k = (R)k[i];
    c.ik = (R)(1.0 / k[i]);
    c.skh = (R)sqrt(0.5 * k[i]);
    c.cR = (R)cR[i];
    c.ce = (R)(0.5 / sqrt(kTwoPi * k[i]));
    c.dlngs = (R)dlngs[i];
    c.lnk_psi = (R)lnk_psi[i];
    c.p = (R)p;
    const EdgeVal<R> e = gg_edge<R, true>(lnx[i], c);
    v[i] = e.v;
    d1[i] = e.d1;
    d2[i] = e.d2;
  }
}

extern "C" {
// Encoded edge values: v >= 0 holds F(x) (lower side), v with its sign bit set
// holds -(1 - F(x)) (upper side); d1 = dF/dk at fixed a, d2 = dF/d ln a.
void edge_f32(int n, const double* ct, const double* k, const double* cR, const double* dlngs,
              const double* lnk_psi, double p, const double* lnx, float* v, float* d1, float* d2) {
  run<float>(n, ct, k, cR, dlngs, lnk_psi, p, lnx, v, d1, d2);
}
void edge_f64(int n, const double* ct, const double* k, const double* cR, const double* dlngs,
              const double* lnk_psi, double p, const double* lnx, double* v, double* d1, double* d2) {
  run<double>(n, ct, k, cR, dlngs, lnk_psi, p, lnx, v, d1, d2);
}
// Cell between two encoded edge values.
float cell_f32(float lo, float hi) { return cell_from<float>(lo, hi); }
}

// Quadrature cells (bin integrals of the density).  Generalized gamma: the
// bin [x0, x1] in ln x, column (ct, k, cR, ln k - psi(k)), exponent p; out:
// value, dR/dk, dR/d ln a.  Gaussian: bin [x0, x1], column (m, 1/sigma); out:
// value, dR/dm, dR/dsigma.  The value is formed in FP64 from the sums of the
// cell precision, the derivatives in the cell precision.
template <class R, int NQ>
static void quad_gg(int n, const double* lnx0, const double* lnx1, double ct, double k, double cR,
                    double lnk_psi, double p, double* out) {
  for (int i = 0; i < n; ++i) {
    const QRowGG<R, NQ> rw = qrow_gg<R, NQ>(lnx0[i], lnx1[i], p);
    const double pum = 0.5 * p * (lnx0[i] + lnx1[i]), h = 0.5 * p * (lnx1[i] - lnx0[i]);
    const CellVal<R> e = gg_cell_quad<R, NQ, true>(pum, h, ct, rw, (R)k, k * cR, (R)lnk_psi, (R)(p * k));
    out[3 * i] = e.v;
    out[3 * i + 1] = e.d1;
    out[3 * i + 2] = e.d2;
  }
}
template <class R, int NQ>
static void quad_gauss(int n, const double* x0, const double* x1, double m, double inv_sigma, double* out) {
  for (int i = 0; i < n; ++i) {
    const CellVal<R> e = gauss_cell_quad<R, NQ, true>(0.5 * (x0[i] + x1[i]), 0.5 * (x1[i] - x0[i]), m, inv_sigma);
    out[3 * i] = e.v;
    out[3 * i + 1] = e.d1;
    out[3 * i + 2] = e.d2;
  }
}
extern "C" {
void quad_gg_f32(int n, const double* a, const double* b, double ct, double k, double cR, double lk, double p,
                 double* o) {
  quad_gg<float, kNQ32>(n, a, b, ct, k, cR, lk, p, o);
}
void quad_gg_f64(int n, const double* a, const double* b, double ct, double k, double cR, double lk, double p,
                 double* o) {
  quad_gg<double, kNQ64>(n, a, b, ct, k, cR, lk, p, o);
}
void quad_gauss_f32(int n, const double* a, const double* b, double m, double is, double* o) {
  quad_gauss<float, kNQ32>(n, a, b, m, is, o);
}
void quad_gauss_f64(int n, const double* a, const double* b, double m, double is, double* o) {
  quad_gauss<double, kNQ64>(n, a, b, m, is, o);
}
}

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

// Host runtime: validation, model placement in device memory, the C ABI of
// the plain path (build / eval / grad / expected counts) and the plain
// quasi-Newton fitter (Sec. 4, workflow steps 1-7 of the paper's package).
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "bx_model.hpp"
#include "bx_fitcore.hpp"

namespace bx {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
bx_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return BX_E_DEVICE;
}
#define BX_HIP(call, what)                  \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

static bx_status inval(const std::string& m) {
  set_error(m);
  return BX_E_INVAL;
}

// ---------------------------------------------------------------------------
// Stirling-series constants of the generalized gamma with exponent p:
// ln Gamma(x + a) ~ (x + a - 1/2) ln x - x + ln sqrt(2 pi)
//                   + sum_n (-1)^(n+1) B_{n+1}(a) / (n (n+1) x^n).
// ---------------------------------------------------------------------------
// Root of e^t - 1 - t = cb on the side sgn of 0 (Newton in FP64 from outside
// the root, where the function is convex and the iteration stays outside).
static double support_root(double cb, int sgn) {
  double t = sgn > 0 ? (cb > 2.0 ? std::log1p(cb) + std::log1p(std::log1p(cb)) : std::sqrt(2.0 * cb))
                     : -(1.0 + cb);
  for (int it = 0; it < 200; ++it) {
    const double e = std::expm1(t);
    const double d = (e - t - cb) / e;
    t -= d;
    if (std::fabs(d) <= 1e-15 * std::fmax(1.0, std::fabs(t))) break;
  }
  return t;
}

// bs: the support cut (k phi = bs) of the model's precision, with margin.
static void make_gg_const(double p, double bs, GGConst* c) {
  long double bern[kSeriesTerms + 3];
  bern[0] = 1.0L;
  for (int n = 1; n < kSeriesTerms + 3; ++n) {  // sum_{k<=n} C(n+1, k) B_k = 0
    long double s = 0.0L, binom = 1.0L;
    for (int k = 0; k < n; ++k) {
      s += binom * bern[k];
      binom = binom * (n + 1 - k) / (k + 1);
    }
    bern[n] = -s / (n + 1);
  }
  auto bpoly = [&](int n, long double a) {  // Bernoulli polynomial B_n(a)
    long double s = 0.0L, binom = 1.0L;
    for (int k = 0; k <= n; ++k) {
      s += binom * bern[k] * powl(a, n - k);
      binom = binom * (n - k) / (k + 1);
    }
    return s;
  };
  c->p = p;
  c->ip = 1.0 / p;
  const long double a1 = 1.0L / p, a2 = 2.0L / p;
  c->cG[0] = c->cD[0] = 0.0;
  for (int n = 1; n <= kSeriesTerms; ++n) {
    const long double sg = (n % 2 == 1) ? 1.0L : -1.0L, den = (long double)n * (n + 1);
    c->cG[n] = (double)(sg * (bpoly(n + 1, 0) + bpoly(n + 1, a2) - 2 * bpoly(n + 1, a1)) / den);
    c->cD[n] = (double)(sg * (bpoly(n + 1, a1) - bpoly(n + 1, 0)) / den);
  }
  // start table of the device shape solve: ln k on a grid of ln tau
  c->has_tab = 0;
  for (int i = 0; i < kKTab; ++i) {
    const double lt = kKTabLo + i * (kKTabHi - kKTabLo) / (kKTab - 1);
    c->lnk_tab[i] = std::log(gg_solve_k(*c, std::exp(lt), nullptr));
  }
  // support roots at ln k_i, rounded outward: for k in [k_i, k_i+1) the
  // roots lie inside those of k_i, so entry i bounds the support from outside
  for (int i = 0; i < kSupTab; ++i) {
    const double cb = bs / std::exp(kSupLo + i * (kSupHi - kSupLo) / (kSupTab - 1));
    const double hi = support_root(cb, 1), lo = support_root(cb, -1);
    float fh = (float)hi, fl = (float)lo;
    if ((double)fh < hi) fh = std::nextafterf(fh, INFINITY);
    if ((double)fl > lo) fl = std::nextafterf(fl, -INFINITY);
    c->sup_hi[i] = std::nextafterf(fh, INFINITY);
    c->sup_lo[i] = std::nextafterf(fl, -INFINITY);
  }
  c->has_tab = 1;
}

Tiles choose_tiles(int T, int N, int kind, int prec, int batched) {
  // True tiles per forward wave (CG) and reco tiles per backward wave (RG),
  // for one fit evaluated alone (latency: CG 1) or inside a batch (throughput:
  // fewer, fuller forward blocks).  A table written by the tuner
  // (BX_TUNE_CACHE: lines "kind prec Tmin Tmax Nmin Nmax batched CG RG")
  // overrides the defaults; BX_TILES="CG,RG" overrides both for sweeps.  CG
  // does not change any result bit (the forward partials are summed in a
  // fixed tree); RG groups the backward partials and does.
  Tiles t{batched ? 4 : 1, 1};
  const char* path = getenv("BX_TUNE_CACHE");
  if (path && *path) {
    FILE* fp = fopen(path, "r");
    if (fp) {
      char line[256];
      while (fgets(line, sizeof line, fp)) {
        int k, pr, tmin, tmax, nmin, nmax, bt, cg, rg;
        if (sscanf(line, "%d %d %d %d %d %d %d %d %d", &k, &pr, &tmin, &tmax, &nmin, &nmax, &bt, &cg, &rg) == 9 &&
            k == kind && pr == prec && T >= tmin && T <= tmax && N >= nmin && N <= nmax && bt == batched &&
            cg > 0 && rg > 0) {
          t.CG = cg;
          t.RG = rg;
          break;
        }
      }
      fclose(fp);
    }
  }
  const char* ov = getenv("BX_TILES");
  if (ov && *ov) {
    int cg = 0, rg = 0;
    if (sscanf(ov, "%d,%d", &cg, &rg) == 2 && cg > 0 && rg > 0) t = Tiles{cg, rg};
  }
  t.RG = std::min(t.RG, kMaxRG);
  // a power of two, at most kMaxCG; the FP64 count-estimator sweep at 8 tiles
  // needs more than the 128 VGPRs of a 16-wave block and spills, so 4 there
  const int cg_max = (kind == kCount && prec == kF64) ? 4 : kMaxCG;
  int cg = 1;
  while (cg * 2 <= std::min(t.CG, cg_max)) cg *= 2;
  t.CG = cg;
  return t;
}

// ---------------------------------------------------------------------------
static bool finite_nonneg(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i]) || v[i] < 0.0) return false;
  return true;
}
static bool increasing(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i]) || (i > 0 && !(v[i] > v[i - 1]))) return false;
  return true;
}

bx_status set_host_data(HostModel* h, const bx_data* x) {
  if (!x) return inval("data is NULL");
  if (h->joint) {  // the joint histogram replaces the vetoed energy, radial and PS histograms
    const size_t nj = (size_t)h->N * h->n_rad * h->n_ps;
    if (!x->joint || !finite_nonneg(x->joint, nj)) return inval("data: joint histogram missing or invalid");
    h->n_j.assign(x->joint, x->joint + nj);
    // the non-zero bins of each row, in bin order
    const int nr = h->n_rad, np = h->n_ps;
    h->jrow.assign(h->N + 1, 0);
    h->jent.clear();
    h->jval.clear();
    for (int j = 0; j < h->N; ++j) {
      for (int k = 0; k < nr; ++k)
        for (int l = 0; l < np; ++l) {
          const double v = x->joint[((size_t)j * nr + k) * np + l];
          if (v > 0.0) {
            h->jent.push_back((uint32_t)k << 16 | (uint32_t)l);
            h->jval.push_back(v);
          }
        }
      h->jrow[j + 1] = (int)h->jent.size();
    }
    if (!x->tagged || !finite_nonneg(x->tagged, h->N)) return inval("data: tagged histogram missing or invalid");
    h->n_t.assign(x->tagged, x->tagged + h->N);
    h->n_e.assign(h->N, 0.0);
    h->n_r.assign(h->n_rad, 0.0);
    h->n_p.assign((size_t)h->N * h->n_ps, 0.0);
    return BX_OK;
  }
  if (!x->energy) return inval("data: energy histogram is NULL");
  if (!finite_nonneg(x->energy, h->N)) return inval("data: energy counts must be finite and >= 0");
  h->n_e.assign(x->energy, x->energy + h->N);
  if (h->mv) {
    if (!x->tagged || !finite_nonneg(x->tagged, h->N)) return inval("data: tagged histogram missing or invalid");
    h->n_t.assign(x->tagged, x->tagged + h->N);
    if (h->n_rad > 0) {
      if (!x->radial || !finite_nonneg(x->radial, h->n_rad)) return inval("data: radial histogram missing or invalid");
      h->n_r.assign(x->radial, x->radial + h->n_rad);
    }
    if (h->n_ps > 0) {
      if (!x->ps || !finite_nonneg(x->ps, (size_t)h->N * h->n_ps)) return inval("data: PS histogram missing or invalid");
      h->n_p.assign(x->ps, x->ps + (size_t)h->N * h->n_ps);
    }
  }
  return BX_OK;
}

bx_status make_host_model(const bx_model_desc* d, const bx_data* x, HostModel* h) {
  if (!d) return inval("desc is NULL");
  if (d->T < 1 || d->N < 1 || d->S < 1 || d->S > kSP) return inval("need T >= 1, N >= 1, 1 <= S <= 16");
  if ((int64_t)d->T * d->N > (int64_t)1 << 31) return inval("T x N too large");
  if (!d->true_edges || !increasing(d->true_edges, d->T + 1)) return inval("true_edges must be finite and strictly increasing");
  if (!d->reco_edges || !increasing(d->reco_edges, d->N + 1)) return inval("reco_edges must be finite and strictly increasing");
  if (!d->spectra || !finite_nonneg(d->spectra, (size_t)d->S * d->T)) return inval("spectra must be finite and >= 0");
  if (d->response != BX_RESP_GAUSS && d->response != BX_RESP_GG && d->response != BX_RESP_TABLE &&
      d->response != BX_RESP_COUNT)
    return inval("unknown response kind");
  if (d->precision != BX_PREC_F32 && d->precision != BX_PREC_F64) return inval("unknown precision");
  if (!std::isfinite(d->exposure) || !(d->exposure > 0)) return inval("exposure must be > 0");
  if (d->response == BX_RESP_COUNT) {
    // one reco bin per count value: integer edges of unit width from >= 0
    if (!(d->reco_edges[0] >= 0) || d->reco_edges[0] != std::floor(d->reco_edges[0]))
      return inval("count estimator: reco edges must be integers >= 0");
    for (int j = 0; j < d->N; ++j)
      if (d->reco_edges[j + 1] != d->reco_edges[j] + 1.0) return inval("count estimator: one count per reco bin");
  }
  if (d->response == BX_RESP_GG || d->response == BX_RESP_COUNT) {
    if (d->response == BX_RESP_GG && (!std::isfinite(d->gg_p) || !(d->gg_p > 0.05) || d->gg_p > 20))
      return inval("gg_p must be in (0.05, 20]");
    if (!d->quench) return inval("this response needs the quenching table");
    for (int i = 0; i < d->T; ++i)
      if (!std::isfinite(d->quench[i]) || !(d->quench[i] > 0)) return inval("quench must be finite and > 0");
  }
  if (d->response == BX_RESP_TABLE) {
    if (d->n_grid < 1 || d->n_grid > kMaxGrid) return inval("n_grid must be in [1, 64]");
    if (!d->grid || !increasing(d->grid, d->n_grid)) return inval("grid must be finite and strictly increasing");
    if (!d->rtab || !finite_nonneg(d->rtab, (size_t)d->n_grid * d->N * d->T)) return inval("rtab must be finite and >= 0");
  }
  if (d->win_lo < 0 || d->win_hi > d->N || d->win_lo >= d->win_hi) return inval("fit window out of range");
  if (d->pu_K < 0 || d->pu_K > kMaxK) return inval("pu_K must be in [0, 256]");
  HostModel& m = *h;
  m.T = d->T; m.N = d->N; m.S = d->S;
  m.kind = d->response == BX_RESP_GAUSS ? kGauss : d->response == BX_RESP_GG ? kGG
         : d->response == BX_RESP_TABLE ? kTable : kCount;
  m.nresp = m.kind == kGauss ? 2 : m.kind == kTable ? (d->n_grid > 1 ? 1 : 0) : 4;
  m.n_grid = 0;
  if (m.kind == kTable) {
    m.n_grid = d->n_grid;
    m.grid.assign(d->grid, d->grid + d->n_grid);
    m.rtab.assign(d->rtab, d->rtab + (size_t)d->n_grid * d->N * d->T);
  }
  m.pu_float = d->pu_float ? 1 : 0;
  if (m.pu_float && !(d->pu_K > 0)) return inval("a floated pile-up fraction needs pu_K > 0");
  m.P = m.S + m.nresp + m.pu_float;
  m.prec = d->precision == BX_PREC_F32 && m.kind != kTable && m.kind != kCount ? kF32 : kF64;
  m.win_lo = d->win_lo; m.win_hi = d->win_hi;
  m.exposure = d->exposure;
  m.p = m.kind == kGG ? d->gg_p : 1.0;
  m.K = 0; m.pu_frac = 0.0;
  if (d->pu_K > 0 && (d->pu_frac != 0.0 || m.pu_float)) {
    if (!d->pu_g || !finite_nonneg(d->pu_g, d->pu_K)) return inval("pu_g must be finite and >= 0");
    if (!m.pu_float && (!std::isfinite(d->pu_frac) || d->pu_frac < 0 || d->pu_frac > 1))
      return inval("pu_frac must be in [0, 1]");
    long double sg = 0.0L;
    for (int k = 0; k < d->pu_K; ++k) sg += d->pu_g[k];
    if (!(sg > 0)) return inval("pu_g has zero sum");
    const double w0 = d->reco_edges[1] - d->reco_edges[0];
    for (int j = 1; j < d->N; ++j) {
      const double w = d->reco_edges[j + 1] - d->reco_edges[j];
      if (std::fabs(w - w0) > 1e-9 * std::fabs(w0)) return inval("pile-up needs uniform reco bins");
    }
    m.K = d->pu_K;
    m.pu_frac = m.pu_float ? 0.0 : d->pu_frac;
    m.ghat.resize(m.K);
    for (int k = 0; k < m.K; ++k) m.ghat[k] = (double)(d->pu_g[k] / sg);
  }
  m.mv = d->multivariate ? 1 : 0;
  m.n_rad = m.n_ps = 0;
  m.rad_lo = m.rad_hi = 0;
  m.tag.assign(kSP, 0.0);
  if (m.mv) {
    if (!d->tag_frac) return inval("multivariate model needs tag_frac");
    for (int s = 0; s < m.S; ++s) {
      if (!std::isfinite(d->tag_frac[s]) || d->tag_frac[s] < 0 || d->tag_frac[s] > 1) return inval("tag_frac must be in [0, 1]");
      m.tag[s] = d->tag_frac[s];
    }
    if (d->n_rad < 0 || d->n_rad > 128) return inval("n_rad must be in [0, 128]");
    if (d->n_ps < 0 || d->n_ps > 64) return inval("n_ps must be in [0, 64]");
    m.n_rad = d->n_rad;
    m.n_ps = d->n_ps;
    if (m.n_rad > 0) {
      if (!d->rad_tmpl || !finite_nonneg(d->rad_tmpl, (size_t)m.S * m.n_rad)) return inval("rad_tmpl invalid");
      if (!d->joint && (d->rad_lo < 0 || d->rad_hi > m.N || d->rad_lo >= d->rad_hi)) return inval("radial window out of range");
      m.rad_lo = d->rad_lo; m.rad_hi = d->rad_hi;
      m.rad.assign((size_t)kSP * m.n_rad, 0.0);
      for (int s = 0; s < m.S; ++s)
        for (int k = 0; k < m.n_rad; ++k) m.rad[s * m.n_rad + k] = d->rad_tmpl[s * m.n_rad + k];
    }
    m.joint = d->joint ? 1 : 0;
    if (m.joint && (m.n_rad < 1 || m.n_ps < 1)) return inval("the joint term needs n_rad >= 1 and n_ps >= 1");
    if (m.joint && (size_t)m.N * m.n_rad * m.n_ps > 0x7fffffff) return inval("joint histogram above 2^31 bins");
    if (m.joint) { m.rad_lo = 0; m.rad_hi = m.N; }
    if (m.n_ps > 0) {
      if (!d->ps_tmpl || !finite_nonneg(d->ps_tmpl, (size_t)m.S * m.n_ps)) return inval("ps_tmpl invalid");
      m.pst.assign((size_t)kSP * m.n_ps, 0.0);
      for (int s = 0; s < m.S; ++s)
        for (int k = 0; k < m.n_ps; ++k) m.pst[s * m.n_ps + k] = d->ps_tmpl[s * m.n_ps + k];
    }
    if (m.joint) {  // sum over a row's bins of rho_sk T_sl
      m.jsig.assign(kSP, 0.0);
      for (int s = 0; s < m.S; ++s) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < m.n_rad; ++k) a += m.rad[s * m.n_rad + k];
        for (int l = 0; l < m.n_ps; ++l) b += m.pst[s * m.n_ps + l];
        m.jsig[s] = a * b;
      }
    }
  }
  // grids
  m.xraw.assign(d->reco_edges, d->reco_edges + m.N + 1);
  m.xe.resize(m.N + 1);
  for (int j = 0; j <= m.N; ++j)
    m.xe[j] = m.kind != kGG ? m.xraw[j] : (m.xraw[j] > 0 ? std::log(m.xraw[j]) : -INFINITY);
  m.Ec.resize(m.T);
  for (int i = 0; i < m.T; ++i) m.Ec[i] = 0.5 * (d->true_edges[i] + d->true_edges[i + 1]);
  m.Qt.assign(m.T, 1.0);
  if (m.kind == kGG || m.kind == kCount) m.Qt.assign(d->quench, d->quench + m.T);
  // quadrature constants of the reco bins (bx_math.h: gg_cell_quad,
  // gauss_cell_quad): a GG bin from x <= 0 has no finite width in ln x and is
  // always a CDF difference
  m.qpum.assign(m.N, 0.0);
  m.qhw.assign(m.N, INFINITY);
  m.qrow32.assign((size_t)m.N * 3 * kNQ32, 0.f);
  m.qrow64.assign((size_t)m.N * 3 * kNQ64, 0.0);
  for (int j = 0; j < m.N; ++j) {
    if (m.kind == kGG && m.xraw[j] > 0.0) {
      m.qpum[j] = 0.5 * m.p * (m.xe[j] + m.xe[j + 1]);
      m.qhw[j] = 0.5 * m.p * (m.xe[j + 1] - m.xe[j]);
      const QRowGG<float, kNQ32> r32 = qrow_gg<float, kNQ32>(m.xe[j], m.xe[j + 1], m.p);
      const QRowGG<double, kNQ64> r64 = qrow_gg<double, kNQ64>(m.xe[j], m.xe[j + 1], m.p);
      static_assert(sizeof r32 == 3 * kNQ32 * sizeof(float) && sizeof r64 == 3 * kNQ64 * sizeof(double),
                    "row table layout");
      memcpy(&m.qrow32[(size_t)j * 3 * kNQ32], &r32, sizeof r32);
      memcpy(&m.qrow64[(size_t)j * 3 * kNQ64], &r64, sizeof r64);
    } else if (m.kind == kGauss) {
      m.qhw[j] = 0.5 * (m.xraw[j + 1] - m.xraw[j]);
    }
  }
  m.fixp.assign((m.N + kRowStep - 1) / kRowStep, 0.0);
  for (int j = 0; j < m.N; ++j) {
    double b = (m.kind == kGG && m.prec == kF32) ? (double)(float)m.qhw[j] : m.qhw[j];
    if (b != b) b = INFINITY;
    m.fixp[j / kRowStep] = std::max(m.fixp[j / kRowStep], b);
  }
  // spectra: unit rows (FP64), times exposure, species padded to 16
  m.F64.assign((size_t)m.T * kSP, 0.0);
  m.F32.assign((size_t)m.T * kSP, 0.f);
  for (int s = 0; s < m.S; ++s) {
    long double sum = 0.0L;
    for (int i = 0; i < m.T; ++i) sum += d->spectra[(size_t)s * m.T + i];
    if (!(sum > 0)) return inval("a spectrum row sums to zero");
    for (int i = 0; i < m.T; ++i) {
      const double v = m.exposure * (double)(d->spectra[(size_t)s * m.T + i] / sum);
      m.F64[(size_t)i * kSP + s] = v;
      m.F32[(size_t)i * kSP + s] = (float)v;
    }
  }
  if (m.kind == kGG) make_gg_const(m.p, 1.05 * (m.prec == kF32 ? kSupportB32 : kSupportB), &m.gg);
  else memset(&m.gg, 0, sizeof m.gg);
  m.tiles = choose_tiles(m.T, m.N, m.kind, m.prec, 0);
  return set_host_data(h, x);
}

double host_lnfact(const HostModel& h) {
  long double s = 0.0L;
  if (h.joint) {
    const size_t nb = (size_t)h.n_rad * h.n_ps;
    for (int j = h.win_lo; j < h.win_hi; ++j) {
      s += std::lgamma(h.n_t[j] + 1.0);
      for (size_t b = 0; b < nb; ++b) s += std::lgamma(h.n_j[(size_t)j * nb + b] + 1.0);
    }
    return (double)s;
  }
  for (int j = h.win_lo; j < h.win_hi; ++j) {
    s += std::lgamma(h.n_e[j] + 1.0);
    if (h.mv) s += std::lgamma(h.n_t[j] + 1.0);
    if (h.mv && h.n_ps > 0)
      for (int k = 0; k < h.n_ps; ++k) s += std::lgamma(h.n_p[(size_t)j * h.n_ps + k] + 1.0);
  }
  if (h.mv)
    for (int k = 0; k < h.n_rad; ++k) s += std::lgamma(h.n_r[k] + 1.0);
  return (double)s;
}

// ---------------------------------------------------------------------------
// Device placement.
// ---------------------------------------------------------------------------
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

void derive_tiles(const HostModel& h, FitDev* f) {
  f->T = h.T;
  f->N = h.N;
  f->n_rt = (h.N + kRowStep - 1) / kRowStep;
  f->n_ct = h.kind == kTable ? 0 : (h.T + kColTile - 1) / kColTile;  // a table has no cell sweeps
  f->CG = h.tiles.CG;
  f->RG = h.tiles.RG;
  // forward partials: one per chunk of kFwdWaves listed true tiles; a forward
  // block holds CG chunks; a backward block kBwdWaves waves of RG reco tiles
  f->n_cg = (f->n_ct + kFwdWaves - 1) / kFwdWaves;
  f->n_fb = (f->n_cg + f->CG - 1) / f->CG;
  f->n_rg = (f->n_rt + kBwdWaves * f->RG - 1) / (kBwdWaves * f->RG);
  f->n_rowblk = (h.N + 15) / 16;
  f->n_cpblk = h.kind == kTable ? 1 : (h.T + kCpBlock - 1) / kCpBlock;  // k_table writes one flag
  f->n_bwdblk = f->n_ct * f->n_rg;
  f->kind = h.kind;
  f->prec = h.prec;
  f->sup_prec = h.prec;
  f->mv = h.mv;
  f->vsum = (!h.mv && h.kind != kTable) ? 1 : 0;
  f->has_fix = (h.kind == kGG || h.kind == kGauss) ? 1 : 0;
  f->n_rad = h.n_rad;
}

// Sub-buffers of one fit in `base`.  With `shared`, the read-only inputs
// (grids, spectra, templates, histograms) are those of an existing placement
// of the same model and only the per-evaluation workspace is carved.
static size_t carve(const HostModel& h, char* base, FitDev* f, double** theta, double** out,
                    const FitDev* shared = nullptr) {
  Carver c{base};
  derive_tiles(h, f);
  if (shared) {
    f->xraw = shared->xraw; f->xe = shared->xe; f->Ec = shared->Ec; f->Qt = shared->Qt;
    f->F32 = shared->F32; f->F64 = shared->F64; f->ghat = shared->ghat; f->tag = shared->tag;
    f->rad = shared->rad; f->pst = shared->pst;
    f->n_e = shared->n_e; f->n_t = shared->n_t; f->n_r = shared->n_r; f->n_p = shared->n_p;
    f->jrow = shared->jrow; f->jent = shared->jent; f->jval = shared->jval; f->jsig = shared->jsig;
    f->qpum = shared->qpum; f->qhw = shared->qhw; f->qrow32 = shared->qrow32; f->qrow64 = shared->qrow64;
    f->fixp = shared->fixp;
  } else {
    f->xraw = c.take<double>(h.N + 1);
    f->xe = c.take<double>(h.N + 1);
    f->Ec = c.take<double>(h.T);
    f->Qt = c.take<double>(h.T);
    f->F32 = c.take<float>((size_t)h.T * kSP);
    f->F64 = c.take<double>((size_t)h.T * kSP);
    f->ghat = c.take<double>(h.K);
    f->tag = c.take<double>(kSP);
    f->rad = c.take<double>((size_t)kSP * h.n_rad);
    f->pst = c.take<double>((size_t)kSP * h.n_ps);
    f->n_e = c.take<double>(h.N);
    f->n_t = c.take<double>(h.N);
    f->n_r = c.take<double>(h.n_rad);
    f->n_p = c.take<double>((size_t)h.N * h.n_ps);
    const size_t nj = h.joint ? (size_t)h.N * h.n_rad * h.n_ps : 0;  // any data fits
    f->jrow = c.take<int>(h.joint ? h.N + 1 : 0);
    f->jent = c.take<uint32_t>(nj);
    f->jval = c.take<double>(nj);
    f->jsig = c.take<double>(h.joint ? kSP : 0);
    f->qpum = c.take<double>(h.N);
    f->qhw = c.take<double>(h.N);
    f->qrow32 = c.take<float>((size_t)h.N * 3 * kNQ32);
    f->qrow64 = c.take<double>((size_t)h.N * 3 * kNQ64);
    f->fixp = c.take<double>(f->n_rt);
  }
  if (h.kind == kTable) {
    if (shared) {
      f->grid = shared->grid;
      f->Mg = shared->Mg;
    } else {
      f->grid = c.take<double>(h.n_grid);
      f->Mg = c.take<double>((size_t)h.n_grid * h.N * kSP);
    }
  }
  *theta = c.take<double>(h.P + 1);  // + the caller's sequence number (host path)
  f->theta = *theta;
  f->cp = c.take<ColPar>(h.kind == kTable ? 0 : h.T);
  f->tb = c.take<int2>(f->n_ct);
  f->Mpart = c.take<double>((size_t)f->n_cg * h.N * (f->vsum ? 1 : kSP));
  f->Mfix = c.take<double>((size_t)kFixSplit * h.N * (f->vsum ? 1 : kSP));
  f->bwdfix = c.take<double>((size_t)f->n_ct * kBwdPart);
  f->fpart = c.take<double>((size_t)kFinBlocks * kFinRow);
  f->fcount = c.take<int>(1);
  f->fixq = c.take<double>((size_t)4 * f->n_ct);
  f->fixflag = c.take<int>((size_t)f->n_rt + f->n_ct);
  f->M = c.take<double>((size_t)h.N * kSP);
  f->Mp = c.take<double>((size_t)h.N * kSP);
  f->H = c.take<double>((size_t)h.N * kSP);
  f->Ht = c.take<double>((size_t)h.N * kSP);
  f->nllpart = c.take<double>(f->n_rowblk);
  f->flagpart = c.take<int>(f->n_rowblk);
  f->gpart = c.take<double>((size_t)f->n_rowblk * kSP);
  f->rad_out = c.take<double>(4 + 2 * kSP);
  f->Dp = c.take<double>((size_t)h.N * kSP);
  f->ppart = c.take<double>(f->n_rowblk);
  if (h.joint) {
    f->jnll = c.take<double>(h.N);
    f->jflag = c.take<int>(h.N);
    f->jg = c.take<double>((size_t)h.N * kSP);
    f->jpp = c.take<double>(h.N);
    f->jtp = c.take<double>(h.N);
  }
  if (h.kind == kTable) {
    f->Dt = c.take<double>((size_t)h.N * kSP);
    f->Dtp = c.take<double>((size_t)h.N * kSP);
    f->tpart = c.take<double>(f->n_rowblk);
  }
  f->cpflag = c.take<int>(f->n_cpblk);
  f->bwdpart = c.take<double>((size_t)f->n_bwdblk * kBwdPart);
  *out = c.take<double>(2 + h.P);
  f->out = *out;
  f->theta_src = nullptr;
  f->out_host = nullptr;
  return (c.off + 255) & ~(size_t)255;
}

HostModel shape_only(const HostModel& h) {
  HostModel s;
  s.T = h.T; s.N = h.N; s.S = h.S; s.P = h.P; s.nresp = h.nresp; s.kind = h.kind; s.prec = h.prec; s.mv = h.mv;
  s.win_lo = h.win_lo; s.win_hi = h.win_hi; s.K = h.K; s.n_rad = h.n_rad; s.rad_lo = h.rad_lo;
  s.rad_hi = h.rad_hi; s.n_ps = h.n_ps;
  s.p = h.p; s.pu_frac = h.pu_frac; s.pu_float = h.pu_float; s.exposure = h.exposure;
  s.n_grid = h.n_grid;
  s.joint = h.joint;
  s.gg = h.gg;
  s.tiles = h.tiles;
  return s;
}

size_t device_fit_bytes(const HostModel& h, bool shared_inputs) {
  FitDev f{}, sh{};
  double *t, *o;
  return carve(h, nullptr, &f, &t, &o, shared_inputs ? &sh : nullptr);
}

LaunchShape shape_of(const FitDev& f) {
  LaunchShape L;
  L.max_T = f.T;
  L.max_fwd_blocks = f.n_rt * f.n_fb;
  L.CG = f.CG;
  L.max_NS = f.N * kSP;
  L.max_rowblk = f.n_rowblk;
  L.max_bwd_blocks = (f.n_ct + 7) / 8 * 8 * f.n_rg;  // true tiles interleaved over the 8 XCDs
  L.max_rt = f.n_rt;
  L.max_ct = f.n_ct;
  L.kind = f.kind;
  L.prec = f.prec;
  L.any_mv = f.mv;
  L.any_rad = f.mv && f.n_rad > 0 && !f.joint;
  L.any_joint = f.mv && f.joint;
  return L;
}

template <class T>
static hipError_t up(const T* dst, const std::vector<T>& v, hipStream_t st) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync((void*)dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

bx_status upload_data(const HostModel& h, const DeviceFit& df, hipStream_t st) {
  BX_HIP(up(df.dev.n_e, h.n_e, st), "upload data");
  BX_HIP(up(df.dev.n_t, h.n_t, st), "upload data");
  BX_HIP(up(df.dev.n_r, h.n_r, st), "upload data");
  BX_HIP(up(df.dev.n_p, h.n_p, st), "upload data");
  if (h.joint) {
    BX_HIP(up(df.dev.jrow, h.jrow, st), "upload data");
    BX_HIP(up(df.dev.jent, h.jent, st), "upload data");
    BX_HIP(up(df.dev.jval, h.jval, st), "upload data");
  }
  return BX_OK;
}

bx_status place_fit(const HostModel& h, void* base, DeviceFit* df, hipStream_t st, const FitDev* shared) {
  FitDev& f = df->dev;
  memset(&f, 0, sizeof f);
  df->base = base;
  df->bytes = carve(h, (char*)base, &f, &df->d_theta, &df->d_out, shared);
  f.T = h.T; f.N = h.N; f.S = h.S; f.P = h.P; f.nresp = h.nresp; f.kind = h.kind; f.prec = h.prec; f.mv = h.mv;
  f.win_lo = h.win_lo; f.win_hi = h.win_hi; f.K = h.K; f.n_rad = h.n_rad; f.rad_lo = h.rad_lo;
  f.rad_hi = h.rad_hi; f.n_ps = h.n_ps;
  f.pu_frac = h.pu_frac;
  f.pu_float = h.pu_float;
  f.n_grid = h.n_grid;
  f.joint = h.joint;
  f.gg = h.gg;
  if (shared) {  // inputs (and what is derived from them) already in place
    f.uniform = shared->uniform;
    f.row0 = shared->row0;
    f.x0 = shared->x0;
    f.inv_w = shared->inv_w;
    return BX_OK;
  }
  // equal reco bins allow a direct edge index in the support search
  const double w0 = h.xraw[1] - h.xraw[0];
  bool uni = true;
  for (int j = 1; j < h.N && uni; ++j) uni = std::fabs((h.xraw[j + 1] - h.xraw[j]) - w0) <= 1e-12 * std::fabs(w0);
  f.uniform = uni ? 1 : 0;
  f.row0 = -1;
  for (int j = 0; j < h.N && h.kind == kGG && f.row0 < 0; ++j)
    if (h.xraw[j] <= 0.0 && h.xraw[j + 1] > 0.0) f.row0 = j;
  f.x0 = h.xraw[0];
  f.inv_w = 1.0 / w0;
  BX_HIP(up(f.xraw, h.xraw, st), "upload");
  BX_HIP(up(f.xe, h.xe, st), "upload");
  BX_HIP(up(f.Ec, h.Ec, st), "upload");
  BX_HIP(up(f.Qt, h.Qt, st), "upload");
  BX_HIP(up(f.F32, h.F32, st), "upload");
  BX_HIP(up(f.F64, h.F64, st), "upload");
  BX_HIP(up(f.ghat, h.ghat, st), "upload");
  BX_HIP(up(f.tag, h.tag, st), "upload");
  BX_HIP(up(f.rad, h.rad, st), "upload");
  BX_HIP(up(f.pst, h.pst, st), "upload");
  if (h.joint) BX_HIP(up(f.jsig, h.jsig, st), "upload");
  BX_HIP(up(f.qpum, h.qpum, st), "upload");
  BX_HIP(up(f.qhw, h.qhw, st), "upload");
  BX_HIP(up(f.fixp, h.fixp, st), "upload");
  BX_HIP(up(f.qrow32, h.qrow32, st), "upload");
  BX_HIP(up(f.qrow64, h.qrow64, st), "upload");
  if (h.kind == kTable) BX_HIP(up(f.grid, h.grid, st), "upload");
  return upload_data(h, *df, st);
}

}  // namespace bx

using namespace bx;

// ---------------------------------------------------------------------------
// Plain-path evaluation.
// ---------------------------------------------------------------------------
static bx_status capture(bx_model* m, const FitDev* d_fit, bool grad, hipGraphExec_t* exec) {
  hipGraph_t g;
  BX_HIP(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal), "graph capture");
  launch_eval(d_fit, nullptr, 1, shape_of(m->df.dev), grad, m->cap_stream);  // fit = blockIdx.y = 0
  BX_HIP(hipStreamEndCapture(m->cap_stream, &g), "graph capture");
  hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  return BX_OK;
}

// host: theta is read from, and the results written to, the pinned buffer
// h_pin by the kernels themselves (no copy nodes); otherwise device buffers.
static bx_status enqueue_eval(bx_model* m, bool grad, bool host, hipStream_t st) {
  hipGraphExec_t* ex = !host ? &m->g_grad_dev : grad ? &m->g_grad : &m->g_eval;
  if (!*ex) {
    bx_status s = capture(m, host ? m->d_fit_h : m->d_fit, grad, ex);
    if (s != BX_OK) return s;
  }
  BX_HIP(hipGraphLaunch(*ex, st), "graph launch");
  return BX_OK;
}

// Work on stream st that uses the model's workspace is ordered after the
// work the previous call enqueued on another stream (an autograd evaluation on
// torch's stream followed by a host-path evaluation on the model's, say):
// record an event there and make st wait for it.
static bx_status order_on(bx_model* m, hipStream_t st) {
  if (m->last_stream && m->last_stream != st) {
    BX_HIP(hipEventRecord(m->ws_event, m->last_stream), "stream ordering");
    BX_HIP(hipStreamWaitEvent(st, m->ws_event, 0), "stream ordering");
  }
  m->last_stream = st;
  return BX_OK;
}

namespace bx {
// The polishing model of a mixed-precision fit: FP64, and the same shapes.
bx_status polish_compatible(const bx_model* m, const bx_model* p) {
  const HostModel &a = m->h, &b = p->h;
  if (b.prec != kF64) return inval("the polishing model must be FP64");
  if (a.T != b.T || a.N != b.N || a.S != b.S || a.P != b.P || a.kind != b.kind || a.mv != b.mv ||
      a.win_lo != b.win_lo || a.win_hi != b.win_hi || a.pu_float != b.pu_float)
    return inval("the polishing model's shapes differ from the fit's");
  return BX_OK;
}

// Evaluate at host theta; fills nll (and grad).  Shared with the plain fitter.
bx_status model_eval(bx_model* m, const double* theta, double* nll, double* grad) {
  const int P = m->h.P;
  for (int q = 0; q < P; ++q)
    if (!std::isfinite(theta[q])) {
      *nll = INFINITY;
      set_error("non-finite parameter");
      return BX_E_DOMAIN;
    }
  // h_pin = [theta[P] | sequence number] (host-written) ... at kPinOut:
  // [out[2 + P] | completion mark] (device-written)
  double* hp = m->h_pin;
  memcpy(hp, theta, P * sizeof(double));
  const double seq = (double)(++m->seq);
  hp[P] = seq;
  flush_lines(hp, P + 1);  // theta in memory before the launch
  bx_status s = order_on(m, m->stream);
  if (s != BX_OK) return s;
  s = enqueue_eval(m, grad != nullptr, true, m->stream);
  if (s != BX_OK) return s;
  // The last kernel writes the sequence number after the results (with a
  // system-scope fence): spin on it, and ask the stream now and then so that
  // a failed launch ends the wait with its error.  Device writes to this
  // buffer do not reliably invalidate a copy of the line the CPU already
  // holds (one fetched by its prefetcher while the results were in flight),
  // so the mark and then the results are read from memory, past the cache.
  const volatile double* mark = hp + kPinOut + 2 + P;
  auto mark_now = [&]() {
    flush_lines(hp + kPinOut + 2 + P, 1);
    return *mark;
  };
  for (unsigned it = 1;; ++it) {
    if (mark_now() == seq) break;
    if ((it & 1023u) == 0u) {
      const hipError_t q = hipStreamQuery(m->stream);
      if (q == hipSuccess && mark_now() == seq) break;
      if (q == hipSuccess) {
        set_error("evaluation finished without its completion mark");
        return BX_E_DEVICE;
      }
      if (q != hipErrorNotReady) return hip_fail(q, "evaluation");
    }
    __builtin_ia32_pause();
  }
  flush_lines(hp + kPinOut, 2 + P);
  std::atomic_thread_fence(std::memory_order_acquire);
  const double* o = hp + kPinOut;
  const int fl = (int)o[1 + P];
  const int hard = fl & (kBadSigma | kBadGG | kBadMu | kBadTheta);
  if (hard || (grad && (fl & kZeroWidth))) {
    *nll = hard ? INFINITY : o[0];
    set_error(hard & kBadMu ? "expected count < 0, or 0 where counts > 0"
              : hard ? "response parameters outside their domain"
                     : "zero-width response: gradient undefined");
    return BX_E_DOMAIN;
  }
  *nll = o[0];
  if (grad) memcpy(grad, o + 1, P * sizeof(double));
  return BX_OK;
}
}  // namespace bx

extern "C" {

const char* bx_last_error(void) { return bx::g_err.c_str(); }

bx_status bx_model_build(const bx_model_desc* desc, const bx_data* data, void* hip_stream, bx_model** out) {
  if (!out) return inval("out is NULL");
  *out = nullptr;
  bx_model* m = new (std::nothrow) bx_model();
  if (!m) return BX_E_NOMEM;
  bx_status s = make_host_model(desc, data, &m->h);  // validation needs no device
  if (s != BX_OK) {
    delete m;
    return s;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete m;
    set_error("no HIP device");
    return BX_E_DEVICE;
  }
  auto fail = [&](bx_status st) {
    bx_model_free(m);
    return st;
  };
  if (hipGetDevice(&m->device) != hipSuccess) return fail(hip_fail(hipErrorNoDevice, "hipGetDevice"));
  if (hip_stream) {
    m->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) return fail(BX_E_DEVICE);
    m->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking) != hipSuccess) return fail(BX_E_DEVICE);
  if (hipEventCreateWithFlags(&m->ws_event, hipEventDisableTiming) != hipSuccess) return fail(BX_E_DEVICE);
  const size_t bytes = device_fit_bytes(m->h);
  void* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    set_error("hipMalloc of the model workspace failed");
    return fail(BX_E_NOMEM);
  }
  s = place_fit(m->h, base, &m->df, m->stream);
  if (s != BX_OK) return fail(s);
  if (m->h.kind == kTable) {  // M_g = R_g F^T once; the matrices themselves are not kept
    const size_t nb = m->h.rtab.size() * sizeof(double);
    double* d_R = nullptr;
    if (hipMalloc(&d_R, nb) != hipSuccess) {
      set_error("hipMalloc of the response tables failed");
      return fail(BX_E_NOMEM);
    }
    const FitDev& fd = m->df.dev;
    hipError_t e = hipMemcpyAsync(d_R, m->h.rtab.data(), nb, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) {
      launch_table_gemm(d_R, fd.F64, const_cast<double*>(fd.Mg), m->h.n_grid, m->h.N, m->h.T, m->stream);
      e = hipStreamSynchronize(m->stream);
    }
    (void)hipFree(d_R);
    if (e != hipSuccess) return fail(hip_fail(e, "response tables"));
    std::vector<double>().swap(m->h.rtab);
  }
  if (hipMalloc(&m->d_fit, 2 * sizeof(FitDev)) != hipSuccess || hipMalloc(&m->d_active, sizeof(int)) != hipSuccess)
    return fail(BX_E_NOMEM);
  m->d_fit_h = m->d_fit + 1;
  // coherent pinned memory: the kernels read theta from it and write the
  // results into it, visible to the host once the stream has synchronised
  if (hipHostMalloc((void**)&m->h_pin, kPinDoubles * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(BX_E_NOMEM);
  memset(m->h_pin, 0, kPinDoubles * sizeof(double));
  flush_lines(m->h_pin, kPinDoubles);  // no dirty host line left over device results
  void* d_pin = nullptr;
  if (hipHostGetDevicePointer(&d_pin, m->h_pin, 0) != hipSuccess)
    return fail(hip_fail(hipErrorUnknown, "hipHostGetDevicePointer"));
  FitDev fh = m->df.dev;
  fh.theta_src = (const double*)d_pin;
  fh.out_host = (double*)d_pin + kPinOut;
  const int zero = 0;
  if (hipMemcpyAsync(m->d_fit, &m->df.dev, sizeof(FitDev), hipMemcpyHostToDevice, m->stream) != hipSuccess ||
      hipMemcpyAsync(m->d_fit_h, &fh, sizeof(FitDev), hipMemcpyHostToDevice, m->stream) != hipSuccess ||
      hipMemcpyAsync(m->d_active, &zero, sizeof(int), hipMemcpyHostToDevice, m->stream) != hipSuccess)
    return fail(BX_E_DEVICE);
  if (hipStreamSynchronize(m->stream) != hipSuccess) return fail(hip_fail(hipErrorUnknown, "model upload"));
  m->lnfact = host_lnfact(m->h);
  *out = m;
  return BX_OK;
}

bx_status bx_model_set_data(bx_model* m, const bx_data* data) {
  if (!m) return inval("model is NULL");
  if (m->users.load() > 0) {
    set_error("model in use by a server fit");
    return BX_E_BUSY;
  }
  bx_status s = set_host_data(&m->h, data);
  if (s != BX_OK) return s;
  s = order_on(m, m->stream);
  if (s != BX_OK) return s;
  s = upload_data(m->h, m->df, m->stream);
  if (s != BX_OK) return s;
  BX_HIP(hipStreamSynchronize(m->stream), "data upload");
  m->lnfact = host_lnfact(m->h);
  return BX_OK;
}

bx_status bx_model_free(bx_model* m) {
  if (!m) return BX_OK;
  if (m->users.load() > 0) {
    set_error("model in use by a server fit");
    return BX_E_BUSY;
  }
  if (m->last_stream) (void)hipStreamSynchronize(m->last_stream);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  if (m->ws_event) (void)hipEventDestroy(m->ws_event);
  if (m->g_eval) (void)hipGraphExecDestroy(m->g_eval);
  if (m->g_grad) (void)hipGraphExecDestroy(m->g_grad);
  if (m->g_grad_dev) (void)hipGraphExecDestroy(m->g_grad_dev);
  if (m->df.base) (void)hipFree(m->df.base);
  if (m->d_fit) (void)hipFree(m->d_fit);
  if (m->d_active) (void)hipFree(m->d_active);
  if (m->h_pin) (void)hipHostFree(m->h_pin);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
  return BX_OK;
}

int32_t bx_model_nparams(const bx_model* m) { return m ? m->h.P : -1; }

bx_status bx_model_lnfact(const bx_model* m, double* out) {
  if (!m || !out) return inval("NULL argument");
  *out = m->lnfact;
  return BX_OK;
}

bx_status bx_nll_eval(bx_model* m, const double* theta, double* nll) {
  if (!m || !theta || !nll) return inval("NULL argument");
  return model_eval(m, theta, nll, nullptr);
}

bx_status bx_nll_grad(bx_model* m, const double* theta, double* nll, double* grad) {
  if (!m || !theta || !nll || !grad) return inval("NULL argument");
  return model_eval(m, theta, nll, grad);
}

bx_status bx_nll_grad_dev(bx_model* m, const double* d_theta, double* d_out, void* stream) {
  if (!m || !d_theta || !d_out) return inval("NULL argument");
  hipStream_t st = stream ? (hipStream_t)stream : m->stream;
  const int P = m->h.P;
  bx_status s = order_on(m, st);
  if (s != BX_OK) return s;
  BX_HIP(hipMemcpyAsync(m->df.d_theta, d_theta, P * sizeof(double), hipMemcpyDeviceToDevice, st), "theta copy");
  s = enqueue_eval(m, true, false, st);
  if (s != BX_OK) return s;
  BX_HIP(hipMemcpyAsync(d_out, m->df.d_out, (1 + P) * sizeof(double), hipMemcpyDeviceToDevice, st), "result copy");
  return BX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free evaluation.  The per-evaluation workspace of
// bx_nll_grad_dev_noalloc (column parameters, forward partials, M, M', the
// adjoint weights, the per-block partials, theta and the results, and the
// fit's descriptor) is carved from one file-scope device array instead of the
// model's own workspace; every kernel writes what it later reads, so nothing
// in it needs clearing between calls.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a stand-in, not a
// device address), only the address hipGetSymbolAddress returns for the
// current device, looked up once per device on the first call there.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)16 << 20;  // 16 MiB per device
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

bx_status scratch_of_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return BX_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return BX_OK;
}
}  // namespace

extern "C" {

bx_status bx_nll_grad_dev_noalloc(bx_model* m, const double* d_theta, double* d_out, void* stream) {
  if (!m || !d_theta || !d_out) return inval("NULL argument");
  int dev = -1;
  BX_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != m->device) return inval("bx_nll_grad_dev_noalloc: the model lives on another device than the current one");
  const size_t ws = (device_fit_bytes(m->h, true) + 255) & ~(size_t)255;  // inputs stay the model's
  const size_t need = ws + ((sizeof(FitDev) + 255) & ~(size_t)255);
  if (need > kScratchBytes) {
    set_error("bx_nll_grad_dev_noalloc: the model's workspace (" + std::to_string(need) +
              " bytes) exceeds the scratch array (" + std::to_string(kScratchBytes) + " bytes)");
    return BX_E_INVAL;
  }
  char* base = nullptr;
  bx_status s = scratch_of_device(dev, &base);
  if (s != BX_OK) return s;
  hipStream_t st = stream ? (hipStream_t)stream : m->stream;
  DeviceFit df;
  s = place_fit(m->h, base, &df, st, &m->df.dev);  // carves only: no allocation, no upload
  if (s != BX_OK) return s;
  FitDev* d_fd = (FitDev*)(base + ws);
  const int P = m->h.P;
  BX_HIP(hipMemcpyAsync(d_fd, &df.dev, sizeof(FitDev), hipMemcpyHostToDevice, st), "descriptor copy");
  BX_HIP(hipMemcpyAsync(df.d_theta, d_theta, P * sizeof(double), hipMemcpyDeviceToDevice, st), "theta copy");
  launch_eval(d_fd, nullptr, 1, shape_of(df.dev), true, st);
  BX_HIP(hipGetLastError(), "launch");
  BX_HIP(hipMemcpyAsync(d_out, df.d_out, (1 + P) * sizeof(double), hipMemcpyDeviceToDevice, st), "result copy");
  return BX_OK;
}

int64_t bx_model_expected_size(const bx_model* m) {
  if (!m) return -1;
  const HostModel& h = m->h;
  return h.mv ? 2 * (int64_t)h.N + h.n_rad + (int64_t)h.N * h.n_ps : h.N;
}

bx_status bx_model_expected(bx_model* m, const double* theta, double* out) {
  if (!m || !theta || !out) return inval("NULL argument");
  double nll;
  bx_status s = model_eval(m, theta, &nll, nullptr);
  if (s != BX_OK && s != BX_E_DOMAIN) return s;
  const int64_t n = bx_model_expected_size(m);
  double* d = nullptr;
  BX_HIP(hipMallocAsync((void**)&d, n * sizeof(double), m->stream), "hipMallocAsync");
  launch_expected(m->d_fit, d, m->h.N, m->h.mv ? m->h.n_rad : 0, m->h.mv ? m->h.n_ps : 0, m->stream);
  BX_HIP(hipMemcpyAsync(out, d, n * sizeof(double), hipMemcpyDeviceToHost, m->stream), "download");
  BX_HIP(hipFreeAsync(d, m->stream), "hipFreeAsync");
  BX_HIP(hipStreamSynchronize(m->stream), "expected");
  return s;
}

bx_status bx_model_stage_times(bx_model* m, const double* theta, int32_t reps, double* ms) {
  if (!m || !theta || !ms || reps < 1) return inval("bad argument");
  double nll;
  bx_status s = model_eval(m, theta, &nll, nullptr);  // uploads theta, warms up
  if (s != BX_OK) return s;
  // Each stage is timed on its own: `reps` back-to-back launches of its
  // kernel between two events (every stage only rewrites what it produces
  // from the previous stages' results, which the evaluation above left in
  // place).  ms[8] times `reps` whole evaluations the same way, ms[9] and
  // ms[10] the forward and backward main sweeps without their fix-up sweeps.
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return hip_fail(hipErrorUnknown, "hipEventCreate");
  const LaunchShape L = shape_of(m->df.dev);
  hipError_t e = hipSuccess;
  for (int k = 0; k < kStageTimes && e == hipSuccess; ++k) {
    e = hipEventRecord(e0, m->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      if (k == kStages) launch_eval(m->d_fit, nullptr, 1, L, true, m->stream);
      else launch_stage(m->d_fit, nullptr, 1, L, true, k < kStages ? k : k - 1, m->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, m->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    ms[k] = (double)t / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "stage timing");
  return BX_OK;
}

bx_status bx_model_cell_ceiling(bx_model* m, const double* theta, int32_t reps, double* cells_per_s) {
  if (!m || !theta || !cells_per_s || reps < 1) return inval("bad argument");
  if (m->h.kind == kTable) return inval("a tabulated response has no cell function");
  double nll;
  bx_status s = model_eval(m, theta, &nll, nullptr);  // column constants and supports at theta
  if (s != BX_OK) return s;
  const int blocks = 256 * 8;  // 8 workgroups of 4 waves per CU
  double* d_sink = nullptr;
  BX_HIP(hipMalloc(&d_sink, sizeof(double)), "hipMalloc");
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    launch_cell_ceiling(m->d_fit, m->h.kind, m->h.prec, blocks, 4, d_sink, m->stream);  // warm-up
    e = hipEventRecord(e0, m->stream);
  }
  if (e == hipSuccess) {
    launch_cell_ceiling(m->d_fit, m->h.kind, m->h.prec, blocks, reps, d_sink, m->stream);
    e = hipEventRecord(e1, m->stream);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_sink);
  if (e != hipSuccess) return hip_fail(e, "cell ceiling");
  *cells_per_s = (double)blocks * 256.0 * 4.0 * reps / (t * 1e-3);  // four cells per lane per repetition
  return BX_OK;
}

bx_status bx_model_batch_times(bx_model* m, const double* theta, int32_t copies, int32_t reps, double* ms) {
  if (!m || !theta || !ms || copies < 1 || reps < 1) return inval("bad argument");
  const int P = m->h.P;
  for (int q = 0; q < P; ++q)
    if (!std::isfinite(theta[q])) {
      set_error("non-finite parameter");
      return BX_E_DOMAIN;
    }
  // `copies` independent fits of this model, placed as the server places
  // them (with the batched tile widths), evaluated together by one launch per
  // stage (blockIdx.y = fit)
  HostModel hb = shape_only(m->h);  // inputs: the model's own placement
  hb.tiles = choose_tiles(hb.T, hb.N, hb.kind, hb.prec, 1);
  const size_t stride = (device_fit_bytes(hb, true) + 255) & ~(size_t)255;
  char* base = nullptr;
  FitDev* d_fd = nullptr;
  if (hipMalloc((void**)&base, stride * copies) != hipSuccess) {
    set_error("hipMalloc of the batch failed");
    return BX_E_NOMEM;
  }
  if (hipMalloc((void**)&d_fd, sizeof(FitDev) * copies) != hipSuccess) {
    (void)hipFree(base);
    set_error("hipMalloc of the batch failed");
    return BX_E_NOMEM;
  }
  std::vector<FitDev> fd(copies);
  bx_status s = BX_OK;
  hipError_t e = hipSuccess;
  for (int c = 0; c < copies && s == BX_OK; ++c) {
    DeviceFit df;
    s = place_fit(hb, base + stride * c, &df, m->stream, &m->df.dev);
    if (s == BX_OK) e = hipMemcpyAsync(df.d_theta, theta, P * sizeof(double), hipMemcpyHostToDevice, m->stream);
    if (e != hipSuccess) s = hip_fail(e, "theta upload");
    fd[c] = df.dev;
  }
  if (s == BX_OK) {
    e = hipMemcpyAsync(d_fd, fd.data(), sizeof(FitDev) * copies, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) s = hip_fail(e, "batch upload");
  }
  if (s == BX_OK) {
    const LaunchShape L = shape_of(fd[0]);
    launch_eval(d_fd, nullptr, copies, L, true, m->stream);  // every stage's inputs in place
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int k = 0; k < kStageTimes && e == hipSuccess; ++k) {
      e = hipEventRecord(e0, m->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        if (k == kStages) launch_eval(d_fd, nullptr, copies, L, true, m->stream);
        else launch_stage(d_fd, nullptr, copies, L, true, k < kStages ? k : k - 1, m->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, m->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      ms[k] = (double)t / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) s = hip_fail(e, "batch timing");
  }
  (void)hipStreamSynchronize(m->stream);
  (void)hipFree(d_fd);
  (void)hipFree(base);
  return s;
}

bx_status bx_fit(bx_model* m, const bx_fit_opts* o, bx_fit_result* r) {
  if (!m || !o || !r || !o->x0) return inval("NULL argument");
  const int P = m->h.P;
  if (P > 32) return inval("too many parameters");
  FitProblem pb;
  bx_status s = fit_problem(P, m->h.S, o, &pb, m->h.pu_float ? P - 1 : -1);
  if (s != BX_OK) return s;
  if (o->polish && (s = polish_compatible(m, o->polish)) != BX_OK) return s;
  pb.f_noise = nll_noise(m->h);
  memset(r, 0, sizeof *r);
  const auto t0 = std::chrono::steady_clock::now().time_since_epoch();
  r->t_submit_ns = r->t_admit_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(t0).count();
  Bfgs opt(pb);
  double x[32], f = 0.0, g[32];
  // the fit's own model, then (mixed precision) the FP64 model from where it stopped
  for (bx_model* em = m; em;) {
    while (opt.next(x)) {
      const bx_status e = model_eval(em, x, &f, g);
      if (e != BX_OK && e != BX_E_DOMAIN) return e;
      opt.feed(e == BX_OK ? f : INFINITY, g);
    }
    em = (em == m && o->polish && opt.polish(pb.final_tol, nll_noise(o->polish->h))) ? o->polish : nullptr;
  }
  opt.result(r);
  const auto t1 = std::chrono::steady_clock::now().time_since_epoch();
  r->t_done_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(t1).count();
  return BX_OK;
}

}  // extern "C"

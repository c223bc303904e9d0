// HIP kernels of one likelihood evaluation (gfx950, wave64).
//
//   k_colparams   per true bin: response column parameters, support, chain
//                 factors to the response parameters (Eq. 1's R_x(N_x, E; p)),
//                 and each wave step's column factor of the one-interval test.
//   k_cells_fwd   per (reco tile, listed true tiles): each lane integrates the
//                 response density of one column over its reco bin (Eq. 1's
//                 cell, Gauss-Legendre in the column's variable) and the cells
//                 are contracted with the spectra in FP64 -- one FMA per cell
//                 for a single histogram, FP64 MFMA 16x16x4 with several species
//                 histograms (M = R F^T).  Tiles are added in a fixed tree;
//                 cells never touch HBM.  Wave steps whose bins are wide
//                 against their columns, or start at x <= 0, are left to
//   k_cells_fwd_fix  (composite quadrature, or a CDF difference).
//   k_reduce_M    FP64 sum of the forward partials (several species histograms;
//                 a single histogram's column is summed by k_rowterms).
//   k_rowterms    pile-up M' = (1-p) M + p g^*M (Eq. 2) from LDS, expected
//                 counts of every likelihood term per reco row (Eqs. 3-4),
//                 Poisson NLL terms, the adjoint weights H, per-block partials.
//   k_radial      radial term (Eq. 4) -- one block per fit.
//   k_joint       joint energy x radius x pulse-shape term per reco row, over
//                 the histogram's non-zero bins (closed-form sum of the
//                 expected counts for the rest).
//   k_adjoint     H~ = P^T H (the pile-up adjoint), from LDS; k_adjoint1 the
//                 single-histogram w~ once per fit for batched launches.
//   k_cells_bwd   per (true tile, RG reco tiles per wave): the cells again,
//                 with their derivatives in the two column parameters;
//                 alpha_i = sum_j W_ji dR_ji/dc1, beta_i = ... dc2 in FP64,
//                 contracted with the chain factors into a per-block partial
//                 (W_ji = w~_j v_i, or an FP64 MFMA product with several
//                 species histograms).  The steps left go to
//   k_cells_bwd_fix  (one fit: k_cells_bwd_fix_final, with the final sums).
//   k_final       fixed-order totals: NLL, rate gradient, response gradient;
//                 also written to the caller's pinned host buffer when set.
//   k_table_gemm  tabulated response, at build: M_g = R_g F^T (FP64 MFMA);
//   k_table       per evaluation: M and dM/dlam interpolated between grid
//                 points (replaces the column and cell kernels).
//   k_fit_start, k_fit_step  the device-minimised batch's quasi-Newton steps
//                 (one wave per fit); k_mark, k_mark_from a server step's
//                 completion mark;
//                 k_cell_ceiling the cell arithmetic alone, for the measured
//                 ceiling.
//
// Every sum has a fixed order, so a fit's result does not depend on what else
// runs in its launch, nor on the form of the launch.  The one device-scope
// counter (the final sums of a single fit) only elects the workgroup that adds
// the rows, in their fixed order; an election in every block of a sweep would
// cost an L2 write-back per block on gfx950 (agent-scope release).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bx_dev.h"
#include "bx_fitcore.hpp"

namespace bx {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float dpp_from_next(float x) {
  // lane l receives lane l+1 of its 16-lane row (row_shl:1); lane 15 keeps x
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x101, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_from_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x101, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x101, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2);
}

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <class R> struct Acc4;
template <> struct Acc4<float> { typedef v4f T; };
template <> struct Acc4<double> { typedef v4d T; };
template <class R> struct Pair;
template <> struct Pair<float> { typedef float2 T; };
template <> struct Pair<double> { typedef double2 T; };

// Workgroups go to the 8 XCDs round-robin (block b to XCD b % 8), each with
// its own L2.  The backward sweep gives true tile ct to XCD ct % 8 with all
// of its blocks: the tile's column parameters are fetched into one L2, and
// neighbouring tiles (similar work) are spread over all eight.
// (block, fit) of this workgroup.  A batch (gridDim.y = fits, a multiple of
// 8) is remapped so that every block of a fit runs on one XCD: the hardware
// deals workgroups to the 8 XCDs round-robin by linear id, and each XCD has
// its own L2, so a fit's column constants, row tables and partials are then
// fetched into one L2 instead of eight.  A single fit keeps the grid as is
// (spread over every XCD).
__device__ __forceinline__ int2 fit_block() {
  const int X = gridDim.x, n = gridDim.y;
  if (n < 8 || (n & 7)) return make_int2(blockIdx.x, blockIdx.y);
  const int L = blockIdx.x + blockIdx.y * X;  // linear workgroup id
  const int s = L >> 3;                       // slot on XCD L % 8
  return make_int2(s % X, 8 * (s / X) + (L & 7));
}

__device__ __forceinline__ int2 bwd_block(int b, int n_rg) {
  const int q = b >> 3;
  return make_int2((b & 7) + 8 * (q / n_rg), q % n_rg);  // (ct, rg)
}

__device__ __forceinline__ double sum16(double x) {  // fixed-order sum over a 16-lane row
  x += __shfl_xor(x, 8, 16);
  x += __shfl_xor(x, 4, 16);
  x += __shfl_xor(x, 2, 16);
  x += __shfl_xor(x, 1, 16);
  return x;
}

// Conservative cell range [jlo, jhi] holding every cell that can exceed
// exp(-B) of the column's mass, from the x-interval [xlo, xhi].
__device__ int2 cell_range(const FitDev& f, double xlo, double xhi) {
  const int N = f.N;
  if (f.uniform) {  // equal bins: direct index, widened by one bin each side
    const double a = fmin(fmax((xlo - f.x0) * f.inv_w, -2.0), (double)N + 2.0);
    const double b = fmin(fmax((xhi - f.x0) * f.inv_w, -2.0), (double)N + 2.0);
    if (!(a == a) || !(b == b)) return make_int2(0, N - 1);
    return make_int2(max((int)floor(a) - 1, 0), min((int)ceil(b) + 1, N - 1));
  }
  const double* x = f.xraw;
  int lo = 0, hi = N;  // first j with x[j+1] > xlo
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid + 1] > xlo) hi = mid; else lo = mid + 1;
  }
  const int jlo = lo;
  lo = 0; hi = N;      // number of edges x[j] < xhi among 0..N-1
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] < xhi) lo = mid + 1; else hi = mid;
  }
  return make_int2(max(jlo - 1, 0), min(lo, N - 1));
}

// ---------------------------------------------------------------------------
// Column parameters of the count estimator: negative binomial with mean
// m = L Q E and shape r = m^2 / (s^2 - m) (c1 = m, c2 = r).  Its support, the
// counts with ln P(n) >= ln P(mode) - B, is bracketed on the continuous
// extension of ln P (unimodal in n).  Each column takes 8 lanes: 4 search
// the lower end and 4 the upper end at once, each round testing 4 interior
// points of the bracket and keeping the sub-interval where the test changes,
// so the bracket shrinks 5-fold per round (a single thread's bisection needs
// ~10 sequential rounds of two lgamma per end).  A block covers the same 64
// columns as a k_colparams block, so the flag partials and tile supports are
// laid out alike.
constexpr int kCpLanes = 8;                      // lanes per column (half per end)
constexpr int kCpCountBlock = kCpLanes * kCpBlock;
__global__ void __launch_bounds__(kCpCountBlock) k_colparams_count(const FitDev* fits, const int* active) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if ((int)blockIdx.x >= f.n_cpblk) return;  // block-uniform
  constexpr int NE = kCpLanes / 2;  // test points per end and round
  const int t = threadIdx.x, lane = t & 63, u = lane & (kCpLanes - 1);
  const int col = t / kCpLanes;  // 0..63 within the block
  const int i = blockIdx.x * kCpBlock + col;
  __shared__ double sth[kMaxP + 1];
  __shared__ int slo[kCpBlock], shi[kCpBlock], sbad[kCpBlock];
  if (blockIdx.x == 0 && t == 0) *f.fcount = 0;  // this evaluation's final sums start their count
  // theta as in k_colparams (pinned host source, device copy by block 0)
  const double* th = f.theta;
  if (f.theta_src) {
    if (t <= f.P) {
      const double v = __hip_atomic_load(f.theta_src + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      sth[t] = v;
      if (blockIdx.x == 0) const_cast<double*>(f.theta)[t] = v;
    }
    __syncthreads();
    th = sth;
  }
  const bool valid = i < f.T;
  const int ic = valid ? i : f.T - 1;
  int bad = 0;
  bool okth = true;
  for (int q = 0; q < f.P; ++q) okth = okth && isfinite(th[q]);
  if (f.pu_float && !(th[f.P - 1] >= 0.0 && th[f.P - 1] <= 1.0)) okth = false;
  if (!okth) bad |= kBadTheta;
  const double E = f.Ec[ic];
  const double L = th[f.S], v0 = th[f.S + 1], v1 = th[f.S + 2], v2 = th[f.S + 3];
  const double m = L * f.Qt[ic] * E;
  const double s2 = v0 + v1 * m + v2 * m * m;
  const bool dom = (m > 0.0) && (s2 > m) && isfinite(s2);
  if (!dom) bad |= kBadGG;
  const double d = s2 - m, r = dom ? m * m / d : 1.0;
  const double lq = dom ? log(r / (r + m)) : 0.0, lp = dom ? log(m / (r + m)) : 0.0;
  const double lgr = lgamma(r);
  auto lnP = [&](double n) { return lgamma(n + r) - lgr - lgamma(n + 1.0) + r * lq + n * lp; };
  const double B = 1.05 * kSupportB;
  const double mode = r > 1.0 ? floor((r - 1.0) * m / r) : 0.0;
  const double top = lnP(mode) - B;
  // first half of the column's lanes: lower end, lnP(a) < top <= lnP(b);
  // second half: upper end, lnP(a) >= top > lnP(b); the test is "lnP(x) on
  // a's side" for either
  const bool upper = u >= NE;
  const int k8 = u & (NE - 1);
  double a, bb;
  bool search;
  if (upper) {
    a = mode;
    bb = mode + 10.0 * sqrt(fmax(s2, 0.0)) + 10.0;
    for (int it = 0; it < 40 && dom && lnP(bb) >= top; ++it) bb = mode + 2.0 * (bb - mode);
    search = dom;
  } else {
    a = 0.0;
    bb = mode;
    search = dom && lnP(0.0) < top;
  }
  for (int it = 0; it < 30; ++it) {
    const bool go = search && bb - a > 0.5;
    if (!__any(go)) break;
    const double w9 = (bb - a) / (double)(NE + 1);
    const double x = a + w9 * (double)(k8 + 1);
    const double lx = go ? lnP(x) : 0.0;
    const bool pred = upper ? (lx >= top) : (lx < top);
    const unsigned long long bal = __ballot(go && pred);
    const unsigned m8 = (unsigned)(bal >> (lane & ~(NE - 1))) & ((1u << NE) - 1u);  // this end's tests
    if (go) {
      const int tf = __builtin_ctz(~m8 | (1u << NE));  // first point not on a's side (NE: none)
      const double na = tf > 0 ? a + w9 * (double)tf : a;
      const double nb = tf < NE ? a + w9 * (double)(tf + 1) : bb;
      a = na;
      bb = nb;
    }
  }
  // the lower end's a (0 without a search) and the upper end's b, to lane 0
  // of the column's lanes
  const double lo_end = search ? a : 0.0;
  const double lo = __shfl(lo_end, lane & ~(kCpLanes - 1), 64);
  const double hi = __shfl(bb, (lane & ~(kCpLanes - 1)) + NE, 64);
  int jlo = 1 << 30, jhi = -1;
  if (u == 0 && valid) {
    ColPar& c = f.cp[i];  // fields stored as formed
    double v = 0.0;
    {  // the spectra row (zero-padded to kSP species) loaded whole, then summed in species order
      const int S = f.S;
      double fr[kSP];
#pragma unroll
      for (int s = 0; s < kSP; ++s) fr[s] = f.F64[i * kSP + s];
#pragma unroll
      for (int s = 0; s < kSP; ++s)
        if (s < S) v += th[s] * fr[s];
    }
    c.v = v;
    for (int q = 0; q < kMaxResp; ++q) c.J[0][q] = c.J[1][q] = 0.0;
    for (int q = 0; q < 8; ++q) { c.f32[q] = 0.f; c.f64[q] = 0.0; }
    if (!dom) {
      c.c0 = 1.0; c.c1 = 1.0;
    } else {
      const double cst[8] = {m, r, lgr, lq, lp, digamma_pos(r), 1.0 / (r + m), 1.0 / m};
      for (int q = 0; q < 8; ++q) { c.f64[q] = cst[q]; c.f32[q] = (float)cst[q]; }
      c.c0 = m;
      c.c1 = r;
      for (int q = 0; q < 4; ++q) {
        const double dm = (q == 0) ? m / L : 0.0;
        const double ds2 = (q == 1 ? 1.0 : q == 2 ? m : q == 3 ? m * m : 0.0) + (v1 + 2.0 * v2 * m) * dm;
        c.J[0][q] = dm;
        c.J[1][q] = (2.0 * m * dm * d - m * m * (ds2 - dm)) / (d * d);
      }
      const int2 rr = cell_range(f, lo, hi + 1.0);
      jlo = rr.x; jhi = rr.y;
    }
    if (bad & (kBadSigma | kBadGG | kBadTheta)) { jlo = 1 << 30; jhi = -1; }
    c.jlo = jlo; c.jhi = jhi; c.bad = bad; c.pad = 0;
  }
  if (u == 0) {
    slo[col] = jlo;
    shi[col] = jhi;
    sbad[col] = valid ? bad : 0;
  }
  __syncthreads();
  // support of each 16-column tile, domain flags of the block
  if (t < kCpBlock / 16) {
    int tl = 1 << 30, th_ = -1;
    for (int q = 0; q < 16; ++q) {
      tl = min(tl, slo[16 * t + q]);
      th_ = max(th_, shi[16 * t + q]);
    }
    const int i0 = blockIdx.x * kCpBlock + 16 * t;
    if (i0 < f.T) f.tb[i0 >> 4] = make_int2(tl, th_);
  }
  if (t == 0) {
    int fl = 0;
    for (int q = 0; q < kCpBlock; ++q) fl |= sbad[q];
    f.cpflag[blockIdx.x] = fl;
  }
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kCpBlock) k_colparams(const FitDev* fits, const int* active) {
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if (fb2.x >= f.n_cpblk) return;  // block-uniform
  const int i = fb2.x * kCpBlock + threadIdx.x;
  int jlo = 1 << 30, jhi = -1, bad = 0;
  // output pointers and T read before the first store (a store through a
  // generic pointer could alias f and force reloads after it)
  ColPar* const cpo = f.cp;
  int2* const tbo = f.tb;
  int* const cpflag = f.cpflag;
  const int T = f.T;
  int* const fixflag = f.fixflag;
  int* const fcount = f.fcount;
  double* const fixq = f.fixq;
  const int n_ct = f.has_fix ? f.n_ct : 0;
  double qv = 0.0;
  const int nflag = f.has_fix ? f.n_rt + f.n_ct : 0, nthr = f.n_cpblk * kCpBlock;
  // this evaluation's fix-up flags start clear (the forward sweep sets them),
  // and so does its final sums' count
  for (int e = i; e < nflag; e += nthr) fixflag[e] = 0;
  if (i == 0) *fcount = 0;
  // theta straight from pinned host memory when the caller passed it there,
  // with system-scope loads (a plain load may hit a line of the previous
  // evaluation's theta still held in the GPU caches); block 0 leaves a device
  // copy for the later kernels, with the caller's sequence number after it
  // (the completion mark of k_final)
  __shared__ double sth[kMaxP + 1];
  // the column's inputs that do not depend on theta (the spectra row,
  // zero-padded to kSP species, its energy and light yield factor), in flight
  // while theta arrives
  const int ic = min(i, T - 1);
  double fr[kSP];
#pragma unroll
  for (int s = 0; s < kSP; ++s) fr[s] = f.F64[ic * kSP + s];
  const double E = f.Ec[ic];
  const double Qt = f.kind == kGG ? f.Qt[ic] : 0.0;
  const double* th = f.theta;
  if (f.theta_src) {
    if ((int)threadIdx.x <= f.P) {
      const double v = __hip_atomic_load(f.theta_src + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      sth[threadIdx.x] = v;
      if (fb2.x == 0) const_cast<double*>(f.theta)[threadIdx.x] = v;
    }
    __syncthreads();
    th = sth;
  }
  if (i < f.T) {
    ColPar c;
    double v = 0.0;
    {  // summed in species order
      const int S = f.S;
#pragma unroll
      for (int s = 0; s < kSP; ++s)
        if (s < S) v += th[s] * fr[s];
    }
    c.v = v;
    for (int q = 0; q < kMaxResp; ++q) c.J[0][q] = c.J[1][q] = 0.0;
    for (int q = 0; q < 8; ++q) { c.f32[q] = 0.f; c.f64[q] = 0.0; }
    bool okth = true;
    for (int q = 0; q < f.P; ++q) okth = okth && isfinite(th[q]);
    if (f.pu_float && !(th[f.P - 1] >= 0.0 && th[f.P - 1] <= 1.0)) okth = false;
    if (!okth) bad |= kBadTheta;
    if (f.kind == kGauss) {
      const double a = th[f.S], b = th[f.S + 1];
      const double var = a * E + b * E * E;
      if (!(var >= 0.0)) bad |= kBadSigma;
      const double sig = sqrt(fmax(var, 0.0));
      c.c0 = E;
      c.c1 = sig > 0.0 ? 1.0 / sig : 0.0;
      if (sig > 0.0) {
        c.J[1][0] = E / (2.0 * sig);
        c.J[1][1] = E * E / (2.0 * sig);
      } else {
        bad |= kZeroWidth;
      }
      const double zb = sqrt(2.0 * (f.sup_prec == kF32 ? kSupportB32 : kSupportB));
      const int2 r = cell_range(f, E - zb * sig, E + zb * sig);
      jlo = r.x; jhi = r.y;
    } else {
      const double L = th[f.S], v0 = th[f.S + 1], v1 = th[f.S + 2], v2 = th[f.S + 3];
      const double m = L * Qt * E;
      const double s2 = v0 + v1 * m + v2 * m * m;
      if (!(m > 0.0) || !(s2 > 0.0)) {
        bad |= kBadGG;
        c.c0 = 0.0; c.c1 = 1.0;
      } else {
        const double tau = log1p(s2 / (m * m));
        // FP32 cells need k to ~1e-8: one Newton step from the table start
        const double k = gg_solve_k(f.gg, tau, nullptr, f.prec == kF32 ? 1e-5 : 1e-9);
        if (!(k > 1e-300) || !(k < 1e12)) bad |= kBadGG;
        const GGShape sh = gg_shape(f.gg, k, true);
        const double p = f.gg.p;
        const double lna = log(m) - sh.D1;
        const double lnk = log(k);
        c.c0 = p * lna + lnk;
        c.c1 = k;
        const double cR = exp(-sh.lngs) / sqrt(kTwoPi * k);
        const double cst[8] = {k, 1.0 / k, sqrt(0.5 * k), cR, 0.5 / sqrt(kTwoPi * k), sh.dlngs, lnk - sh.psi, p};
        for (int q = 0; q < 8; ++q) { c.f64[q] = cst[q]; c.f32[q] = (float)cst[q]; }
        // chain factors d(k, ln a)/d(L, v0, v1, v2)
        const double im = 1.0 / m, im2 = im * im;
        const double itau = 1.0 / ((1.0 + s2 * im2) * sh.dG);  // dk = dtau' * itau
        const double dsdm = v1 + 2.0 * v2 * m;
        for (int q = 0; q < 4; ++q) {
          const double dm = (q == 0) ? m / L : 0.0;
          const double ds2 = (q == 1 ? 1.0 : q == 2 ? m : q == 3 ? m * m : 0.0) + dsdm * dm;
          const double dk = (ds2 * im2 - 2.0 * s2 * dm * im2 * im) * itau;
          c.J[0][q] = dk;
          c.J[1][q] = dm * im - sh.dD1 * dk;
        }
        // support: k (lambda - 1 - ln lambda) <= B, lambda = e^t, x = exp((ct + t)/p),
        // with B raised by 5 % (the bounds only need to be conservative).  The
        // roots come from the table of the nearest grid point below ln k,
        // which bounds them from outside; off the table, FP32 Newton from
        // outside each root stays outside it.
        float th_, tl;
        const double spos = (lnk - kSupLo) * ((kSupTab - 1) / (kSupHi - kSupLo));
        if (f.gg.has_tab && spos >= 0.0 && spos < kSupTab - 1) {
          const int si = (int)spos;
          th_ = f.gg.sup_hi[si];
          tl = f.gg.sup_lo[si];
        } else {
          const float cb = (float)(1.05 * (f.sup_prec == kF32 ? kSupportB32 : kSupportB) / k);
          th_ = cb > 2.f ? log1pf(cb) + log1pf(log1pf(cb)) : sqrtf(2.f * cb);
          for (int it = 0; it < 12; ++it) {
            const float e = expm1f(th_);
            const float d = (e - th_ - cb) * rcp(e);
            th_ -= d;
            if (fabsf(d) < 1e-4f * fmaxf(1.f, th_)) break;
          }
          tl = -(1.f + cb);
          for (int it = 0; it < 12; ++it) {
            const float e = expm1f(tl);
            const float d = (e - tl - cb) * rcp(e);
            tl -= d;
            if (fabsf(d) < 1e-4f * fmaxf(1.f, -tl)) break;
          }
        }
        const double xlo = exp((c.c0 + (double)tl) / p), xhi = exp((c.c0 + (double)th_) / p);
        const int2 r = cell_range(f, xlo, xhi);
        jlo = r.x; jhi = r.y;
      }
    }
    if (bad & (kBadSigma | kBadGG | kBadTheta)) { jlo = 1 << 30; jhi = -1; }
    c.jlo = jlo; c.jhi = jhi; c.bad = bad; c.pad = 0;
    // GG: the cell of the reco bin from x <= 0, F(x) at its upper edge (the
    // value in FP64, the derivatives in the cell precision, as the fix-up
    // sweeps form a CDF-difference cell), for a support that reaches it
    c.e1[0] = c.e1[1] = c.e1[2] = 0.0;
    if (f.kind == kGG && f.row0 >= 0 && jlo <= f.row0 && f.row0 <= jhi) {
      const double lnx1 = f.xe[f.row0 + 1];
      GGCol<double> g;
      g.ct = c.c0;
      g.k = c.f64[0]; g.ik = c.f64[1]; g.skh = c.f64[2]; g.cR = c.f64[3]; g.ce = c.f64[4];
      g.dlngs = c.f64[5]; g.lnk_psi = c.f64[6]; g.p = c.f64[7];
      c.e1[0] = cell_from(0.0, gg_edge<double, false>(lnx1, g).v);
      if (f.prec == kF32) {
        GGCol<float> h;
        h.ct = c.c0;
        h.k = c.f32[0]; h.ik = c.f32[1]; h.skh = c.f32[2]; h.cR = c.f32[3]; h.ce = c.f32[4];
        h.dlngs = c.f32[5]; h.lnk_psi = c.f32[6]; h.p = c.f32[7];
        const EdgeVal<float> e = gg_edge<float, true>(lnx1, h);
        c.e1[1] = e.d1;
        c.e1[2] = e.d2;
      } else {
        const EdgeVal<double> e = gg_edge<double, true>(lnx1, g);
        c.e1[1] = e.d1;
        c.e1[2] = e.d2;
      }
    }
    cpo[i] = c;
    // the column's factor of the sweeps' one-interval test, as the cells
    // form it (step_lean)
    if (f.kind == kGauss) {
      qv = c.c1 > 0.0 ? c.c1 : INFINITY;
    } else if (f.prec == kF32) {
      const float w = 1.4142135623730950488f * c.f32[2];
      qv = w == w ? (double)w : INFINITY;
    } else {
      const double w = 1.4142135623730950488 * c.f64[2];
      qv = w == w ? w : INFINITY;
    }
  }
  // largest over the four columns of each wave step (columns past T: none)
  qv = fmax(qv, __shfl_xor(qv, 1, 4));
  qv = fmax(qv, __shfl_xor(qv, 2, 4));
  if ((i & 3) == 0 && (i >> 2) < 4 * n_ct) fixq[i >> 2] = qv;
  // support of each 16-column tile, domain flags of the block
  for (int m = 8; m >= 1; m >>= 1) {
    jlo = min(jlo, __shfl_xor(jlo, m, 16));
    jhi = max(jhi, __shfl_xor(jhi, m, 16));
  }
  if ((threadIdx.x & 15) == 0 && i < T) tbo[i >> 4] = make_int2(jlo, jhi);
  for (int m = 32; m >= 1; m >>= 1) bad |= __shfl_xor(bad, m, 64);
  if (threadIdx.x == 0) cpflag[fb2.x] = bad;
}

// A column's constants as one lane holds them in the sweeps.
typedef __attribute__((address_space(1))) const ColPar GColPar;

template <class R>
struct ColPre {
  double c0, c1;  // Gauss: m, 1/sigma; GG: ct, k cR (the quadrature's column scale, FP64)
  R s[8];         // GG constants (count: its FP64 constants)
  double v;       // single histogram: v_i = sum_s r_s F^_si; multivariate: F^[i, species of the lane]
  GColPar* cp;    // the column's parameters (FP64 constants of the CDF at the edges)
};

// The CDF at a reco edge (GG, Gaussian) and its two column-parameter
// derivatives, for bins too wide for the quadrature (or a GG bin from x <= 0,
// whose cell is the single value F(x_1)).  The value is formed in FP64 (the
// value alone: no derivative carried through the series), the derivatives in
// the cell precision: an FP32 value would leave the per-column rounding of its
// constants in the cell, which the gradient amplifies; FP32 derivatives do not
// matter there.
template <class R, int KIND, bool D>
__device__ __forceinline__ EdgeVal<double> edge_mixed(const ColPre<R>& c, double xe) {
  EdgeVal<double> o;
  GColPar* cp = c.cp;
  if constexpr (KIND == kGauss) {
    o.v = gauss_edge<double, false>(xe, cp->c0, cp->c1).v;
    if (D) {
      const EdgeVal<R> e = gauss_edge<R, true>(xe, c.c0, c.c1);
      o.d1 = e.d1;
      o.d2 = e.d2;
    }
  } else {
    GGCol<double> g;
    g.ct = cp->c0;
    g.k = cp->f64[0]; g.ik = cp->f64[1]; g.skh = cp->f64[2]; g.cR = cp->f64[3]; g.ce = cp->f64[4];
    g.dlngs = cp->f64[5]; g.lnk_psi = cp->f64[6]; g.p = cp->f64[7];
    o.v = gg_edge<double, false>(xe, g).v;
    if (D) {
      GGCol<R> h;
      h.ct = c.c0;
      h.k = c.s[0]; h.ik = c.s[1]; h.skh = c.s[2]; h.cR = c.s[3]; h.ce = c.s[4];
      h.dlngs = c.s[5]; h.lnk_psi = c.s[6]; h.p = c.s[7];
      const EdgeVal<R> e = gg_edge<R, true>(xe, h);
      o.d1 = e.d1;
      o.d2 = e.d2;
    }
  }
  if (!D) o.d1 = o.d2 = 0.0;
  return o;
}

// Quadrature constants of a lane's reco bin: GG the bin centre in p ln x, its
// half-width in t and the node constants (FP32: 4 nodes, FP64: 5); Gaussian
// the bin's centre and half-width.
template <class R>
struct RowQ {
  static constexpr int NQ = sizeof(R) == 4 ? kNQ32 : kNQ64;
  double a, b;
  QRowGG<R, NQ> g;
};

template <class R, int KIND>
__device__ __forceinline__ RowQ<R> load_rowq(const FitDev& f, int j) {
  typedef __attribute__((address_space(1))) const double GD;
  RowQ<R> r;
  r.a = r.b = 0.0;
  if constexpr (KIND == kGG) {
    constexpr int NQ = RowQ<R>::NQ;
    typedef __attribute__((address_space(1))) const R GR;
    GR* q;
    if constexpr (sizeof(R) == 4) q = (GR*)f.qrow32 + (size_t)j * 3 * NQ;
    else q = (GR*)f.qrow64 + (size_t)j * 3 * NQ;
    r.a = ((GD*)f.qpum)[j];
    r.b = ((GD*)f.qhw)[j];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {  // the layout of QRowGG: d, fd, ed
      r.g.d[u] = q[u];
      r.g.fd[u] = q[NQ + u];
      r.g.ed[u] = q[2 * NQ + u];
    }
  } else if constexpr (KIND == kGauss) {
    const double x0 = ((GD*)f.xraw)[j], x1 = ((GD*)f.xraw)[j + 1];
    r.a = 0.5 * (x0 + x1);
    r.b = 0.5 * (x1 - x0);
  }
  return r;
}

// The cell R_ji of the lane's reco bin j for column c, and with D its
// derivatives in the column parameters (Gaussian: m, sigma; GG: k, ln a;
// count: m, r).  Analytic responses integrate the density over the bin by
// Gauss-Legendre quadrature.  The sweeps take the common case (cell_lean):
// every lane of the wave a single quadrature interval (step_lean), all but
// about 0.4 % of the wave steps of the 3000 x 900 sweep; the other steps are
// left to the fix-up sweeps (k_cells_fwd_fix, k_cells_bwd_fix), which take
// every case (cell_general): a composite rule of up to kMaxSub intervals when
// the bin is wide against the column (quad_intervals), and a bin wider than
// that (or a GG bin from x <= 0) as the difference of the CDF at its edges,
// the upper one from the next lane of the row (DPP row_shl:1).  Kept out of
// the main sweeps, the general code no longer sets their register allocation
// (with it inlined they ran several times slower).  The count estimator's
// cell is its pmf at the lane's count (always the lean case).  ok = false (no
// such bin or column) gives zeros.  Both are called by all lanes of the wave.
// The one-interval test of a wave step (reco tile, true tile, q): every lane's
// bin half-width times its column's inverse width at most kQuadMax, taken as
// the product of the step's largest factors (p of the reco tile, q of the
// four columns), in the precision the cells form it (GG: R; Gauss: FP64).
// Rounding is monotonic, so this is exactly the test over all the lanes.
template <class R, int KIND>
__device__ __forceinline__ bool step_lean(double q, double p) {
  if constexpr (KIND == kGG) return (R)q * (R)p <= (R)kQuadMax;
  else if constexpr (KIND == kGauss) return q * p <= kQuadMax;
  return true;
}

template <class R, int KIND, bool D>
__device__ __forceinline__ CellVal<R> cell_lean(const ColPre<R>& c, const RowQ<R>& rq, double xe, double lnf,
                                                bool ok) {
  CellVal<R> o;
  if constexpr (KIND == kCount) {
    const EdgeVal<R> e = count_cell<D>(xe, lnf, c.s);
    o.v = e.v;
    o.d1 = e.d1;
    o.d2 = e.d2;
  } else if constexpr (KIND == kGG) {
    o = gg_cell_lean<R, RowQ<R>::NQ, D>((R)(rq.a - c.c0), rq.b * (c.c1 * gl_norm<R, RowQ<R>::NQ>()), rq.g,
                                        c.s[0] * (R)kLog2e, c.s[6], c.s[7] * c.s[0]);
  } else {
    o = gauss_cell_quad<R, RowQ<R>::NQ, D>(rq.a, rq.b, c.c0, c.c1);
  }
  if (!ok) {
    o.v = 0.0;
    o.d1 = o.d2 = (R)0;
  }
  return o;
}

template <class R, int KIND, bool D>
__device__ __forceinline__ CellVal<R> cell_general(const ColPre<R>& c, const RowQ<R>& rq, double xe, bool ok,
                                                   bool zrow) {
  CellVal<R> o;
  o.v = 0.0;
  o.d1 = o.d2 = (R)0;
  // inverse width of the column in the quadrature variable: GG sqrt(k) in
  // t = ln(y/k); Gaussian 1/sigma (none for a zero width)
  const double iw = KIND == kGG ? 1.4142135623730950488 * (double)c.s[2] : (c.c1 > 0.0 ? c.c1 : NAN);
  // lanes without a cell side with quadrature; the GG bin from x <= 0 (zrow)
  // takes the cell k_colparams formed, and needs no edge from its neighbour
  const int ns = ok && !zrow ? quad_intervals(rq.b, iw) : 1;
  const unsigned long long eb = __ballot(ns == 0);
  const int lane = threadIdx.x & 63;
  const bool row_edge = ((eb >> (lane & 48)) & 0xffffull) != 0;  // row-uniform
  // the edge values the row needs: the lower edge of each CDF-difference cell
  // (the lane's own) and its upper edge (the next lane's); the FP64 CDF runs
  // a series or continued fraction of up to ~100 terms, so the other lanes
  // leave it alone
  const bool need = ((eb >> lane) & 1) || ((lane & 15) > 0 && ((eb >> (lane - 1)) & 1));
  if (ns > 0 && !zrow) {
    if constexpr (KIND == kGG)
      o = gg_cell_quad<R, RowQ<R>::NQ, D>(rq.a, rq.b, c.c0, rq.g, c.s[0], c.c1, c.s[6], c.s[7] * c.s[0], ns);
    else
      o = gauss_cell_quad<R, RowQ<R>::NQ, D>(rq.a, rq.b, c.c0, c.c1, ns);
  }
  if (row_edge) {
    EdgeVal<double> e;
    e.v = e.d1 = e.d2 = 0.0;
    if (need) e = edge_mixed<R, KIND, D>(c, xe);
    const double vh = dpp_from_next(e.v);
    const double d1h = D ? dpp_from_next(e.d1) : 0.0;
    const double d2h = D ? dpp_from_next(e.d2) : 0.0;
    if (ns == 0) {
      o.v = cell_from(e.v, vh);
      if (D) {
        o.d1 = (R)(d1h - e.d1);
        o.d2 = (R)(d2h - e.d2);
      }
    }
  }
  if (zrow) {
    GColPar* cp = c.cp;
    o.v = cp->e1[0];
    if (D) {
      o.d1 = (R)cp->e1[1];
      o.d2 = (R)cp->e1[2];
    }
  }
  if (!ok) {
    o.v = 0.0;
    o.d1 = o.d2 = (R)0;
  }
  return o;
}

// ---------------------------------------------------------------------------
// Tabulated response (the Monte Carlo alternative to the analytic R of
// Eq. 1).  At build: M_g = R_g F^T for every grid matrix, FP64 MFMA 16x16x4.
// Block = (16 reco rows, g), 8 waves; wave w takes the 16-column chunks
// c = w, w + 8, ... of the true axis (each lane loads its MFMA operands
// straight from R_g and F: the four steps of a chunk read 16 rows x 128
// contiguous bytes), and the 8 partial products are added in a fixed order.
constexpr int kGemmWaves = 8;
__global__ void __launch_bounds__(kGemmWaves * 64) k_table_gemm(const double* R, const double* F64, double* Mg,
                                                                 int N, int T) {
  typedef __attribute__((address_space(1))) const double GD;
  __shared__ double part[kGemmWaves][4][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, g = blockIdx.y, j0 = blockIdx.x * 16;
  const int m = lane & 15, kq = lane >> 4;
  GD* Rrow = (GD*)R + ((size_t)g * N + min(j0 + m, N - 1)) * T;
  GD* F = (GD*)F64;
  const bool rok = j0 + m < N;
  v4d acc = {0, 0, 0, 0};
  for (int i0 = 16 * wv; i0 < T; i0 += 16 * kGemmWaves) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int i = i0 + 4 * kk + kq;
      const double A = (rok && i < T) ? Rrow[i] : 0.0;                // A[m = reco row][k]
      const double B = i < T ? F[(size_t)i * kSP + m] : 0.0;          // B[k][n = species]
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wv][r][lane] = acc[r];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = part[0][r][lane];
      for (int w = 1; w < kGemmWaves; ++w) v += part[w][r][lane];
      const int j = j0 + (lane >> 4) + 4 * r;  // FP64 result layout: row l/16 + 4r, column l%16
      if (j < N) Mg[((size_t)g * N + j) * kSP + (lane & 15)] = v;
    }
  }
}

void launch_table_gemm(const double* d_R, const double* d_F64, double* d_Mg, int G, int N, int T, hipStream_t st) {
  hipLaunchKernelGGL(k_table_gemm, dim3((N + 15) / 16, G), dim3(kGemmWaves * 64), 0, st, d_R, d_F64, d_Mg, N, T);
}

// Per evaluation: M = (1 - w) M_g + w M_g+1 for the grid cell [lam_g, lam_g+1]
// holding lam = theta[S] (the cell above at an interior grid point), and
// dM/dlam = (M_g+1 - M_g) / (lam_g+1 - lam_g).  theta comes from pinned host
// memory when the caller passed it there (block 0 leaves the device copy and
// the domain flags).
__global__ void __launch_bounds__(kBlock) k_table(const FitDev* fits, const int* active) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if ((int)blockIdx.x * kBlock >= f.N * kSP) return;  // block-uniform
  __shared__ double sth[kMaxP + 1];
  __shared__ int sg, sbad;
  __shared__ double sw, sdl;
  if ((int)threadIdx.x <= f.P) {
    const double v = f.theta_src ? __hip_atomic_load(f.theta_src + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)
                                 : f.theta[threadIdx.x];
    sth[threadIdx.x] = v;
    if (f.theta_src && blockIdx.x == 0) const_cast<double*>(f.theta)[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int q = 0; q < f.P; ++q)
      if (!isfinite(sth[q])) bad |= kBadTheta;
    if (f.pu_float && !(sth[f.P - 1] >= 0.0 && sth[f.P - 1] <= 1.0)) bad |= kBadTheta;
    int g = 0;
    double w = 0.0, dl = 1.0;
    const int G = f.n_grid;
    if (G > 1) {
      const double lam = sth[f.S];
      if (!(lam >= f.grid[0] && lam <= f.grid[G - 1])) bad |= kBadTheta;
      while (g + 1 < G - 1 && f.grid[g + 1] <= lam) ++g;  // last grid point <= lam, at most G - 2
      dl = f.grid[g + 1] - f.grid[g];
      w = bad ? 0.0 : (lam - f.grid[g]) / dl;
    }
    sg = g;
    sw = w;
    sdl = dl;
    sbad = bad;
    if (blockIdx.x == 0) {
      f.cpflag[0] = bad;
      *f.fcount = 0;  // this evaluation's final sums start their count
    }
  }
  __syncthreads();
  if (t >= f.N * kSP) return;
  const double* M0 = f.Mg + (size_t)sg * f.N * kSP;
  if (f.n_grid > 1) {
    const double a = M0[t], b = M0[(size_t)f.N * kSP + t];
    f.M[t] = (1.0 - sw) * a + sw * b;
    f.Dt[t] = (b - a) / sdl;
  } else {
    f.M[t] = M0[t];
  }
}

// ---------------------------------------------------------------------------
// Balanced pairwise sum of item(OFF), ..., item(OFF + N - 1), N a power of
// two: ((i0 + i1) + (i2 + i3)) + ...  Any aligned sub-range is a subtree, so
// partial sums formed over sub-ranges and combined the same way give the same
// bits.
template <int N, int OFF, class V, class F>
__device__ __forceinline__ V tree_sum(const F& item) {
  if constexpr (N == 1) {
    return item(OFF);
  } else {
    const V a = tree_sum<N / 2, OFF, V>(item);
    const V b = tree_sum<N / 2, OFF + N / 2, V>(item);
    return a + b;
  }
}

// Block (rt, fb): reco rows [15 rt, 15 rt + 15).  The true tiles whose
// support meets these rows (a contiguous band for a smooth response, about a
// third of them on the 3000 x 900 grid) are listed in ascending order; the
// list is cut into chunks of 16 entries, and each chunk's tiles are summed in
// the balanced tree of tree_sum into one partial, Mpart[chunk].  A block takes
// CG chunks: wave w holds entries [w CG, w CG + CG) of its window (a subtree),
// so the partials do not depend on CG, which sets only how many tiles a wave
// evaluates in a row.  The working waves fill the first blocks of each reco
// tile; the rest find their window empty and write zero partials.
// Lane (j = l%16, g = l/16) holds reco bin j of the tile and column 4q + g of
// the true tile at step q.  The cells are contracted in FP64: with a single
// histogram (vsum) each lane accumulates R_ji v_i, summed over its four
// column groups at the end; with several species histograms (MV) the cells
// are the A operand of FP64 MFMA 16x16x4 with B = F^[i, s] (M = R F^T).
template <class R, int KIND, int CG, bool MV>
__global__ void __launch_bounds__(kFwdWaves * 64) k_cells_fwd(const FitDev* fits, const int* active) {
  typedef typename std::conditional<MV, v4d, double>::type V;
  constexpr int NR = MV ? 4 : 1;
  typedef __attribute__((address_space(1))) const double GD;
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int rt = fb2.x / f.n_fb, fb = fb2.x % f.n_fb;
  // block-uniform; a launch holds fits of one contraction kind only (a fit of
  // the other kind is left alone rather than written with the wrong layout)
  if (rt >= f.n_rt || f.vsum == (int)MV) return;
  __shared__ double part[kFwdWaves][NR][64];
  __shared__ int wcount[kFwdWaves];
  __shared__ int mylist[kFwdWaves * CG];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, jr = lane & 15, g = lane >> 4;
  const int j0 = rt * kRowStep;
  // this block's window [lo, lo + kFwdWaves CG) of the list of active tiles
  constexpr int win = kFwdWaves * CG;
  const int lo = win * fb;
  int n_act = 0;
  for (int c0 = 0; c0 < f.n_ct; c0 += kFwdWaves * 64) {
    const int ct = c0 + (int)threadIdx.x;
    bool act = false;
    if (ct < f.n_ct) {
      const __attribute__((address_space(1))) int* tbp = (const __attribute__((address_space(1))) int*)f.tb;
      const int bx = tbp[2 * ct], by = tbp[2 * ct + 1];  // the tile's support [bx, by] (by < bx: empty)
      act = by >= bx && !(by < j0 || bx > j0 + kRowStep - 1);
    }
    const unsigned long long m = __ballot(act);
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int off = n_act, tot = n_act;
    for (int w = 0; w < kFwdWaves; ++w) {
      off += w < wv ? wcount[w] : 0;
      tot += wcount[w];
    }
    const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
    if (act && pos >= lo && pos < lo + win) mylist[pos - lo] = ct;
    n_act = tot;
    __syncthreads();
  }
  // Fields of f in registers, accesses through global-address-space views
  // (flat accesses would make every wait for a load also wait for all older
  // memory operations).
  GColPar* const cpar = (GColPar*)f.cp;
  GD* const F64 = (GD*)f.F64;
  const int T = f.T, N = f.N, n_cg = f.n_cg;
  double* const Mpart = f.Mpart;
  int* const fixflag = f.fixflag;
  GD* const fixq = (GD*)f.fixq;
  const int n_rt = f.n_rt;
  const double pmax = KIND == kCount ? 0.0 : ((GD*)f.fixp)[rt];
  const int je = min(j0 + jr, N);
  const double xe = ((GD*)f.xe)[je];
  const double lnf = KIND == kCount ? lgamma(xe + 1.0) : 0.0;  // count estimator: ln n! of the row
  const bool row_ok = (jr < kRowStep) && (j0 + jr < N);
  const RowQ<R> rq = load_rowq<R, KIND>(f, min(j0 + jr, N - 1));
  const int n_here = n_act - lo;  // entries of this window in the list
  // a lane's column constants, fetched one column ahead of their use so that
  // the loads overlap the cell arithmetic
  auto fetch = [&](int i) -> ColPre<R> {
    ColPre<R> p;
    const bool iok = i < T;
    GColPar& cpi = cpar[iok ? i : T - 1];
    p.cp = &cpi;
    p.c0 = cpi.c0;
    p.c1 = KIND == kGauss ? cpi.c1 : KIND == kGG ? cpi.c1 * cpi.f64[3] : 0.0;
    if (KIND != kGauss) {
#pragma unroll
      for (int u = 0; u < 8; ++u) p.s[u] = sizeof(R) == 4 ? (R)cpi.f32[u] : (R)cpi.f64[u];
    }
    p.v = !iok ? 0.0 : MV ? F64[i * kSP + jr] : cpi.v;
    return p;
  };
  // one tile's contribution (zero past the end of the list)
  auto tile = [&](int c) -> V {
    V acc = {};
    const int e = wv * CG + c;
    if (e >= n_here) return acc;  // wave-uniform
    const int ct = mylist[e];
    ColPre<R> cur = fetch(ct * kColTile + g);
    int left = 0;  // steps left to the fix-up sweeps (bit q)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ColPre<R> nxt;
      if (q < 3) nxt = fetch(ct * kColTile + 4 * (q + 1) + g);
      const int i = ct * kColTile + 4 * q + g;
      const bool ok = row_ok && i < T;
      if (KIND == kCount || step_lean<R, KIND>(fixq[ct * 4 + q], pmax)) {  // wave-uniform
        const CellVal<R> ev = cell_lean<R, KIND, false>(cur, rq, xe, lnf, ok);
        if constexpr (MV) acc = mfma16(ev.v, cur.v, acc);
        else acc = fma(ev.v, cur.v, acc);
      } else {
        left |= 1 << q;
      }
      if (q < 3) cur = nxt;
    }
    if constexpr (KIND != kCount) {
      if (lane == 0 && left) {  // the fix-up sweeps of this reco tile and this true tile have work
        atomicOr(fixflag + rt, 1);
        atomicOr(fixflag + n_rt + ct, 1);
      }
    }
    return acc;
  };
  const V sub = tree_sum<CG, 0, V>(tile);
  if constexpr (MV) {
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wv][r][lane] = sub[r];
  } else {
    part[wv][0][lane] = sub;
  }
  __syncthreads();
  // chunk k of this block = waves [k W, k W + W), W = 16 / CG: wave k adds
  // their subtrees in the same tree and writes the chunk's partial
  constexpr int W = kFwdWaves / CG;
  const int chunk = fb * CG + wv;
  if (wv < CG && chunk < n_cg) {
    const V v = tree_sum<W, 0, V>([&](int w) -> V {
      V x;
      if constexpr (MV) {
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = part[wv * W + w][r][lane];
      } else {
        x = part[wv * W + w][0][lane];
      }
      return x;
    });
    if constexpr (MV) {
      double* out = Mpart + (size_t)chunk * N * kSP;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // FP64 MFMA 16x16x4 result layout: lane l, register r holds row l/16 + 4r, column l%16
        const int row = g + 4 * r;
        if (row < kRowStep && j0 + row < N) out[(size_t)(j0 + row) * kSP + jr] = v[r];
      }
    } else {
      // the four column groups of row jr, added in a fixed order
      double x = v;
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (g == 0 && row_ok) Mpart[(size_t)chunk * N + j0 + jr] = x;
    }
  }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double nll_term(double mu, double n, double* w, int* bad) {
  if (!(mu >= 0.0) || (mu == 0.0 && n > 0.0) || !isfinite(mu)) {
    *bad |= kBadMu;
    *w = 0.0;
    return 0.0;
  }
  if (n > 0.0) {
    *w = 1.0 - n / mu;
    return mu - n * log(mu);
  }
  *w = 1.0;
  return mu;
}

__device__ __forceinline__ int pu_len(const FitDev& f) {
  return (f.K > 0 && (f.pu_float || f.pu_frac != 0.0)) ? f.K : 1;
}

// Pile-up fraction: the last parameter when it is floated, else fixed.
__device__ __forceinline__ double pu_p(const FitDev& f) {
  return f.pu_float ? f.theta[f.P - 1] : f.pu_frac;
}

// M[j, s] = sum over the forward chunks of the partials, FP64, fixed order.
// A single histogram (vsum) has one partial per row: mu0_j goes to M[j, 0]
// and the other species columns are zero.
// M[j, s] (single histogram: s = 0) as the sum of the forward sweep's chunk
// partials and then, for a reco tile with steps left, the fix-up sweep's
// shares, in a fixed order.
__device__ __forceinline__ double m_sum(const FitDev& f, int j, int s) {
  typedef __attribute__((address_space(1))) const double GD;
  const int n = f.n_cg;
  const size_t stride = f.vsum ? (size_t)f.N : (size_t)f.N * kSP;
  const size_t off = f.vsum ? (size_t)j : (size_t)j * kSP + s;
  GD* const p = (GD*)f.Mpart + off;
  // the first U partials, the tile's fix-up flag and its shares are loaded
  // together (the shares whatever the flag: a tile without steps left holds
  // stale values there, which are then not added)
  constexpr int U = 16;
  const bool fx = f.has_fix != 0;
  double v[U], w[kFixSplit];
#pragma unroll
  for (int c = 0; c < U; ++c) v[c] = c < n ? p[c * stride] : 0.0;
  const int fl = fx ? ((const __attribute__((address_space(1))) int*)f.fixflag)[j / kRowStep] : 0;
  GD* const q = (GD*)f.Mfix + off;
#pragma unroll
  for (int b = 0; b < kFixSplit; ++b) w[b] = fx ? q[b * stride] : 0.0;
  double a = 0.0;
#pragma unroll
  for (int c = 0; c < U; ++c)
    if (c < n) a += v[c];
  for (int c = U; c < n; ++c) a += p[c * stride];
  if (fl) {
#pragma unroll
    for (int b = 0; b < kFixSplit; ++b) a += w[b];
  }
  return a;
}

// Several species histograms: M from the partials (a single histogram's M
// column is summed by k_rowterms as it stages the rows).
__global__ void __launch_bounds__(kBlock) k_reduce_M(const FitDev* fits, const int* active) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= f.N * kSP || f.vsum) return;
  f.M[t] = m_sum(f, t >> 4, t & 15);
}

// (g * M)_j = sum_k g_k M_(j-k) over the taps k <= kmax, with row j - k of
// M staged at Ml[jl - k] and the taps at gl[]: four chains over k (mod 4),
// added pairwise.
__device__ __forceinline__ double pu_conv(const double* gl, const double (*Ml)[kSP], int jl, int s, int kmax) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = 0;
  for (; k + 3 <= kmax; k += 4) {
    a0 = fma(gl[k], Ml[jl - k][s], a0);
    a1 = fma(gl[k + 1], Ml[jl - k - 1][s], a1);
    a2 = fma(gl[k + 2], Ml[jl - k - 2][s], a2);
    a3 = fma(gl[k + 3], Ml[jl - k - 3][s], a3);
  }
  if (k <= kmax) a0 = fma(gl[k], Ml[jl - k][s], a0);
  if (k + 1 <= kmax) a1 = fma(gl[k + 1], Ml[jl - k - 1][s], a1);
  if (k + 2 <= kmax) a2 = fma(gl[k + 2], Ml[jl - k - 2][s], a2);
  return (a0 + a1) + (a2 + a3);
}

// 16 rows x 16 species per block.
__global__ void __launch_bounds__(kBlock) k_rowterms(const FitDev* fits, const int* active) {
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if (fb2.x >= f.n_rowblk) return;  // block-uniform
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) double GDw;
  typedef __attribute__((address_space(1))) int GIw;
  // every field used is read into registers before the first store (a store
  // through a generic pointer could alias f and force reloads after it)
  const int N = f.N, S = f.S, mv = f.mv, joint = f.joint, n_ps = f.n_ps, pu_float = f.pu_float, vsum = f.vsum;
  const int win_lo = f.win_lo, win_hi = f.win_hi;
  const bool tab = f.kind == kTable && f.nresp > 0;
  const int K = pu_len(f);
  const double pp = pu_p(f);
  GD* const Mg = (GD*)f.M;
  GD* const ghat = (GD*)f.ghat;
  GD* const Dt = (GD*)f.Dt;
  GD* const th = (GD*)f.theta;
  GD* const tag = (GD*)f.tag;
  GD* const pst = (GD*)f.pst;
  GD* const n_e = (GD*)f.n_e;
  GD* const n_t = (GD*)f.n_t;
  GD* const n_p = (GD*)f.n_p;
  GDw* const Mp = (GDw*)f.Mp;
  GDw* const Dp = (GDw*)f.Dp;
  GDw* const Dtp = (GDw*)f.Dtp;
  GDw* const H = (GDw*)f.H;
  GDw* const nllpart = (GDw*)f.nllpart;
  GIw* const flagpart = (GIw*)f.flagpart;
  GDw* const gpart = (GDw*)f.gpart;
  GDw* const ppart = (GDw*)f.ppart;
  GDw* const tpart = (GDw*)f.tpart;
  __shared__ double Ml[16 + kMaxK - 1][kSP];
  __shared__ double mp[16][kSP];
  __shared__ double red[kBlock];
  __shared__ int redf[kBlock];
  __shared__ double wps[16][64];
  __shared__ double gl[kMaxK];
  const int rl = threadIdx.x >> 4, s = threadIdx.x & 15;
  const int j0 = fb2.x * 16;
  const int r0 = max(j0 - (K - 1), 0), r1 = min(j0 + 16, N);
  for (int e = threadIdx.x; e < K; e += kBlock) gl[e] = ghat[e];
  // M rows [r0, r1) staged in LDS for the pile-up sums (a single histogram's
  // column summed here from the forward partials)
  if (vsum) {
    for (int e = threadIdx.x; e < (r1 - r0) * kSP; e += kBlock)
      if (e & 15) Ml[e >> 4][e & 15] = 0.0;
    for (int e = threadIdx.x; e < r1 - r0; e += kBlock) Ml[e][0] = m_sum(f, r0 + e, 0);
  } else {
    for (int e = threadIdx.x; e < (r1 - r0) * kSP; e += kBlock) Ml[e >> 4][e & 15] = Mg[(size_t)r0 * kSP + e];
  }
  __syncthreads();
  const int j = j0 + rl;
  const bool jok = j < N;
  double m = 0.0, dmp = 0.0;  // M'_js and dM'_js/dp = (g^*M)_js - M_js
  if (jok) {
    m = Ml[j - r0][s];
    if (K > 1) {
      const double acc = pu_conv(gl, Ml, j - r0, s, min(j, K - 1));
      dmp = acc - m;
      m = (1.0 - pp) * m + pp * acc;
    }
    Mp[j * kSP + s] = m;
    if (pu_float) Dp[j * kSP + s] = dmp;
  }
  mp[rl][s] = m;
  __syncthreads();
  // tabulated response: dM'/dlam, the pile-up applied to dM/dlam (rows
  // staged in the same LDS rows as M)
  double dmt = 0.0;
  if (tab) {  // block-uniform
    for (int e = threadIdx.x; e < (r1 - r0) * kSP; e += kBlock) Ml[e >> 4][e & 15] = Dt[(size_t)r0 * kSP + e];
    __syncthreads();
    if (jok) {
      dmt = Ml[j - r0][s];
      if (K > 1) {
        const double acc = pu_conv(gl, Ml, j - r0, s, min(j, K - 1));
        dmt = (1.0 - pp) * dmt + pp * acc;
      }
      Dtp[j * kSP + s] = dmt;
    }
  }
  // vsum: M' holds mu0 after pile-up in species column 0 (the rates are in v)
  const double r_s = vsum ? (s == 0 ? 1.0 : 0.0) : s < S ? th[s] : 0.0;
  const bool inwin = jok && j >= win_lo && j < win_hi;
  double term = 0.0, h = 0.0;
  int bad = 0;
  if (!mv) {
    const double mu = sum16(m * r_s);
    double w = 0.0;
    if (inwin) {
      const double t = nll_term(mu, n_e[j], &w, &bad);
      if (s == 0) term = t;
    }
    h = w;
  } else {
    const double t_s = s < S ? tag[s] : 0.0;
    const double musub = sum16(m * (1.0 - t_s) * r_s);
    const double mutag = sum16(m * t_s * r_s);
    double wsub = 0.0, wtag = 0.0;
    if (inwin) {
      // with the joint term (k_joint) the vetoed events are not a term here
      const double t1 = joint ? 0.0 : nll_term(musub, n_e[j], &wsub, &bad);
      const double t2 = nll_term(mutag, n_t[j], &wtag, &bad);
      if (s == 0) term = t1 + t2;
    }
    // pulse-shape row j: lambda_jk = sum_s M'_js (1 - t_s) r_s T_sk
    for (int k = s; k < (joint ? 0 : n_ps); k += 16) {
      double w = 0.0;
      if (inwin) {
        double lam = 0.0;
        for (int u = 0; u < S; ++u) lam += mp[rl][u] * (1.0 - tag[u]) * th[u] * pst[u * n_ps + k];
        term += nll_term(lam, n_p[(size_t)j * n_ps + k], &w, &bad);
      }
      wps[rl][k] = w;
    }
    __syncthreads();
    double hps = 0.0;
    if (s < S && !joint)
      for (int k = 0; k < n_ps; ++k) hps += wps[rl][k] * pst[s * n_ps + k];
    // H_js = w_sub (1 - t_s) + w_tag t_s + (1 - t_s) sum_k w_ps,jk T_sk
    h = wsub * (1.0 - t_s) + wtag * t_s + (1.0 - t_s) * hps;
  }
  if (jok) H[j * kSP + s] = (s < S) ? h : 0.0;
  // block partials: NLL (fixed tree), flags, rate gradient sum_j H_js M'_js
  red[threadIdx.x] = term;
  redf[threadIdx.x] = bad;
  __syncthreads();
  for (int st = kBlock / 2; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[threadIdx.x] += red[threadIdx.x + st];
      redf[threadIdx.x] |= redf[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nllpart[fb2.x] = red[0];
    flagpart[fb2.x] = redf[0];
  }
  __syncthreads();
  red[threadIdx.x] = (jok && s < S) ? h * m : 0.0;
  __syncthreads();
  if (threadIdx.x < 16) {
    double a = 0.0;
    for (int r = 0; r < 16; ++r) a += red[r * 16 + threadIdx.x];
    gpart[fb2.x * kSP + threadIdx.x] = a;
  }
  if (pu_float) {  // block-uniform: dNLL/dp without the radial part, sum_js H_js r_s dM'_js/dp
    __syncthreads();
    red[threadIdx.x] = (jok && s < S) ? h * r_s * dmp : 0.0;
    __syncthreads();
    for (int st = kBlock / 2; st >= 1; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) ppart[fb2.x] = red[0];
  }
  if (tab) {  // block-uniform: dNLL/dlam without the radial part, sum_js H_js r_s dM'_js/dlam
    __syncthreads();
    red[threadIdx.x] = (jok && s < S) ? h * r_s * dmt : 0.0;
    __syncthreads();
    for (int st = kBlock / 2; st >= 1; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) tpart[fb2.x] = red[0];
  }
}

// Radial term: nu_k = sum_s (1 - t_s) r_s (sum_{j in W} M'_js) rho_sk.
__global__ void __launch_bounds__(kBlock) k_radial(const FitDev* fits, const int* active) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if (!f.mv || f.n_rad <= 0 || f.joint) return;  // block-uniform
  __shared__ double part[16][kSP], partd[16][kSP], partt[16][kSP];
  __shared__ double SW[kSP], SD[kSP], ST[kSP], A[kSP], pgs[kSP], tgs[kSP], wr[128], red[kBlock];
  __shared__ int redf[kBlock];
  const int s = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const bool tab = f.kind == kTable && f.nresp > 0;
  double acc = 0.0, accd = 0.0, acct = 0.0;
  for (int j = f.rad_lo + grp; j < f.rad_hi; j += 16) {
    acc += f.Mp[j * kSP + s];
    if (f.pu_float) accd += f.Dp[j * kSP + s];
    if (tab) acct += f.Dtp[j * kSP + s];
  }
  part[grp][s] = acc;
  partd[grp][s] = accd;
  partt[grp][s] = acct;
  __syncthreads();
  if (threadIdx.x < 16) {
    double t = 0.0, td = 0.0, tt = 0.0;
    for (int g = 0; g < 16; ++g) {
      t += part[g][threadIdx.x];
      td += partd[g][threadIdx.x];
      tt += partt[g][threadIdx.x];
    }
    SW[threadIdx.x] = t;
    SD[threadIdx.x] = td;
    ST[threadIdx.x] = tt;
    A[threadIdx.x] = (int)threadIdx.x < f.S ? (1.0 - f.tag[threadIdx.x]) * f.theta[threadIdx.x] * t : 0.0;
  }
  __syncthreads();
  double term = 0.0;
  int bad = 0;
  for (int k = threadIdx.x; k < f.n_rad; k += kBlock) {
    double nu = 0.0;
    for (int u = 0; u < f.S; ++u) nu += A[u] * f.rad[u * f.n_rad + k];
    double w;
    term += nll_term(nu, f.n_r[k], &w, &bad);
    wr[k] = w;
  }
  red[threadIdx.x] = term;
  redf[threadIdx.x] = bad;
  __syncthreads();
  for (int st = kBlock / 2; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[threadIdx.x] += red[threadIdx.x + st];
      redf[threadIdx.x] |= redf[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x < 16) {
    double rw = 0.0;
    if ((int)threadIdx.x < f.S)
      for (int k = 0; k < f.n_rad; ++k) rw += wr[k] * f.rad[threadIdx.x * f.n_rad + k];
    f.rad_out[2 + threadIdx.x] = rw;
    f.rad_out[2 + 16 + threadIdx.x] =
        (int)threadIdx.x < f.S ? (1.0 - f.tag[threadIdx.x]) * SW[threadIdx.x] * rw : 0.0;
    // radial part of dNLL/dp: sum_s (1 - t_s) r_s (sum_{j in W} dM'_js/dp) rho.w_s
    pgs[threadIdx.x] = (int)threadIdx.x < f.S ? (1.0 - f.tag[threadIdx.x]) * f.theta[threadIdx.x] * SD[threadIdx.x] * rw : 0.0;
    // and of dNLL/dlam (tabulated response) with dM'/dlam
    tgs[threadIdx.x] = (int)threadIdx.x < f.S ? (1.0 - f.tag[threadIdx.x]) * f.theta[threadIdx.x] * ST[threadIdx.x] * rw : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    f.rad_out[0] = red[0];
    f.rad_out[1] = (double)redf[0];
    double pg = 0.0, tg = 0.0;
    for (int u = 0; u < 16; ++u) {
      pg += pgs[u];
      tg += tgs[u];
    }
    f.rad_out[2 + 32] = pg;
    f.rad_out[2 + 33] = tg;
  }
}

// H~ = P^T H_tot, H_tot = H + [j in W](1 - t_s) rho.w_s; 16 rows per block.
__global__ void __launch_bounds__(kBlock) k_adjoint(const FitDev* fits, const int* active) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if ((int)blockIdx.x >= f.n_rowblk) return;  // block-uniform
  __shared__ double Hl[16 + kMaxK - 1][kSP];
  const int j0 = blockIdx.x * 16;
  const int K = pu_len(f);
  const int r1 = min(j0 + 16 + K - 1, f.N);
  const bool rad = f.mv && f.n_rad > 0 && !f.joint;
  for (int e = threadIdx.x; e < (r1 - j0) * kSP; e += kBlock) {
    const int jj = j0 + (e >> 4), s = e & 15;
    double h = f.H[jj * kSP + s];
    if (rad && s < f.S && jj >= f.rad_lo && jj < f.rad_hi) h += (1.0 - f.tag[s]) * f.rad_out[2 + s];
    Hl[e >> 4][s] = h;
  }
  __syncthreads();
  const int rl = threadIdx.x >> 4, s = threadIdx.x & 15;
  const int j = j0 + rl;
  if (j >= f.N) return;
  double h = Hl[rl][s];
  if (K > 1) {
    double acc = 0.0;
    const int kmax = min(K - 1, f.N - 1 - j);
    for (int k = 0; k <= kmax; ++k) acc += f.ghat[k] * Hl[rl + k][s];
    h = (1.0 - pu_p(f)) * h + pu_p(f) * acc;
  }
  f.Ht[j * kSP + s] = h;
}

// Single histogram: w~ = P^T w into column 0 of H~, 64 rows per block, four
// threads per row over the taps k = part (mod 4), the partials added in the
// same order and with the same explicit fused multiply-adds as in the
// backward sweep's own prologue (same bits).
__global__ void __launch_bounds__(kBlock) k_adjoint1(const FitDev* fits, const int* active) {
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int j0 = fb2.x * 64;
  if (f.mv || j0 >= f.N) return;  // block-uniform
  __shared__ double hs[64 + kMaxK - 1], gl[kMaxK];
  const int K = pu_len(f);
  const int r1 = min(j0 + 64 + K - 1, f.N);
  for (int e = threadIdx.x; e < r1 - j0; e += kBlock) hs[e] = f.H[(size_t)(j0 + e) * kSP];
  for (int e = threadIdx.x; e < K; e += kBlock) gl[e] = K > 1 ? f.ghat[e] : 0.0;
  __syncthreads();
  const int e = threadIdx.x >> 2, part = threadIdx.x & 3, j = j0 + e;
  double acc = 0.0;
  if (K > 1 && j < f.N) {
    const int kmax = min(K - 1, f.N - 1 - j);
    for (int k = part; k <= kmax; k += 4) acc = fma(gl[k], hs[e + k], acc);
  }
  const int l0 = (threadIdx.x & 63) & ~3;
  const double p0 = __shfl(acc, l0, 64), p1 = __shfl(acc, l0 + 1, 64);
  const double p2 = __shfl(acc, l0 + 2, 64), p3 = __shfl(acc, l0 + 3, 64);
  if (part == 0 && j < f.N) {
    double h = hs[e];
    const double pp = pu_p(f);
    if (K > 1) h = fma(pp, (p0 + p1) + (p2 + p3), (1.0 - pp) * h);
    f.Ht[(size_t)j * kSP] = h;
  }
}

// ---------------------------------------------------------------------------
// Logical block (ct, rg): true tile ct; its support covers the contiguous reco
// tiles [rt_a, rt_b], and wave w of the kBwdWaves takes
// rt = rt_a + (kBwdWaves rg + w) RG + c, c < RG.  The working blocks of a true
// tile are thus its first ones (one block for a support of up to kBwdWaves RG
// reco tiles); the others write zero partials and leave.  Each lane holds the
// constants of its four columns (4q + g) for all of its reco tiles and
// evaluates each cell's derivatives in the two column parameters again (by
// quadrature, or from the CDF's edge derivatives), weighted by
// W_ji = dNLL/dmu0_j dmu0_j/dR_ji: alpha_i = sum_j W_ji dR_ji/dc1,
// beta_i = sum_j W_ji dR_ji/dc2 in FP64, contracted with the column chain
// factors into the block's response-gradient partial.  Single histogram:
// W_ji = w~_j v_i with w~ = P^T w (the pile-up adjoint, formed here from the
// block's rows staged in LDS, or read from k_adjoint1 for batched launches,
// with the same bits), and the same pass accumulates u_i = sum_j w~_j R_ji for
// the rate gradient sum_i F^_si u_i.  Multivariate (MV): W_ji = sum_s H~_js
// r_s F^_is, the FP64 MFMA product of F (16 columns x 16 species) and
// (H~ r)^T, whose result layout (lane l, register q: column l/16 + 4q, row
// l%16) is the cells' lane layout.
template <class R, int KIND, bool MV>
__global__ void __launch_bounds__(kBwdWaves * 64) k_cells_bwd(const FitDev* fits, const int* active, int pre) {
  constexpr int NT = kBwdWaves * 64;
  constexpr int kRows = kBwdWaves * kMaxRG * kRowStep;
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int2 cr = bwd_block(fb2.x, f.n_rg);
  const int ct = cr.x, rg = cr.y, bl = ct * f.n_rg + rg;
  if (ct >= f.n_ct || f.mv != (int)MV) return;  // block-uniform (one contraction kind per launch)
  __shared__ double colA[kBwdWaves][16], colB[kBwdWaves][16], colU[kBwdWaves][16];
  __shared__ double hst[kRows + kMaxK], htl[kRows], gl[kMaxK];
  __shared__ double pq[kRows][4];
  __shared__ double rsum[16][kSP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, jr = lane & 15, g = lane >> 4;
  const int T = f.T, N = f.N, RG = f.RG;
  GColPar* const cpar = (GColPar*)f.cp;
  GD* const Hg = (GD*)f.H;
  GD* const F64 = (GD*)f.F64;
  double* const bwdpart = f.bwdpart + (size_t)bl * kBwdPart;
  const int bx = ((GI*)f.tb)[2 * ct], by = ((GI*)f.tb)[2 * ct + 1];  // support [bx, by]
  const int rt_a = by >= bx ? max(bx, 0) / kRowStep : 0;
  const int rt_b = by >= bx ? min(by / kRowStep, f.n_rt - 1) : -1;
  const int rt_blk = rt_a + kBwdWaves * rg * RG;  // first reco tile of this block
  if (rt_blk > rt_b) {                            // block-uniform: nothing in range
    if (threadIdx.x < kBwdPart) bwdpart[threadIdx.x] = 0.0;
    return;
  }
  // chain factors of the column totals (threads < 64: column c16, parameter q)
  const int c16 = threadIdx.x & 15, qp = (threadIdx.x >> 4) & 3;
  const int icol = ct * kColTile + c16;
  double J0 = 0.0, J1 = 0.0;
  if (threadIdx.x < 64 && icol < T && qp < f.nresp) {
    J0 = cpar[icol].J[0][qp];
    J1 = cpar[icol].J[1][qp];
  }
  // the constants of the lane's four columns, for all of its reco tiles
  ColPre<R> col[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = min(ct * kColTile + 4 * q + g, T - 1);
    GColPar& cpi = cpar[i];
    col[q].cp = &cpi;
    col[q].c0 = cpi.c0;
    col[q].c1 = KIND == kGauss ? cpi.c1 : KIND == kGG ? cpi.c1 * cpi.f64[3] : 0.0;
    if (KIND != kGauss) {
#pragma unroll
      for (int u = 0; u < 8; ++u) col[q].s[u] = sizeof(R) == 4 ? (R)cpi.f32[u] : (R)cpi.f64[u];
    }
    col[q].v = MV ? 0.0 : cpi.v;
  }
  const int rt0 = rt_blk + wv * RG;
  const int rt_end = min(rt0 + RG, rt_b + 1);
  const int S = f.S;
  double fa[4] = {0, 0, 0, 0}, thv[4] = {0, 0, 0, 0};
  if (MV) {  // F operands of the weights (lane: column lane%16, species 4 kb + lane/16)
    const int i = ct * kColTile + jr;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int s = 4 * kb + g;
      fa[kb] = (i < T && s < S) ? F64[(size_t)i * kSP + s] : 0.0;
      thv[kb] = s < S ? ((GD*)f.theta)[s] : 0.0;
    }
  }
  // single histogram: the pile-up adjoint w~ = P^T w of this block's reco
  // rows, from the rows it needs staged in LDS (multivariate fits read the
  // full adjoint H~ written by k_adjoint)
  const int r0 = rt_blk * kRowStep;
  const int nr = max(min((min(rt_b + 1, rt_blk + kBwdWaves * RG) - rt_blk) * kRowStep, N - r0), 0);
  if (!MV && !pre) {
    const int K = pu_len(f);
    const int ns = min(nr + K - 1, N - r0);
    for (int e = threadIdx.x; e < ns; e += NT) hst[e] = Hg[(size_t)(r0 + e) * kSP];
    for (int e = threadIdx.x; e < K; e += NT) gl[e] = K > 1 ? ((GD*)f.ghat)[e] : 0.0;
    __syncthreads();
    if (K > 1) {
      // four threads per row, taps k = part (mod 4); partials added in a fixed order
      for (int e4 = threadIdx.x; e4 < 4 * nr; e4 += NT) {
        const int e = e4 >> 2, part = e4 & 3;
        const int kmax = min(K - 1, N - 1 - (r0 + e));
        double acc = 0.0;
        for (int k = part; k <= kmax; k += 4) acc = fma(gl[k], hst[e + k], acc);
        pq[e][part] = acc;
      }
      __syncthreads();
    }
    const double pp = pu_p(f);
    // a true tile with fix-up steps left leaves w~ of its rows for
    // k_cells_bwd_fix (the adjoint H~ is otherwise unused without pre; tiles
    // that share rows write the same bits)
    const bool keep = K > 1 && f.has_fix && ((GI*)f.fixflag)[f.n_rt + ct];
    double* const Ht = f.Ht;
    for (int e = threadIdx.x; e < nr; e += NT) {
      double h = hst[e];
      if (K > 1) h = fma(pp, (pq[e][0] + pq[e][1]) + (pq[e][2] + pq[e][3]), (1.0 - pp) * h);
      htl[e] = h;
      if (keep) Ht[(size_t)(r0 + e) * kSP] = h;
    }
    __syncthreads();
  }
  double aA[4] = {0, 0, 0, 0}, aB[4] = {0, 0, 0, 0}, aU[4] = {0, 0, 0, 0};
  double qf[4] = {0, 0, 0, 0};  // the step test's column factors
  if (KIND != kCount)
    for (int q = 0; q < 4; ++q) qf[q] = ((GD*)f.fixq)[ct * 4 + q];
  for (int rt = rt0; rt < rt_end; ++rt) {
    const int j = rt * kRowStep + jr;
    const bool row_ok = (jr < kRowStep) && (j < N);
    const double xe = ((GD*)f.xe)[min(j, N)];
    const double lnf = KIND == kCount ? lgamma(xe + 1.0) : 0.0;
    const double pmax = KIND == kCount ? 0.0 : ((GD*)f.fixp)[rt];
    const RowQ<R> rq = load_rowq<R, KIND>(f, min(j, N - 1));
    const double w1 = (row_ok && !MV) ? (pre ? ((GD*)f.Ht)[(size_t)j * kSP] : htl[j - r0]) : 0.0;
    v4d Wm = {0, 0, 0, 0};
    if (MV) {  // wave-uniform
      GD* hr = (GD*)f.Ht + (size_t)min(j, N - 1) * kSP + g;
      const double hb0 = (row_ok && g < S) ? hr[0] : 0.0;
      const double hb1 = (row_ok && 4 + g < S) ? hr[4] : 0.0;
      const double hb2 = (row_ok && 8 + g < S) ? hr[8] : 0.0;
      const double hb3 = (row_ok && 12 + g < S) ? hr[12] : 0.0;
      Wm = mfma16(fa[0], hb0 * thv[0], Wm);
      Wm = mfma16(fa[1], hb1 * thv[1], Wm);
      Wm = mfma16(fa[2], hb2 * thv[2], Wm);
      Wm = mfma16(fa[3], hb3 * thv[3], Wm);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ct * kColTile + 4 * q + g;
      // the same steps as the forward sweep's; the others are k_cells_bwd_fix's
      const bool ok = row_ok && i < T;
      if (KIND == kCount || step_lean<R, KIND>(qf[q], pmax)) {  // wave-uniform
        const CellVal<R> ev = cell_lean<R, KIND, true>(col[q], rq, xe, lnf, ok);
        const double Wq = MV ? Wm[q] : w1 * col[q].v;
        aA[q] = fma(Wq, (double)ev.d1, aA[q]);
        aB[q] = fma(Wq, (double)ev.d2, aB[q]);
        if (!MV) aU[q] = fma(w1, ev.v, aU[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double A = sum16(aA[q]), B = sum16(aB[q]);
    const double U = MV ? 0.0 : sum16(aU[q]);
    if (jr == 0) {
      colA[wv][4 * q + g] = A;
      colB[wv][4 * q + g] = B;
      colU[wv][4 * q + g] = U;
    }
  }
  __syncthreads();
  // column totals (fixed order over the waves), times the chain factors
  if (threadIdx.x < 64) {
    double A = colA[0][c16], B = colB[0][c16];
#pragma unroll
    for (int w = 1; w < kBwdWaves; ++w) {
      A += colA[w][c16];
      B += colB[w][c16];
    }
    double v = (icol < T && qp < f.nresp) ? A * J0 + B * J1 : 0.0;
    v = sum16(v);
    if (c16 == 0) bwdpart[qp] = v;
  }
  if (!MV) {  // rate partials sum_i F^_si u_i over the tile's 16 columns
    const int s = threadIdx.x & 15, c = threadIdx.x >> 4;  // 256 threads: (column c, species s)
    const int i = ct * kColTile + c;
    double u = colU[0][c];
#pragma unroll
    for (int w = 1; w < kBwdWaves; ++w) u += colU[w][c];
    rsum[c][s] = (i < T && s < S) ? F64[(size_t)i * kSP + s] * u : 0.0;
    __syncthreads();
    if (threadIdx.x < kSP) {
      double a = 0.0;
      for (int cc = 0; cc < 16; ++cc) a += rsum[cc][threadIdx.x];
      bwdpart[4 + threadIdx.x] = a;
    }
  } else if (threadIdx.x < kSP) {
    bwdpart[4 + threadIdx.x] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Fix-up sweeps: the wave steps the sweeps above leave (step_lean false: some
// lane of the wave not a single quadrature interval), with the general cell:
// composite quadrature, or the CDF at the bin's edges.  An entry is one such
// step; the fix-up sweeps find them by the same test on the same operands
// (k_colparams' column factors and the row tiles' half-widths).  Launched
// after the main sweep (use_flags), a block first reads the flag the forward
// sweep set for its tile and leaves at once when nothing is left there (a
// graph branch beside the main sweep was measured to cost as much in
// cross-queue synchronisation as it hid).  Each block lists
// the entries of its tile in a fixed order, its waves take every NW-th entry
// (the forward spreads a reco tile over kFixSplit blocks, which take turns),
// and the sums over the waves and blocks are added in a fixed order, so these
// partials do not depend on the launch either.  In the 3000 x 900 generalized-gamma sweep
// they are about 0.4 % of the wave steps: the reco bin from x <= 0 (its cell
// the CDF at x_1) and wide low-energy bins against narrow columns.

constexpr int kFixWaves = 8;     // waves per forward fix-up block
constexpr int kBwdFixWaves = 4;  // waves per backward fix-up block (a true tile has few entries:
                                 // idle waves would only hold a CU's registers)

// Compacts the entries with want = true of one chunk of NW * 64 candidates
// (candidate c at thread c) into list[], in candidate order; returns their
// count.  Called by the whole block.
template <int NW>
__device__ __forceinline__ int fix_compact(bool want, int value, int* list, int* wcount) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned long long m = __ballot(want);
  if (lane == 0) wcount[wv] = __popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < NW; ++w) {
    off += w < wv ? wcount[w] : 0;
    tot += wcount[w];
  }
  if (want) list[off + __popcll(m & ((1ull << lane) - 1ull))] = value;
  __syncthreads();
  return tot;
}

// Column i's constants as the sweeps hold them (i >= T: those of column T - 1
// with a zero contraction weight; the cell is masked by the caller).
// v: forward MV F^[i, jr]; otherwise the single-histogram v_i, and (backward
// MV) zero.
template <class R, int KIND>
__device__ __forceinline__ ColPre<R> fix_col(const FitDev& f, int i, double vmv, bool mv) {
  GColPar& cpi = ((GColPar*)f.cp)[i < f.T ? i : f.T - 1];
  ColPre<R> c;
  c.cp = &cpi;
  c.c0 = cpi.c0;
  c.c1 = KIND == kGauss ? cpi.c1 : cpi.c1 * cpi.f64[3];
  if (KIND != kGauss) {
#pragma unroll
    for (int u = 0; u < 8; ++u) c.s[u] = sizeof(R) == 4 ? (R)cpi.f32[u] : (R)cpi.f64[u];
  }
  c.v = i >= f.T ? 0.0 : mv ? vmv : cpi.v;
  return c;
}

// Block (reco tile rt, share b < kFixSplit).  Candidates: (true tile, step)
// pairs in order; writes share b of rt's rows of Mfix (zeros where nothing is
// left).
template <class R, int KIND, bool MV>
__global__ void __launch_bounds__(kFixWaves * 64) k_cells_fwd_fix(const FitDev* fits, const int* active,
                                                                   int use_flags, int nsplit) {
  constexpr int NW = kFixWaves, NTH = NW * 64;
  typedef typename std::conditional<MV, v4d, double>::type V;
  constexpr int NR = MV ? 4 : 1;
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int rt = fb2.x / nsplit, sh = fb2.x % nsplit;
  // block-uniform; nothing left in this reco tile: its shares of Mfix are not read
  if (rt >= f.n_rt || f.vsum == (int)MV || (use_flags && ((GI*)f.fixflag)[rt] == 0)) return;
  __shared__ int list[NTH], wcount[NW];
  __shared__ double part[NW][NR][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, jr = lane & 15, g = lane >> 4;
  const int T = f.T, N = f.N, n_ct = f.n_ct, j0 = rt * kRowStep;
  GD* const F64 = (GD*)f.F64;
  GI* const tbp = (GI*)f.tb;
  GD* const fixq = (GD*)f.fixq;
  const double pmax = ((GD*)f.fixp)[rt];
  const bool row_ok = (jr < kRowStep) && (j0 + jr < N);
  const double xe = ((GD*)f.xe)[min(j0 + jr, N)];
  const RowQ<R> rq = load_rowq<R, KIND>(f, min(j0 + jr, N - 1));
  const bool zrow = KIND == kGG && row_ok && j0 + jr == f.row0;  // the bin from x <= 0
  // logical share ls takes the entries e = ls NW + wv (mod kFixSplit NW),
  // whatever the number of blocks that run the shares (same sums either way)
  for (int ls = sh; ls < kFixSplit; ls += nsplit) {
    V acc = {};
    for (int c0 = 0; c0 < 4 * n_ct; c0 += NTH) {
      const int cand = c0 + (int)threadIdx.x, ct = cand >> 2;
      bool want = false;
      if (ct < n_ct) {
        const int bx = tbp[2 * ct], by = tbp[2 * ct + 1];
        // a tile the forward sweep lists for this reco tile, and a step it leaves
        if (by >= bx && !(by < j0 || bx > j0 + kRowStep - 1)) want = !step_lean<R, KIND>(fixq[cand], pmax);
      }
      const int n = fix_compact<NW>(want, cand, list, wcount);
      for (int e = ls * NW + wv; e < n; e += kFixSplit * NW) {
        const int ent = list[e];
        const int i = (ent >> 2) * kColTile + 4 * (ent & 3) + g;
        const ColPre<R> c = fix_col<R, KIND>(f, i, MV && i < T ? F64[i * kSP + jr] : 0.0, MV);
        const CellVal<R> ev = cell_general<R, KIND, false>(c, rq, xe, row_ok && i < T, zrow);
        if constexpr (MV) acc = mfma16(ev.v, c.v, acc);
        else acc = fma(ev.v, c.v, acc);
      }
      __syncthreads();  // list[] is rewritten by the next chunk
    }
    if constexpr (MV) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part[wv][r][lane] = acc[r];
    } else {
      part[wv][0][lane] = acc;
    }
    __syncthreads();
    if (wv == 0) {
      if constexpr (MV) {
        double* const out = f.Mfix + (size_t)ls * N * kSP;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double x = part[0][r][lane];
          for (int w = 1; w < NW; ++w) x += part[w][r][lane];
          const int row = g + 4 * r;  // FP64 MFMA result layout: row l/16 + 4r, column l%16
          if (row < kRowStep && j0 + row < N) out[(size_t)(j0 + row) * kSP + jr] = x;
        }
      } else {
        double x = part[0][0][lane];
        for (int w = 1; w < NW; ++w) x += part[w][0][lane];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (g == 0 && row_ok) f.Mfix[(size_t)ls * N + j0 + jr] = x;
      }
    }
    __syncthreads();  // part[] is rewritten by the next share
  }
}

// Block = true tile ct.  Candidates: (reco tile of ct's support, step) pairs
// in order; a wave forms its entry's weights as the backward sweep does (a
// single histogram's w~ with pile-up as k_cells_bwd left it in H~) and
// evaluates the step.  Writes bwdfix[ct] (zeros where nothing is left).
template <class R, int KIND, bool MV>
__device__ __forceinline__ void bwd_fix_tile(const FitDev& f, int ct, int pre) {
  constexpr int NW = kBwdFixWaves, NTH = NW * 64;
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  __shared__ int list[NTH], wcount[NW];
  __shared__ double colA[NW][16], colB[NW][16], colU[NW][16];
  __shared__ double rsum[16][kSP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, jr = lane & 15, g = lane >> 4;
  const int T = f.T, N = f.N, S = f.S, n_ct = f.n_ct;
  GColPar* const cpar = (GColPar*)f.cp;
  GD* const F64 = (GD*)f.F64;
  GD* const fixp = (GD*)f.fixp;
  double* const out = f.bwdfix + (size_t)ct * kBwdPart;
  const int bx = ((GI*)f.tb)[2 * ct], by = ((GI*)f.tb)[2 * ct + 1];  // support [bx, by]
  const int rt_a = by >= bx ? max(bx, 0) / kRowStep : 0;
  const int rt_b = by >= bx ? min(by / kRowStep, f.n_rt - 1) : -1;
  double fa[4] = {0, 0, 0, 0}, thv[4] = {0, 0, 0, 0};
  if (MV) {  // F operands of the weights (lane: column lane%16, species 4 kb + lane/16)
    const int i = ct * kColTile + jr;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int s = 4 * kb + g;
      fa[kb] = (i < T && s < S) ? F64[(size_t)i * kSP + s] : 0.0;
      thv[kb] = s < S ? ((GD*)f.theta)[s] : 0.0;
    }
  }
  // w~ (single histogram): H~ with pile-up (k_adjoint1 or k_cells_bwd wrote it), else H
  GD* const wsrc = (GD*)(pre || pu_len(f) > 1 ? f.Ht : f.H);
  // the tail's factors, in flight with the entries: chain factors (threads
  // < 64: column c16, parameter qp) and spectra (column t / 16, species t % 16)
  const int c16 = threadIdx.x & 15, qp = (threadIdx.x >> 4) & 3;
  const int icol = ct * kColTile + c16;
  double J0 = 0.0, J1 = 0.0, Fs = 0.0;
  if (threadIdx.x < 64 && icol < T && qp < f.nresp) {
    J0 = cpar[icol].J[0][qp];
    J1 = cpar[icol].J[1][qp];
  }
  if (!MV && threadIdx.x < 256) {
    const int s = threadIdx.x & 15, i = ct * kColTile + (threadIdx.x >> 4);
    Fs = (i < T && s < S) ? F64[(size_t)i * kSP + s] : 0.0;
  }
  double aA[4] = {0, 0, 0, 0}, aB[4] = {0, 0, 0, 0}, aU[4] = {0, 0, 0, 0};
  const int ncand = 4 * (rt_b - rt_a + 1);
  for (int c0 = 0; c0 < ncand; c0 += NTH) {
    const int cand = c0 + (int)threadIdx.x, rt = rt_a + (cand >> 2);
    const bool want = cand < ncand && !step_lean<R, KIND>(((GD*)f.fixq)[ct * 4 + (cand & 3)], fixp[rt]);
    const int n = fix_compact<NW>(want, cand, list, wcount);
    for (int e = wv; e < n; e += NW) {
      const int ent = list[e], qe = ent & 3;
      const int j = (rt_a + (ent >> 2)) * kRowStep + jr;
      const bool row_ok = (jr < kRowStep) && (j < N);
      const double xe = ((GD*)f.xe)[min(j, N)];
      const RowQ<R> rq = load_rowq<R, KIND>(f, min(j, N - 1));
      const int i = ct * kColTile + 4 * qe + g;
      const ColPre<R> c = fix_col<R, KIND>(f, i, 0.0, MV);
      double Wq;
      double w1 = 0.0;
      if (MV) {  // W for the 16 columns of the tile (wave-uniform), then the lane's column 4 qe + g
        v4d Wm = {0, 0, 0, 0};
        GD* hr = (GD*)f.Ht + (size_t)min(j, N - 1) * kSP + g;
        const double hb0 = (row_ok && g < S) ? hr[0] : 0.0;
        const double hb1 = (row_ok && 4 + g < S) ? hr[4] : 0.0;
        const double hb2 = (row_ok && 8 + g < S) ? hr[8] : 0.0;
        const double hb3 = (row_ok && 12 + g < S) ? hr[12] : 0.0;
        Wm = mfma16(fa[0], hb0 * thv[0], Wm);
        Wm = mfma16(fa[1], hb1 * thv[1], Wm);
        Wm = mfma16(fa[2], hb2 * thv[2], Wm);
        Wm = mfma16(fa[3], hb3 * thv[3], Wm);
        Wq = qe == 0 ? Wm[0] : qe == 1 ? Wm[1] : qe == 2 ? Wm[2] : Wm[3];
      } else {
        if (row_ok) w1 = wsrc[(size_t)j * kSP];
        Wq = w1 * c.v;
      }
      const CellVal<R> ev = cell_general<R, KIND, true>(c, rq, xe, row_ok && i < T, KIND == kGG && j == f.row0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q != qe) continue;  // wave-uniform
        aA[q] = fma(Wq, (double)ev.d1, aA[q]);
        aB[q] = fma(Wq, (double)ev.d2, aB[q]);
        if (!MV) aU[q] = fma(w1, ev.v, aU[q]);
      }
    }
    __syncthreads();  // list[] is rewritten by the next chunk
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double A = sum16(aA[q]), B = sum16(aB[q]);
    const double U = MV ? 0.0 : sum16(aU[q]);
    if (jr == 0) {
      colA[wv][4 * q + g] = A;
      colB[wv][4 * q + g] = B;
      colU[wv][4 * q + g] = U;
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // column totals (fixed order over the waves), times the chain factors
    double A = colA[0][c16], B = colB[0][c16];
    for (int w = 1; w < NW; ++w) {
      A += colA[w][c16];
      B += colB[w][c16];
    }
    double v = (icol < T && qp < f.nresp) ? A * J0 + B * J1 : 0.0;
    v = sum16(v);
    if (c16 == 0) out[qp] = v;
  }
  if (!MV) {  // rate partials sum_i F^_si u_i over the tile's 16 columns
    static_assert(NTH >= 256, "one thread per (column, species)");
    if (threadIdx.x < 256) {
      const int s = threadIdx.x & 15, c = threadIdx.x >> 4;
      const int i = ct * kColTile + c;
      double u = colU[0][c];
      for (int w = 1; w < NW; ++w) u += colU[w][c];
      rsum[c][s] = (i < T && s < S) ? Fs * u : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < kSP) {
      double a = 0.0;
      for (int cc = 0; cc < 16; ++cc) a += rsum[cc][threadIdx.x];
      out[4 + threadIdx.x] = a;
    }
  } else if (threadIdx.x < kSP) {
    out[4 + threadIdx.x] = 0.0;
  }
}

template <class R, int KIND, bool MV>
__global__ void __launch_bounds__(kBwdFixWaves * 64) k_cells_bwd_fix(const FitDev* fits, const int* active, int pre,
                                                                   int use_flags) {
  const int2 fb2 = fit_block();
  const FitDev& f = fits[active ? active[fb2.y] : fb2.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  const int ct = fb2.x;
  // block-uniform; nothing left in this true tile: its partials are not read
  if (ct >= f.n_ct || f.mv != (int)MV || (use_flags && f.fixflag[f.n_rt + ct] == 0)) return;
  bwd_fix_tile<R, KIND, MV>(f, ct, pre);
}

// ---------------------------------------------------------------------------
// Fixed-order sums of the per-block partials into out[].  The partials other
// than the backward fix-up sweep's are split into kFinBlocks logical blocks
// of kFinThreads threads, each summing a fixed share of every kind of partial
// into a row (wave sums in lane order, the block's waves in order).  The
// finish adds the rows in block order and then the fix-up sweep's partials
// of the true tiles with steps left (per column: runs of tiles in tile order,
// then the runs in order; tile t + 256 m at thread t), and writes the
// results.  A single
// fit runs its logical blocks as workgroups of their own (spread over many
// CUs, the partials stream in at the rate of many CUs, where one workgroup
// would wait on its own few outstanding loads): with the gradient inside the
// backward fix-up sweep's launch, beside its true tiles, else in k_final;
// the workgroup counted last on a device-scope counter finishes.  A launch of
// many fits runs one 1024-thread workgroup per fit, four logical blocks at a
// time, with the rows in LDS.  The arithmetic, and so every bit, is the same
// in each of these forms.
__device__ __forceinline__ double sum64(double x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ int or64(int x) {
  for (int o = 32; o >= 1; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

constexpr int kFinA = 7;  // sums per row before the flags: NLL, 4 response-parameter
                          // gradients, pile-up-fraction gradient, table-coordinate gradient
constexpr int kFinFixParts = 12;  // runs of tiles of the fix-up partials' sums (x kBwdPart threads)
constexpr int kFinFixRun = (kFinThreads + kFinFixParts - 1) / kFinFixParts;
static_assert(kFinFixParts * kBwdPart <= kFinThreads, "one thread per (run, column)");

// LDS of the final sums in a workgroup of PT threads.
template <int PT>
struct FinLds {
  double wred[PT / 64][kFinA + kSP];
  int wflag[PT / 64];
  double rowl[kFinBlocks][kFinRow];  // the rows (one workgroup per fit)
  double fx[kFinThreads][kBwdPart + 1];  // the fix-up partials by tile (odd stride: no bank conflicts)
  double fpsum[kFinFixParts][kBwdPart];  // their sums over kFinFixParts runs of tiles
  int last;
};

// The rows of logical blocks lb = lb0 + p (PT / kFinThreads) + t / kFinThreads,
// p < npass, to fpart (each writing wave fences its row) or to L.rowl.
template <int PT>
__device__ __forceinline__ void fin_rows(const FitDev& f, int with_grad, int lb0, int npass, bool global,
                                         FinLds<PT>& L) {
  constexpr int NT = kFinThreads, G = NT * kFinBlocks, NA = kFinA, LPB = PT / NT;
  static_assert(PT % NT == 0, "whole logical blocks per workgroup");
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  // every field used is read into registers before the first store (a store
  // through a generic pointer could alias f and force reloads after it)
  const int n_rowblk = f.n_rowblk, n_cpblk = f.n_cpblk, n_bwdblk = f.n_bwdblk, N = f.N;
  const int pu_float = f.pu_float, vsum = f.vsum;
  const bool tab = f.kind == kTable && f.nresp > 0;
  const bool jt = f.mv && f.joint;
  GD* const nllpart = (GD*)f.nllpart;
  GI* const flagpart = (GI*)f.flagpart;
  GD* const ppart = (GD*)f.ppart;
  GD* const tpart = (GD*)f.tpart;
  GI* const cpflag = (GI*)f.cpflag;
  GD* const bwdpart = (GD*)f.bwdpart;
  GD* const gpart = (GD*)f.gpart;
  GD* const jnll = (GD*)f.jnll;
  GI* const jflag = (GI*)f.jflag;
  GD* const jpp = (GD*)f.jpp;
  GD* const jtp = (GD*)f.jtp;
  GD* const jg = (GD*)f.jg;
  double* const fpart = f.fpart;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // In rounds: every load of a round is issued before any of its values is
  // added, so a round costs one memory round trip (the 3000 x 900 fit needs
  // one).  Thread gt of the G threads takes, per round, the row and
  // cell-parameter partials b = gt + G r, UQ backward blocks' response parts
  // and, for species s = gt % 16, UR blocks' rate parts (or the row blocks'
  // species sums).  Sums within a round are pairwise in a fixed order, rounds
  // are added in order.
  constexpr int ST = G / 16, UQ = 2, UR = 4;
  const bool wg = with_grad != 0;
  const int nA = max(max(n_rowblk, n_cpblk), jt ? N : 0);
  const int nQ = wg ? n_bwdblk : 0;
  const int nR = vsum ? (wg ? n_bwdblk : 0) : n_rowblk;
  const int rounds = max(max((nA + G - 1) / G, (nQ + UQ * G - 1) / (UQ * G)), (nR + UR * ST - 1) / (UR * ST));
  for (int pass = 0; pass < npass; ++pass) {
    const int lb = lb0 + pass * LPB + t / NT;  // logical block, its thread gt
    const int gt = lb * NT + (t & (NT - 1));
    const int sp = gt & 15, tb = gt >> 4;
    double acc[NA] = {0, 0, 0, 0, 0, 0, 0};
    int fl = 0;
    double gr = 0.0;
    for (int r = 0; r < rounds; ++r) {
      const int b = gt + G * r;
      const bool inR = b < n_rowblk, inJ = jt && b < N;
      const double x0 = inR ? nllpart[b] : 0.0;
      const int xf = inR ? flagpart[b] : 0;
      const double x5 = inR && pu_float && wg ? ppart[b] : 0.0;
      const double x6 = inR && tab && wg ? tpart[b] : 0.0;
      const int xc = b < n_cpblk ? cpflag[b] : 0;
      const double y0 = inJ ? jnll[b] : 0.0;
      const int yf = inJ ? jflag[b] : 0;
      const double y5 = inJ && pu_float && wg ? jpp[b] : 0.0;
      const double y6 = inJ && tab && wg ? jtp[b] : 0.0;
      double qv[UQ][4], rv[UR];
#pragma unroll
      for (int u = 0; u < UQ; ++u) {
        const int bb = gt + G * (UQ * r + u);
#pragma unroll
        for (int q = 0; q < 4; ++q) qv[u][q] = bb < nQ ? bwdpart[(size_t)bb * kBwdPart + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int bb = tb + ST * (UR * r + u);
        rv[u] = bb >= nR ? 0.0 : vsum ? bwdpart[(size_t)bb * kBwdPart + 4 + sp] : gpart[bb * kSP + sp];
      }
      acc[0] += x0 + y0;
      fl |= xf | xc | yf;
      acc[5] += x5 + y5;
      acc[6] += x6 + y6;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = qv[0][q];
#pragma unroll
        for (int u = 1; u < UQ; ++u) v += qv[u][q];
        acc[1 + q] += v;
      }
#pragma unroll
      for (int h = 1; h < UR; h *= 2)
#pragma unroll
        for (int u = 0; u + h < UR; u += 2 * h) rv[u] += rv[u + h];
      gr += rv[0];
    }
    if (jt && wg)  // the joint term's species sums, one per reco row
      for (int b = tb; b < N; b += ST) gr += jg[b * kSP + sp];
    gr += __shfl_xor(gr, 16, 64);
    gr += __shfl_xor(gr, 32, 64);
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = sum64(acc[q]);
    fl = or64(fl);
    if (lane == 0) {
      for (int q = 0; q < NA; ++q) L.wred[w][q] = acc[q];
      L.wflag[w] = fl;
    }
    if (lane < kSP) L.wred[w][NA + lane] = gr;
    __syncthreads();
    // the first wave of each logical block forms its row (lane c: column c,
    // summed over the block's waves in order; column NA holds the flags)
    if ((w & (NT / 64 - 1)) == 0) {
      double v = 0.0;
      if (lane < kFinRow && lane != NA) {
        const int col = lane < NA ? lane : lane - 1;
        v = L.wred[w][col];
        for (int u = 1; u < NT / 64; ++u) v += L.wred[w + u][col];
      }
      int fw = 0;
      for (int u = 0; u < NT / 64; ++u) fw |= L.wflag[w + u];
      if (lane == NA) v = (double)fw;
      if (lane < kFinRow) {
        if (global) fpart[lb * kFinRow + lane] = v;
        else L.rowl[lb][lane] = v;
      }
      if (global) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the row, device-wide
    }
    __syncthreads();  // wred[] is rewritten by the next pass
  }
}

// Counts the workgroup done (every wave that stored what the finish reads
// has fenced it device-wide, release); true in the workgroup counted last of
// `target`, which then sees every counted workgroup's stores (acquire).
template <int PT>
__device__ __forceinline__ bool fin_count(int* fcount, int target, FinLds<PT>& L) {
  __syncthreads();
  if (threadIdx.x == 0)
    L.last = __hip_atomic_fetch_add(fcount, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == target - 1;
  __syncthreads();
  const bool last = L.last != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// The finish, by a whole workgroup of PT >= 256 threads (rows from fpart or
// L.rowl).
template <int PT>
__device__ __forceinline__ void fin_finish(const FitDev& f, int with_grad, bool global, FinLds<PT>& L) {
  constexpr int NB = kFinBlocks, NA = kFinA;
  static_assert(PT >= kFinThreads, "the fix-up partials' tree needs 256 threads");
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  typedef __attribute__((address_space(1))) double GDw;
  const int S = f.S, P = f.P, nresp = f.nresp, pu_float = f.pu_float, n_ct = f.n_ct, n_rt = f.n_rt;
  const bool tab = f.kind == kTable && f.nresp > 0;
  const bool rad = f.mv && f.n_rad > 0 && !f.joint;
  const bool fixg = f.has_fix && with_grad;
  GI* const fixflag = (GI*)f.fixflag;
  GD* const bwdfix = (GD*)f.bwdfix;
  GD* const rad_out = (GD*)f.rad_out;
  GD* const rows = (GD*)f.fpart;
  GDw* const out = (GDw*)f.out;
  int* const fcount = f.fcount;
  double* const out_host = f.out_host;
  const double* const theta = f.theta;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // every load first: the rows (wave 0, lane c < kFinRow: column c of every
  // row), the radial parts, the caller's sequence number and the fix-up
  // partials (threads < 256: tiles t + 256 m)
  double x[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u)
    x[u] = (w == 0 && lane < kFinRow) ? (global ? rows[u * kFinRow + lane] : L.rowl[u][lane]) : 0.0;
  double rad_g = 0.0, rad_nll = 0.0, rad_fl = 0.0, rad_p = 0.0, rad_t = 0.0, seq = 0.0;
  if (rad && w == 0) {
    if (lane < S) rad_g = rad_out[2 + 16 + lane];
    if (lane == 0) {
      rad_nll = rad_out[0];
      rad_fl = rad_out[1];
      rad_p = rad_out[2 + 32];
      rad_t = rad_out[2 + 33];
    }
  }
  if (out_host && t == 0) seq = theta[P];
  double fq[kBwdPart];
  const bool f0 = fixg && t < kFinThreads && t < n_ct;
  const int fl0 = f0 ? fixflag[n_rt + t] : 0;
#pragma unroll
  for (int c = 0; c < kBwdPart; ++c)  // whatever the flag (a tile without steps left holds stale values)
    fq[c] = f0 ? bwdfix[(size_t)t * kBwdPart + c] : 0.0;
  if (!fl0) {
#pragma unroll
    for (int c = 0; c < kBwdPart; ++c) fq[c] = 0.0;
  }
  if (fixg && t < kFinThreads)
    for (int ct = t + kFinThreads; ct < n_ct; ct += kFinThreads)
      if (fixflag[n_rt + ct]) {
#pragma unroll
        for (int c = 0; c < kBwdPart; ++c) fq[c] += bwdfix[(size_t)ct * kBwdPart + c];
      }
  if (fixg) {  // block-uniform: the fix-up partials through LDS, by column over runs of tiles
    if (t < kFinThreads) {
#pragma unroll
      for (int c = 0; c < kBwdPart; ++c) L.fx[t][c] = fq[c];
    }
    __syncthreads();
    if (t < kFinFixParts * kBwdPart) {
      const int c = t / kFinFixParts, part = t % kFinFixParts;
      const int k0 = part * kFinFixRun, k1 = min(k0 + kFinFixRun, kFinThreads);
      double a = 0.0;
      for (int k = k0; k < k1; ++k) a += L.fx[k][c];
      L.fpsum[part][c] = a;
    }
    __syncthreads();
  }
  if (w != 0) return;
  double v = 0.0;
  int fv = 0;
  if (lane == NA) {
#pragma unroll
    for (int u = 0; u < NB; ++u) fv |= (int)x[u];
  } else if (lane < kFinRow) {
    v = x[0];
#pragma unroll
    for (int u = 1; u < NB; ++u) v += x[u];
    // row columns 1-4 (response parameters) and 8-23 (rates) take the fix-up
    // partials' columns 0-3 and 4-19
    const int fc = lane >= 1 && lane <= 4 ? lane - 1 : lane >= NA + 1 ? lane - NA - 1 + 4 : -1;
    if (fixg && fc >= 0) {
      double s = L.fpsum[0][fc];
      for (int u = 1; u < kFinFixParts; ++u) s += L.fpsum[u][fc];
      v += s;
    }
  }
  if (global && lane == 0) *fcount = 0;  // for the next launch (the stage timer repeats a launch alone)
  double tot[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) tot[q] = __shfl(v, q, 64);
  int flags = __shfl(fv, NA, 64);
  const double gs = __shfl(v, (NA + 1 + lane) & 63, 64);  // the rate gradient of species `lane`
  // results go to f.out and, when set, straight into the caller's pinned
  // host buffer as well (no separate copy node)
  if (lane < S) {
    const double a = rad ? gs + rad_g : gs;
    out[1 + lane] = a;
    if (out_host) out_host[1 + lane] = a;
  }
  if (lane == 0) {
    double pg = tot[5];  // dNLL/dp: row terms, then the radial term
    if (rad) pg += rad_p;
    if (tab) {  // the table coordinate takes the response gradient's place
      tot[1] = tot[6];
      if (rad) tot[1] += rad_t;
    }
    double nll = tot[0];
    if (rad) {
      nll += rad_nll;
      flags |= (int)rad_fl;
    }
    // a zero-width Gaussian column leaves the NLL defined but not its
    // gradient: with the gradient requested it is a domain error like the
    // others (+inf in out[0], which is all the device-pointer entry point hands
    // back)
    if (!with_grad) flags &= ~kZeroWidth;
    const double v0 = flags ? INFINITY : nll;
    out[0] = v0;
    out[1 + P] = (double)flags;
#pragma unroll
    for (int q = 0; q < kMaxResp; ++q)  // static indices keep tot[] in registers
      if (q < nresp) out[1 + S + q] = with_grad ? tot[1 + q] : 0.0;
    if (pu_float) out[P] = with_grad ? pg : 0.0;
    if (out_host) {
      out_host[0] = v0;
      out_host[1 + P] = (double)flags;
#pragma unroll
      for (int q = 0; q < kMaxResp; ++q)
        if (q < nresp) out_host[1 + S + q] = with_grad ? tot[1 + q] : 0.0;
      if (pu_float) out_host[P] = with_grad ? pg : 0.0;
    }
  }
  if (out_host) {  // then the completion mark the caller spins on (all writers are in this wave)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the results before the mark
    if (lane == 0) {
      out_host[2 + P] = seq;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    }
  }
}

template <int PT>  // threads per workgroup: kFinThreads (kFinBlocks workgroups per fit) or 1024 (one)
__global__ void __launch_bounds__(PT) k_final(const FitDev* fits, const int* active, int with_grad) {
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  __shared__ FinLds<PT> L;
  if (PT == kFinThreads) {  // one logical block per workgroup
    fin_rows<PT>(f, with_grad, blockIdx.x, 1, true, L);
    if (!fin_count<PT>(f.fcount, kFinBlocks, L)) return;
    fin_finish<PT>(f, with_grad, true, L);
  } else {
    fin_rows<PT>(f, with_grad, 0, kFinBlocks / (PT / kFinThreads), false, L);
    fin_finish<PT>(f, with_grad, false, L);
  }
}

// Few fits: kFinBlocks workgroups each; many: one 1024-thread workgroup each.
static void launch_final(const FitDev* d_fits, const int* d_active, int n, bool with_grad, hipStream_t st) {
  if (n < 8)
    hipLaunchKernelGGL(k_final<kFinThreads>, dim3(kFinBlocks, n), dim3(kFinThreads), 0, st, d_fits, d_active,
                       with_grad ? 1 : 0);
  else
    hipLaunchKernelGGL(k_final<1024>, dim3(1, n), dim3(1024), 0, st, d_fits, d_active, with_grad ? 1 : 0);
}

// One fit's backward fix-up sweep and final sums in one launch: workgroups
// ct < n_ct as k_cells_bwd_fix, the kFinBlocks after them one logical block
// of the final sums each; the workgroup counted last finishes.
template <class R, int KIND, bool MV>
__global__ void __launch_bounds__(kBwdFixWaves * 64) k_cells_bwd_fix_final(const FitDev* fits, const int* active,
                                                                         int pre) {
  constexpr int NTH = kBwdFixWaves * 64, LPB = NTH / kFinThreads;
  static_assert(kFinBlocks % LPB == 0, "whole workgroups of logical blocks");
  const FitDev& f = fits[active ? active[0] : 0];
  if (f.skip) return;  // uniform: a device-minimised fit that has finished
  __shared__ FinLds<NTH> L;
  const int b = blockIdx.x, n_ct = f.n_ct;
  if (b >= n_ct) {
    fin_rows<NTH>(f, 1, (b - n_ct) * LPB, 1, true, L);
  } else if (f.mv == (int)MV && f.fixflag[f.n_rt + b]) {
    bwd_fix_tile<R, KIND, MV>(f, b, pre);
    if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // wave 0 wrote the partials
  }
  if (!fin_count<NTH>(f.fcount, n_ct + kFinBlocks / LPB, L)) return;
  fin_finish<NTH>(f, 1, true, L);
}

template <class R, int KIND>
static void launch_bwd_fix_final(bool mv, int n_ct, hipStream_t st, const FitDev* d_fits, const int* d_active,
                                 int pre) {
  const dim3 g(n_ct + kFinBlocks / (kBwdFixWaves * 64 / kFinThreads)), b(kBwdFixWaves * 64);
  if (mv) hipLaunchKernelGGL((k_cells_bwd_fix_final<R, KIND, true>), g, b, 0, st, d_fits, d_active, pre);
  else hipLaunchKernelGGL((k_cells_bwd_fix_final<R, KIND, false>), g, b, 0, st, d_fits, d_active, pre);
}

// Joint energy x radius x pulse-shape term (the alternative to the additive
// terms) of reco row j: lambda_jkl = sum_s c_s rho_sk T_sl with
// c_s = M'_js (1 - t_s) r_s over the n_rad x n_ps bins of the row.  The
// expected counts of a row sum to sum_s c_s sigma_s, sigma_s =
// (sum_k rho_sk)(sum_l T_sl), so the Poisson NLL sum_kl (lambda - n ln lambda)
// and G_s = dNLL/dc_s = sigma_s - sum_kl (n / lambda) rho_sk T_sl need the
// logarithm and the ratio at the bins with counts only: the histogram is held
// as the list of its non-zero bins per row.  With every c_s >= 0 (the
// templates are >= 0) no bin can have lambda < 0; otherwise the whole row is
// scanned for the domain check.  kJointWPR waves share a row (entries
// round-robin over their lanes), then fixed-order sums.  The term's part of
// H_js = dNLL/d(r_s M'_js), (1 - t_s) G_s, is added to H (k_rowterms wrote
// the tagged part) before the adjoint and the backward sweep read it; the
// row's NLL, flags and the rate, pile-up and table-coordinate gradient parts
// go to per-row partials.
constexpr int kJointBlock = 256;
constexpr int kJointWPR = 2;                                       // waves per row
constexpr int kJointRows = kJointBlock / 64 / kJointWPR;           // rows per block
template <bool D>
__global__ void __launch_bounds__(kJointBlock) k_joint(const FitDev* fits, const int* active) {
  typedef __attribute__((address_space(1))) const double GD;
  typedef __attribute__((address_space(1))) const int GI;
  typedef __attribute__((address_space(1))) const uint32_t GU;
  const FitDev& f = fits[active ? active[blockIdx.y] : blockIdx.y];
  if (f.skip) return;  // block-uniform: a batched fit whose minimiser has finished
  if (!f.mv || !f.joint || (int)blockIdx.x * kJointRows >= f.N) return;  // block-uniform
  constexpr int NW = kJointBlock / 64;
  // rows of 18 doubles (144 B): lanes reading different radial or pulse-shape
  // bins start 4 banks apart
  __shared__ __align__(16) double Rk[128][kSP + 2];
  __shared__ __align__(16) double Tl[64][kSP + 2];
  __shared__ double wsum[NW][kSP + 2], hs[kJointRows][kSP], ht[kJointRows][kSP];
  __shared__ int wfl[NW];
  const int nr = f.n_rad, np = f.n_ps, S = f.S;
  // every field used is read into registers before the first store (a store
  // through a generic pointer could alias f and force reloads after it)
  typedef __attribute__((address_space(1))) double GDw;
  typedef __attribute__((address_space(1))) int GIw;
  const int N = f.N, win_lo = f.win_lo, win_hi = f.win_hi, pu_float = f.pu_float;
  const bool tab = f.kind == kTable && f.nresp > 0;
  GD* const Mp = (GD*)f.Mp;
  GD* const tag = (GD*)f.tag;
  GD* const th = (GD*)f.theta;
  GD* const jsig = (GD*)f.jsig;
  GD* const Dp = (GD*)f.Dp;
  GD* const Dtp = (GD*)f.Dtp;
  GD* const rad = (GD*)f.rad;
  GD* const pst = (GD*)f.pst;
  GI* const jrow = (GI*)f.jrow;
  GU* const jent = (GU*)f.jent;
  GD* const jval = (GD*)f.jval;
  GDw* const H = (GDw*)f.H;
  GDw* const jg = (GDw*)f.jg;
  GDw* const jnll = (GDw*)f.jnll;
  GIw* const jflag = (GIw*)f.jflag;
  GDw* const jpp = (GDw*)f.jpp;
  GDw* const jtp = (GDw*)f.jtp;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int r = w / kJointWPR, sub = w - r * kJointWPR;
  const int j = blockIdx.x * kJointRows + r;
  const bool inwin = j < N && j >= win_lo && j < win_hi;
  // the row's coefficients and first entries are loaded before the staging
  double c[kSP];
#pragma unroll
  for (int s = 0; s < kSP; ++s)
    c[s] = (inwin && s < S) ? Mp[j * kSP + s] * (1.0 - tag[s]) * th[s] : 0.0;
  const int e0 = inwin ? jrow[j] : 0, e1 = inwin ? jrow[j + 1] : 0;
  int e = e0 + sub * 64 + lane;
  uint32_t bn = 0;
  double nn = 0.0;
  if (e < e1) {
    bn = jent[e];
    nn = jval[e];
  }
  for (int x = t; x < kSP * 128; x += kJointBlock) {
    const int s = x >> 7, k = x & 127;
    if (k < nr) Rk[k][s] = s < S ? rad[s * nr + k] : 0.0;
  }
  for (int x = t; x < kSP * 64; x += kJointBlock) {
    const int s = x >> 6, l = x & 63;
    if (l < np) Tl[l][s] = s < S ? pst[s * np + l] : 0.0;
  }
  bool dense = false;
  double mu = 0.0;  // sum_kl lambda_jkl = sum_s c_s sigma_s
#pragma unroll
  for (int s = 0; s < kSP; ++s) {
    dense |= !(c[s] >= 0.0) || !isfinite(c[s]);
    mu += c[s] * jsig[s];
  }
  __syncthreads();
  double term = 0.0, A[kSP];
#pragma unroll
  for (int s = 0; s < kSP; ++s) A[s] = 0.0;
  int bad = 0;
  for (; e < e1; e += 64 * kJointWPR) {
    const uint32_t b = bn;
    const double n = nn;  // > 0
    if (e + 64 * kJointWPR < e1) {  // next entry in flight
      bn = jent[e + 64 * kJointWPR];
      nn = jval[e + 64 * kJointWPR];
    }
    const double2* rk = (const double2*)&Rk[b >> 16][0];
    const double2* tl = (const double2*)&Tl[b & 0xffff][0];
    double q[kSP], lam = 0.0;
#pragma unroll
    for (int h = 0; h < kSP / 2; ++h) {
      const double2 u = rk[h], v = tl[h];
      q[2 * h] = u.x * v.x;
      q[2 * h + 1] = u.y * v.y;
    }
#pragma unroll
    for (int s = 0; s < kSP; ++s) lam += c[s] * q[s];
    if (!(lam > 0.0) || !isfinite(lam)) {
      bad |= kBadMu;
      continue;
    }
    term += n * log(lam);
    if (D) {
      const double g = n / lam;
#pragma unroll
      for (int s = 0; s < kSP; ++s) A[s] += g * q[s];
    }
  }
  if (inwin && dense)  // some c_s < 0 (or not finite): lambda >= 0 at every bin?
    for (int x = sub * 64 + lane; x < nr * np; x += 64 * kJointWPR) {
      const int k = x / np, l = x - k * np;
      double lam = 0.0;
#pragma unroll
      for (int s = 0; s < kSP; ++s) lam += c[s] * (Rk[k][s] * Tl[l][s]);
      if (!(lam >= 0.0) || !isfinite(lam)) bad |= kBadMu;
    }
  term = sum64(term);
  bad = or64(bad);
  if (D) {
#pragma unroll
    for (int s = 0; s < kSP; ++s) A[s] = sum64(A[s]);
  }
  if (lane == 0) {
    wsum[w][kSP] = term;
    wsum[w][kSP + 1] = mu;
    wfl[w] = bad;
    if (D) {
#pragma unroll
      for (int s = 0; s < kSP; ++s) wsum[w][s] = A[s];
    }
  }
  __syncthreads();
  // per row: sub-wave partials in order
  if (D && t < kJointRows * kSP) {
    const int rr = t / kSP, s = t - rr * kSP, jj = blockIdx.x * kJointRows + rr;
    const bool in = jj < N && jj >= win_lo && jj < win_hi;
    double a = wsum[rr * kJointWPR][s];
    for (int v = 1; v < kJointWPR; ++v) a += wsum[rr * kJointWPR + v][s];
    const double hadd = (in && s < S) ? (1.0 - tag[s]) * (jsig[s] - a) : 0.0;  // (1 - t_s) G_s
    // pile-up-fraction and table-coordinate parts (summed over s below),
    // loaded before the stores
    hs[rr][s] = pu_float && jj < N ? hadd * th[s] * Dp[jj * kSP + s] : 0.0;
    ht[rr][s] = tab && jj < N ? hadd * th[s] * Dtp[jj * kSP + s] : 0.0;
    if (jj < N) {
      const double mpv = Mp[jj * kSP + s];
      H[jj * kSP + s] += hadd;
      jg[jj * kSP + s] = hadd * mpv;
    }
  }
  if (D) __syncthreads();
  if (t < kJointRows) {
    const int jj = blockIdx.x * kJointRows + t;
    if (jj >= N) return;
    double lt = wsum[t * kJointWPR][kSP];
    int fl = wfl[t * kJointWPR];
    for (int v = 1; v < kJointWPR; ++v) {
      lt += wsum[t * kJointWPR + v][kSP];
      fl |= wfl[t * kJointWPR + v];
    }
    jnll[jj] = wsum[t * kJointWPR][kSP + 1] - lt;
    jflag[jj] = fl;
    if (D) {
      double pp = 0.0, tp = 0.0;
      for (int s = 0; s < S; ++s) {
        pp += hs[t][s];
        tp += ht[t][s];
      }
      if (pu_float) jpp[jj] = pp;
      if (tab) jtp[jj] = tp;
    }
  }
}

// Ceiling microbenchmark of the cell arithmetic, with the sweeps' lane
// layout: each wave takes one (true tile, reco tile) pair inside a tile
// support (chosen by a hash of its index, so the mix of shapes, arguments and
// paths is the workload's), lane (j = l%16, g = l/16) holds the constants of
// columns 4q+g, q = 0..3, and its bin's constants in registers, and evaluates
// the four cells (value and the two column-parameter derivatives, by the same
// path as the backward sweep) `reps` times.  No list building, contraction or
// memory traffic in the loop: the rate the cell arithmetic alone reaches.
// eps is 0 at run time (it only keeps each repetition's arguments from being
// hoisted); sink is written only if the sum equals `never`, which keeps the
// results live.
template <class R, int KIND>
__global__ void __launch_bounds__(256) k_cell_ceiling(const FitDev* fits, int reps, double eps, double never,
                                                      double* sink) {
  const FitDev& f = fits[0];
  const unsigned wid = blockIdx.x * 4u + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, jr = lane & 15, g = lane >> 4;
  const int ct = (int)((wid * 2654435761u) % (unsigned)f.n_ct);
  const int2 b = f.tb[ct];
  const int rt_a = b.y >= b.x ? max(b.x, 0) / kRowStep : 0;
  const int rt_b = b.y >= b.x ? min(b.y / kRowStep, f.n_rt - 1) : 0;
  const int rt = rt_a + (int)((wid / 7u) % (unsigned)(rt_b - rt_a + 1));
  const double xe = f.xe[min(rt * kRowStep + jr, f.N)];
  const double lnf = KIND == kCount ? lgamma(xe + 1.0) : 0.0;
  const RowQ<R> rq = load_rowq<R, KIND>(f, min(rt * kRowStep + jr, f.N - 1));
  const bool ok = rt * kRowStep + jr < f.N && jr < kRowStep;
  ColPre<R> c[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    GColPar& cp = ((GColPar*)f.cp)[min(ct * kColTile + 4 * q + g, f.T - 1)];
    c[q].cp = &cp;
    c[q].c0 = cp.c0;
    c[q].c1 = KIND == kGauss ? cp.c1 : KIND == kGG ? cp.c1 * cp.f64[3] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) c[q].s[u] = sizeof(R) == 4 ? (R)cp.f32[u] : (R)cp.f64[u];
    c[q].v = 0.0;
  }
  double acc = 0.0;
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ColPre<R> cc = c[q];
      cc.c0 += eps * r;
      const CellVal<R> ev = cell_lean<R, KIND, true>(cc, rq, xe + eps * r, lnf, ok);
      acc += ev.v + (double)(ev.d1 + ev.d2);
    }
  }
  if ((double)acc == never) sink[0] = (double)acc;
}

void launch_cell_ceiling(const FitDev* d_fit, int kind, int prec, int blocks, int reps, double* d_sink,
                         hipStream_t st) {
  const double eps = 0.0, never = -1.2345e300;
  if (kind == kGG && prec == kF32)
    hipLaunchKernelGGL((k_cell_ceiling<float, kGG>), dim3(blocks), dim3(256), 0, st, d_fit, reps, eps, never, d_sink);
  else if (kind == kGG)
    hipLaunchKernelGGL((k_cell_ceiling<double, kGG>), dim3(blocks), dim3(256), 0, st, d_fit, reps, eps, never, d_sink);
  else if (kind == kGauss && prec == kF32)
    hipLaunchKernelGGL((k_cell_ceiling<float, kGauss>), dim3(blocks), dim3(256), 0, st, d_fit, reps, eps, never, d_sink);
  else if (kind == kGauss)
    hipLaunchKernelGGL((k_cell_ceiling<double, kGauss>), dim3(blocks), dim3(256), 0, st, d_fit, reps, eps, never, d_sink);
  else if (kind == kCount)
    hipLaunchKernelGGL((k_cell_ceiling<double, kCount>), dim3(blocks), dim3(256), 0, st, d_fit, reps, eps, never, d_sink);
}

// Completion mark of a batched step: launched after its last kernel, it
// writes v into pinned host memory once everything before it on the stream
// is done and its results are visible to the host.
__global__ void k_mark(double* mark, double v) {
  __threadfence_system();
  *mark = v;
  __threadfence_system();
}

void launch_mark(double* d_mark, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_mark, dim3(1), dim3(1), 0, st, d_mark, v);
}

// The same with the value read from pinned host memory at run time (a
// captured step then marks the step number the host wrote for this replay).
__global__ void k_mark_from(double* mark, const double* src) {
  const double v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
  *mark = v;
  __threadfence_system();
}

void launch_mark_from(double* d_mark, const double* d_src, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_from, dim3(1), dim3(1), 0, st, d_mark, d_src);
}

// ---------------------------------------------------------------------------
template <class R, int KIND, bool MV>
static void launch_fwd_m(int cg, dim3 grid, dim3 blk, hipStream_t st, const FitDev* d_fits, const int* d_active) {
  switch (cg) {
    case 1: hipLaunchKernelGGL((k_cells_fwd<R, KIND, 1, MV>), grid, blk, 0, st, d_fits, d_active); break;
    case 2: hipLaunchKernelGGL((k_cells_fwd<R, KIND, 2, MV>), grid, blk, 0, st, d_fits, d_active); break;
    case 4: hipLaunchKernelGGL((k_cells_fwd<R, KIND, 4, MV>), grid, blk, 0, st, d_fits, d_active); break;
    default: hipLaunchKernelGGL((k_cells_fwd<R, KIND, 8, MV>), grid, blk, 0, st, d_fits, d_active); break;
  }
}
template <class R, int KIND>
static void launch_fwd(int cg, bool mv, dim3 grid, dim3 blk, hipStream_t st, const FitDev* d_fits,
                       const int* d_active) {
  if (mv) launch_fwd_m<R, KIND, true>(cg, grid, blk, st, d_fits, d_active);
  else launch_fwd_m<R, KIND, false>(cg, grid, blk, st, d_fits, d_active);
}
template <class R, int KIND>
static void launch_fix(bool fwd, bool mv, dim3 grid, hipStream_t st, const FitDev* d_fits, const int* d_active,
                       int pre, int use_flags, int nsplit) {
  const dim3 b((fwd ? kFixWaves : kBwdFixWaves) * 64);
  if (fwd && mv)
    hipLaunchKernelGGL((k_cells_fwd_fix<R, KIND, true>), grid, b, 0, st, d_fits, d_active, use_flags, nsplit);
  if (fwd && !mv)
    hipLaunchKernelGGL((k_cells_fwd_fix<R, KIND, false>), grid, b, 0, st, d_fits, d_active, use_flags, nsplit);
  if (!fwd && mv)
    hipLaunchKernelGGL((k_cells_bwd_fix<R, KIND, true>), grid, b, 0, st, d_fits, d_active, pre, use_flags);
  if (!fwd && !mv)
    hipLaunchKernelGGL((k_cells_bwd_fix<R, KIND, false>), grid, b, 0, st, d_fits, d_active, pre, use_flags);
}
// The fix-up sweep of stage 1 (fwd) or 6, after the main sweep (use_flags).
static void launch_fix_stage(const LaunchShape& L, bool fwd, dim3 grid, hipStream_t st, const FitDev* d_fits,
                             const int* d_active, int pre, int use_flags, int ns) {
  const bool f32 = L.prec == kF32;
  if (f32 && L.kind == kGauss) launch_fix<float, kGauss>(fwd, L.any_mv, grid, st, d_fits, d_active, pre, use_flags, ns);
  if (f32 && L.kind == kGG) launch_fix<float, kGG>(fwd, L.any_mv, grid, st, d_fits, d_active, pre, use_flags, ns);
  if (!f32 && L.kind == kGauss)
    launch_fix<double, kGauss>(fwd, L.any_mv, grid, st, d_fits, d_active, pre, use_flags, ns);
  if (!f32 && L.kind == kGG) launch_fix<double, kGG>(fwd, L.any_mv, grid, st, d_fits, d_active, pre, use_flags, ns);
}
template <class R, int KIND>
static void launch_bwd(bool mv, dim3 grid, hipStream_t st, const FitDev* d_fits, const int* d_active, int pre) {
  if (mv) hipLaunchKernelGGL((k_cells_bwd<R, KIND, true>), grid, dim3(kBwdWaves * 64), 0, st, d_fits, d_active, pre);
  else hipLaunchKernelGGL((k_cells_bwd<R, KIND, false>), grid, dim3(kBwdWaves * 64), 0, st, d_fits, d_active, pre);
}

// One stage of an evaluation: 0 colparams, 1 cells_fwd, 2 reduce_M,
// 3 rowterms, 4 radial, 5 adjoint, 6 cells_bwd, 7 final.  Stages that do not
// apply (radial/adjoint without multivariate terms, the backward stages
// without the gradient) launch nothing.
static void launch_joint(const LaunchShape& L, int n, bool with_grad, hipStream_t st, const FitDev* d_fits,
                         const int* d_active) {
  const dim3 g((L.max_NS / kSP + kJointRows - 1) / kJointRows, n);
  if (with_grad) hipLaunchKernelGGL(k_joint<true>, g, dim3(kJointBlock), 0, st, d_fits, d_active);
  else hipLaunchKernelGGL(k_joint<false>, g, dim3(kJointBlock), 0, st, d_fits, d_active);
}

void launch_stage(const FitDev* d_fits, const int* d_active, int n, const LaunchShape& L, bool with_grad,
                  int stage, hipStream_t st) {
  const dim3 blk(kBlock);
  const dim3 gf(L.max_fwd_blocks, n), gb(L.max_bwd_blocks, n), grow(L.max_rowblk, n);
  const dim3 gred((L.max_NS + kBlock - 1) / kBlock, n), bf(kFwdWaves * 64);
  // forward fix-up blocks per reco tile (each runs kFixSplit / nsplit of its
  // shares): a single fit spreads its few busy tiles over more waves; a batch
  // keeps the (mostly idle) grid small
  const int nsplit = n > 1 ? 2 : kFixSplit;
  const dim3 gfx(L.max_rt * nsplit, n), gbx(L.max_ct, n);  // fix-up sweeps (per reco / true tile)
  const bool fixk = L.kind == kGG || L.kind == kGauss;
  const bool f32 = L.prec == kF32, gauss = L.kind == kGauss;
  // batches form a single histogram's pile-up adjoint once per fit
  const int pre = n >= kPreAdjFits ? 1 : 0;
  if (L.kind == kTable) {  // no cell sweeps: the interpolated table, then the row terms
    switch (stage) {
      case 0:
        hipLaunchKernelGGL(k_table, dim3((L.max_NS + kBlock - 1) / kBlock, n), blk, 0, st, d_fits, d_active);
        break;
      case 3:
        hipLaunchKernelGGL(k_rowterms, grow, blk, 0, st, d_fits, d_active);
        break;
      case 4:
        if (L.any_rad) hipLaunchKernelGGL(k_radial, dim3(1, n), blk, 0, st, d_fits, d_active);
        if (L.any_joint)
          launch_joint(L, n, with_grad, st, d_fits, d_active);
        break;
      case 7:
        launch_final(d_fits, d_active, n, with_grad, st);
        break;
      default:
        break;
    }
    return;
  }
  switch (stage) {
    case 0:
      if (L.kind == kCount)
        hipLaunchKernelGGL(k_colparams_count, dim3((L.max_T + kCpBlock - 1) / kCpBlock, n), dim3(kCpCountBlock), 0,
                           st, d_fits, d_active);
      else
        hipLaunchKernelGGL(k_colparams, dim3((L.max_T + kCpBlock - 1) / kCpBlock, n), dim3(kCpBlock), 0, st,
                           d_fits, d_active);
      break;
    case 1:
    case kStageFwdMain:
      if (f32 && gauss) launch_fwd<float, kGauss>(L.CG, L.any_mv, gf, bf, st, d_fits, d_active);
      if (f32 && L.kind == kGG) launch_fwd<float, kGG>(L.CG, L.any_mv, gf, bf, st, d_fits, d_active);
      if (!f32 && gauss) launch_fwd<double, kGauss>(L.CG, L.any_mv, gf, bf, st, d_fits, d_active);
      if (!f32 && L.kind == kGG) launch_fwd<double, kGG>(L.CG, L.any_mv, gf, bf, st, d_fits, d_active);
      if (L.kind == kCount) launch_fwd<double, kCount>(L.CG, L.any_mv, gf, bf, st, d_fits, d_active);
      if (fixk && stage == 1) launch_fix_stage(L, true, gfx, st, d_fits, d_active, 0, 1, nsplit);  // the steps left
      break;
    case 2:
      if (L.any_mv) hipLaunchKernelGGL(k_reduce_M, gred, blk, 0, st, d_fits, d_active);
      break;
    case 3:
      hipLaunchKernelGGL(k_rowterms, grow, blk, 0, st, d_fits, d_active);
      break;
    case 4:
      if (L.any_rad) hipLaunchKernelGGL(k_radial, dim3(1, n), blk, 0, st, d_fits, d_active);
      if (L.any_joint)
        launch_joint(L, n, with_grad, st, d_fits, d_active);
      break;
    case 5:  // a single histogram's adjoint: here for batches, else inside k_cells_bwd
      if (with_grad && L.any_mv) hipLaunchKernelGGL(k_adjoint, grow, blk, 0, st, d_fits, d_active);
      if (with_grad && pre)
        hipLaunchKernelGGL(k_adjoint1, dim3((L.max_rowblk + 3) / 4, n), blk, 0, st, d_fits, d_active);
      break;
    case 6:
    case kStageBwdMain:
      if (!with_grad) break;
      if (f32 && gauss) launch_bwd<float, kGauss>(L.any_mv, gb, st, d_fits, d_active, pre);
      if (f32 && L.kind == kGG) launch_bwd<float, kGG>(L.any_mv, gb, st, d_fits, d_active, pre);
      if (!f32 && gauss) launch_bwd<double, kGauss>(L.any_mv, gb, st, d_fits, d_active, pre);
      if (!f32 && L.kind == kGG) launch_bwd<double, kGG>(L.any_mv, gb, st, d_fits, d_active, pre);
      if (L.kind == kCount) launch_bwd<double, kCount>(L.any_mv, gb, st, d_fits, d_active, pre);
      if (fixk && stage == 6) launch_fix_stage(L, false, gbx, st, d_fits, d_active, pre, 1, 1);
      break;
    case 7:
      launch_final(d_fits, d_active, n, with_grad, st);
      break;
  }
}

void launch_eval(const FitDev* d_fits, const int* d_active, int n, const LaunchShape& L, bool with_grad,
                 hipStream_t st) {
  // one fit with the gradient: the final sums in the backward fix-up sweep's launch
  const bool fused = n == 1 && with_grad && (L.kind == kGG || L.kind == kGauss);
  for (int k = 0; k < kStages; ++k) {
    if (fused && k == 6) {
      launch_stage(d_fits, d_active, n, L, with_grad, kStageBwdMain, st);
      const bool f32 = L.prec == kF32, mv = L.any_mv;
      if (f32 && L.kind == kGauss) launch_bwd_fix_final<float, kGauss>(mv, L.max_ct, st, d_fits, d_active, 0);
      if (f32 && L.kind == kGG) launch_bwd_fix_final<float, kGG>(mv, L.max_ct, st, d_fits, d_active, 0);
      if (!f32 && L.kind == kGauss) launch_bwd_fix_final<double, kGauss>(mv, L.max_ct, st, d_fits, d_active, 0);
      if (!f32 && L.kind == kGG) launch_bwd_fix_final<double, kGG>(mv, L.max_ct, st, d_fits, d_active, 0);
    } else if (!(fused && k == 7)) {
      launch_stage(d_fits, d_active, n, L, with_grad, k, st);
    }
  }
}

// Expected counts of every term over the full reco range (diagnostics):
// out = [mu_energy[N] | mu_tagged[N] | nu[n_rad] | lambda[N][n_ps]].
__global__ void __launch_bounds__(kBlock) k_expected(const FitDev* fits, double* out) {
  const FitDev& f = fits[0];
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const double* th = f.theta;
  if (!f.mv) {
    if (t < f.N) {
      double mu = 0.0;
      if (f.vsum) mu = f.Mp[t * kSP];
      else
        for (int s = 0; s < f.S; ++s) mu += f.Mp[t * kSP + s] * th[s];
      out[t] = mu;
    }
    return;
  }
  if (t < f.N) {
    double a = 0.0, b = 0.0;
    for (int s = 0; s < f.S; ++s) {
      a += f.Mp[t * kSP + s] * (1.0 - f.tag[s]) * th[s];
      b += f.Mp[t * kSP + s] * f.tag[s] * th[s];
    }
    out[t] = a;
    out[f.N + t] = b;
  }
  if (t < f.n_rad) {
    double nu = 0.0;
    for (int s = 0; s < f.S; ++s) {
      double sw = 0.0;
      for (int j = f.rad_lo; j < f.rad_hi; ++j) sw += f.Mp[j * kSP + s];
      nu += (1.0 - f.tag[s]) * th[s] * sw * f.rad[s * f.n_rad + t];
    }
    out[2 * f.N + t] = nu;
  }
  if (t < f.N * f.n_ps) {
    const int j = t / f.n_ps, k = t % f.n_ps;
    double lam = 0.0;
    for (int s = 0; s < f.S; ++s) lam += f.Mp[j * kSP + s] * (1.0 - f.tag[s]) * th[s] * f.pst[s * f.n_ps + k];
    out[2 * f.N + f.n_rad + t] = lam;
  }
}

void launch_expected(const FitDev* d_fit, double* d_out, int N, int n_rad, int n_ps, hipStream_t st) {
  const int n = max(max(N, n_rad), N * n_ps);
  hipLaunchKernelGGL(k_expected, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d_fit, d_out);
}

// ---------------------------------------------------------------------------
// Device-minimised batched fits (Sec. 4, steps 5-6 for many fits at once):
// the minimiser of every fit runs on the device, one wave per fit, between
// the evaluation launches of a captured graph, so that an iteration of all
// the fits needs no host round trip.  The minimiser is the host's own code
// (bx_fitcore.hpp, contraction off), so a fit takes the same steps as on the
// plain path.
__global__ void __launch_bounds__(64) k_fit_start(Bfgs* opts, FitSlot* slots, FitDev* fits, int n) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  FitDev& f = fits[slots[i].fit];
  opts[i].next(const_cast<double*>(f.theta));
}

__global__ void k_zero_count(int* c) { *c = 0; }

// running[i]: 0 finished, 1 on its first model, 2 waiting for its polishing
// placement to join the graph, 3 on the polishing model.  ready[i]: the
// polishing placement is in the graph now.  One block (one wave) per fit:
// the wave stages the minimiser state in LDS, runs the step on it with every
// lane (the loops over independent elements shared out, the rest computed
// alike by all lanes, so the control flow is uniform) and writes it back;
// lane 0 alone does the bookkeeping in global memory.
__global__ void __launch_bounds__(64) k_fit_step(Bfgs* opts, FitSlot* slots, FitDev* fits, int n, int* count,
                                                 int* running, const int* ready) {
  const int i = blockIdx.x;
  if (i >= n) return;
  constexpr int kWords = (int)(sizeof(Bfgs) / sizeof(double));
  static_assert(sizeof(Bfgs) % sizeof(double) == 0, "minimiser state in whole words");
  __shared__ int go;
  __shared__ __align__(16) double sw[kWords];  // the fit's minimiser (raw words: no constructor runs)
  Bfgs& o = *reinterpret_cast<Bfgs*>(sw);
  const bool lead = threadIdx.x == 0;
  FitSlot& sl = slots[i];
  if (lead) {
    const Bfgs& og = opts[i];
    go = !og.done() || (sl.fit_p >= 0 && sl.phase == 0 && og.can_polish());
    if (!go) running[i] = 0;
  }
  __syncthreads();
  if (!go) return;  // block-uniform: a finished fit
  // the state in (all of a lane's loads issued before its first store: one
  // memory latency, not one per word), and the last evaluation's result row
  // (NLL, gradient, flags), which the step reads in serial loops
  double* const gw = reinterpret_cast<double*>(opts + i);
  constexpr int kPer = (kWords + 63) / 64;
  {
    double v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int w = threadIdx.x + 64 * k;
      v[k] = w < kWords ? gw[w] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int w = threadIdx.x + 64 * k;
      if (w < kWords) sw[w] = v[k];
    }
  }
  // the slot's fields, read once by every lane (lane 0 may rewrite phase)
  const int fit = sl.fit, fit_p = sl.fit_p, P = sl.P;
  int phase = sl.phase;
  __shared__ double res[kMaxP + 2];
  {
    const double* out = fits[phase ? fit_p : fit].out;
    if ((int)threadIdx.x < P + 2) res[threadIdx.x] = out[threadIdx.x];
  }
  __syncthreads();
  if (lead) running[i] = 0;
  if (!o.done()) {  // the results of the last evaluation (only a fit about to move to its polishing model is done)
    const int fl = (int)res[1 + P];
    const bool bad = (fl & (kBadSigma | kBadGG | kBadMu | kBadTheta | kZeroWidth)) != 0;
    o.feed(bad ? INFINITY : res[0], res + 1);
  }
  bool held = false;
  if (o.done() && fit_p >= 0 && phase == 0 && o.can_polish()) {
    if (lead) fits[fit].skip = 1;
    if (!ready[i]) {  // wait (no evaluation) until the host adds the FP64 placement
      if (lead) {
        running[i] = 2;
        atomicAdd(count, 1);
      }
      held = true;
    } else {
      o.polish(sl.final_tol, sl.noise_p);  // on to the polishing placement (same theta and result rows)
      phase = 1;
      if (lead) {
        sl.phase = 1;
        fits[fit_p].skip = 0;
      }
    }
  }
  if (!held && lead) {
    FitDev& g = fits[phase ? fit_p : fit];
    if (o.done()) {
      g.skip = 1;
    } else {
      o.next(const_cast<double*>(g.theta));
      running[i] = 1 + 2 * phase;
      atomicAdd(count, 1);
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < kWords; w += 64) gw[w] = sw[w];
}

void launch_fit_start(void* opts, FitSlot* slots, FitDev* fits, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fit_start, dim3((n + 63) / 64), dim3(64), 0, st, (Bfgs*)opts, slots, fits, n);
}

void launch_fit_step(void* opts, FitSlot* slots, FitDev* fits, int n, int* d_count, int* d_running,
                     const int* d_ready, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, d_count);
  hipLaunchKernelGGL(k_fit_step, dim3(n), dim3(64), 0, st, (Bfgs*)opts, slots, fits, n, d_count, d_running,
                     d_ready);
}

}  // namespace bx

// Device-side data layout of one fit (model + data + per-evaluation
// workspace).  All pointers are device pointers; a batch of fits is an array
// of these in device memory, and every kernel takes (fits, active list) with
// blockIdx.y selecting the fit, so one fit and a batch of thousands run the
// same code with the same per-fit arithmetic.
#pragma once
#include <stdint.h>

#include "bx_math.h"

namespace bx {

constexpr int kSP = 16;        // species padded to the MFMA width
constexpr int kRowTile = 16;   // reco edges per tile (15 cells)
constexpr int kRowStep = 15;   // cells per row tile
constexpr int kColTile = 16;   // true bins per tile
constexpr int kMaxResp = 4;    // response parameters (Gauss 2, GG 4)
constexpr int kBlock = 256;    // threads per block (4 waves)
constexpr int kCpBlock = 64;   // threads per block of the column-parameter kernel
constexpr int kFwdWaves = 16;  // waves per forward block (one reco tile, 16 CG true tiles)
constexpr int kMaxK = 256;     // longest random-trigger spectrum
constexpr int kMaxRG = 4;      // reco tiles per backward wave (LDS staging bound)
constexpr int kBwdWaves = 4;   // waves per backward block (one reco tile each, times RG)
constexpr int kFixSplit = 8;   // forward fix-up blocks per reco tile (their shares of Mfix)
constexpr int kPreAdjFits = 8; // launches of this many fits form the pile-up adjoint in its own kernel
constexpr int kMaxCG = 8;      // true tiles per forward wave
constexpr int kMaxP = 32;      // parameters (16 rates + response parameters)
constexpr int kBwdPart = 4 + kSP;  // backward partials per block: response parameters, then rates
constexpr int kFinBlocks = 16;  // blocks of the final sums (each a share of every partial)
constexpr int kFinThreads = 256;
constexpr int kFinRow = 8 + kSP;  // per final-sums block: NLL, 4 response-parameter gradients,
                                  // pile-up fraction, table coordinate, flags; then the rates

enum : int { kGauss = 0, kGG = 1, kTable = 2, kCount = 3 };
constexpr int kMaxGrid = 64;   // grid points of a tabulated response
enum : int { kF32 = 0, kF64 = 1 };
enum : int {                   // domain flags
  kBadSigma = 1,               // Gaussian sigma^2 < 0
  kBadGG = 2,                  // GG mean or variance <= 0, or shape out of range; count
                               // estimator mean <= 0 or variance <= mean
  kBadMu = 4,                  // an expected count < 0, or 0 with counts > 0
  kBadTheta = 8,               // non-finite parameter
  kZeroWidth = 16              // sigma = 0 somewhere: response derivative undefined
};

struct ColPar {
  double c0;        // Gauss: m;        GG: ct = p ln a + ln k;  count: m
  double c1;        // Gauss: 1/sigma;  GG: k;                 count: r
  double v;         // sum_s r_s F^_si  (expected deposited counts in true bin i)
  float f32[8];     // GG edge constants (k, 1/k, sqrt(k/2), cR, ce, dlnG*, ln k - psi, p)
  double f64[8];    // the same in FP64 (count: m, r, ln Gamma(r), ln(r/(r+m)), ln(m/(r+m)), psi(r),
                    // 1/(r+m), 1/m)
  double J[2][kMaxResp];  // d(c1, c2)/d(response parameter q)
  int jlo, jhi;     // cells that may be non-zero (support)
  int bad;          // domain flags
  int pad;
  double e1[3];     // GG: the cell of the reco bin from x <= 0 (row0), the CDF at its upper edge,
                    // and its two derivatives as the fix-up sweeps form them; 0 beyond the support
};

struct FitDev {
  // shape
  int T, N, S, P, nresp, kind, prec, mv;
  int win_lo, win_hi, K, n_rad, rad_lo, rad_hi, n_ps;
  int n_rt, n_ct, CG, n_cg, n_fb, RG, n_rg, n_rowblk;  // n_cg: forward chunks, n_fb: forward blocks per reco tile
  int n_cpblk, n_bwdblk;  // column-parameter blocks, backward blocks
  int uniform;            // reco bins of equal width
  int row0;               // GG: the reco bin from x <= 0 into x > 0 (its cell is F(x_row0+1)), or -1
  int vsum;               // one energy histogram with analytic cells: the sweeps contract the cells
                          // with v_i = sum_s r_s F^_si (mu0 = R v) and the rate gradient is
                          // F^T (R^T w~); otherwise per-species M = R F^T (FP64 MFMA)
  int sup_prec;           // precision whose support cut the column supports use (the model's);
                          // prec is the precision of this evaluation's cells
  int pu_float;           // the pile-up fraction is theta[P - 1] (else pu_frac)
  int n_grid;             // tabulated response: grid points (kind kTable)
  int joint;              // joint energy x radius x PS term replaces the vetoed/radial/PS terms
  double x0, inv_w;       // first reco edge, 1 / bin width (uniform bins)
  double pu_frac;
  GGConst gg;
  // inputs (device)
  const double* xraw;   // [N+1] reco edges
  const double* xe;     // [N+1] Gauss: edges; GG: ln edges (-inf at x <= 0)
  const double* Ec;     // [T] true-bin centres
  const double* Qt;     // [T] quenching (GG)
  const float* F32;     // [T][16] exposure * normalised spectra
  const double* F64;    // [T][16]
  const double* ghat;   // [K] normalised random-trigger spectrum
  const double* tag;    // [16] tag fractions
  const double* rad;    // [16][n_rad]
  const double* pst;    // [16][n_ps]
  const double* n_e;    // [N] energy (vetoed) histogram
  const double* n_t;    // [N] tagged
  const double* n_r;    // [n_rad]
  const double* n_p;    // [N][n_ps]
  const int* jrow;      // [N + 1] joint histogram of the vetoed events ([N][n_rad][n_ps]) as
  const uint32_t* jent; //   its non-zero bins per row: entries jrow[j] .. jrow[j+1]-1 hold
  const double* jval;   //   (k << 16 | l) and the count (room for every bin)
  const double* jsig;   // [16] (sum_k rho_sk)(sum_l T_sl) of the joint term's templates
  const double* grid;   // [n_grid] tabulated response: coordinate of each matrix
  // quadrature of the cells (analytic responses): per reco bin j the centre
  // qpum[j] = p (ln x_j + ln x_j+1)/2 and half-width qhw[j] = p/2 ln(x_j+1/x_j)
  // in t (GG, +inf for a bin from x <= 0; Gaussian: qhw = (x_j+1 - x_j)/2)
  // and the GG node constants QRowGG in FP32 (4 nodes) and FP64 (5 nodes)
  const double* qpum;   // [N]
  const double* qhw;    // [N]
  const float* qrow32;  // [N][3 kNQ32]
  const double* qrow64; // [N][3 kNQ64]
  const double* Mg;     // [n_grid][N][16] exposure * R_g F^T, formed at build
  // per-evaluation state
  const double* theta;  // [P]
  ColPar* cp;           // [T]
  int2* tb;             // [n_ct] support of each column tile (cells)
  double* Mpart;        // [n_cg][N][16] (multivariate) or [n_cg][N] (vsum): one partial per
                        // chunk of 16 listed true tiles
  double* Mfix;         // [kFixSplit][N][16] or [kFixSplit][N]: the forward fix-up sweep's
                        // shares (cells outside the sweeps' common case), added last
  int has_fix;          // analytic cells: the fix-up sweeps run (not for the count estimator)
  int skip;             // 1: every kernel leaves this fit alone (a device-minimised fit that
                        // has finished, or the placement it does not use now)
  double* fixq;         // [n_ct][4]: per wave step (true tile, q), the largest column factor of
                        // the one-interval test (GG sqrt(k) in the cell precision, Gauss 1/sigma;
                        // +inf for a column without a width), written by k_colparams
  const double* fixp;   // [n_rt]: per reco tile, the largest half-width of its bins in the
                        // column's variable (model constant; +inf for the GG bin from x <= 0)
  int* fixflag;         // [n_rt + n_ct]: reco tiles, then true tiles, with a step left (cleared
                        // by k_colparams, set by the forward sweep)
  double* M;            // [N][16] sum of the partials (FP64)
  double* Mp;           // [N][16] after pile-up
  double* H;            // [N][16] dNLL/d(r_s M'_js) / r_s, without the radial part
  double* Ht;           // [N][16] pile-up adjoint of H
  double* nllpart;      // [n_rowblk]
  int* flagpart;        // [n_rowblk]
  double* gpart;        // [n_rowblk][16] rate-gradient partials
  double* rad_out;      // [4 + 2*16]: nll_rad, flag, rho.w[16], rate grad[16], pile-up-fraction
                        // grad, table-coordinate grad
  double* Dp;           // [N][16] dM'/dp = g^*M - M (a floated pile-up fraction)
  double* ppart;        // [n_rowblk] pile-up-fraction gradient partials
  double* Dt;           // [N][16] tabulated response: dM/dlam in the current grid cell
  double* Dtp;          // [N][16] dM'/dlam (after pile-up)
  double* tpart;        // [n_rowblk] table-coordinate gradient partials
  double* jnll;         // [N] joint term per reco row: NLL, flags, rate gradient [N][16],
  int* jflag;           //   pile-up-fraction and table-coordinate gradients
  double* jg;
  double* jpp;
  double* jtp;
  int* cpflag;          // [n_cpblk] domain flags of the column parameters
  double* bwdpart;      // [n_bwdblk][kBwdPart] response-gradient partials, then (vsum) the
                        // rate-gradient partials sum_i F^_si u_i, u = R^T w~
  double* bwdfix;       // [n_ct][kBwdPart] the backward fix-up sweep's partials
  double* fpart;        // [kFinBlocks][kFinRow] the final-sums blocks' rows
  int* fcount;          // final-sums blocks done (zeroed by the first kernel of an evaluation
                        // and by the block that adds the rows)
  double* out;          // [2 + P]: nll, grad[P], flags
  const double* theta_src;  // pinned host [P + 1]: theta and the caller's sequence number, or null
  double* out_host;         // pinned host [3 + P]: the results, then the sequence number as
                            // completion mark (written last, after a system-scope fence), or null
};

// Grid sizes of one batched launch (maxima over the fits in it).
struct LaunchShape {
  int max_T, max_fwd_blocks, max_NS, max_rowblk, max_bwd_blocks, max_rt, max_ct;
  int kind, prec, any_mv, any_rad, any_joint;
  int CG;  // forward tiles per wave (one value per launch)
};
constexpr int kStages = 8;  // colparams, cells_fwd, reduce_M, rowterms, radial, adjoint, cells_bwd, final
// launch_stage's extra codes (timing only): the main sweep of stage 1 or 6
// without its fix-up sweep
constexpr int kStageFwdMain = 8, kStageBwdMain = 9;
constexpr int kStageTimes = kStages + 3;  // the stages, a whole evaluation, the two main sweeps
void launch_stage(const FitDev* d_fits, const int* d_active, int n, const LaunchShape& L, bool with_grad,
                  int stage, hipStream_t st);
void launch_eval(const FitDev* d_fits, const int* d_active, int n, const LaunchShape& L,
                 bool with_grad, hipStream_t st);
void launch_expected(const FitDev* d_fit, double* d_out, int N, int n_rad, int n_ps, hipStream_t st);

// One device-minimised fit (bx_fit_batch): its placements in the FitDev
// array (fit_p: the FP64 polishing placement, or -1), its parameter count,
// the phase (0: first model, 1: polishing model), the polishing model's
// tolerance and NLL rounding noise.
struct FitSlot {
  int fit, fit_p, P, phase;
  double final_tol, noise_p;
};
// opts: the fits' minimisers (bx::Bfgs[n], device memory).  start: every fit
// names its first point (theta rows); step: hands each unfinished fit the
// results of its last evaluation, moves it to its polishing placement when
// the first model is done, names its next point, and counts the fits still
// running into *d_count (zeroed in the same launch sequence) and their state
// into d_running[n] (0 finished, 1 first model, 2 waiting for its polishing
// placement, 3 polishing model).  A fit whose first model is done moves on
// only when d_ready[i] says its polishing placement is in the graph.
void launch_fit_start(void* opts, FitSlot* slots, FitDev* fits, int n, hipStream_t st);
void launch_fit_step(void* opts, FitSlot* slots, FitDev* fits, int n, int* d_count, int* d_running,
                     const int* d_ready, hipStream_t st);
void launch_mark(double* d_mark, double v, hipStream_t st);
void launch_mark_from(double* d_mark, const double* d_src, hipStream_t st);
void launch_table_gemm(const double* d_R, const double* d_F64, double* d_Mg, int G, int N, int T, hipStream_t st);
void launch_cell_ceiling(const FitDev* d_fit, int kind, int prec, int blocks, int reps, double* d_sink,
                         hipStream_t st);

}  // namespace bx

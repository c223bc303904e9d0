// Host-side model object and helpers shared by the C ABI, the plain fitter
// and the fit server.
#pragma once
#include <hip/hip_runtime.h>
#include <immintrin.h>
#include <stdint.h>

#include <atomic>
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/bx.h"
#include "bx_dev.h"

namespace bx {



void set_error(const std::string& msg);
bx_status hip_fail(hipError_t e, const char* what);

// Tile choice for a fit of this shape (depends only on the fit's own shape).
struct Tiles {
  int CG, RG;
};
Tiles choose_tiles(int T, int N, int kind, int prec, int batched);

// Host copy of everything a fit needs, independent of device placement.
struct HostModel {
  int T, N, S, P, nresp, kind, prec, mv;
  int win_lo, win_hi, K, n_rad, rad_lo, rad_hi, n_ps;
  double p, pu_frac, exposure;
  int pu_float;  // the pile-up fraction is the last parameter
  int n_grid = 0;                 // tabulated response: grid points
  std::vector<double> grid, rtab;  // its coordinates; the matrices (kept only until build)
  std::vector<double> xraw, xe, Ec, Qt, F64, ghat, tag, rad, pst;
  std::vector<float> F32;
  std::vector<double> n_e, n_t, n_r, n_p;
  int joint = 0;             // joint energy x radius x PS term (multivariate)
  std::vector<double> n_j;   // its histogram [N][n_rad][n_ps]
  std::vector<int> jrow;     // and its non-zero bins per row (row starts [N + 1],
  std::vector<uint32_t> jent;  // k << 16 | l, counts)
  std::vector<double> jval;
  std::vector<double> jsig;   // [16] (sum_k rho_sk)(sum_l T_sl)
  // quadrature of the cells: per reco bin the GG bin centre p (ln x_j + ln x_j+1)/2,
  // the half-width in the quadrature variable and the node constants (FP32 4
  // nodes, FP64 5 nodes)
  std::vector<double> qpum, qhw, qrow64;
  std::vector<float> qrow32;
  // per reco tile: the largest half-width of its bins, as the sweeps' one-
  // interval test takes it (the cell precision for GG, FP64 for Gauss)
  std::vector<double> fixp;
  GGConst gg;
  Tiles tiles;
};

bx_status make_host_model(const bx_model_desc* d, const bx_data* x, HostModel* h);
// Relative rounding noise of the NLL values: FP32 cells leave ~1e-10 of the
// NLL, FP64 cells ~1e-15 (the minimiser accepts changes within it when the
// gradient shows progress).
inline double nll_noise(const HostModel& h) { return h.prec == kF32 ? 1e-9 : 1e-13; }

// Writes back and evicts the CPU cache lines of n doubles at p, then a full
// fence, so that later loads come from memory and earlier stores have left.
// Pinned buffers shared with the kernels need it: device writes do not
// reliably invalidate a copy of the line the CPU already holds (one fetched
// by its prefetcher while the results were in flight).
inline void flush_lines(const double* p, int n) {
  const uintptr_t a = (uintptr_t)p & ~(uintptr_t)63, e = (uintptr_t)(p + n);
  for (uintptr_t l = a; l < e; l += 64) _mm_clflush((const void*)l);
  _mm_mfence();
}
bx_status set_host_data(HostModel* h, const bx_data* x);
// The scalars, per-model constants and tiles of h, without its arrays.
HostModel shape_only(const HostModel& h);
double host_lnfact(const HostModel& h);

// Device placement of one fit: one allocation holding inputs and workspace.
struct DeviceFit {
  void* base = nullptr;
  size_t bytes = 0;
  FitDev dev{};          // host copy with device pointers
  double* d_theta = nullptr;
  double* d_out = nullptr;
};
// shared_inputs: the read-only inputs live in another placement (see place_fit)
size_t device_fit_bytes(const HostModel& h, bool shared_inputs = false);
void derive_tiles(const HostModel& h, FitDev* f);
// Carve `base` (device memory of device_fit_bytes(h, shared != null)) and
// upload h; stream-ordered.  With `shared` (a placed fit of the same model
// and data), the read-only inputs are that fit's and only the workspace is
// carved here.
bx_status place_fit(const HostModel& h, void* base, DeviceFit* df, hipStream_t st, const FitDev* shared = nullptr);
bx_status upload_data(const HostModel& h, const DeviceFit& df, hipStream_t st);
LaunchShape shape_of(const FitDev& f);
// Launch group of a placed fit: kind, precision, single histogram or several
// (the sweeps' contraction differs, so the two never share a launch), and the
// forward tiles per wave.
constexpr int kGroups = 64;
inline int group_of(const LaunchShape& l) {
  int cgl = 0;
  while ((1 << cgl) < l.CG) ++cgl;
  return ((l.kind * 2 + l.prec) * 2 + l.any_mv) * 4 + cgl;
}
// The grid needs of a launch covering both shapes.
inline void widen(LaunchShape* L, const LaunchShape& l) {
  L->kind = l.kind;
  L->prec = l.prec;
  L->CG = l.CG;
  L->max_T = std::max(L->max_T, l.max_T);
  L->max_fwd_blocks = std::max(L->max_fwd_blocks, l.max_fwd_blocks);
  L->max_NS = std::max(L->max_NS, l.max_NS);
  L->max_rowblk = std::max(L->max_rowblk, l.max_rowblk);
  L->max_bwd_blocks = std::max(L->max_bwd_blocks, l.max_bwd_blocks);
  L->max_rt = std::max(L->max_rt, l.max_rt);
  L->max_ct = std::max(L->max_ct, l.max_ct);
  L->any_mv |= l.any_mv;
  L->any_rad |= l.any_rad;
  L->any_joint |= l.any_joint;
}

}  // namespace bx

constexpr int kPinOut = 64;       // doubles: device-written half of h_pin (512 B in)
constexpr int kPinDoubles = 128;  // 1 KiB: room for 2 + 32 results and the mark

struct bx_model {
  bx::HostModel h;
  bx::DeviceFit df;
  bx::FitDev* d_fit = nullptr;   // device copy of df.dev (theta and results in device memory)
  bx::FitDev* d_fit_h = nullptr; // the same, reading theta from and writing results to h_pin
  int* d_active = nullptr;       // {0}
  hipStream_t stream = nullptr;  // launches
  bool own_stream = false;
  // The evaluation workspace (theta, column parameters, partials, results) is
  // shared by every entry point; a call on another stream than the previous
  // one waits for the work already enqueued there (order_on).
  hipStream_t last_stream = nullptr;
  hipEvent_t ws_event = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used for graph capture
  hipGraphExec_t g_eval = nullptr, g_grad = nullptr;  // host-buffer path (d_fit_h)
  hipGraphExec_t g_grad_dev = nullptr;                // device-buffer path (d_fit)
  // pinned, coherent: theta[P] | seq at 0 (written by the host), out[2 + P] |
  // completion mark at kPinOut (written by the device).  The two halves never
  // share a cache line: a host line holding a stale copy of a device-written
  // value would otherwise be written back over it.  Device writes do not
  // reliably invalidate lines the CPU holds, so the host flushes its lines of
  // theta after writing them and those of the mark and results before reading.
  double* h_pin = nullptr;
  uint64_t seq = 0;              // evaluations on the host path (completion marks)
  double lnfact = 0.0;
  std::atomic<int> users{0};     // server fits referencing this model
  int device = 0;
};

namespace bx {
// The polishing model of a mixed-precision fit: FP64 and the same shapes
// (BX_E_INVAL otherwise).
bx_status polish_compatible(const bx_model* m, const bx_model* p);
}  // namespace bx

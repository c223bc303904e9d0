// Batched fits with their minimisers on the device (Sec. 4, steps 5-7 for
// many fits at once, e.g. a toy study): every fit is placed once (inputs
// shared with its model, its own workspace, theta and result rows), and one
// iteration of all of them -- the evaluation launches of every launch group,
// then the minimisers' step kernel -- is captured as a HIP graph and replayed
// until no fit is left running.  The host only checks which fits are still
// running every few replays; when half of the fits in the graph have
// finished, it captures the iteration again over the running ones (their
// grids shrink with them, so the long tail of slow fits costs little).  A
// mixed-precision fit whose first model is done waits (no evaluation) until
// a capture puts its FP64 placement in the graph in place of the first one.  The minimiser is the plain path's (bx_fitcore.hpp,
// compiled for the device with the same arithmetic), so every fit ends with
// the plain path's result bit for bit.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "bx_fitcore.hpp"
#include "bx_model.hpp"

using namespace bx;

namespace {

constexpr int kRow = 40;  // doubles per theta / result row (P <= 32, plus flags)

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Everything the call allocates, released on every exit path.
struct Batch {
  hipStream_t st = nullptr;
  void* mem = nullptr;          // all placements
  double* rows = nullptr;       // theta rows, then result rows
  FitDev* d_fits = nullptr;
  FitSlot* d_slots = nullptr;
  Bfgs* d_opts = nullptr;
  int* d_lists = nullptr;       // active lists of the launch groups
  int* d_count = nullptr;       // running fits, then their states [n]
  int* h_count = nullptr;       // pinned copy of the same
  int* d_ready = nullptr;       // [n]: the fit's polishing placement is in the graph
  std::vector<int> h_ready;
  hipGraphExec_t exec = nullptr;
  ~Batch() {
    if (st) (void)hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    for (void* p : {(void*)d_fits, (void*)d_slots, (void*)d_opts, (void*)d_lists, (void*)d_count, (void*)d_ready,
                    (void*)rows, mem})
      if (p) (void)hipFree(p);
    if (h_count) (void)hipHostFree(h_count);
    if (st) (void)hipStreamDestroy(st);
  }
};

size_t align4k(size_t b) { return (b + 4095) & ~(size_t)4095; }

}  // namespace

extern "C" bx_status bx_fit_batch(bx_model* const* models, const bx_fit_opts* opts, int32_t n,
                                  bx_fit_result* results, int32_t check_every) {
  if (!models || !opts || !results || n < 1) {
    set_error("NULL argument or no fits");
    return BX_E_INVAL;
  }
  const int64_t t0 = now_ns();
  const int K = check_every > 0 ? check_every : 4;
  std::vector<Bfgs> opt(n);
  std::vector<FitSlot> slot(n);
  std::vector<HostModel> hm, hp;
  hm.reserve(n);
  hp.reserve(n);
  size_t bytes = 0;
  std::vector<size_t> off(n), offp(n);
  int npl = n, max_eval = 0;
  for (int i = 0; i < n; ++i) {
    bx_model* m = models[i];
    const bx_fit_opts* o = opts + i;
    if (!m || !o->x0) {
      set_error("NULL model or start point");
      return BX_E_INVAL;
    }
    if (m->device != models[0]->device) {
      set_error("the fits' models are on different devices");
      return BX_E_INVAL;
    }
    FitProblem pb;
    bx_status s = fit_problem(m->h.P, m->h.S, o, &pb, m->h.pu_float ? m->h.P - 1 : -1);
    if (s != BX_OK) return s;
    if (o->polish && (s = polish_compatible(m, o->polish)) != BX_OK) return s;
    pb.f_noise = nll_noise(m->h);
    opt[i] = Bfgs(pb);
    max_eval = std::max(max_eval, pb.max_eval);
    HostModel h = shape_only(m->h);
    h.tiles = choose_tiles(h.T, h.N, h.kind, h.prec, 1);
    off[i] = bytes;
    bytes += align4k(device_fit_bytes(h, true));
    hm.push_back(h);
    slot[i] = FitSlot{i, -1, m->h.P, 0, pb.final_tol, 0.0};
    if (o->polish) {
      HostModel g = shape_only(o->polish->h);
      g.tiles = choose_tiles(g.T, g.N, g.kind, g.prec, 1);
      offp[i] = bytes;
      bytes += align4k(device_fit_bytes(g, true));
      slot[i].fit_p = npl++;
      slot[i].noise_p = nll_noise(o->polish->h);
    }
    hp.push_back(o->polish ? shape_only(o->polish->h) : HostModel{});
    if (o->polish) hp.back().tiles = choose_tiles(hp.back().T, hp.back().N, hp.back().kind, hp.back().prec, 1);
  }
  Batch b;
  if (hipSetDevice(models[0]->device) != hipSuccess || hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess)
    return hip_fail(hipErrorUnknown, "stream");
  // the models' inputs are read in place: their pending work (a new data
  // set, say) first
  for (int i = 0; i < n; ++i)
    for (const bx_model* m : {(const bx_model*)models[i], (const bx_model*)opts[i].polish})
      if (m && m->last_stream && hipStreamSynchronize(m->last_stream) != hipSuccess)
        return hip_fail(hipErrorUnknown, "model stream");
  if (hipMalloc(&b.mem, bytes) != hipSuccess || hipMalloc((void**)&b.rows, sizeof(double) * 2 * kRow * n) != hipSuccess ||
      hipMalloc((void**)&b.d_fits, sizeof(FitDev) * (npl + 1)) != hipSuccess ||
      hipMalloc((void**)&b.d_slots, sizeof(FitSlot) * n) != hipSuccess ||
      hipMalloc((void**)&b.d_opts, sizeof(Bfgs) * n) != hipSuccess ||
      hipMalloc((void**)&b.d_lists, sizeof(int) * (npl + 8 * kGroups)) != hipSuccess ||
      hipMalloc((void**)&b.d_count, sizeof(int) * (1 + n)) != hipSuccess ||
      hipMalloc((void**)&b.d_ready, sizeof(int) * n) != hipSuccess ||
      hipHostMalloc((void**)&b.h_count, sizeof(int) * (1 + n), hipHostMallocDefault) != hipSuccess) {
    set_error("device memory for the batch could not be allocated");
    return BX_E_NOMEM;
  }
  // placements: theta and result rows per fit, shared by its two placements
  std::vector<FitDev> fd(npl + 1);  // + one that never runs: the padding of the launch lists
  std::vector<int> grp(npl);
  std::vector<LaunchShape> shp(npl);
  for (int i = 0; i < n; ++i) {
    for (int ph = 0; ph < 2; ++ph) {
      if (ph == 1 && slot[i].fit_p < 0) break;
      const bx_model* src = ph ? opts[i].polish : models[i];
      DeviceFit df;
      const bx_status s = place_fit(ph ? hp[i] : hm[i], (char*)b.mem + (ph ? offp[i] : off[i]), &df, b.st,
                                    &src->df.dev);
      if (s != BX_OK) return s;
      df.dev.theta = b.rows + (size_t)i * kRow;
      df.dev.out = b.rows + (size_t)(n + i) * kRow;
      df.dev.theta_src = nullptr;
      df.dev.out_host = nullptr;
      df.dev.skip = ph;  // the polishing placement waits
      const int k = ph ? slot[i].fit_p : i;
      fd[k] = df.dev;
      shp[k] = shape_of(df.dev);
      grp[k] = group_of(shp[k]);
    }
  }
  fd[npl] = fd[0];
  fd[npl].skip = 1;
  hipError_t e = hipMemcpyAsync(b.d_fits, fd.data(), sizeof(FitDev) * (npl + 1), hipMemcpyHostToDevice, b.st);
  if (e == hipSuccess) e = hipMemcpyAsync(b.d_slots, slot.data(), sizeof(FitSlot) * n, hipMemcpyHostToDevice, b.st);
  if (e == hipSuccess) e = hipMemcpyAsync(b.d_opts, opt.data(), sizeof(Bfgs) * n, hipMemcpyHostToDevice, b.st);
  if (e == hipSuccess) e = hipStreamSynchronize(b.st);  // the host arrays above are temporaries
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  for (int i = 0; i < n; ++i) results[i] = bx_fit_result{};
  launch_fit_start(b.d_opts, b.d_slots, b.d_fits, n, b.st);  // every fit's first point
  // One iteration of the running fits as a graph: each launch group lists
  // the placement each fit evaluates now (state 1: its first model; 2 or 3:
  // its polishing model, which a waiting fit moves to at its next step).
  std::vector<int> lists, state(n, 1), cur;
  auto capture = [&]() -> bx_status {
    cur.clear();
    b.h_ready.assign(n, 0);
    for (int i = 0; i < n; ++i)
      if (state[i]) {
        cur.push_back(i);
        b.h_ready[i] = state[i] >= 2;
      }
    struct G {
      int first, count;
      LaunchShape L;
    };
    std::vector<G> groups;
    lists.clear();
    for (int g = 0; g < kGroups; ++g) {
      G gr{(int)lists.size(), 0, LaunchShape{}};
      for (int i : cur) {
        const int k = state[i] >= 2 ? slot[i].fit_p : i;
        if (grp[k] == g) {
          lists.push_back(k);
          widen(&gr.L, shp[k]);
          ++gr.count;
        }
      }
      // a multiple of 8 fits: the kernels then keep each fit's blocks on one
      // XCD (a group of a few fits stays spread over all of them)
      while (gr.count >= 64 && (gr.count & 7)) {
        lists.push_back(npl);
        ++gr.count;
      }
      if (gr.count) groups.push_back(gr);
    }
    hipError_t er = hipMemcpyAsync(b.d_lists, lists.data(), sizeof(int) * lists.size(), hipMemcpyHostToDevice, b.st);
    if (er == hipSuccess) er = hipMemcpyAsync(b.d_ready, b.h_ready.data(), sizeof(int) * n, hipMemcpyHostToDevice, b.st);
    if (er == hipSuccess) er = hipStreamSynchronize(b.st);  // the host arrays are rewritten by the next capture
    if (er != hipSuccess) return hip_fail(er, "batch lists");
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
    hipGraph_t graph;
    er = hipStreamBeginCapture(b.st, hipStreamCaptureModeThreadLocal);
    if (er != hipSuccess) return hip_fail(er, "graph capture");
    for (const G& g : groups) launch_eval(b.d_fits, b.d_lists + g.first, g.count, g.L, true, b.st);
    launch_fit_step(b.d_opts, b.d_slots, b.d_fits, n, b.d_count, b.d_count + 1, b.d_ready, b.st);
    er = hipStreamEndCapture(b.st, &graph);
    if (er != hipSuccess) return hip_fail(er, "graph capture");
    er = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (er != hipSuccess) return hip_fail(er, "graph instantiate");
    return BX_OK;
  };
  bx_status cs = capture();
  if (cs != BX_OK) return cs;
  // replay until no fit is running (every fit ends within its evaluation
  // budget, one evaluation per iteration, and waits for its polishing
  // placement for fewer iterations than another fit runs)
  const int64_t t_start = now_ns();
  int steps = 0;
  for (bool running = true; running && steps <= 2 * max_eval + 4 * K + 8;) {
    for (int k = 0; k < K && e == hipSuccess; ++k, ++steps) e = hipGraphLaunch(b.exec, b.st);
    if (e == hipSuccess) e = hipMemcpyAsync(b.h_count, b.d_count, sizeof(int) * (1 + n), hipMemcpyDeviceToHost, b.st);
    if (e == hipSuccess) e = hipStreamSynchronize(b.st);
    if (e != hipSuccess) return hip_fail(e, "batch iteration");
    const int left = *b.h_count;
    running = left > 0;
    int waiting = 0;
    for (int i : cur) waiting += b.h_count[1 + i] == 2;
    // capture again when half of the graph's fits are done (their grids go),
    // or when an eighth of them (or all that run) wait for their polishing
    // placement
    const int nc = (int)cur.size();
    if (running && (2 * left <= nc || 8 * waiting >= nc || waiting == left)) {
      for (int i = 0; i < n; ++i) state[i] = b.h_count[1 + i];
      if ((cs = capture()) != BX_OK) return cs;
    }
  }
  e = hipMemcpyAsync(opt.data(), b.d_opts, sizeof(Bfgs) * n, hipMemcpyDeviceToHost, b.st);
  if (e == hipSuccess) e = hipStreamSynchronize(b.st);
  if (e != hipSuccess) return hip_fail(e, "batch results");
  const int64_t t_end = now_ns();
  for (int i = 0; i < n; ++i) {
    opt[i].result(results + i);
    results[i].t_submit_ns = t0;
    results[i].t_admit_ns = t_start;
    results[i].t_done_ns = t_end;
  }
  return BX_OK;
}

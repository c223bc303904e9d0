// Fit server: HBM-budget admission, resident per-fit state, and continuous
// batching -- every scheduler step evaluates the NLL and gradient of all
// active fits in one batched launch (per response kind and precision), then
// advances each fit's own minimiser by one step.  Fits join when memory and a
// slot free up and leave when they finish.  A fit's arithmetic depends only
// on its own shape and parameters (tile shapes from its own T and N, fixed
// reduction orders), so its result does not depend on the rest of the batch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bx_fitcore.hpp"
#include "bx_model.hpp"

namespace bx {

// Parallel for over the fits of a step: the scheduler thread and a few
// helpers take indices from a shared counter.  Each fit's minimiser state is
// touched by one thread only, so results do not depend on the pool.
class StepPool {
 public:
  explicit StepPool(int helpers) {
    for (int k = 0; k < helpers; ++k) th_.emplace_back([this] { loop(); });
  }
  ~StepPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int n, const std::function<void(int)>& f) {
    if (th_.empty() || n < 64) {  // small steps: not worth the hand-off
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      n_ = n;
      next_.store(0);
      busy_ = (int)th_.size();
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [this] { return busy_ == 0; });
    job_ = nullptr;
  }

 private:
  void work() {
    for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) (*job_)(i);
  }
  void loop() {
    uint64_t seen = 0;
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
      std::lock_guard<std::mutex> lk(mu_);
      if (--busy_ == 0) done_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* job_ = nullptr;
  int n_ = 0, busy_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr int kThetaStride = 40;  // theta[P] and the step number, 5 cache lines
constexpr int kOutStride = 40;    // nll, grad[P], flags, completion mark
constexpr int kSeqAt = 64;        // the step number in the mark's allocation (its own cache line)
constexpr int kGraphFits = 16;    // steps of at most this many fits are replayed from a graph

struct Req {
  uint64_t ticket = 0;
  bx_model* model = nullptr;
  HostModel h;             // shape and constants of the model (its arrays stay in the model)
  FitProblem pb;
  std::unique_ptr<Bfgs> opt;
  size_t bytes = 0;
  int slot = -1;
  void* mem = nullptr;
  DeviceFit df;            // host copy of the slot's FitDev (source of its upload)
  LaunchShape shape{};     // grid needs of this fit (set at admission)
  int group = 0;           // launch group: (kind, precision, multivariate, forward tiles per wave)
  bx_fit_result res{};
  bool done = false;
  // mixed precision: the FP64 model the fit moves to, and its placement in
  // the same allocation (after the first one's bytes1)
  bx_model* polish = nullptr;
  HostModel hp;
  DeviceFit dfp;
  LaunchShape shape_p{};
  int group_p = 0;
  size_t bytes1 = 0;
  bool polished = false;
};



}  // namespace bx

using namespace bx;

struct bx_server {
  size_t budget = 0, used = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  FitDev* d_fits = nullptr;       // [max_slots + 1]: the last one never runs (list padding)
  int* d_active = nullptr;        // [kGroups][max_slots + 8] active lists, one region per launch group
  double* d_theta = nullptr;      // [max_slots][kThetaStride] device copies of theta
  double* d_out = nullptr;        // [max_slots][kOutStride]
  // pinned, coherent: theta and the step number written by the host and read
  // by k_colparams; the results written by k_final; the step's completion
  // mark written by k_mark (each in its own allocation, so host-written and
  // device-written values never share a cache line)
  double* h_theta = nullptr;
  double* h_out = nullptr;
  double* h_mark = nullptr;
  double* dh_theta = nullptr;     // their device addresses
  double* dh_out = nullptr;
  double* dh_mark = nullptr;
  double seq = 0.0;               // steps so far (completion marks)
  int* h_active = nullptr;        // pinned
  // A step over the same fits as the last two is replayed from a graph
  // captured once (a few fits: their launches would otherwise cost the host
  // more than the device's work); the step number comes from h_mark[kSeqAt].
  hipGraphExec_t step_exec = nullptr;
  std::vector<uint64_t> step_key;
  int stable = 0;
  std::vector<int> free_slots;
  std::deque<std::shared_ptr<Req>> queue;
  std::vector<std::shared_ptr<Req>> active;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> tickets;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::thread worker;
  std::unique_ptr<StepPool> pool;  // helpers for the per-fit minimiser updates
  bool stop = false;
  int pending = 0;
  int device = 0;
};

static void retire(bx_server* s, const std::shared_ptr<Req>& r);

// Admit queued requests while slots and budget allow (called with mu held).
static void admit(bx_server* s) {
  while (!s->queue.empty() && !s->free_slots.empty()) {
    auto r = s->queue.front();
    if (s->used + r->bytes > s->budget) break;
    void* mem = nullptr;
    const bool got = hipMallocAsync(&mem, r->bytes, s->stream) == hipSuccess;
    if (!got && !s->active.empty()) break;  // retry when a fit leaves
    s->queue.pop_front();
    r->mem = mem;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->used += r->bytes;
    DeviceFit& df = r->df;
    bool placed = got && place_fit(r->h, mem, &df, s->stream, &r->model->df.dev) == BX_OK;
    if (placed && r->polish)
      placed = place_fit(r->hp, (char*)mem + r->bytes1, &r->dfp, s->stream, &r->polish->df.dev) == BX_OK;
    if (!placed) {
      r->res.status = BX_FAILED;
      retire(s, r);
      continue;
    }
    for (DeviceFit* d : {&r->df, &r->dfp}) {  // both read theta and write results in the slot's rows
      d->dev.theta = s->d_theta + (size_t)r->slot * kThetaStride;
      d->dev.out = s->d_out + (size_t)r->slot * kOutStride;
      d->dev.theta_src = s->dh_theta + (size_t)r->slot * kThetaStride;
      d->dev.out_host = s->dh_out + (size_t)r->slot * kOutStride;
    }
    r->shape = shape_of(df.dev);
    r->group = group_of(r->shape);
    if (r->polish) {
      r->shape_p = shape_of(r->dfp.dev);
      r->group_p = group_of(r->shape_p);
    }
    (void)hipMemcpyAsync(s->d_fits + r->slot, &df.dev, sizeof(FitDev), hipMemcpyHostToDevice, s->stream);
    r->res.t_admit_ns = now_ns();
    s->active.push_back(r);
  }
}

static void retire(bx_server* s, const std::shared_ptr<Req>& r) {
  if (r->mem) (void)hipFreeAsync(r->mem, s->stream);
  r->mem = nullptr;
  s->used -= r->bytes;
  s->free_slots.push_back(r->slot);
  r->res.t_done_ns = now_ns();
  r->done = true;
  r->model->users.fetch_sub(1);
  if (r->polish) r->polish->users.fetch_sub(1);
  --s->pending;
}

// One step: every active fit's next point in one batched launch per group.
// The kernels read theta from pinned memory and write the results there; the
// host spins on the step's completion mark, reading it (and then the
// results) past its own cache.  launch_step stages and enqueues (returning
// the step number), finish_step waits and hands the results to the
// minimisers (false when the launch failed); the worker admits new fits in
// between, while the step runs on the GPU.
// One batched launch per group of (kind, precision, forward tiles per wave),
// then the step's mark; with lists = false the groups' device lists are
// taken as in place.
static void enqueue_step(bx_server* s, const std::vector<std::shared_ptr<Req>>& act, bool lists) {
  for (int grp = 0; grp < kGroups; ++grp) {
    int n = 0;
    LaunchShape L{};
    int* act_list = s->h_active + (size_t)grp * (s->max_slots + 8);  // each group stages its own list
    int* d_list = s->d_active + (size_t)grp * (s->max_slots + 8);
    for (auto& r : act) {
      if (r->group != grp) continue;
      widen(&L, r->shape);
      act_list[n++] = r->slot;
    }
    if (!n) continue;
    // a multiple of 8 fits (the slot past the last never runs): the kernels
    // then keep each fit's blocks on one XCD
    while (n >= 64 && (n & 7)) act_list[n++] = s->max_slots;
    if (lists) (void)hipMemcpyAsync(d_list, act_list, sizeof(int) * n, hipMemcpyHostToDevice, s->stream);
    launch_eval(s->d_fits, d_list, n, L, true, s->stream);
  }
  launch_mark_from(s->dh_mark, s->dh_mark + kSeqAt, s->stream);
}

// Captures a step's launches (without the list copies) as a graph in
// s->step_exec; on failure it stays null and the step is launched directly.
static void capture_step(bx_server* s, const std::vector<std::shared_ptr<Req>>& act) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return;
  enqueue_step(s, act, false);
  if (hipStreamEndCapture(s->stream, &g) != hipSuccess || !g) return;
  if (hipGraphInstantiate(&s->step_exec, g, nullptr, nullptr, 0) != hipSuccess) s->step_exec = nullptr;
  (void)hipGraphDestroy(g);
}

static double launch_step(bx_server* s, std::vector<std::shared_ptr<Req>>& act) {
  const double seq = (s->seq += 1.0);
  // stage every active fit's next point (with the step number after it)
  s->pool->run((int)act.size(), [&](int k) {
    auto& r = act[k];
    double* th = s->h_theta + (size_t)r->slot * kThetaStride;
    r->opt->next(th);
    th[r->h.P] = seq;
    flush_lines(th, r->h.P + 1);
  });
  s->h_mark[kSeqAt] = seq;
  flush_lines(s->h_mark + kSeqAt, 1);
  // the same fits (and placements) as the last step?
  std::vector<uint64_t> key;
  key.reserve(act.size());
  for (auto& r : act) key.push_back(2 * r->ticket + (r->polished ? 1 : 0));
  if (key == s->step_key) {
    ++s->stable;
  } else {
    s->step_key.swap(key);
    s->stable = 0;
    if (s->step_exec) (void)hipGraphExecDestroy(s->step_exec);
    s->step_exec = nullptr;
  }
  // their device lists are in place since the last step: replay (capturing
  // the launches once)
  if (s->stable >= 2 && (int)act.size() <= kGraphFits) {
    if (!s->step_exec) capture_step(s, act);
    if (s->step_exec && hipGraphLaunch(s->step_exec, s->stream) == hipSuccess) return seq;
  }
  enqueue_step(s, act, true);
  return seq;
}

static bool finish_step(bx_server* s, std::vector<std::shared_ptr<Req>>& act, double seq) {
  const volatile double* mark = s->h_mark;
  for (unsigned it = 1;; ++it) {
    flush_lines(s->h_mark, 1);
    if (*mark == seq) break;
    if ((it & 1023u) == 0u) {
      const hipError_t q = hipStreamQuery(s->stream);
      flush_lines(s->h_mark, 1);
      if (*mark == seq) break;
      if (q != hipErrorNotReady) return false;  // failed, or finished without its mark
    }
    __builtin_ia32_pause();
  }
  s->pool->run((int)act.size(), [&](int k) {
    auto& r = act[k];
    const double* o = s->h_out + (size_t)r->slot * kOutStride;
    const int P = r->h.P;
    flush_lines(o, 2 + P);
    const int fl = (int)o[1 + P];
    const bool bad = (fl & (kBadSigma | kBadGG | kBadMu | kBadTheta | kZeroWidth)) != 0;
    r->opt->feed(bad ? INFINITY : o[0], o + 1);
  });
  return true;
}

static void worker_loop(bx_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    admit(s);
    if (s->active.empty()) {
      if (s->stop) break;
      s->cv.wait(lk);
      continue;
    }
    std::vector<std::shared_ptr<Req>> act = s->active;
    lk.unlock();
    const double seq = launch_step(s, act);
    lk.lock();
    admit(s);  // while the step runs; the new fits join the next one
    lk.unlock();
    const bool ok = finish_step(s, act, seq);
    lk.lock();
    if (!ok) {  // the device failed: every active fit ends as failed
      for (auto& r : s->active) {
        r->res.status = BX_FAILED;
        retire(s, r);
      }
      s->active.clear();
      s->cv_done.notify_all();
      continue;
    }
    std::vector<std::shared_ptr<Req>> keep;
    for (auto& r : s->active) {
      if (r->opt->done() && r->polish && !r->polished &&
          r->opt->polish(r->pb.final_tol, nll_noise(r->polish->h))) {
        // mixed precision: on to the FP64 placement, from the same point
        r->h = r->hp;
        r->df = r->dfp;
        r->shape = r->shape_p;
        r->group = r->group_p;
        r->polished = true;
        (void)hipMemcpyAsync(s->d_fits + r->slot, &r->df.dev, sizeof(FitDev), hipMemcpyHostToDevice, s->stream);
      }
      if (r->opt->done()) {
        r->opt->result(&r->res);
        retire(s, r);
      } else {
        keep.push_back(r);
      }
    }
    s->active.swap(keep);
    s->cv_done.notify_all();
  }
}

extern "C" {

bx_status bx_server_create(size_t hbm_budget_bytes, int32_t max_slots, void* hip_stream, bx_server** out) {
  if (!out) {
    set_error("out is NULL");
    return BX_E_INVAL;
  }
  *out = nullptr;
  bx_server* s = new (std::nothrow) bx_server();
  if (!s) return BX_E_NOMEM;
  s->max_slots = max_slots > 0 ? max_slots : 4096;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    set_error("no HIP device");
    return BX_E_DEVICE;
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete s;
    set_error("hipMemGetInfo failed");
    return BX_E_DEVICE;
  }
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return BX_E_DEVICE;
    }
    s->own_stream = true;
  }
  const size_t M = s->max_slots;
  if (hipMalloc(&s->d_fits, sizeof(FitDev) * (M + 1)) != hipSuccess ||
      hipMalloc(&s->d_active, sizeof(int) * kGroups * (M + 8)) != hipSuccess ||
      hipMalloc(&s->d_theta, sizeof(double) * kThetaStride * M) != hipSuccess ||
      hipMalloc(&s->d_out, sizeof(double) * kOutStride * M) != hipSuccess ||
      hipHostMalloc((void**)&s->h_theta, sizeof(double) * kThetaStride * M, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&s->h_out, sizeof(double) * kOutStride * M, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&s->h_mark, 4096, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&s->h_active, sizeof(int) * kGroups * (M + 8), hipHostMallocDefault) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->dh_theta, s->h_theta, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->dh_out, s->h_out, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&s->dh_mark, s->h_mark, 0) != hipSuccess) {
    bx_server_destroy(s);
    set_error("server allocation failed");
    return BX_E_NOMEM;
  }
  memset(s->h_theta, 0, sizeof(double) * kThetaStride * M);
  memset(s->h_out, 0, sizeof(double) * kOutStride * M);
  memset(s->h_mark, 0, 4096);
  // no dirty host line may later be written back over device results
  flush_lines(s->h_theta, kThetaStride * (int)M);
  flush_lines(s->h_out, kOutStride * (int)M);
  flush_lines(s->h_mark, 512);
  for (int i = (int)M - 1; i >= 0; --i) s->free_slots.push_back(i);
  {  // the padding entry of the launch lists: a fit that never runs
    FitDev pad{};
    pad.skip = 1;
    if (hipMemcpy(s->d_fits + M, &pad, sizeof pad, hipMemcpyHostToDevice) != hipSuccess) {
      bx_server_destroy(s);
      set_error("server allocation failed");
      return BX_E_DEVICE;
    }
  }
  const unsigned hc = std::thread::hardware_concurrency();
  s->pool.reset(new StepPool((int)std::min(7u, hc > 1 ? hc - 1 : 0u)));
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return BX_OK;
}

bx_status bx_server_destroy(bx_server* s) {
  if (!s) return BX_OK;
  if (s->worker.joinable()) {
    bx_server_drain(s);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
  }
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->step_exec) (void)hipGraphExecDestroy(s->step_exec);
  if (s->d_fits) (void)hipFree(s->d_fits);
  if (s->d_active) (void)hipFree(s->d_active);
  if (s->d_theta) (void)hipFree(s->d_theta);
  if (s->d_out) (void)hipFree(s->d_out);
  if (s->h_theta) (void)hipHostFree(s->h_theta);
  if (s->h_out) (void)hipHostFree(s->h_out);
  if (s->h_mark) (void)hipHostFree(s->h_mark);
  if (s->h_active) (void)hipHostFree(s->h_active);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return BX_OK;
}

bx_status bx_fit_submit(bx_server* s, bx_model* m, const bx_fit_opts* o, uint64_t* ticket) {
  if (!s || !m || !o || !o->x0 || !ticket) {
    set_error("NULL argument");
    return BX_E_INVAL;
  }
  auto r = std::make_shared<Req>();
  r->res.t_submit_ns = now_ns();
  bx_status st = fit_problem(m->h.P, m->h.S, o, &r->pb, m->h.pu_float ? m->h.P - 1 : -1);
  if (st != BX_OK) return st;
  r->pb.f_noise = nll_noise(m->h);
  if (o->polish && (st = polish_compatible(m, o->polish)) != BX_OK) return st;
  // the fit reads the model's inputs in place (the model stays busy while it
  // is pending) and gets its own workspace, with the batched tile widths
  r->h = shape_only(m->h);
  r->h.tiles = choose_tiles(r->h.T, r->h.N, r->h.kind, r->h.prec, 1);
  r->bytes = r->bytes1 = (device_fit_bytes(r->h, true) + 4095) & ~(size_t)4095;
  if (o->polish) {  // and a second workspace for the FP64 model's iterations
    r->hp = shape_only(o->polish->h);
    r->hp.tiles = choose_tiles(r->hp.T, r->hp.N, r->hp.kind, r->hp.prec, 1);
    r->bytes += (device_fit_bytes(r->hp, true) + 4095) & ~(size_t)4095;
  }
  if (r->bytes > s->budget) {
    set_error("request larger than the server's memory budget");
    return BX_E_BUSY;
  }
  r->opt.reset(new Bfgs(r->pb));
  r->model = m;
  m->users.fetch_add(1);
  if (o->polish) {
    r->polish = o->polish;
    r->polish->users.fetch_add(1);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->tickets[r->ticket] = r;
    s->queue.push_back(r);
    ++s->pending;
    *ticket = r->ticket;
  }
  s->cv.notify_all();
  return BX_OK;
}

bx_status bx_fit_poll(bx_server* s, uint64_t ticket, bx_fit_result* res) {
  if (!s || !res) {
    set_error("NULL argument");
    return BX_E_INVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) {
    set_error("unknown ticket");
    return BX_E_NOTFOUND;
  }
  if (!it->second->done) return BX_PENDING;
  *res = it->second->res;
  s->tickets.erase(it);
  return BX_OK;
}

bx_status bx_server_drain(bx_server* s) {
  if (!s) return BX_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending == 0; });
  return BX_OK;
}

}  // extern "C"

"""Benchmark: NLL + gradient evaluations per second of the full single fit
(3000 true x 900 reco bins, 12 species, generalized-gamma response, 2 %
pile-up, 3e6 events) on one MI355X, with its error against the FP64 oracle,
plus the batched form of the same evaluation, the other workloads (configs 1,
3a, 3b and the other response kinds), the batched toy fits, the served fits,
the roofline of the dominant kernel and the FP64 oracle on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--toys N] [--no-cpu]

One step = one NLL + gradient evaluation through the C ABI (theta uploaded
from the host, NLL and gradient downloaded, as a host minimiser needs them).
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

# the CPU baseline (oracle) is timed on one core
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad evals/s; toy fits/s batched vs plain; p50/p99 fit latency"
WORKLOAD = ("single fit, 3000 true x 900 reco bins (1 keV x 1 p.e.), 12 species, "
            "generalized-gamma response (light yield, 3 resolution params, quenching), "
            "2% pile-up (K=128), 3e6 events")
PEAK_FP32 = 157.3e12   # MI355X published dense FP32 vector FLOP/s
PEAK_HBM = 8.0e12      # MI355X published HBM3E bandwidth, bytes/s
# Algorithmic operations per cell of Eq. 1 (the response integrated over one
# reco bin) on the sweeps' path: the one-interval, four-node Gauss-Legendre
# quadrature of the generalized-gamma density in t = ln(y/k) (FP32), counted
# from the formula with add/mul/exp2 = 1 and FMA = 2.  Forward: the bin centre
# in t, the scale, phi(t) by its series (23), four nodes of 8 (phi at the
# node from the centre's, -k log2(e) phi, 2^x, weight, sum), the FP64 scale
# and the one FMA of the single-histogram contraction mu0 = R v: 63.  Backward:
# the same cell with its two column-parameter derivatives (7 more per node,
# 6 after the nodes) and the adjoint weights (7), without the contraction:
# 102.  The cells counted are those the method needs (oracle-counted: the
# cells between each column's [1e-12, 1 - 1e-12] quantile edges and the edges
# bracketing them), not the ones a kernel happens to evaluate.
FLOP_FWD_CELL = 63
FLOP_BWD_CELL = 102


def profiled(fname, key, name):
    """A per-kernel figure measured with rocprofv3 counters (a `key ...` line
    of profiles/fname), or None when the kernel sources changed since the
    counters were taken."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1805_11125_amd", "csrc")
    h = hashlib.sha256()
    for f in ("bx_kernels.hip", "bx_math.h", "bx_dev.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    try:
        text = open(os.path.join(ROOT, "profiles", fname)).read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith(key + " "):
            kv = dict(t.split("=") for t in line.split()[1:])
            if kv.get("src_sha") == h.hexdigest()[:16] and name in kv:
                return float(kv[name])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--toys", type=int, default=4096, help="batched toy fits to time (0 = skip)")
    ap.add_argument("--plain-toys", type=int, default=64, help="toys fitted on the plain path")
    ap.add_argument("--edm", type=float, default=1e-12, help="toy fits stop at EDM below this")
    ap.add_argument("--qps", type=str, default="10,30,100,300,1000", help="serving arrival rates ('' = skip)")
    ap.add_argument("--requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-seconds", type=float, default=15.0,
                    help="cap on each rate's arrival window: min(requests, rate x this) requests")
    ap.add_argument("--batch", type=int, default=512,
                    help="resident copies of the fit for the batched-launch timing (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle-check", dest="oracle_check", action="store_false",
                    help="skip the oracle errors of the GPU results")
    ap.add_argument("--no-table", dest="table", action="store_false",
                    help="skip the per-config, tabulated-response, count-estimator and joint-term legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def support():
    z = np.load(os.path.join(ROOT, "tests", "golden", "c2_support.npz"))
    return int(z["cells"]), int(z["edges"])


def host_info():
    """CPU model and the cores this process may use (where the oracle ran)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def oracle_errors(d, x, th, v, g):
    """The GPU result's error against the FP64 oracle at the same point: NLL
    absolute and relative, and the largest gradient component error over its
    magnitude scale sum_b |(1 - n_b/mu_b) dmu_b/dq| (the absolute summands of
    dNLL/dq).  Also returns the oracle's own wall time for the NLL+gradient."""
    import oracle
    t0 = time.perf_counter()
    v0, g0 = oracle.nll_grad(d, x, th)
    dt = time.perf_counter() - t0
    sc = oracle.grad_scale(d, x, th)
    sc = np.maximum(sc, 1e-20 * sc.max())
    e = np.abs(np.asarray(g) - g0) / sc
    return {"nll_abs": abs(v - v0), "nll_rel": abs(v - v0) / abs(v0), "grad_max_over_scale": float(e.max()),
            "grad_scale": "sum_b |(1 - n_b/mu_b) dmu_b/dq|"}, dt


def cpu_baseline(timed):
    """The FP64 oracle's NLL+gradient on the host, one thread: the config-2
    evaluation timed beside the GPU error check, and configs 1, 3a (median of
    5 at theta_true and at a perturbed theta) and 3b (one evaluation)."""
    import oracle
    import synth
    per = {}
    for name, reps in (("c1", 5), ("c3a", 5), ("c3b", 1)):
        d, x = synth.load(name)
        ts = []
        for th in (d.theta_true, d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))):
            for _ in range(reps):
                t0 = time.perf_counter()
                oracle.nll_grad(d, x, th)
                ts.append(time.perf_counter() - t0)
        per[name] = {"median_s": float(np.median(ts)), "evals": len(ts)}
    if "c2" in timed:
        per["c2"] = {"median_s": timed["c2"], "evals": 1}
    v = 1.0 / per["c2"]["median_s"] if "c2" in per else None
    return {"value": v, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 oracle NLL+gradient (dense scipy incomplete-gamma or ndtr cells, "
                      "numpy contraction, explicit pile-up, fsum NLL, Richardson response "
                      "derivatives), one thread: 1 evaluation of the 3000 x 900 workload "
                      "(value), plus per-config medians",
            "per_config_s": per, **host_info()}


def toy_study(bx, synth, n_toys, n_plain, edm):
    """Toy study (config 4): ragged Poisson pseudo-experiments of the config-2
    model, each fitted with FP32 cells until EDM < 1e-8 and then with its
    FP64 model until EDM < edm (mixed precision).  Three ways: the device-
    minimised batch (every fit's minimiser on the GPU, one iteration of all
    fits replayed as a HIP graph), the fit server (continuous batching, host
    minimisers), and the plain path one fit at a time (a sample).  Models and
    histograms are resident before any timing starts."""
    base, per_species, theta = synth.catalogue()
    t0 = time.perf_counter()
    toys = []
    for b in range(n_toys):
        t = synth.toy(b, per_species, theta)
        d = synth.toy_desc(base, t)
        x = synth.Data(energy=t.counts)
        toys.append((bx.Model(d, x, precision=bx.BX_PREC_F32), bx.Model(d, x, precision=bx.BX_PREC_F64), d, t))
    build_s = time.perf_counter() - t0
    m32 = [m for m, _, _, _ in toys]
    m64 = [p for _, p, _, _ in toys]
    x0s = [t.theta0 for _, _, _, t in toys]
    masks = [d.float_mask for _, _, d, _ in toys]
    t1 = time.perf_counter()
    graph = bx.fit_batch(m32, x0s, masks, edm_tol=edm, max_iter=500, polish=m64)
    el_g = time.perf_counter() - t1
    srv = bx.Server()
    t2 = time.perf_counter()
    tickets = [srv.submit(m, x0, float_mask=mk, edm_tol=edm, max_iter=500, polish=p)
               for m, p, x0, mk in zip(m32, m64, x0s, masks)]
    served = [srv.wait(k, sleep=2e-4) for k in tickets]
    el_s = time.perf_counter() - t2
    srv.close()
    n_plain = min(n_plain, n_toys)
    t3 = time.perf_counter()
    plain = [m.fit(x0, float_mask=mk, edm_tol=edm, max_iter=500, polish=p)
             for m, p, x0, mk in list(zip(m32, m64, x0s, masks))[:n_plain]]
    el_p = time.perf_counter() - t3
    same_g = all(np.array_equal(p.x, r.x) and p.nll == r.nll for p, r in zip(plain, graph))
    same_s = all(np.array_equal(g.x, r.x) and g.nll == r.nll for g, r in zip(graph, served))
    for m, p, _, _ in toys:
        m.close()
        p.close()
    st = np.array([r.status for r in graph])
    n_eval = np.array([r.n_eval for r in graph])
    return {"toys": n_toys, "edm_tol": edm, "precision": "FP32 cells, FP64 from EDM < 1e-8",
            "device_minimised_fits_per_s": n_toys / el_g, "server_fits_per_s": n_toys / el_s,
            "plain_fits_per_s": n_plain / el_p, "plain_sample": n_plain,
            "speedup_device_vs_plain": (n_toys / el_g) / (n_plain / el_p),
            "device_minimised_evals_per_s": float(n_eval.sum()) / el_g,
            "converged": int((st == bx.BX_CONVERGED).sum()),
            "median_iters": float(np.median([r.n_iter for r in graph])),
            "median_evals": float(np.median(n_eval)), "max_evals": int(n_eval.max()),
            "device_equals_plain_bitwise": bool(same_g), "server_equals_device_bitwise": bool(same_s),
            "model_build_s": build_s}


def config_leg(bx, synth, name, prec, steps, warmup, copies, check, timed):
    """Plain-path NLL+gradient evaluations per second of one of the other
    workloads (config 1: 400 x 200 Gaussian; 3a / 3b: the multivariate
    likelihood of Eqs. 3-4 on configs 1 and 2), the batched form of the same
    evaluation, and the result's error against the oracle."""
    d, x = synth.load(name)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    m = bx.Model(d, x, precision=prec)
    for _ in range(warmup):
        m.nll_grad(th)
    t1 = time.perf_counter()
    for _ in range(steps):
        m.nll_grad(th)
    evals = steps / (time.perf_counter() - t1)
    v, g = m.nll_grad(th)
    rec = {"workload": f"{d.T} true x {d.N} reco bins, {d.S} species, {d.kind} response, "
                       f"{'multivariate' if d.multivariate else 'single histogram'}",
           "precision": "FP32 cells" if prec == bx.BX_PREC_F32 else "FP64", "evals_per_s": evals}
    if copies > 0:
        bt = m.batch_times(th, copies, reps=5)
        rec["batched"] = {"copies": copies, "evals_per_s": copies / (bt["total"] * 1e-3)}
    m.close()
    if check:
        rec["oracle_error"], timed[name] = oracle_errors(d, x, th, v, g)
    return rec


def table_leg(bx, synth, x, steps, warmup):
    """Tabulated (Monte Carlo) response on the config-2 grid: five 900 x 3000
    tables at light yields 480-520 p.e./MeV, the light yield the fitted
    coordinate.  The build forms M_g = R_g F^T once (FP64 MFMA); each
    evaluation interpolates M and runs the row terms."""
    d = synth.table_config()
    t0 = time.perf_counter()
    m = bx.Model(d, x, precision=bx.BX_PREC_F64)
    build_s = time.perf_counter() - t0
    th = d.theta_true.copy()
    th[d.S] = 503.7
    for _ in range(warmup):
        m.nll_grad(th)
    t1 = time.perf_counter()
    for _ in range(steps):
        m.nll_grad(th)
    evals = steps / (time.perf_counter() - t1)
    st = m.stage_times(th, reps=200)
    m.close()
    G, N, T = d.table_R.shape
    return {"workload": f"{G} tables {N} x {T}, {d.S} species, FP64", "evals_per_s": evals,
            "build_s": build_s, "build_gemm_flop": 2 * G * N * T * 16, "build_gemm_bytes": G * N * T * 8,
            "stage_ms": {("table" if k == "colparams" else k): round(v, 5) for k, v in st.items()
                         if v > 0 or k == "total"}}


def count_leg(bx, synth, steps, warmup):
    """Count estimator (fired PMTs, one reco bin per count) on the config-2
    species: 3000 true bins x 1000 counts, negative-binomial cells in FP64."""
    d = synth.count_config()
    x = synth.count_events(d, d.theta_true, seed=0)
    m = bx.Model(d, x, precision=bx.BX_PREC_F64)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    for _ in range(warmup):
        m.nll_grad(th)
    t1 = time.perf_counter()
    for _ in range(steps):
        m.nll_grad(th)
    evals = steps / (time.perf_counter() - t1)
    st = m.stage_times(th, reps=100)
    m.close()
    return {"workload": f"{d.T} true bins x {d.N} counts, {d.S} species, FP64", "evals_per_s": evals,
            "stage_ms": {k: round(v, 5) for k, v in st.items() if v > 0 or k == "total"}}


def joint_leg(bx, synth, steps, warmup):
    """Joint energy x radius x pulse-shape term on the config-3b model (900 reco
    bins x 100 radial x 50 pulse-shape bins = 4.5e6 bins, generalized-gamma
    cells in FP32), histograms from simulated events."""
    d = synth.config3b(synth.pileup_spectrum())
    d.joint = True
    x = synth.joint_events(d, d.theta_true, seed=0)
    m = bx.Model(d, x, precision=bx.BX_PREC_F32)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    for _ in range(warmup):
        m.nll_grad(th)
    t1 = time.perf_counter()
    for _ in range(steps):
        m.nll_grad(th)
    evals = steps / (time.perf_counter() - t1)
    st = m.stage_times(th, reps=100)
    m.close()
    nb = d.N * d.rad_tmpl.shape[1] * d.ps_tmpl.shape[1]
    nnz = int(np.count_nonzero(x.joint))
    jms = st["radial"]  # stage 4: the joint kernel
    # the kernel reads the non-zero bins (4-byte bin index + 8-byte count) and
    # the row starts; the closed-form sum covers the empty bins
    sparse = 12 * nnz + 4 * (d.N + 1)
    return {"workload": f"{d.N} x {d.rad_tmpl.shape[1]} x {d.ps_tmpl.shape[1]} joint bins, {d.S} species",
            "evals_per_s": evals, "stage_ms": {("joint" if k == "radial" else k): round(v, 5) for k, v in st.items()},
            "joint_kernel": {"bins": nb, "nonzero_bins": nnz, "bytes_read": sparse, "ms": jms,
                             "GB_per_s": sparse / (jms * 1e-3) / 1e9 if jms > 0 else None,
                             "bins_per_s": nb / (jms * 1e-3) if jms > 0 else None}}


def serving(bx, synth, qps_list, n_max, window_s):
    import torch
    """Poisson arrivals mixing config-1 fits (Gaussian, FP64), config-2 fits
    (generalized gamma, FP32) with fresh Poisson data, and NLL+gradient
    requests through the autograd path; latency = done - submit.  The plain
    baseline serves the same stream first-in first-out through the plain path
    on one thread."""
    d1, d2 = synth.config1(), synth.config2(pu_g=synth.pileup_spectrum())
    tab1, tab2 = synth.species_table("c1"), synth.species_table("c2")
    out = {}
    for qps in qps_list:
        n_req = int(min(n_max, max(100, round(qps * window_s))))
        reqs, rng = synth.request_stream(qps, n_req)
        jobs = []
        for r in reqs:
            d, tab, prec = (d1, tab1, bx.BX_PREC_F64) if r.kind == "fit1" else (d2, tab2, bx.BX_PREC_F32)
            n = synth.draw_species_sum(rng, tab, d.theta_true[: d.S])
            m = bx.Model(d, synth.Data(energy=n), precision=prec)
            z = rng.standard_normal(d.P)
            x0 = d.theta_true * (1 + (0.01 if r.kind == "evalgrad" else 0.05) * z)
            x0[~d.float_mask] = d.theta_true[~d.float_mask]
            jobs.append((r, m, x0, d.float_mask))
        srv = bx.Server()
        t0 = time.perf_counter()
        tickets, ag = [], {}
        for n_r, (r, m, x0, mask) in enumerate(jobs):
            dt = t0 + r.t_arrival - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            if r.kind == "evalgrad":
                # the autograd path (torch's stream), while the server's fits run
                s0 = time.perf_counter_ns()
                th_t = torch.tensor(x0, dtype=torch.float64, device="cuda", requires_grad=True)
                loss = bx.NLLFunction.apply(m, th_t)
                loss.backward()
                th_t.grad.cpu()
                ag[n_r] = (s0, time.perf_counter_ns())
                tickets.append(None)
            else:
                tickets.append(srv.submit(m, x0, float_mask=mask, edm_tol=1e-8, max_iter=500))
        res = [srv.wait(k, sleep=2e-4) if k is not None else None for k in tickets]
        t_sub = [ag[i][0] if x is None else x.t_submit_ns for i, x in enumerate(res)]
        t_done = [ag[i][1] if x is None else x.t_done_ns for i, x in enumerate(res)]
        srv.close()
        fits = [x for x in res if x is not None]
        span = (max(x.t_done_ns for x in fits) - min(x.t_submit_ns for x in fits)) * 1e-9 if fits else 0.0
        lat = (np.array(t_done) - np.array(t_sub)) * 1e-9
        kinds = np.array([r.kind for r, *_ in jobs])
        # plain FIFO baseline on the same stream
        t_free, plat = 0.0, []
        for r, m, x0, mask in jobs:
            s0 = time.perf_counter()
            if r.kind == "evalgrad":
                m.nll_grad(x0)
            else:
                m.fit(x0, float_mask=mask, edm_tol=1e-8, max_iter=500)
            dur = time.perf_counter() - s0
            start = max(r.t_arrival, t_free)
            t_free = start + dur
            plat.append(t_free - r.t_arrival)
        plat = np.array(plat)
        n_fit = int((kinds != "evalgrad").sum())
        rec = {"requests": n_req, "fits_per_s": n_fit / (span + 1e-12) if span > 0 else None,
               "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
               "plain_p50_s": float(np.percentile(plat, 50)), "plain_p99_s": float(np.percentile(plat, 99)),
               "plain_fits_per_s": n_fit / max(t_free, 1e-12),
               "converged": int(sum(x.status == bx.BX_CONVERGED for x in fits)),
               "evalgrad_path": "autograd (NLLFunction on torch's stream)"}
        for k in ("fit1", "fit2", "evalgrad"):
            sel = lat[kinds == k]
            if len(sel):
                rec[f"{k}_p50_s"] = float(np.percentile(sel, 50))
                rec[f"{k}_p99_s"] = float(np.percentile(sel, 99))
        out[str(qps)] = rec
        for _, m, _, _ in jobs:
            m.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1805_11125_amd as bx
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    if a.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 5}))
        return
    d, x = synth.load("c2")
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    m = bx.Model(d, x, precision=bx.BX_PREC_F32)
    for _ in range(a.warmup):
        m.nll_grad(th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        m.nll_grad(th)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    evals = a.steps / el
    v_gpu, g_gpu = m.nll_grad(th)

    # device-pointer path (autograd entry point), stream-ordered, no host sync per eval
    thd = torch.tensor(th, dtype=torch.float64, device="cuda")
    out = torch.empty(d.P + 1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(a.warmup):
        m.nll_grad_dev(thd.data_ptr(), out.data_ptr(), stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(a.steps):
        m.nll_grad_dev(thd.data_ptr(), out.data_ptr(), stream)
    torch.cuda.synchronize()
    dev_evals = a.steps / (time.perf_counter() - t1)

    # the dominant kernel: the backward cell sweep (cells, their two
    # derivatives and the adjoint weights), main sweep plus its fix-up sweep,
    # timed with HIP events on the model's stream (each stage launched back
    # to back on its own)
    st = m.stage_times(th, reps=200)
    cells, edges = support()

    def roofline(bwd_ms, bwd_main_ms, units):
        ach = units * cells * FLOP_BWD_CELL / (bwd_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": ach * 1e12 / PEAK_FP32, "kernel": "k_cells_bwd + k_cells_bwd_fix",
                "kernel_ms": bwd_ms, "main_sweep_ms": bwd_main_ms, "cells_per_launch": units * cells,
                "flop_per_cell": FLOP_BWD_CELL}

    rl = roofline(st["cells_bwd"], st["cells_bwd_main"], 1)
    t_main = profiled("config2_hbm_counters.md", "traffic_bytes", "k_cells_bwd")
    t_fix = profiled("config2_hbm_counters.md", "traffic_bytes", "k_cells_bwd_fix")
    rl["traffic"] = t_main + t_fix if t_main is not None and t_fix is not None else None
    rl["traffic_unit"] = ("HBM bytes per launch of k_cells_bwd and k_cells_bwd_fix (rocprofv3 FETCH_SIZE + "
                          "WRITE_SIZE, calibrated against a 256 MiB copy)")
    rl["valu_issue_frac"] = profiled("config2_valu_counters.md", "valu_issue", "k_cells_bwd")
    ceil_cps = m.cell_ceiling(th, reps=64)
    rl["measured_ceiling"] = {
        "cells_per_s": ceil_cps, "TFLOP_s": ceil_cps * FLOP_BWD_CELL / 1e12,
        "backward_cells_per_s": cells / (st["cells_bwd"] * 1e-3),
        "what": "registers-only evaluation of the backward cell (value and two derivatives) in the "
                "sweeps' lane layout, one (true tile, reco tile) of the workload per wave"}
    fwd = {"kernel": "k_cells_fwd + k_cells_fwd_fix", "kernel_ms": st["cells_fwd"],
           "main_sweep_ms": st["cells_fwd_main"], "flop_per_cell": FLOP_FWD_CELL,
           "TFLOP_s": cells * FLOP_FWD_CELL / (st["cells_fwd"] * 1e-3) / 1e12}
    fwd["frac"] = fwd["TFLOP_s"] * 1e12 / PEAK_FP32
    res = {
        "metric": METRIC, "value": evals, "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 / evals,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "T": d.T, "N": d.N, "S": d.S,
                   "path": "plain (host theta in, NLL+grad out, per evaluation)"},
        "dev_path_evals_per_s": dev_evals,
        "stage_ms": {k: round(v, 5) for k, v in st.items()},
        "roofline": rl, "forward_sweep": fwd,
        "support": {"cells": cells, "edges": edges, "q": 1e-12},
    }
    if a.batch > 0:
        # one launch per stage over `batch` resident copies (HIP events on the
        # model's stream): throughput of the batched form of the same evaluation
        bt = m.batch_times(th, a.batch, reps=10)
        brl = roofline(bt["cells_bwd"], bt["cells_bwd_main"], a.batch)
        brl["forward_TFLOP_s"] = a.batch * cells * FLOP_FWD_CELL / (bt["cells_fwd"] * 1e-3) / 1e12
        brl["frac_of_ceiling"] = a.batch * cells / (bt["cells_bwd"] * 1e-3) / ceil_cps
        brl["valu_issue_frac"] = profiled("config2_valu_counters.md", "valu_issue", "k_cells_bwd_batched")
        res["batched_eval"] = {
            "copies": a.batch, "evals_per_s": a.batch / (bt["total"] * 1e-3),
            "us_per_eval": bt["total"] * 1e3 / a.batch,
            "stage_us_per_eval": {k: round(v * 1e3 / a.batch, 4) for k, v in bt.items()},
            "roofline": brl}
        print(f"batched: {res['batched_eval']}", file=sys.stderr, flush=True)
    m.close()
    timed = {}
    if a.oracle_check:
        res["oracle_error"], timed["c2"] = oracle_errors(d, x, th, v_gpu, g_gpu)
        print(f"oracle error: {res['oracle_error']}", file=sys.stderr, flush=True)
    if a.table:
        # the other workloads, response kinds and likelihood forms (reported
        # beside the headline; a failure is recorded, not fatal to the line)
        ck = a.oracle_check
        legs = (("config1", lambda: config_leg(bx, synth, "c1", bx.BX_PREC_F64, min(a.steps, 3000), a.warmup,
                                                a.batch, ck, timed)),
                ("config3a", lambda: config_leg(bx, synth, "c3a", bx.BX_PREC_F64, min(a.steps, 3000), a.warmup,
                                                 a.batch, ck, timed)),
                ("config3b", lambda: config_leg(bx, synth, "c3b", bx.BX_PREC_F32, min(a.steps, 2000), a.warmup,
                                                 min(a.batch, 128), ck, timed)),
                ("tabulated_response", lambda: table_leg(bx, synth, x, min(a.steps, 3000), a.warmup)),
                ("count_estimator", lambda: count_leg(bx, synth, min(a.steps, 500), min(a.warmup, 20))),
                ("joint_term", lambda: joint_leg(bx, synth, min(a.steps, 500), min(a.warmup, 20))))
        for key, fn in legs:
            try:
                res[key] = fn()
            except Exception as e:  # noqa: BLE001
                res[key] = {"error": f"{type(e).__name__}: {e}"}
            print(f"{key}: {res[key]}", file=sys.stderr, flush=True)
    if a.toys > 0:
        res["toy_study"] = toy_study(bx, synth, a.toys, a.plain_toys, a.edm)
        print(f"toys: {res['toy_study']}", file=sys.stderr, flush=True)
    if a.qps:
        res["serving"] = serving(bx, synth, [float(q) for q in a.qps.split(",")], a.requests,
                                 a.serve_seconds)
        print(f"serving: {res['serving']}", file=sys.stderr, flush=True)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(timed)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

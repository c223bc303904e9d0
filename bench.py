"""Benchmark: NLL + gradient evaluations per second of the full single fit
(3000 true x 900 reco bins, 12 species, generalized-gamma response, 2 %
pile-up, 3e6 events) on one MI355X, plus the batched toy-fit and served-fit
figures, the roofline of the dominant kernel and the FP64 oracle on the host.

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
# Algorithmic operations per CDF edge evaluation on the dominant code path
# (the uniform expansion of the incomplete gamma, |eta| < 1), counted from the
# formula: add/mul/transcendental = 1, FMA = 2.  The forward sweep of an
# NLL+gradient evaluation forms the edge CDF (130) and its two column-
# parameter derivatives (27), plus the species contraction of its cell, 2 S;
# the backward sweep then only weights the stored derivative differences by
# the adjoint (5 per edge: one product, two multiply-adds) and is bound by
# reading them (one FP32 pair, 8 bytes, per edge).  The edges counted are
# those the method needs (oracle-counted: each column's [1e-12, 1 - 1e-12]
# quantile support plus its two bracketing edges), not the ones a kernel
# happens to evaluate.
FLOP_FWD_EDGE = 157
FLOP_BWD_EDGE = 5
BYTES_BWD_EDGE = 8
PEAK_HBM = 8.0e12      # MI355X published HBM3E bandwidth, bytes/s


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
    ap.add_argument("--toys", type=int, default=1024, help="batched toy fits to time (0 = skip)")
    ap.add_argument("--plain-toys", type=int, default=64, help="toys fitted on the plain path")
    ap.add_argument("--qps", type=str, default="30,300", help="serving arrival rates ('' = skip)")
    ap.add_argument("--requests", type=int, default=200, help="requests per arrival rate")
    ap.add_argument("--batch", type=int, default=512,
                    help="resident copies of the fit for the batched-launch timing (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-table", dest="table", action="store_false",
                    help="skip the tabulated-response, count-estimator and joint-term legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def support_edges():
    z = np.load(os.path.join(ROOT, "tests", "golden", "c2_support.npz"))
    return int(z["edges"])


def cpu_baseline(d, x, th, budget_s=12.0):
    import oracle
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.nll_grad(d, x, th)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 5:
            break
    return {"value": n / el, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} FP64 oracle NLL+gradient evaluations of the same workload "
                      f"(dense scipy incomplete-gamma cells, Richardson dR/dk), one thread"}


def toy_study(bx, synth, n_toys, n_plain):
    """Batched toy fits through the fit server vs the same toys fitted one
    at a time through the plain path (histograms resident before timing)."""
    base, per_species, theta = synth.catalogue()
    toys = []
    for b in range(n_toys):
        t = synth.toy(b, per_species, theta)
        d = synth.toy_desc(base, t)
        toys.append((bx.Model(d, synth.Data(energy=t.counts), precision=bx.BX_PREC_F32), d, t))
    srv = bx.Server()
    t0 = time.perf_counter()
    tickets = [srv.submit(m, t.theta0, float_mask=d.float_mask, edm_tol=1e-8, max_iter=500)
               for m, d, t in toys]
    res = [srv.wait(k, sleep=2e-4) for k in tickets]
    el = time.perf_counter() - t0
    srv.close()
    n_plain = min(n_plain, n_toys)
    t1 = time.perf_counter()
    plain = [m.fit(t.theta0, float_mask=d.float_mask, edm_tol=1e-8, max_iter=500)
             for m, d, t in toys[:n_plain]]
    el_p = time.perf_counter() - t1
    same = all(np.array_equal(p.x, r.x) for p, r in zip(plain, res))
    for m, _, _ in toys:
        m.close()
    st = np.array([r.status for r in res])
    # NLL+gradient evaluations the fits asked for, per second of wall time
    ev_b = sum(r.n_eval for r in res) / el
    ev_p = sum(r.n_eval for r in plain) / el_p
    return {"toys": n_toys, "batched_fits_per_s": n_toys / el, "plain_fits_per_s": n_plain / el_p,
            "batched_evals_per_s": ev_b, "plain_evals_per_s": ev_p,
            "plain_sample": n_plain, "speedup": (n_toys / el) / (n_plain / el_p),
            "converged": int((st == bx.BX_CONVERGED).sum()),
            "median_iters": float(np.median([r.n_iter for r in res])),
            "median_evals": float(np.median([r.n_eval for r in res])),
            "batched_equals_plain_bitwise": bool(same), "edm_tol": 1e-8}


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


def serving(bx, synth, qps_list, n_req):
    """Poisson arrivals mixing config-1 fits (Gaussian, FP64), config-2 fits
    (generalized gamma, FP32) with fresh Poisson data, and NLL+gradient
    requests; latency = done - submit.  The plain baseline serves the same
    stream first-in first-out through the plain path on one thread."""
    d1, d2 = synth.config1(), synth.config2(pu_g=synth.pileup_spectrum())
    tab1, tab2 = synth.species_table("c1"), synth.species_table("c2")
    out = {}
    for qps in qps_list:
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
        tickets = []
        for r, m, x0, mask in jobs:
            dt = t0 + r.t_arrival - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            kind = bx.BX_EVAL_GRAD if r.kind == "evalgrad" else bx.BX_FIT
            tickets.append(srv.submit(m, x0, float_mask=mask, edm_tol=1e-8, max_iter=500, kind=kind))
        res = [srv.wait(k, sleep=2e-4) for k in tickets]
        span = (max(x.t_done_ns for x in res) - min(x.t_submit_ns for x in res)) * 1e-9
        srv.close()
        lat = np.array([x.latency_s for x in res])
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
               "converged": int(sum(x.status == bx.BX_CONVERGED for x in res))}
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

    # device-pointer path (autograd entry point), stream-ordered, no host sync per eval
    thd = torch.tensor(th, dtype=torch.float64, device="cuda")
    out = torch.empty(d.P + 1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(a.warmup):
        m.nll_grad_dev(thd.data_ptr(), out.data_ptr(), stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ndev = a.steps
    for _ in range(ndev):
        m.nll_grad_dev(thd.data_ptr(), out.data_ptr(), stream)
    torch.cuda.synchronize()
    dev_evals = ndev / (time.perf_counter() - t1)

    st = m.stage_times(th, reps=200)
    edges = support_edges()
    fwd_ms, bwd_ms = st["cells_fwd"], st["cells_bwd"]
    if bwd_ms >= fwd_ms:  # the backward sweep reads the stored differences: HBM-bound
        kname, kms = "k_cells_bwd", bwd_ms
        rl = {"bound": "hbm", "achieved": edges * BYTES_BWD_EDGE / (kms * 1e-3) / 1e9,
              "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    else:
        kname, kms = "k_cells_fwd", fwd_ms
        rl = {"bound": "alu", "achieved": edges * (FLOP_FWD_EDGE + 2 * d.S) / (kms * 1e-3) / 1e12,
              "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s"}
    rl["frac"] = rl["achieved"] / rl["peak"]
    # measured ceiling: the edge arithmetic alone, same column/edge mix
    ceil_eps = m.edge_ceiling(th, reps=64)
    fwd_eps = edges / (fwd_ms * 1e-3)
    ceiling = {"edges_per_s": ceil_eps, "TFLOP_s": ceil_eps * FLOP_FWD_EDGE / 1e12,
               "forward_edges_per_s": fwd_eps, "forward_frac_of_ceiling": fwd_eps / ceil_eps,
               "what": "registers-only evaluation of the edge CDF and its two derivatives in the "
                       "forward sweep's lane layout, one (true tile, reco tile) of the workload per wave"}
    traffic = profiled("config2_hbm_counters.md", "traffic_bytes", kname)
    valu = profiled("config2_valu_counters.md", "valu_issue", kname)
    res = {
        "metric": METRIC, "value": evals, "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 / evals,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "T": d.T, "N": d.N, "S": d.S,
                   "path": "plain (host theta in, NLL+grad out, per evaluation)"},
        "dev_path_evals_per_s": dev_evals,
        "stage_ms": {k: round(v, 5) for k, v in st.items()},
        "roofline": {**rl, "kernel": kname, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "edges_per_launch": edges,
                     "flop_per_edge": FLOP_FWD_EDGE + 2 * d.S if kname == "k_cells_fwd" else FLOP_BWD_EDGE,
                     "valu_issue_frac": valu,
                     "kernel_ms": kms, "measured_ceiling": ceiling},
    }
    if a.batch > 0:
        # one launch per stage over `batch` resident copies (HIP events on the
        # model's stream): throughput of the batched form of the same evaluation
        bt = m.batch_times(th, a.batch, reps=10)
        bk = "cells_bwd" if bt["cells_bwd"] >= bt["cells_fwd"] else "cells_fwd"
        if bk == "cells_bwd":
            brl = {"bound": "hbm", "achieved": a.batch * edges * BYTES_BWD_EDGE / (bt[bk] * 1e-3) / 1e9,
                   "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
        else:
            brl = {"bound": "alu", "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                   "achieved": a.batch * edges * (FLOP_FWD_EDGE + 2 * d.S) / (bt[bk] * 1e-3) / 1e12}
        brl["frac"] = brl["achieved"] / brl["peak"]
        fwd_tf = a.batch * edges * (FLOP_FWD_EDGE + 2 * d.S) / (bt["cells_fwd"] * 1e-3) / 1e12
        bwd_gb = a.batch * edges * BYTES_BWD_EDGE / (bt["cells_bwd"] * 1e-3) / 1e9
        res["batched_eval"] = {
            "copies": a.batch, "evals_per_s": a.batch / (bt["total"] * 1e-3),
            "us_per_eval": bt["total"] * 1e3 / a.batch,
            "stage_us_per_eval": {k: round(v * 1e3 / a.batch, 4) for k, v in bt.items()},
            "roofline": {**brl, "kernel": "k_" + bk, "edges_per_launch": a.batch * edges,
                         "kernel_ms": bt[bk]},
            "forward_TFLOP_s": fwd_tf, "forward_frac": fwd_tf * 1e12 / PEAK_FP32,
            "forward_frac_of_ceiling": a.batch * edges / (bt["cells_fwd"] * 1e-3) / ceil_eps,
            "backward_GB_s": bwd_gb, "backward_frac": bwd_gb * 1e9 / PEAK_HBM}
        print(f"batched: {res['batched_eval']}", file=sys.stderr, flush=True)
    m.close()
    if a.table:
        # the other response kinds and likelihood forms (reported beside the
        # headline; a failure is recorded, not fatal to the line)
        legs = (("tabulated_response", lambda: table_leg(bx, synth, x, min(a.steps, 3000), a.warmup)),
                ("count_estimator", lambda: count_leg(bx, synth, min(a.steps, 500), min(a.warmup, 20))),
                ("joint_term", lambda: joint_leg(bx, synth, min(a.steps, 500), min(a.warmup, 20))))
        for key, fn in legs:
            try:
                res[key] = fn()
            except Exception as e:  # noqa: BLE001
                res[key] = {"error": f"{type(e).__name__}: {e}"}
            print(f"{key}: {res[key]}", file=sys.stderr, flush=True)
    if a.toys > 0:
        res["toy_study"] = toy_study(bx, synth, a.toys, a.plain_toys)
        print(f"toys: {res['toy_study']}", file=sys.stderr, flush=True)
    if a.qps:
        res["serving"] = serving(bx, synth, [float(q) for q in a.qps.split(",")], a.requests)
        print(f"serving: {res['serving']}", file=sys.stderr, flush=True)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d, x, th)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

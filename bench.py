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
# algorithmic FP32 operations per response cell (see the design notes):
# forward = CDF at the cell's upper edge (uniform expansion, 149) + species
# contraction (2 S = 24); backward = CDF with both parameter derivatives (185)
FLOP_FWD_PER_CELL = 149 + 24
FLOP_BWD_PER_CELL = 185


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--toys", type=int, default=0, help="batched toy fits to time (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def support_cells():
    z = np.load(os.path.join(ROOT, "tests", "golden", "c2_support.npz"))
    return int(z["cells"])


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


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1805_11125_amd as bx
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
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
    cells = support_cells()
    fwd_ms, bwd_ms = st["cells_fwd"], st["cells_bwd"]
    if bwd_ms >= fwd_ms:
        kname, kms, flops = "k_cells_bwd", bwd_ms, cells * FLOP_BWD_PER_CELL
    else:
        kname, kms, flops = "k_cells_fwd", fwd_ms, cells * FLOP_FWD_PER_CELL
    achieved = flops / (kms * 1e-3)
    res = {
        "metric": METRIC, "value": evals, "unit": "evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 / evals,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "T": d.T, "N": d.N, "S": d.S,
                   "path": "plain (host theta in, NLL+grad out, per evaluation)"},
        "dev_path_evals_per_s": dev_evals,
        "stage_ms": {k: round(v, 5) for k, v in st.items()},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": None,
                     "cells_per_launch": cells, "kernel_ms": kms},
    }
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d, x, th)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

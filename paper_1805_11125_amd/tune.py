"""Tile autotuner for the cell sweeps.

For each shape class it builds a representative model and times every
candidate pair of true tiles per forward wave (CG) and reco tiles per
backward wave (RG) on the device, once for a fit evaluated alone
(whole-evaluation time of the back-to-back stage launches,
`bx_model_stage_times`) and once for a batch of resident fits
(`bx_model_batch_times`, time per fit).  It writes the table the library
reads at model build and at admission to the fit server (BX_TUNE_CACHE):

    kind prec Tmin Tmax Nmin Nmax batched CG RG

CG changes no result bit (the forward partials are summed in a fixed tree),
so the two modes take their own best CG.  RG groups the backward partials, so
both modes share one RG (a fit gives the same bits alone and in a batch): the
one whose best times, alone and batched, are together the least above the
best of each mode, the time alone counted `ws` times (3 for the shape class of
the 3000 x 900 single fit, whose latency the plain path serves; 1 otherwise).  The block sizes (waves per forward and backward
workgroup, fits per workgroup = 1) are compile-time constants of the kernels,
chosen by the measurements recorded with them.

    python -m paper_1805_11125_amd.tune --out paper_1805_11125_amd/tiles_mi355x.txt
"""
import argparse
import os
import sys

import numpy as np

CANDIDATES = (1, 2, 4, 8)      # CG
RG_CANDIDATES = (1, 2, 4)      # RG


def _time(bx, desc, data, prec, theta, cg, rg, copies):
    os.environ["BX_TILES"] = f"{cg},{rg}"
    try:
        m = bx.Model(desc, data, precision=prec)
        single = m.stage_times(theta, reps=100)["total"]
        batched = m.batch_times(theta, copies, reps=5)["total"] / copies
        m.close()
    finally:
        del os.environ["BX_TILES"]
    return single, batched


def tune(classes, copies=128, log=print):
    """classes: list of (kind, prec, Tmin, Tmax, Nmin, Nmax, desc, data, theta, ws).
    Returns the table lines."""
    import paper_1805_11125_amd as bx
    lines = []
    for kind, prec, tmin, tmax, nmin, nmax, desc, data, theta, ws in classes:
        res = {(cg, rg): _time(bx, desc, data, prec, theta, cg, rg, copies)
               for rg in RG_CANDIDATES for cg in CANDIDATES}
        best_mode = [min(v[mode] for v in res.values()) for mode in (0, 1)]

        def cost(rg):  # relative excess over each mode's best, at the best CG for this RG
            return sum((ws if mode == 0 else 1) * min(res[(cg, rg)][mode] for cg in CANDIDATES) / best_mode[mode]
                       for mode in (0, 1))

        rg = min(RG_CANDIDATES, key=cost)
        for batched in (0, 1):
            cg = min(CANDIDATES, key=lambda c: res[(c, rg)][batched])
            lines.append(f"{kind} {prec} {tmin} {tmax} {nmin} {nmax} {batched} {cg} {rg}")
            log(f"class kind={kind} prec={prec} T=[{tmin},{tmax}] N=[{nmin},{nmax}] "
                f"{'batched' if batched else 'single'}: " +
                " ".join(f"CG{c}/RG{r}={res[(c, r)][batched] * 1e3:.2f}us" for r in RG_CANDIDATES
                         for c in CANDIDATES) + f" -> CG {cg} RG {rg}")
    return lines


def standard_classes():
    """Shape classes of the synthetic workloads (generator in synth/)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth
    out = []
    d1, x1 = synth.load("c1")
    out.append((0, 1, 1, 2000, 1, 2000, d1, x1, d1.theta_true, 1))
    d2, x2 = synth.load("c2")
    th2 = d2.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d2.P))
    base, per_species, theta = synth.catalogue()
    t = synth.toy(9, per_species, theta)   # a short reco window (303 bins)
    out.append((1, 0, 1, 100000, 1, 600, synth.toy_desc(base, t), synth.Data(energy=t.counts), t.theta0, 1))
    out.append((1, 0, 1, 100000, 601, 100000, d2, x2, th2, 3))
    out.append((1, 1, 1, 100000, 1, 100000, d2, x2, th2, 1))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--copies", type=int, default=128)
    a = ap.parse_args()
    lines = tune(standard_classes(), copies=a.copies, log=lambda s: print(s, flush=True))
    with open(a.out, "w") as f:
        f.write("# kind prec Tmin Tmax Nmin Nmax batched CG RG  (written by paper_1805_11125_amd.tune)\n")
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()

"""Write the frozen synthetic datasets used by the tests, smoke check and bench.

Run from the repository root:  python tests/golden/make_fixtures.py

Every stored expectation comes from the FP64 oracle; the histograms are
Poisson draws of those expectations with the stated seeds.  Freezing them
keeps the targets fixed if numpy's samplers ever change.

Files
  c1.npz   config 1: energy histogram (seed 0); per-species expectations
  c2.npz   config 2: random-trigger spectrum g[128]; energy histogram (seed 0)
  c3a.npz  config 3a: vetoed, tagged, radial, pulse-shape histograms (seed 0)
  c3b.npz  config 3b: the same on the config-2 model (seed 0)
  c4.npz   toy catalogue: expectations per unit rate [900, 14] at the truth
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import model as om  # noqa: E402


def mv_draw(desc, seed):
    mu = om.forward(desc, desc.theta_true).mu
    rng = np.random.default_rng(seed)
    N = desc.N
    j0, j1 = desc.win
    sub = np.zeros(N)
    tag = np.zeros(N)
    ps = np.zeros((N, desc.ps_tmpl.shape[1]))
    sub[j0:j1] = rng.poisson(mu["energy"])
    tag[j0:j1] = rng.poisson(mu["tagged"])
    rad = rng.poisson(mu["radial"]).astype(np.float64)
    ps[j0:j1] = rng.poisson(mu["ps"])
    return dict(sub=sub, tag=tag, radial=rad, ps=ps)


def main():
    # config 1
    d1 = synth.config1()
    mp1 = oracle.per_species_expected(d1, d1.theta_true)
    mu1 = om.forward(d1, d1.theta_true).mu["energy"]
    n1 = synth.draw_poisson(np.random.default_rng(0), mu1)
    np.savez_compressed(os.path.join(HERE, "c1.npz"), energy=n1, per_species=mp1)

    # config 2: g = response applied to the low-energy beta shape, first 128
    # reco bins (p.e.), at the true response parameters
    d2np = synth.config2()
    g = oracle.per_species_expected(d2np, d2np.theta_true)[:synth.C2_PU_K, 0].copy()
    d2 = synth.config2(pu_g=g)
    mu2 = om.forward(d2, d2.theta_true).mu["energy"]
    n2 = synth.draw_poisson(np.random.default_rng(0), mu2)
    np.savez_compressed(os.path.join(HERE, "c2.npz"), pu_g=g, energy=n2)

    # the algorithmic work of one response sweep: make_support.py

    # config 3a / 3b
    np.savez_compressed(os.path.join(HERE, "c3a.npz"), **mv_draw(synth.config3a(), 0))
    np.savez_compressed(os.path.join(HERE, "c3b.npz"), **mv_draw(synth.config3b(g), 0))

    # toy catalogue (config-2 species + flat + exponential) with pile-up
    d4 = synth.config2(pu_g=g, catalogue=True)
    np.savez_compressed(os.path.join(HERE, "c4.npz"),
             per_species=oracle.per_species_expected(d4, d4.theta_true),
             theta=d4.theta_true)
    print("fixtures written to", HERE)


if __name__ == "__main__":
    main()

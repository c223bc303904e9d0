"""Oracle fits of the frozen datasets (slow: the config-2 fit takes minutes).

    python tests/golden/make_fit_fixtures.py [c1 c2 c3a c3b]

Writes fit_<name>.npz with the oracle's minimum (theta, NLL, EDM, parameter
errors from the inverse Hessian) from the start point theta_true * (1 + 5%
deterministic offsets), the same start the GPU fit tests use.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def start_point(d):
    z = np.random.default_rng(11).standard_normal(d.P)
    th0 = d.theta_true * (1 + 0.05 * z)
    mask = d.float_mask if d.float_mask is not None else np.ones(d.P, bool)
    th0[~mask] = d.theta_true[~mask]
    return th0, mask


def main(names):
    for name in names:
        d, x = synth.load(name)
        th0, mask = start_point(d)
        t0 = time.time()
        # the Newton polish finishes what a bounded number of L-BFGS-B steps leaves
        res = oracle.fit(d, x, th0, float_mask=mask, lbfgs_maxiter=150 if d.T > 1000 else 5000)
        np.savez_compressed(os.path.join(HERE, f"fit_{name}.npz"), theta0=th0, theta=res.theta,
                            nll=res.nll, edm=res.edm, err=res.err, mask=mask)
        print(name, "nll", res.nll, "edm", res.edm, "evals", res.n_eval, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c3a", "c2", "c3b"])

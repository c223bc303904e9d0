"""Write c2_support.npz: the algorithmic work of one response sweep of the
3000 x 900 generalized-gamma workload at the benchmark's parameter point,
counted by the oracle: the edges inside each column's [1e-12, 1 - 1e-12]
quantile support plus the bracketing edges, and the cells between them.

    python tests/golden/make_support.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    d2, _ = synth.load("c2")
    th_b = d2.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d2.P))
    edges = oracle.support_edges(d2, th_b, q=1e-12)
    cells = oracle.support_cells(d2, th_b, q=1e-12)
    np.savez_compressed(os.path.join(HERE, "c2_support.npz"), edges=edges, cells=cells, q=1e-12, theta=th_b)
    print("support edges", edges, "cells", cells)


if __name__ == "__main__":
    main()

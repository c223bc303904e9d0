"""Shared checks of GPU results against the FP64 oracle (test helpers).

Gradient tolerance: component q within 1e-6 of sum_b |(1 - n_b/mu_b) dmu_b/dq|,
the sum of the absolute summands of dNLL/dq (oracle.grad_scale).  The error
is also printed against the looser scale sum_b |dmu_b/dq| (1 + n_b/mu_b)
(oracle.grad_scale_abs) for comparison.

A component whose scale is below 1e-20 of the largest component's comes only
from the far tails of the response columns, which the library drops beyond
its support cut (less than 1e-32 of a column's mass for FP64 cells, 1e-14 for
FP32): such a component is held to 1e-6 of that floor instead (e.g. the rate
of a line species whose columns reach a count of zero only at 1e-136).
"""
import numpy as np

import oracle


def grad_errors(d, x, th, g, g0):
    """(error / grad_scale, error / grad_scale_abs) per component."""
    e = np.abs(np.asarray(g) - np.asarray(g0))
    sc = oracle.grad_scale(d, x, th)
    sc = np.maximum(sc, 1e-20 * sc.max())
    return e / sc, e / oracle.grad_scale_abs(d, x, th)


def check_nll_grad(label, d, x, th, v, g, v0=None, g0=None, nll_rel=1e-9, grad_tol=1e-6):
    if v0 is None:
        v0, g0 = oracle.nll_grad(d, x, th)
    rel = abs(v - v0) / abs(v0)
    e10, eabs = grad_errors(d, x, th, g, g0)
    print(f"{label}: NLL {v:.12g} oracle {v0:.12g} |d|={abs(v - v0):.3g} rel={rel:.2e}; "
          f"grad max err/scale={e10.max():.2e} (q={int(np.argmax(e10))}; "
          f"looser scale {eabs.max():.2e})", flush=True)
    assert rel <= nll_rel, (v, v0)
    assert np.all(e10 <= grad_tol), e10
    return rel, e10

"""Oracle fitter -- TEST INFRASTRUCTURE.

The paper's package hands the likelihood to a minimiser that varies the
parameters until it finds the optimum (Sec. 4, workflow steps 5-7).  The
oracle does that with scipy's L-BFGS-B on the analytic gradient (bounds keep
the rates and response parameters non-negative), then polishes with Newton
steps on a finite-difference Hessian of the analytic gradient until the
estimated distance to the minimum, EDM = g^T H^-1 g / 2, is tiny.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
from scipy import optimize

from .model import DomainError, nll_grad


def _hessian(desc, data, theta, idx, scale):
    """Central-difference Hessian of the analytic gradient over idx."""
    n = len(idx)
    H = np.zeros((n, n))
    for a, q in enumerate(idx):
        h = 1e-5 * scale[a]
        tp = theta.copy()
        tm = theta.copy()
        tp[q] += h
        tm[q] -= h
        gp = nll_grad(desc, data, tp)[1][idx]
        gm = nll_grad(desc, data, tm)[1][idx]
        H[:, a] = (gp - gm) / (2 * h)
    return 0.5 * (H + H.T)


def fit(desc, data, theta0, float_mask=None, edm_tol=1e-14, max_polish=20, lbfgs_maxiter=5000):
    theta0 = np.asarray(theta0, np.float64).copy()
    mask = np.ones(desc.P, bool) if float_mask is None else np.asarray(float_mask, bool)
    idx = np.flatnonzero(mask)
    scale = np.where(np.abs(theta0[idx]) > 0, np.abs(theta0[idx]), 1.0)
    n_eval = [0]

    def full(u):
        th = theta0.copy()
        th[idx] = u * scale
        return th

    def fun(u):
        n_eval[0] += 1
        try:
            f, g = nll_grad(desc, data, full(u))
        except DomainError:
            return np.inf, np.zeros_like(u)
        return f, g[idx] * scale

    # rates are bounded at zero; response parameters are free, their domain
    # (sigma^2 >= 0, GG mean and variance > 0) is enforced by the NLL being
    # +inf outside it
    pu_q = desc.P - 1 if getattr(desc, "pu_float", False) else -1  # pile-up fraction in [0, 1]
    bounds = [(0.0, None) if q < desc.S else (0.0, 1.0) if q == pu_q else (None, None) for q in idx]
    res = optimize.minimize(fun, np.ones(len(idx)), jac=True, method="L-BFGS-B",
                            bounds=bounds,
                            options=dict(ftol=0.0, gtol=1e-12, maxiter=lbfgs_maxiter,
                                         maxfun=4 * lbfgs_maxiter))
    theta = full(res.x)
    f, g = nll_grad(desc, data, theta)
    edm = np.inf
    H = None
    for _ in range(max_polish):
        H = _hessian(desc, data, theta, idx, scale)
        gi = g[idx]
        at_bound = (idx < desc.S) & (theta[idx] <= 0) & (gi > 0)
        free = ~at_bound
        if not np.any(free):
            edm = 0.0
            break
        Hf = H[np.ix_(free, free)]
        step = np.linalg.solve(Hf, gi[free])
        edm = 0.5 * float(gi[free] @ step)
        if edm < edm_tol:
            break
        trial = theta.copy()
        sub = idx[free]
        trial[sub] = theta[sub] - step
        trial[: desc.S] = np.maximum(trial[: desc.S], 0.0)
        try:
            ft, gt = nll_grad(desc, data, trial)
        except DomainError:
            break
        if ft > f + 1e-9 * abs(f):
            break
        theta, f, g = trial, ft, gt
    cov = None
    if H is not None:
        try:
            cov = np.linalg.inv(H)
        except np.linalg.LinAlgError:
            cov = None
    err = np.full(desc.P, np.nan)
    if cov is not None:
        err[idx] = np.sqrt(np.maximum(np.diag(cov), 0.0))
    return SimpleNamespace(theta=theta, nll=f, grad=g, edm=edm, err=err,
                           n_eval=n_eval[0], success=bool(edm < 1e-6))

"""Host build of the quadrature cells (bin integrals of the response density
over one reco bin, the discretised form of Eq. 1) against 30-digit mpmath
values of the same integrals and of their derivatives.

Generalized gamma (Stacy, exponent p): cell = P(k, y1) - P(k, y0) with
y = (x/a)^p; dR/dk at fixed x and a by mpmath differentiation of that
difference; dR/d ln a = -p (g(y1) - g(y0)), g(y) = y^k e^-y / Gamma(k).
Gaussian: cell = Phi(z1) - Phi(z0); dR/dm = -(phi(z1) - phi(z0))/sigma,
dR/dsigma = -(z1 phi(z1) - z0 phi(z0))/sigma.  Bins are as narrow as the
kernels integrate by quadrature: half-width / column width <= 0.25.

Bounds: FP64 (five nodes) values within 5e-11 (2e-11 at k = 2.5, whose
upper tail is narrower than the core width that sets the bin size; 2e-12
from k = 14 on) and derivatives within 1e-9 of their size (the truncation
of the quadrature; a bias of that order moves
a fitted rate by ~1e-9 of its error); FP32 (four nodes) within 3e-6, where
the rounding of the bin centre in FP32 dominates (relative error ~ k t^2 eps
at t = ln(y/k)).  Bins with less than 1e-3 of the column's largest value (3e-2 for the
derivatives, which change sign inside the column) are held to the same
bounds times that fraction of the largest value.
"""
import ctypes as C
import math
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_11125_amd", "csrc")
P_EXP = 1.25
QUAD_MAX = 0.25
TOL64 = np.array([5e-11, 1e-9, 1e-9])   # value, two derivatives
TOL32 = np.array([3e-6, 3e-6, 3e-6])
# floors (fractions of the column's largest value): the derivatives change
# sign inside the column, where their bin values pass through zero
FLOOR = np.array([1e-3, 3e-2, 3e-2])


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("quad") / "edge_shim.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "edge_shim.cpp"), "-o", so]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    lib = C.CDLL(so)
    dp = np.ctypeslib.ndpointer(np.float64, flags="C")
    for name in ("quad_gg_f32", "quad_gg_f64"):
        getattr(lib, name).argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, dp]
    for name in ("quad_gauss_f32", "quad_gauss_f64"):
        getattr(lib, name).argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, dp]
    return lib


def gg_exact(k, a, x0, x1):
    mp.mp.dps = 30
    k, a, p = mp.mpf(k), mp.mpf(a), mp.mpf(P_EXP)
    y0, y1 = (mp.mpf(x0) / a) ** p, (mp.mpf(x1) / a) ** p
    cell = mp.gammainc(k, y0, y1, regularized=True)
    dk = mp.diff(lambda kk: mp.gammainc(kk, y0, y1, regularized=True), k)
    g = lambda y: mp.exp(k * mp.log(y) - y - mp.loggamma(k))
    da = -p * (g(y1) - g(y0))
    return float(cell), float(dk), float(da)


def gg_bins(k, a, n_bins, f32):
    """Bins across the column's support, each of half-width QUAD_MAX (or less)
    in units of the column width 1/(p sqrt(k)) in ln x."""
    sd = 1.0 / (P_EXP * math.sqrt(k))                     # width in ln x
    lo, hi = math.log(a * k ** (1 / P_EXP)) - 6 * sd, math.log(a * k ** (1 / P_EXP)) + 6 * sd
    c = np.linspace(lo, hi, n_bins)
    rng = np.random.default_rng(int(k))
    h = sd * QUAD_MAX * rng.uniform(0.2, 1.0, n_bins)
    return c - h, c + h


@pytest.mark.parametrize("k", [2.5, 14.0, 60.0, 310.0, 900.0])
def test_gg_quad_cells(shim, k):
    a = 3.4
    lnx0, lnx1 = gg_bins(k, a, 13, False)
    lngs = special.gammaln(k) - ((k - 0.5) * math.log(k) - k + 0.5 * math.log(2 * math.pi))
    cR = math.exp(-lngs) / math.sqrt(2 * math.pi * k)
    lnk_psi = math.log(k) - special.digamma(k)
    ct = P_EXP * math.log(a) + math.log(k)
    ex = np.array([gg_exact(k, a, math.exp(u0), math.exp(u1)) for u0, u1 in zip(lnx0, lnx1)])
    colmax = np.abs(ex).max(axis=0)
    for f32, name, tol in ((False, "quad_gg_f64", TOL64), (True, "quad_gg_f32", TOL32)):
        out = np.zeros(3 * len(lnx0))
        getattr(shim, name)(len(lnx0), lnx0, lnx1, ct, k, cR, lnk_psi, P_EXP, out)
        got = out.reshape(-1, 3)
        # each quantity relative to its own size in bins holding at least 1e-3
        # of the column's largest value, and relative to 1e-3 of that largest
        # value in the tails
        err = np.abs(got - ex) / np.maximum(np.abs(ex), FLOOR * colmax)
        assert np.all(err.max(axis=0) <= tol), (name, k, err.max(axis=0))


@pytest.mark.parametrize("sigma", [0.03, 0.2, 1.7])
def test_gauss_quad_cells(shim, sigma):
    m = 1.3
    c = m + sigma * np.linspace(-7, 7, 15)
    h = QUAD_MAX * sigma * np.random.default_rng(3).uniform(0.2, 1.0, 15)
    x0, x1 = c - h, c + h
    mp.mp.dps = 30
    ex = []
    for a, b in zip(x0, x1):
        z0, z1 = (mp.mpf(a) - m) / sigma, (mp.mpf(b) - m) / sigma
        ph = lambda z: mp.npdf(z)
        ex.append((float(mp.ncdf(z1) - mp.ncdf(z0)), float(-(ph(z1) - ph(z0)) / sigma),
                   float(-(z1 * ph(z1) - z0 * ph(z0)) / sigma)))
    ex = np.array(ex)
    colmax = np.abs(ex).max(axis=0)
    for f32, name, tol in ((False, "quad_gauss_f64", TOL64), (True, "quad_gauss_f32", TOL32)):
        out = np.zeros(3 * len(x0))
        getattr(shim, name)(len(x0), x0, x1, m, 1.0 / sigma, out)
        got = out.reshape(-1, 3)
        err = np.abs(got - ex) / np.maximum(np.abs(ex), FLOOR * colmax)
        assert np.all(err.max(axis=0) <= tol), (name, sigma, err.max(axis=0))

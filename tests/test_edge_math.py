"""Host build of the per-edge generalized-gamma arithmetic against scipy's
regularized incomplete gamma ratios, over shapes on both sides of the FP32
method switch and deep into both tails (beyond the support cut, where tiles
still evaluate edges of narrow columns that share them with wide ones).

F(x) = P(k, (x/a)^p) for the Stacy law (the response model of the paper's
energy-response section).  Checked: the encoded side of every edge, the CDF
value, and every cell formed from neighbouring edges.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_11125_amd", "csrc")
P_EXP = 1.25
A_SCALE = 3.4


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("edge") / "edge_shim.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "edge_shim.cpp"), "-o", so]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    lib = C.CDLL(so)
    dp = np.ctypeslib.ndpointer(np.float64, flags="C")
    for name, t in (("edge_f32", np.float32), ("edge_f64", np.float64)):
        tp = np.ctypeslib.ndpointer(t, flags="C")
        getattr(lib, name).argtypes = [C.c_int, dp, dp, dp, dp, dp, C.c_double, dp, tp, tp, tp]
    lib.cell_f32.argtypes = [C.c_float, C.c_float]
    lib.cell_f32.restype = C.c_float
    return lib


def edges(lib, k, y, f32):
    """Encoded edge values at y = (x/a)^p for shape k (constants from their
    definitions: Gamma*(k) = Gamma(k) / (sqrt(2 pi / k) k^k e^-k))."""
    n = len(y)
    k = np.full(n, float(k))
    lngs = special.gammaln(k) - ((k - 0.5) * np.log(k) - k + 0.5 * np.log(2 * np.pi))
    cR = np.exp(-lngs) / np.sqrt(2 * np.pi * k)
    psi = special.digamma(k)
    dlngs = psi - np.log(k) + 0.5 / k
    lnk_psi = np.log(k) - psi
    ct = P_EXP * np.log(A_SCALE) + np.log(k)
    lnx = np.log(A_SCALE) + np.log(y) / P_EXP
    t = np.float32 if f32 else np.float64
    v, d1, d2 = (np.zeros(n, t) for _ in range(3))
    getattr(lib, "edge_f32" if f32 else "edge_f64")(n, ct, k, cR, dlngs, lnk_psi, P_EXP, lnx, v, d1, d2)
    return v


def decode(v):
    a = np.abs(v.astype(np.float64))
    return np.where(np.signbit(v), 1.0 - a, a)


SHAPES = [0.05, 0.7, 3.0, 11.5, 12.0, 16.409, 40.0, 150.0, 900.0, 4000.0]


def lam_at(k, c, upper):
    """lambda with k (lambda - 1 - ln lambda) = c on the given side of 1 (bisection)."""
    lo, hi = (1.0, 1e6) if upper else (1e-300, 1.0)
    for _ in range(200):
        mid = np.exp(0.5 * (np.log(lo) + np.log(hi))) if not upper else 0.5 * (lo + hi)
        val = k * (mid - 1.0 - np.log(mid))
        if (val < c) == upper:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("f32", [True, False])
@pytest.mark.parametrize("k", SHAPES)
def test_edges_and_cells_through_both_tails(shim, k, f32):
    # lambda = y/k from far below to far above the mode: k (lambda - 1 - ln lambda)
    # reaches several hundred on both sides for every shape here
    lam = np.geomspace(1e-9 if k < 1 else 1e-4, 40.0, 3000)
    # densely through k phi = 70..120, where FP32 terms of the tail go subnormal
    dense = [np.linspace(lam_at(k, 70.0, up), lam_at(k, 120.0, up), 2000) for up in (True, False)]
    lam = np.unique(np.concatenate([lam] + [d[d > 0] for d in dense]))
    y = k * lam
    v = edges(shim, k, y, f32)
    P = special.gammainc(k, y)
    Q = special.gammaincc(k, y)
    F = decode(v)
    # side: where the smaller tail is clearly below 1/2 the encoding must name it
    clear = np.minimum(P, Q) < 0.45
    assert np.array_equal(np.signbit(v)[clear], (P > 0.5)[clear])
    tol = 1e-6 if f32 else 1e-13
    assert np.max(np.abs(F - P)) <= tol
    # cells from neighbouring edges, as the kernels form them
    if f32:
        cells = np.array([shim.cell_f32(float(a), float(b)) for a, b in zip(v[:-1], v[1:])])
    else:
        lo, hi = v[:-1], v[1:]
        cells = (hi - lo) + (np.signbit(hi) & ~np.signbit(lo))
    exact = np.diff(P)
    assert np.max(np.abs(cells - exact)) <= 2 * tol
    assert np.min(cells) >= -2 * tol


def test_far_upper_tail_keeps_its_side(shim):
    # the case that once put a whole column into one far-tail cell: k = 16.4,
    # y/k = 9.33 (Q ~ e^-100, FP32 subnormal terms)
    k = 16.409034254226853
    y = np.array([148.0, 150.0, 153.07104394984174, 156.0, 160.0])
    v = edges(shim, k, y, True)
    assert np.all(np.signbit(v))
    assert np.all(np.abs(v) < 1e-30)

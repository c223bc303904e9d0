"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances: NLL within 1e-9 relative; every gradient component within 1e-6
of its magnitude scale sum_b |(1 - n_b/mu_b) dmu_b/dq| (the absolute summands
of dNLL/dq); expected counts per bin within 1e-11 relative (FP64 cells)
or 1e-6 relative per bin (FP32 cells; 1e-9 absolute below 1e-3 counts).
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import model as om
from parity_util import check_nll_grad

pytestmark = pytest.mark.gpu

F32, F64 = 0, 1


@pytest.fixture(scope="module")
def bx():
    import paper_1805_11125_amd as bx
    return bx


def perturbed(d, seed=3, eps=0.01):
    z = np.random.default_rng(seed).standard_normal(d.P)
    th = d.theta_true * (1 + eps * z)
    return th


def check_point(bx, d, x, th, prec, label):
    m = bx.Model(d, x, precision=prec)
    v, g = m.nll_grad(th)
    check_nll_grad(label, d, x, th, v, g)
    ve = m.nll(th)
    assert ve == v
    return m, v, g


@pytest.mark.parametrize("name,prec", [("c1", F64), ("c1", F32), ("c2", F32), ("c2", F64),
                                       ("c3a", F64), ("c3a", F32), ("c3b", F32)])
def test_nll_grad_parity(bx, name, prec):
    d, x = synth.load(name)
    check_point(bx, d, x, perturbed(d), prec, f"{name}/prec{prec}")


# Toy start points (5 % perturbed truth) with short reco windows: narrow
# generalized-gamma columns share tiles with wide ones, so their edges are
# evaluated deep in the tail (k phi ~ 100 for toy 143's column 81).
@pytest.mark.parametrize("b", [143, 3, 13])
@pytest.mark.parametrize("prec", [F32, F64])
def test_toy_start_parity(bx, b, prec):
    base, per_species, theta = synth.catalogue()
    t = synth.toy(b, per_species, theta)
    d = synth.toy_desc(base, t)
    x = synth.Data(energy=t.counts)
    check_point(bx, d, x, t.theta0, prec, f"toy{b}/prec{prec}")


def _pu_float(d):
    d = d.copy()
    d.pu_float = True
    d.theta_true = np.concatenate([d.theta_true, [d.pu_frac]])
    if d.float_mask is not None:
        d.float_mask = np.concatenate([d.float_mask, [True]])
    return d


# The pile-up fraction as a fit parameter (last entry of theta), with its
# gradient; the multivariate model carries it through the radial term too.
@pytest.mark.parametrize("name,prec", [("c2", F32), ("c2", F64), ("c3b", F32)])
def test_pu_float_parity(bx, name, prec):
    d, x = synth.load(name)
    d = _pu_float(d)
    th = perturbed(d, seed=9)
    check_point(bx, d, x, th, prec, f"{name}+p/prec{prec}")


def test_pu_float_domain(bx):
    d, x = synth.load("c2")
    d = _pu_float(d)
    m = bx.Model(d, x, precision=F32)
    th = d.theta_true.copy()
    th[-1] = 1.2
    with pytest.raises(bx.DomainError):
        m.nll_grad(th)
    th[-1] = 0.0  # the boundary is inside the domain
    v, g = m.nll_grad(th)
    assert np.isfinite(v) and np.all(np.isfinite(g))


@pytest.mark.parametrize("name,prec", [("c1", F64), ("c2", F32), ("c3a", F64)])
def test_expected_counts_parity(bx, name, prec):
    d, x = synth.load(name)
    th = perturbed(d, seed=5)
    m = bx.Model(d, x, precision=prec)
    mu = m.expected(th)
    f = om.forward(d, th)
    full = d.copy()
    full.win = (0, d.N)
    ref = om.expected(full, f.Mp, f.r)
    for key, arr in ref.items():
        got = np.asarray(mu[key]).reshape(arr.shape)
        if prec == F64:
            np.testing.assert_allclose(got, arr, rtol=1e-11, atol=1e-12 * np.abs(arr).max())
    if prec == F32:
        _per_bin_check(mu, ref, f"{name}/F32")


# Per-bin parity of the expected counts of every term (Eqs. 1-4) with FP32
# cells: each bin against its own oracle value.  The cells carry ~1e-7 of
# relative rounding (FP32 nodes; FP64 scale and sums), and a bin's expected
# count is a positive sum of cells, so its relative error stays at that
# level wherever the bin is populated (4.1e-7 at worst, a tagged bin of the
# 3000 x 900 multivariate model); bins far in the tails of every column
# (expected counts below 1e-3) are held to an absolute 1e-9 instead.
PER_BIN_REL = 1e-6


def _per_bin_check(mu, ref, label):
    worst = {}
    for key, arr in ref.items():
        got = np.asarray(mu[key]).reshape(arr.shape)
        big = np.abs(arr) >= 1e-3
        rel = np.abs(got - arr)[big] / np.abs(arr)[big]
        small = np.abs(got - arr)[~big]
        worst[key] = (float(rel.max()) if rel.size else 0.0, float(small.max()) if small.size else 0.0)
        assert rel.size == 0 or rel.max() <= PER_BIN_REL, (label, key, rel.max())
        assert small.size == 0 or small.max() <= 1e-9, (label, key, small.max())
    print(label, {k: f"rel {a:.2e} abs(small) {b:.1e}" for k, (a, b) in worst.items()})


@pytest.mark.parametrize("name", ["c3b", "c3a", "c2"])
def test_expected_counts_per_bin_fp32(bx, name):
    d, x = synth.load(name)
    th = perturbed(d, seed=5)
    m = bx.Model(d, x, precision=F32)
    mu = m.expected(th)
    f = om.forward(d, th)
    full = d.copy()
    full.win = (0, d.N)
    _per_bin_check(mu, om.expected(full, f.Mp, f.r), f"{name}/F32")


@pytest.mark.parametrize("b", [143, 3, 13])
def test_expected_counts_per_bin_toys(bx, b):
    base, per_species, theta = synth.catalogue()
    t = synth.toy(b, per_species, theta)
    d = synth.toy_desc(base, t)
    m = bx.Model(d, synth.Data(energy=t.counts), precision=F32)
    mu = m.expected(t.theta0)
    f = om.forward(d, t.theta0)
    full = d.copy()
    full.win = (0, d.N)
    _per_bin_check(mu, om.expected(full, f.Mp, f.r), f"toy{b}/F32")


def test_lnfact_matches_oracle(bx):
    for name in ["c1", "c3a"]:
        d, x = synth.load(name)
        m = bx.Model(d, x, precision=F64)
        assert abs(m.lnfact() - oracle.lnfact(d, x)) <= 1e-12 * oracle.lnfact(d, x)


def ragged_gauss(T, N, S, seed, win=None):
    rng = np.random.default_rng(seed)
    te = np.sort(rng.uniform(0.0, 2.0, T + 1))
    te[0], te[-1] = 0.0, 2.0
    re = np.linspace(0.0, 2.1, N + 1)
    F = rng.random((S, T)) + 0.05
    th = np.concatenate([rng.uniform(1e3, 1e4, S), [0.03, 0.002]])
    d = synth.ModelDesc(kind="gauss", true_edges=te, reco_edges=re, spectra=F,
                        species=[f"s{i}" for i in range(S)], win=win or (0, N), theta_true=th)
    mu = om.forward(d, th).mu["energy"]
    x = synth.Data(energy=np.zeros(N))
    x.energy[d.win[0]:d.win[1]] = rng.poisson(mu)
    return d, x


@pytest.mark.parametrize("T,N,S", [(1, 1, 1), (17, 16, 3), (33, 31, 16), (250, 151, 5), (16, 15, 2)])
def test_ragged_shapes(bx, T, N, S):
    d, x = ragged_gauss(T, N, S, seed=T + N)
    for prec in (F64, F32):
        check_point(bx, d, x, perturbed(d, eps=0.05), prec, f"ragged T{T} N{N} S{S} p{prec}")


def test_window_subset(bx):
    d, x = ragged_gauss(120, 90, 3, seed=9, win=(17, 71))
    check_point(bx, d, x, perturbed(d), F64, "window")


def test_gg_ragged_with_pileup(bx):
    d = synth.config2(pu_g=synth.pileup_spectrum())
    keep = [0, 1, 5, 9]
    d.true_edges = d.true_edges[:701]
    d.spectra = d.spectra[keep][:, :700]
    d.quench = d.quench[:700]
    d.species = [d.species[i] for i in keep]
    d.reco_edges = d.reco_edges[:334]
    d.win = (3, 333)
    d.theta_true = np.concatenate([d.theta_true[keep], d.theta_true[-4:]])
    mu = om.forward(d, d.theta_true).mu["energy"]
    e = np.zeros(d.N)
    e[3:333] = np.random.default_rng(2).poisson(mu)
    x = synth.Data(energy=e)
    for prec in (F32, F64):
        check_point(bx, d, x, perturbed(d), prec, f"gg ragged p{prec}")


def test_zero_width_gauss_eval_and_grad_domain(bx):
    d, x = synth.load("c1")
    th = d.theta_true.copy()
    th[d.S:] = 0.0
    m = bx.Model(d, x, precision=F64)
    v = m.nll(th)
    v0 = oracle.nll(d, x, th) if np.all(np.isfinite(om.forward(d, th).mu["energy"])) else None
    if v0 is not None and math.isfinite(v0):
        assert abs(v - v0) <= 1e-9 * abs(v0)
    with pytest.raises(bx.DomainError):
        m.nll_grad(th)
    # the device-pointer entry point (autograd) reports it as NLL = +inf
    import torch
    t = torch.tensor(th, dtype=torch.float64, device="cuda")
    out = torch.empty(d.P + 1, dtype=torch.float64, device="cuda")
    m.nll_grad_dev(t.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert math.isinf(out[0].item()) and out[0].item() > 0


def test_domain_errors(bx):
    d, x = synth.load("c1")
    m = bx.Model(d, x, precision=F64)
    th = d.theta_true.copy()
    th[d.S] = -1.0                       # sigma^2 < 0
    with pytest.raises(bx.DomainError):
        m.nll(th)
    th = d.theta_true.copy()
    th[0] = np.nan
    with pytest.raises(bx.DomainError):
        m.nll(th)
    th = d.theta_true.copy()
    th[: d.S] = 0.0                      # mu = 0 where counts > 0
    with pytest.raises(bx.DomainError):
        m.nll(th)
    # the model still works after domain errors
    assert math.isfinite(m.nll(d.theta_true))


def test_repeatable_bitwise(bx):
    d, x = synth.load("c2")
    m = bx.Model(d, x, precision=F32)
    th = perturbed(d)
    a = m.nll_grad(th)
    for _ in range(3):
        b = m.nll_grad(th)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_cell_ceiling_bounds_the_sweep(bx):
    # the edge arithmetic alone (registers only) must run faster than the
    # forward sweep's algorithmic edge rate, which adds tiles, the
    # contraction and the stored differences
    d, x = synth.load("c2")
    m = bx.Model(d, x, precision=F32)
    th = perturbed(d)
    ceiling = m.cell_ceiling(th, reps=32)
    st = m.stage_times(th, reps=20)
    edges = int(np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_support.npz"))["edges"])
    rate = edges / (st["cells_fwd"] * 1e-3)
    print(f"edge ceiling {ceiling:.3e}/s, forward sweep {rate:.3e} algorithmic edges/s")
    assert np.isfinite(ceiling) and ceiling > rate
    t = synth.table_config(grid_L=(500.0,), true_step=0.05, reco_step=30.0, n_mc=100)
    mt = bx.Model(t, synth.Data(energy=np.ones(t.N)), precision=F64)
    with pytest.raises(bx.BxError):
        mt.cell_ceiling(t.theta_true)

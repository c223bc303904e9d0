"""Pins of the FP64 oracle against things other than itself: brute-force
quadrature, closed forms, invariants and special cases that reduce to
library routines (the paper prints no worked example with values)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

import oracle
import synth
from oracle import model as om


# ---------------------------------------------------------------------------
# small models
# ---------------------------------------------------------------------------
def tiny_gauss(T=6, N=8, S=2, seed=0):
    rng = np.random.default_rng(seed)
    te = np.linspace(0.1, 1.3, T + 1)
    re = np.linspace(0.0, 1.6, N + 1)
    F = rng.random((S, T)) + 0.1
    F /= F.sum(1, keepdims=True)
    th = np.concatenate([rng.uniform(50, 200, S), [0.05, 0.01]])
    return synth.ModelDesc(kind="gauss", true_edges=te, reco_edges=re, spectra=F,
                           species=[f"s{i}" for i in range(S)], win=(0, N), theta_true=th)


def tiny_gg(T=5, N=7, S=2, p=1.25, seed=0):
    rng = np.random.default_rng(seed)
    te = np.linspace(0.002, 0.08, T + 1)
    re = np.linspace(0.0, 40.0, N + 1)
    F = rng.random((S, T)) + 0.1
    F /= F.sum(1, keepdims=True)
    Q = 1 - 0.25 * np.exp(-0.5 * (te[:-1] + te[1:]) / 0.2)
    th = np.concatenate([rng.uniform(50, 200, S), [500.0, 4.0, 1.1, 4e-4]])
    return synth.ModelDesc(kind="gg", true_edges=te, reco_edges=re, spectra=F, gg_p=p,
                           quench=Q, species=[f"s{i}" for i in range(S)], win=(0, N),
                           theta_true=th)


def poisson_data(desc, theta, seed=1):
    mu = om.forward(desc, theta).mu["energy"]
    return synth.Data(energy=np.random.default_rng(seed).poisson(mu).astype(float))


# ---------------------------------------------------------------------------
# brute force in mpmath (30 digits): density integrated over every reco bin
# ---------------------------------------------------------------------------
def mp_gauss_cells(E, sig, x):
    out = np.zeros((len(x) - 1, len(E)))
    for i, (m, s) in enumerate(zip(E, sig)):
        dens = lambda u: mp.exp(-(u - m) ** 2 / (2 * s * s)) / (s * mp.sqrt(2 * mp.pi))  # noqa
        for j in range(len(x) - 1):
            out[j, i] = float(mp.quad(dens, [x[j], m, x[j + 1]] if x[j] < m < x[j + 1]
                                      else [x[j], x[j + 1]]))
    return out


def mp_gg_cells(k, a, p, x):
    out = np.zeros((len(x) - 1, len(k)))
    for i, (kk, aa) in enumerate(zip(k, a)):
        kk, aa = mp.mpf(kk), mp.mpf(aa)
        lg = mp.loggamma(kk)

        def dens(u):
            if u <= 0:
                return mp.mpf(0)
            return p * mp.exp((p * kk - 1) * mp.log(u) - (u / aa) ** p - p * kk * mp.log(aa) - lg)
        for j in range(len(x) - 1):
            out[j, i] = float(mp.quad(dens, [max(x[j], 0), x[j + 1]])) if x[j + 1] > 0 else 0.0
    return out


def test_gauss_cells_vs_quadrature():
    mp.mp.dps = 40
    d = tiny_gauss()
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    ref = mp_gauss_cells(cp.m, cp.sigma, d.reco_edges)
    assert np.all(np.abs(R - ref) <= 1e-16 + 1e-13 * np.abs(ref))


@pytest.mark.parametrize("p", [1.25, 0.8, 2.0])
def test_gg_cells_vs_quadrature(p):
    mp.mp.dps = 30
    d = tiny_gg(p=p)
    cp = om.column_params(d, d.theta_true[d.S:])
    assert cp.k.min() < 3 and cp.k.max() > 5      # spans small and large shapes
    R = om.response_matrix(d, cp)
    ref = mp_gg_cells(cp.k, cp.a, p, d.reco_edges)
    assert np.all(np.abs(R - ref) <= 1e-15 + 1e-11 * np.abs(ref))


def test_gg_cdf_vs_mpmath_gammainc():
    mp.mp.dps = 30
    d = tiny_gg(T=3, N=5)
    cp = om.column_params(d, d.theta_true[d.S:])
    tail, lower = om.edge_tails(d, cp)
    for i in range(d.T):
        for j, x in enumerate(d.reco_edges):
            y = (mp.mpf(x) / cp.a[i]) ** cp.p if x > 0 else mp.mpf(0)
            P = mp.gammainc(cp.k[i], 0, y, regularized=True)
            ref = P if lower[i, j] else 1 - P
            assert abs(tail[i, j] - float(ref)) <= 1e-15 + 1e-12 * float(ref)


def test_gg_p1_is_gamma_closed_form():
    """p = 1: moment matching has the closed form k = m^2/s^2, a = s^2/m and
    the CDF is the gamma distribution's."""
    d = tiny_gg(p=1.0)
    cp = om.column_params(d, d.theta_true[d.S:])
    np.testing.assert_allclose(cp.k, cp.m ** 2 / cp.s2, rtol=1e-9)
    np.testing.assert_allclose(cp.a, cp.s2 / cp.m, rtol=1e-9)
    R = om.response_matrix(d, cp)
    cdf = stats.gamma.cdf(d.reco_edges[None, :], cp.k[:, None], scale=cp.a[:, None])
    np.testing.assert_allclose(R, np.diff(cdf, axis=1).T, rtol=1e-10, atol=1e-15)


def test_gg_moment_matching_mpmath():
    mp.mp.dps = 30
    d = synth.config2()
    cp = om.column_params(d, d.theta_true[d.S:])
    for i in [0, 3, 20, 150, 900, 2999]:
        k, a, p = mp.mpf(cp.k[i]), mp.mpf(cp.a[i]), mp.mpf(cp.p)
        g0 = mp.gamma(k)
        mean = a * mp.gamma(k + 1 / p) / g0
        var = a * a * mp.gamma(k + 2 / p) / g0 - mean ** 2
        assert abs(float(mean) / cp.m[i] - 1) < 1e-12
        assert abs(float(var) / cp.s2[i] - 1) < 1e-7


@pytest.mark.parametrize("kind", ["gauss", "gg"])
def test_column_normalisation_with_under_overflow(kind):
    d = synth.config1() if kind == "gauss" else synth.config2()
    d.reco_edges = np.concatenate([[-np.inf], d.reco_edges, [np.inf]])
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    np.testing.assert_allclose(R.sum(axis=0), 1.0, rtol=0, atol=1e-14)


def test_delta_spectrum_gives_kernel_column():
    d = synth.config1()
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    for i in [0, 57, 160, 399]:
        e = d.copy()
        e.spectra = np.zeros((1, d.T))
        e.spectra[0, i] = 1.0
        e.species = ["delta"]
        mu = om.forward(e, np.concatenate([[1.0], d.theta_true[d.S:]])).mu["energy"]
        np.testing.assert_array_equal(mu, R[:, i])


def test_delta_kernel_rebins_spectrum():
    d = synth.config1()
    th = d.theta_true.copy()
    th[d.S:] = 0.0                      # sigma = 0 everywhere
    mu = om.forward(d, th).mu["energy"]
    E = om.true_centres(d)
    ref = np.zeros(d.N)
    vals = (th[: d.S, None] * d.spectra).sum(0)
    for i, e in enumerate(E):
        j = np.searchsorted(d.reco_edges, e, side="right") - 1
        if 0 <= j < d.N:
            ref[j] += vals[i]
    np.testing.assert_allclose(mu, ref, rtol=1e-13, atol=1e-9)


def test_delta_kernel_on_edge_goes_to_upper_bin():
    d = tiny_gauss(T=2, N=4)
    d.true_edges = np.array([0.3, 0.5, 0.7])       # centres 0.4 (on an edge) and 0.6
    d.reco_edges = np.array([0.0, 0.2, 0.4, 0.6, 0.8])
    th = np.concatenate([[1.0, 1.0], [0.0, 0.0]])
    d.spectra = np.array([[1.0, 0.0], [0.0, 1.0]])
    mu = om.forward(d, th).mu["energy"]
    np.testing.assert_array_equal(mu, [0.0, 0.0, 1.0, 1.0])


# ---------------------------------------------------------------------------
# pile-up (Eq. 2)
# ---------------------------------------------------------------------------
def _pu_desc(N, g, p):
    d = tiny_gauss(N=N)
    d.pu_g, d.pu_frac = np.asarray(g, float), p
    return d


def test_pileup_zero_fraction_is_identity():
    M = np.random.default_rng(0).random((30, 3))
    d = _pu_desc(30, np.ones(5), 0.0)
    assert np.array_equal(om.pileup(d, M), M)


def test_pileup_delta_is_identity():
    M = np.random.default_rng(0).random((30, 3))
    d = _pu_desc(30, [2.0, 0.0, 0.0], 0.3)
    np.testing.assert_allclose(om.pileup(d, M), M, rtol=3e-16, atol=0)


def test_pileup_brute_force_loop():
    rng = np.random.default_rng(3)
    N, K, p = 12, 5, 0.17
    M = rng.random((N, 2))
    g = rng.random(K)
    gh = g / g.sum()
    ref = np.zeros_like(M)
    for s in range(2):
        for j in range(N):
            acc = 0.0
            for k in range(K):
                if j - k >= 0:
                    acc += gh[k] * M[j - k, s]
            ref[j, s] = (1 - p) * M[j, s] + p * acc
    np.testing.assert_allclose(om.pileup(_pu_desc(N, g, p), M), ref, rtol=1e-14)


def test_pileup_conserves_mass_on_padded_window():
    rng = np.random.default_rng(4)
    N, K = 40, 8
    M = np.zeros((N, 2))
    M[: N - K] = rng.random((N - K, 2))
    out = om.pileup(_pu_desc(N, rng.random(K), 0.4), M)
    np.testing.assert_allclose(out.sum(0), M.sum(0), rtol=1e-14)


def test_pileup_composition():
    rng = np.random.default_rng(5)
    N = 50
    M = rng.random((N, 1))
    g1, g2 = rng.random(6), rng.random(4)
    g1, g2 = g1 / g1.sum(), g2 / g2.sum()
    twice = om.pileup(_pu_desc(N, g2, 1.0), om.pileup(_pu_desc(N, g1, 1.0), M))
    once = om.pileup(_pu_desc(N, np.convolve(g1, g2), 1.0), M)
    np.testing.assert_allclose(twice, once, rtol=1e-13)


# ---------------------------------------------------------------------------
# expected counts and the NLL
# ---------------------------------------------------------------------------
def test_rate_linearity():
    d = synth.config1()
    resp = d.theta_true[d.S:]
    r1, r2 = np.array([1.0, 2, 3, 4]), np.array([5.0, -1, 0.5, 2])
    mu = lambda r: om.forward(d, np.concatenate([r, resp])).mu["energy"]  # noqa
    np.testing.assert_allclose(mu(2 * r1 + 3 * r2), 2 * mu(r1) + 3 * mu(r2), rtol=1e-12, atol=1e-12)


def test_nll_matches_poisson_logpmf():
    d, data = synth.load("c1")
    mu = om.forward(d, d.theta_true).mu["energy"]
    ref = -np.sum(stats.poisson.logpmf(data.energy, mu)) - np.sum(special.gammaln(data.energy + 1))
    assert abs(oracle.nll(d, data, d.theta_true) - ref) < 1e-9 * abs(ref)
    lnf = oracle.lnfact(d, data)
    assert abs(oracle.nll(d, data, d.theta_true) + lnf + np.sum(stats.poisson.logpmf(data.energy, mu))) < 1e-6


def test_nll_constant_mu_closed_form():
    n = np.array([0.0, 3, 7, 1, 0, 12])
    c = 2.5
    t = om.nll_terms(np.full(6, c), n)
    assert math.isclose(math.fsum(t), 6 * c - math.log(c) * n.sum(), rel_tol=1e-15)


def test_nll_conventions():
    assert list(om.nll_terms([0.0, 2.0], [0.0, 0.0])) == [0.0, 2.0]
    with pytest.raises(om.DomainError):
        om.nll_terms([0.0], [1.0])
    with pytest.raises(om.DomainError):
        om.nll_terms([-1e-3], [0.0])
    with pytest.raises(om.DomainError):
        om.nll_terms([np.nan], [0.0])


@pytest.mark.parametrize("name", ["c1", "c3a"])
def test_euler_identity_rates(name):
    d, data = synth.load(name)
    th = d.theta_true * 1.01
    g = oracle.grad(d, data, th)
    f = om.forward(d, th)
    obs = om.observed(d, data)
    lhs = float(th[: d.S] @ g[: d.S])
    rhs = math.fsum(math.fsum((f.mu[k] - obs[k]).ravel()) for k in f.mu)
    assert abs(lhs - rhs) < 1e-9 * math.fsum(math.fsum(np.abs(f.mu[k]).ravel()) for k in f.mu)


def _richardson(fun, x, h):
    D = lambda hh: (fun(x + hh) - fun(x - hh)) / (2 * hh)  # noqa
    return (4 * D(h / 2) - D(h)) / 3


@pytest.mark.parametrize("maker", ["gauss", "gg", "mv"])
def test_gradient_vs_richardson(maker):
    if maker == "gauss":
        d = synth.config1()
    elif maker == "gg":
        d = tiny_gg(T=60, N=45)
        d.pu_g, d.pu_frac = np.exp(-np.arange(6) / 2.0), 0.05
    else:
        d = synth.config3a()
    th0 = d.theta_true * (1 + 0.02 * np.random.default_rng(7).standard_normal(d.P))
    if d.multivariate:
        data = synth.load("c3a")[1]
    else:
        data = poisson_data(d, d.theta_true)
    g = oracle.grad(d, data, th0)
    for q in range(d.P):
        def f(v):
            t = th0.copy()
            t[q] = v
            return oracle.nll(d, data, t)
        fd = _richardson(f, th0[q], 1e-3 * abs(th0[q]))
        assert abs(g[q] - fd) <= 1e-6 * max(abs(fd), 1e-3) + 1e-7, (q, g[q], fd)


def test_gg_dF_dk_vs_mpmath_diff():
    mp.mp.dps = 30
    d = tiny_gg(T=3, N=6)
    cp = om.column_params(d, d.theta_true[d.S:])
    dk = om._gg_dF_dk(d, cp)
    for i in range(d.T):
        for j, x in enumerate(d.reco_edges):
            if x <= 0:
                continue
            y = (mp.mpf(x) / cp.a[i]) ** cp.p
            ref = mp.diff(lambda kk: mp.gammainc(kk, 0, y, regularized=True), cp.k[i])
            assert abs(dk[i, j] - float(ref)) < 1e-9 * max(1e-6, abs(float(ref)))


def mp_tiny_nll(d, data, theta):
    """The whole NLL of a tiny single-histogram model in 30-digit mpmath:
    moment matching by findroot, cells by quadrature of the density,
    contraction, pile-up and NLL as explicit sums."""
    S, T, N = d.S, d.T, d.N
    r = theta[:S]
    resp = theta[S:]
    E = [(mp.mpf(d.true_edges[i]) + mp.mpf(d.true_edges[i + 1])) / 2 for i in range(T)]
    x = [mp.mpf(v) for v in d.reco_edges]
    R = [[mp.mpf(0)] * T for _ in range(N)]
    for i in range(T):
        if d.kind == "gauss":
            m, s = E[i], mp.sqrt(resp[0] * E[i] + resp[1] * E[i] ** 2)
            dens = lambda u, m=m, s=s: mp.exp(-(u - m) ** 2 / (2 * s * s)) / (s * mp.sqrt(2 * mp.pi))  # noqa
        else:
            p = mp.mpf(d.gg_p)
            m = resp[0] * mp.mpf(d.quench[i]) * E[i]
            s2 = resp[1] + resp[2] * m + resp[3] * m * m
            tau = mp.log(1 + s2 / m ** 2)
            G = lambda k: mp.loggamma(k) + mp.loggamma(k + 2 / p) - 2 * mp.loggamma(k + 1 / p) - tau  # noqa
            k = mp.findroot(G, mp.mpf(1) / (p * p * tau))
            a = m * mp.exp(mp.loggamma(k) - mp.loggamma(k + 1 / p))

            def dens(u, k=k, a=a, p=p):
                if u <= 0:
                    return mp.mpf(0)
                return p * mp.exp((p * k - 1) * mp.log(u) - (u / a) ** p - p * k * mp.log(a) - mp.loggamma(k))
        for j in range(N):
            R[j][i] = mp.quad(dens, [max(x[j], 0) if d.kind != "gauss" else x[j], x[j + 1]])
    F = [[mp.mpf(v) for v in row] for row in d.spectra]
    F = [[v / mp.fsum(row) for v in row] for row in F]
    mu0 = [mp.fsum(R[j][i] * mp.fsum(r[s] * F[s][i] for s in range(S)) for i in range(T))
           for j in range(N)]
    if d.pu_frac and d.pu_g is not None:
        g = [mp.mpf(v) for v in d.pu_g]
        gs = mp.fsum(g)
        pf = mp.mpf(d.pu_frac)
        mu = [(1 - pf) * mu0[j] + pf * mp.fsum(g[k] / gs * mu0[j - k] for k in range(len(g)) if j - k >= 0)
              for j in range(N)]
    else:
        mu = mu0
    n = [mp.mpf(v) for v in data.energy]
    return mp.fsum(mu[j] - n[j] * mp.log(mu[j]) if n[j] > 0 else mu[j] for j in range(N))


@pytest.mark.parametrize("kind", ["gauss", "gg"])
def test_full_nll_and_gradient_vs_mpmath(kind):
    mp.mp.dps = 30
    if kind == "gauss":
        d = tiny_gauss(T=4, N=5)
    else:
        d = tiny_gg(T=3, N=5)
        d.pu_g, d.pu_frac = np.array([1.0, 0.5, 0.25]), 0.1
    data = poisson_data(d, d.theta_true)
    th = d.theta_true * 1.03
    v, g = oracle.nll_grad(d, data, th)
    thm = [mp.mpf(t) for t in th]
    ref = mp_tiny_nll(d, data, thm)
    assert abs(v - float(ref)) < 1e-12 * abs(float(ref))
    for q in range(d.S, d.P):       # response parameters (the rates are linear)
        def f(u, q=q):
            t = list(thm)
            t[q] = u
            return mp_tiny_nll(d, data, t)
        dref = float(mp.diff(f, thm[q], h=mp.mpf(th[q]) * mp.mpf("1e-8")))
        assert abs(g[q] - dref) < 1e-8 * max(abs(dref), 1e-6), (q, g[q], dref)


# ---------------------------------------------------------------------------
# fits (workflow steps 5-7)
# ---------------------------------------------------------------------------
def test_single_species_fit_closed_form():
    d = tiny_gauss(S=1, T=20, N=15)
    data = poisson_data(d, d.theta_true)
    mask = np.array([True, False, False])
    res = oracle.fit(d, data, d.theta_true * np.array([1.3, 1, 1]), float_mask=mask)
    Mp = oracle.per_species_expected(d, d.theta_true)[:, 0]
    assert abs(res.theta[0] - data.energy.sum() / Mp.sum()) < 1e-9 * res.theta[0]


@pytest.mark.slow
def test_asimov_fit_recovers_truth_and_interior_sum():
    d = synth.config1()
    mu = om.forward(d, d.theta_true).mu["energy"]
    asimov = synth.Data(energy=mu)
    th0 = d.theta_true * np.array([1.1, 0.9, 1.05, 0.95, 1.2, 0.8])
    res = oracle.fit(d, asimov, th0)
    np.testing.assert_allclose(res.theta, d.theta_true, rtol=1e-8)
    # Poisson data: at an interior optimum sum(mu) = sum(n)
    d, data = synth.load("c1")
    res = oracle.fit(d, data, th0)
    muh = om.forward(d, res.theta).mu["energy"]
    assert abs(muh.sum() - data.energy.sum()) < 1e-6 * data.energy.sum()
    assert res.edm < 1e-10


# ---------------------------------------------------------------------------
# multivariate terms (Eqs. 3-4)
# ---------------------------------------------------------------------------
def test_mv_zero_tagging_reduces_to_plain():
    d, data = synth.load("c1")
    m = d.copy()
    m.tag_frac = np.zeros(d.S)
    mdata = synth.Data(energy=data.energy, tagged=np.zeros(d.N))
    assert oracle.nll(m, mdata, d.theta_true) == oracle.nll(d, data, d.theta_true)


def test_mv_half_tagging_splits_evenly():
    d = synth.config3a()
    d.tag_frac = np.full(d.S, 0.5)
    mu = om.forward(d, d.theta_true).mu
    plain = om.forward(synth.config1(), d.theta_true).mu["energy"]
    np.testing.assert_allclose(mu["energy"], plain / 2, rtol=1e-14)
    np.testing.assert_allclose(mu["tagged"], plain / 2, rtol=1e-14)


def test_mv_single_ps_bin_equals_vetoed_term():
    d, data = synth.load("c3a")
    d.ps_tmpl = np.ones((d.S, 1))
    d.rad_tmpl = None
    data.ps = data.energy[:, None].copy()
    f = om.forward(d, d.theta_true)
    np.testing.assert_allclose(f.mu["ps"][:, 0], f.mu["energy"], rtol=1e-14)


def test_mv_brute_force_radial_and_ps():
    d = synth.config3a()
    d.rad_win = (20, 150)
    rng = np.random.default_rng(11)
    r = rng.uniform(1e3, 1e4, d.S)
    Mp = rng.random((d.N, d.S))
    mu = om.expected(d, Mp, r)
    t, rho, Tps = d.tag_frac, d.rad_tmpl, d.ps_tmpl
    for k in [0, 37, 99]:
        acc = 0.0
        for s in range(d.S):
            acc += (1 - t[s]) * r[s] * sum(Mp[j, s] for j in range(20, 150)) * rho[s, k]
        assert abs(mu["radial"][k] - acc) < 1e-12 * acc
    for j in [0, 77, 199]:
        for k in [0, 20, 49]:
            acc = sum(Mp[j, s] * (1 - t[s]) * r[s] * Tps[s, k] for s in range(d.S))
            assert abs(mu["ps"][j, k] - acc) < 1e-12 * acc
    for j in [3, 150]:
        assert abs(mu["tagged"][j] - sum(Mp[j, s] * t[s] * r[s] for s in range(d.S))) < 1e-9


def test_support_edges_gauss_quantiles():
    # Gaussian columns: the edges with Phi((x - m)/sigma) in [q, 1 - q] are
    # those within z = -ndtri(q) standard deviations of the mean; add the
    # bracketing edge on each side (clipped to the grid).
    d = synth.config1()
    q = 1e-12
    z = -special.ndtri(q)
    cp = om.column_params(d, d.theta_true[d.S:])
    x = np.asarray(d.reco_edges, np.float64)
    expect = 0
    for m, s in zip(cp.m, cp.sigma):
        idx = np.flatnonzero((x >= m - z * s) & (x <= m + z * s))
        if idx.size:
            expect += min(idx[-1] + 1, len(x) - 1) - max(idx[0] - 1, 0) + 1
    assert oracle.support_edges(d, d.theta_true, q=q) == expect


def _quantile_count(d, th, q, cells=False):
    # GG columns: y = (x/a)^p is Gamma(k, 1); F(x) >= q and 1 - F(x) >= q
    # hold between the q and 1 - q quantiles, which come from the inverse
    # incomplete gamma (a route independent of the forward P, Q the oracle
    # compares against q); add the bracketing edge on each side.
    cp = om.column_params(d, th[d.S:])
    x = np.asarray(d.reco_edges, np.float64)
    total = 0
    for k, a in zip(cp.k, cp.a):
        xl = a * special.gammaincinv(k, q) ** (1.0 / cp.p)
        xh = a * special.gammainccinv(k, q) ** (1.0 / cp.p)
        idx = np.flatnonzero((x > 0) & (x >= xl) & (x <= xh))
        if idx.size:
            total += min(idx[-1] + 1, len(x) - 1) - max(idx[0] - 1, 0) + (0 if cells else 1)
    return total


@pytest.mark.parametrize("T,N", [(60, 45), (200, 120)])
def test_support_edges_gg_quantiles(T, N):
    d = tiny_gg(T=T, N=N)
    th = d.theta_true
    for q in (1e-12, 1e-6):
        assert oracle.support_edges(d, th, q=q) == _quantile_count(d, th, q)
        assert oracle.support_cells(d, th, q=q) == _quantile_count(d, th, q, cells=True)


def test_support_cells_gauss_is_edges_minus_columns():
    d = synth.config1()
    th = d.theta_true
    cp = om.column_params(d, th[d.S:])
    assert np.all(cp.sigma > 0)  # every column has support on this grid
    assert oracle.support_cells(d, th) == oracle.support_edges(d, th) - d.T


# ---------------------------------------------------------------------------
# Pile-up fraction as a fit parameter (the last entry of theta)
# ---------------------------------------------------------------------------
def _pu_float_model():
    d = tiny_gg(T=60, N=45)
    d.pu_g, d.pu_frac = np.exp(-np.arange(6) / 2.0), 0.0
    d.pu_float = True
    d.theta_true = np.concatenate([d.theta_true, [0.05]])
    return d


def test_pu_float_mu_is_affine_in_p():
    d = _pu_float_model()
    th = d.theta_true.copy()
    mu = {}
    for p in (0.0, 0.3, 0.7, 1.0):
        th[-1] = p
        mu[p] = om.forward(d, th).mu["energy"]
    np.testing.assert_allclose(mu[0.7] - mu[0.0], (0.7 / 0.3) * (mu[0.3] - mu[0.0]), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(mu[1.0] - mu[0.0], (1.0 / 0.3) * (mu[0.3] - mu[0.0]), rtol=1e-12, atol=1e-12)


def test_pu_float_zero_equals_no_pileup():
    d = _pu_float_model()
    th = d.theta_true.copy()
    th[-1] = 0.0
    d0 = d.copy()
    d0.pu_float, d0.pu_g, d0.pu_frac = False, None, 0.0
    assert np.array_equal(om.forward(d, th).mu["energy"], om.forward(d0, th[:-1]).mu["energy"])


def test_pu_float_gradient_from_the_two_ends():
    # mu is affine in p, so dmu/dp = mu(p=1) - mu(p=0) and
    # dNLL/dp = sum (1 - n/mu(p)) (mu(1) - mu(0)): no derivative formula needed
    d = _pu_float_model()
    data = poisson_data(d, d.theta_true)
    th = d.theta_true * (1 + 0.02 * np.random.default_rng(11).standard_normal(d.P))
    g = oracle.grad(d, data, th)
    ends = []
    for p in (0.0, 1.0):
        t = th.copy()
        t[-1] = p
        ends.append(om.forward(d, t).mu["energy"])
    mu = om.forward(d, th).mu["energy"]
    n = data.energy
    lo, hi = d.win
    w = np.where(n > 0, 1.0 - n / mu, 1.0)[lo:hi]
    ref = math.fsum((w * (ends[1] - ends[0])[lo:hi]).tolist())
    assert abs(g[-1] - ref) <= 1e-12 * np.sum(np.abs(w * (ends[1] - ends[0])[lo:hi]))


def test_pu_float_gradient_vs_richardson():
    d = _pu_float_model()
    data = poisson_data(d, d.theta_true)
    th = d.theta_true * (1 + 0.02 * np.random.default_rng(12).standard_normal(d.P))
    g = oracle.grad(d, data, th)
    for q in (0, d.S, d.P - 1):
        def f(v):
            t = th.copy()
            t[q] = v
            return oracle.nll(d, data, t)
        fd = _richardson(f, th[q], 1e-3 * abs(th[q]))
        assert abs(g[q] - fd) <= 1e-6 * max(abs(fd), 1e-3) + 1e-7, (q, g[q], fd)


def test_pu_float_outside_unit_interval_is_a_domain_error():
    d = _pu_float_model()
    th = d.theta_true.copy()
    th[-1] = 1.5
    with pytest.raises(oracle.DomainError):
        om.forward(d, th)


# ---------------------------------------------------------------------------
# tabulated response (Monte Carlo matrices interpolated in one coordinate)
# ---------------------------------------------------------------------------
def tiny_table(G=3, T=6, N=9, S=2, seed=3, pu=False):
    rng = np.random.default_rng(seed)
    te = np.linspace(0.1, 1.3, T + 1)
    re = np.linspace(0.0, 1.6, N + 1)
    F = rng.random((S, T)) + 0.1
    F /= F.sum(1, keepdims=True)
    R = rng.random((G, N, T))
    R /= R.sum(1, keepdims=True) * 1.05  # columns lose 1/21 of their mass
    grid = np.cumsum(rng.uniform(0.5, 1.5, G)) + 2.0
    lam = [0.5 * (grid[0] + grid[1])] if G > 1 else []
    th = np.concatenate([rng.uniform(50, 200, S), lam, [0.03] if pu else []])
    g = np.array([0.6, 0.3, 0.1]) if pu else None
    return synth.ModelDesc(kind="table", true_edges=te, reco_edges=re, spectra=F,
                           species=[f"s{i}" for i in range(S)], win=(0, N), theta_true=th,
                           table_grid=grid, table_R=R, pu_g=g, pu_float=pu)


def test_table_at_grid_point_is_that_matrix():
    # at lam = lam_g the model is the single-matrix model of R_g, bit for bit
    # in M and to rounding in the NLL (a one-point table has no coordinate)
    d = tiny_table()
    x = poisson_data(d, d.theta_true)
    for g in range(3):
        th = d.theta_true.copy()
        th[d.S] = d.table_grid[g]
        one = d.copy()
        one.table_grid = d.table_grid[g:g + 1]
        one.table_R = d.table_R[g:g + 1]
        assert one.P == d.S
        assert np.array_equal(om.forward(d, th).M, om.forward(one, th[: d.S]).M)
        assert om.nll(d, x, th) == pytest.approx(om.nll(one, x, th[: d.S]), rel=1e-15)


def test_table_of_analytic_matrices_reproduces_analytic_model():
    # tabulate the generalized-gamma response at light yields L_g; at each
    # L_g the table model must give the analytic model's NLL (two independent
    # routes through the oracle: interpolated table vs Eq. 1 cells)
    a = tiny_gg(T=7, N=9)
    x = poisson_data(a, a.theta_true)
    grid = np.array([480.0, 500.0, 515.0])
    R = []
    for L in grid:
        resp = a.theta_true[a.S:].copy()
        resp[0] = L
        R.append(om.response_matrix(a, om.column_params(a, resp)))
    t = synth.ModelDesc(kind="table", true_edges=a.true_edges, reco_edges=a.reco_edges,
                        spectra=a.spectra, species=a.species, win=a.win,
                        table_grid=grid, table_R=np.array(R))
    for L in grid:
        tha = a.theta_true.copy()
        tha[a.S] = L
        tht = np.concatenate([a.theta_true[: a.S], [L]])
        assert om.nll(t, x, tht) == pytest.approx(om.nll(a, x, tha), rel=1e-13)


def test_table_expectations_affine_inside_a_cell():
    d = tiny_table(G=4)
    th = d.theta_true.copy()
    lo, hi = d.table_grid[1], d.table_grid[2]
    ms = []
    for lam in (lo, 0.25 * lo + 0.75 * hi, hi):
        th[d.S] = lam
        ms.append(om.forward(d, th).M)
    assert np.allclose(ms[1], 0.25 * ms[0] + 0.75 * ms[2], rtol=1e-14, atol=0)


def test_table_gradient_vs_richardson_and_slope_at_grid_point():
    d = tiny_table(G=4, pu=True)
    x = poisson_data(d, d.theta_true)
    th = d.theta_true.copy()
    th[d.S] = 0.3 * d.table_grid[1] + 0.7 * d.table_grid[2]
    _, g = om.nll_grad(d, x, th)
    for q in range(d.P):
        def f(v, q=q):
            t = th.copy()
            t[q] = v
            return om.nll(d, x, t)
        h = 1e-3 * abs(th[q]) if q != d.S else 1e-3 * (d.table_grid[2] - d.table_grid[1])
        assert g[q] == pytest.approx(_richardson(f, th[q], h), rel=1e-7, abs=1e-7)
    # at an interior grid point the coordinate takes the slope of the cell above
    th[d.S] = d.table_grid[2]
    _, g2 = om.nll_grad(d, x, th)
    t = th.copy()
    h = 1e-6 * (d.table_grid[3] - d.table_grid[2])
    t[d.S] += h
    assert g2[d.S] == pytest.approx((om.nll(d, x, t) - om.nll(d, x, th)) / h, rel=1e-5)


def test_table_domain():
    d = tiny_table(G=3)
    x = poisson_data(d, d.theta_true)
    for lam in (d.table_grid[0] - 1e-9, d.table_grid[-1] + 1e-9, np.inf):
        th = d.theta_true.copy()
        th[d.S] = lam
        with pytest.raises(om.DomainError):
            om.nll(d, x, th)
    th = d.theta_true.copy()
    th[d.S] = d.table_grid[-1]  # the top of the grid is inside
    assert np.isfinite(om.nll(d, x, th))


def test_mc_tables_are_column_probabilities():
    # each column of a Monte Carlo table is a histogram of n_mc events over
    # the reco bins: multiples of 1/n_mc summing to at most 1
    te = np.linspace(0.0, 1.0, 11)
    re = np.linspace(0.0, 600.0, 31)
    R = synth.mc_response_tables(te, re, np.ones(10), [480.0, 520.0], 500, 5)
    assert R.shape == (2, 30, 10)
    assert np.allclose(R * 500, np.round(R * 500))
    assert np.all(R.sum(axis=1) <= 1.0 + 1e-12)
    # the light yield moves the mean charge: column means scale with L
    xc = 0.5 * (re[:-1] + re[1:])
    m = (R * xc[None, :, None]).sum(1) / R.sum(1)
    assert np.all(m[1, 2:8] > m[0, 2:8])


# ---------------------------------------------------------------------------
# count estimator (negative binomial in the number of fired PMTs)
# ---------------------------------------------------------------------------
def tiny_count(T=6, N=60, S=2, seed=4, resp=(40.0, 2.0, 1.0, 0.02)):
    rng = np.random.default_rng(seed)
    te = np.linspace(0.1, 1.3, T + 1)
    re = np.arange(N + 1, dtype=float)
    F = rng.random((S, T)) + 0.1
    F /= F.sum(1, keepdims=True)
    Q = 1 - 0.25 * np.exp(-0.5 * (te[:-1] + te[1:]) / 0.2)
    th = np.concatenate([rng.uniform(50, 200, S), resp])
    return synth.ModelDesc(kind="count", true_edges=te, reco_edges=re, spectra=F, quench=Q,
                           species=[f"s{i}" for i in range(S)], win=(0, N), theta_true=th)


def test_count_cells_vs_mpmath():
    d = tiny_count(T=4, N=12)
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    mp.mp.dps = 30
    for i in range(4):
        m, r = mp.mpf(cp.m[i]), mp.mpf(cp.r[i])
        for j in range(12):
            n = mp.mpf(j)
            ref = mp.exp(mp.loggamma(n + r) - mp.loggamma(r) - mp.loggamma(n + 1)
                         + r * mp.log(r / (r + m)) + n * mp.log(m / (r + m)))
            assert R[j, i] == pytest.approx(float(ref), rel=1e-12, abs=1e-300)


def test_count_poisson_limit():
    # v0 -> 0+, v2 = 0, v1 = 1: the variance tends to the mean and the law to
    # Poisson (here r ~ 1e9: the two differ by ~n^2/2r, below 2e-5)
    d = tiny_count(resp=(40.0, 1e-6, 1.0, 0.0))
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    n = np.arange(d.N)
    P = stats.poisson.pmf(n[:, None], cp.m[None, :])
    assert np.allclose(R, P, rtol=2e-5, atol=1e-15)


def test_count_columns_have_the_moments():
    d = tiny_count(N=200)
    cp = om.column_params(d, d.theta_true[d.S:])
    R = om.response_matrix(d, cp)
    n = np.arange(d.N)[:, None]
    assert np.allclose(R.sum(0), 1.0, rtol=0, atol=1e-12)
    assert np.allclose((n * R).sum(0), cp.m, rtol=1e-11)
    assert np.allclose(((n - cp.m) ** 2 * R).sum(0), cp.s2, rtol=1e-10)


def test_count_gradient_vs_richardson():
    d = tiny_count()
    x = poisson_data(d, d.theta_true)
    th = d.theta_true * 1.01
    _, g = om.nll_grad(d, x, th)
    for q in range(d.P):
        def f(v, q=q):
            t = th.copy()
            t[q] = v
            return om.nll(d, x, t)
        assert g[q] == pytest.approx(_richardson(f, th[q], 1e-3 * abs(th[q])), rel=1e-7, abs=1e-7)


def test_count_domain():
    d = tiny_count()
    x = poisson_data(d, d.theta_true)
    th = d.theta_true.copy()
    th[d.S + 2] = 0.5  # v1 < 1 with v0, v2 small: variance below the mean somewhere
    th[d.S + 1] = 0.0
    th[d.S + 3] = 0.0
    with pytest.raises(om.DomainError):
        om.nll(d, x, th)


# ---------------------------------------------------------------------------
# joint energy x radius x pulse-shape term
# ---------------------------------------------------------------------------
def tiny_joint(n_rad=3, n_ps=4, seed=5):
    d = tiny_gauss(T=7, N=9, S=3, seed=seed)
    rng = np.random.default_rng(seed + 1)
    d.tag_frac = np.array([0.9, 0.0, 0.2])
    d.rad_tmpl = rng.random((3, n_rad)) + 0.05
    d.rad_tmpl /= d.rad_tmpl.sum(1, keepdims=True)
    d.ps_tmpl = rng.random((3, n_ps)) + 0.05
    d.ps_tmpl /= d.ps_tmpl.sum(1, keepdims=True)
    d.rad_win = (0, d.N)
    d.joint = True
    return d


def joint_data(d, theta, seed=2):
    mu = om.forward(d, theta).mu
    rng = np.random.default_rng(seed)
    return synth.Data(energy=np.zeros(d.N), tagged=rng.poisson(mu["tagged"]).astype(float),
                      joint=rng.poisson(mu["joint"]).astype(float))


def test_joint_expectations_brute_force_loops():
    d = tiny_joint()
    f = om.forward(d, d.theta_true)
    r, t = f.r, d.tag_frac
    lam = f.mu["joint"]
    for j in range(d.N):
        for k in range(3):
            for l in range(4):
                ref = math.fsum(f.Mp[j, s] * (1 - t[s]) * r[s] * d.rad_tmpl[s, k] * d.ps_tmpl[s, l]
                                for s in range(3))
                assert lam[j, k, l] == pytest.approx(ref, rel=1e-14)


def test_joint_marginal_is_vetoed_energy_term():
    d = tiny_joint()
    lam = om.forward(d, d.theta_true).mu["joint"]
    flat = d.copy()
    flat.joint = False
    flat.rad_tmpl = flat.ps_tmpl = None
    assert np.allclose(lam.sum(axis=(1, 2)), om.forward(flat, d.theta_true).mu["energy"], rtol=1e-13)


def test_joint_single_bin_templates_reduce_to_energy_and_tagged_terms():
    d = tiny_joint(n_rad=1, n_ps=1)
    x = joint_data(d, d.theta_true)
    flat = d.copy()
    flat.joint = False
    flat.rad_tmpl = flat.ps_tmpl = None
    xf = synth.Data(energy=x.joint[:, 0, 0], tagged=x.tagged)
    th = d.theta_true * 1.02
    assert om.nll(d, x, th) == pytest.approx(om.nll(flat, xf, th), rel=1e-14)
    assert np.allclose(om.grad(d, x, th), om.grad(flat, xf, th), rtol=1e-11, atol=1e-9)


def test_joint_gradient_vs_richardson():
    d = tiny_joint()
    x = joint_data(d, d.theta_true)
    th = d.theta_true * 1.01
    g = om.grad(d, x, th)
    for q in range(d.P):
        def f(v, q=q):
            t = th.copy()
            t[q] = v
            return om.nll(d, x, t)
        assert g[q] == pytest.approx(_richardson(f, th[q], 1e-3 * abs(th[q])), rel=1e-7, abs=1e-7)


# ---------------------------------------------------------------------------
# The gradient tolerance scale, sum_b |(1 - n_b/mu_b) dmu_b/dq| over every bin
# of every term, against a per-bin loop over Richardson differences of the
# expected counts (nothing of oracle.grad_scale's own contraction is reused).
# ---------------------------------------------------------------------------
def _bruteforce_scale(d, data, th):
    f0 = om.forward(d, th)
    obs = om.observed(d, data)
    keys = list(f0.mu)
    mu0 = {k: np.asarray(f0.mu[k], float).ravel() for k in keys}
    n = {k: np.asarray(obs[k], float).ravel() for k in keys}
    out = []
    for q in range(d.P):
        h = 1e-4 * max(abs(th[q]), 1e-3)

        def mu_at(v, key):
            t = th.copy()
            t[q] = v
            return np.asarray(om.forward(d, t).mu[key], float).ravel()

        total = 0.0
        for key in keys:
            dmu = _richardson(lambda v: mu_at(v, key), th[q], h)
            for b in range(len(mu0[key])):
                w = 1.0 - n[key][b] / mu0[key][b] if n[key][b] > 0 else 1.0
                total += abs(w) * abs(dmu[b])
        out.append(total)
    return np.array(out)


@pytest.mark.parametrize("maker", ["gauss", "gg_pileup", "mv"])
def test_grad_scale_is_the_sum_of_absolute_summands(maker):
    if maker == "gauss":
        d = tiny_gauss(T=10, N=9, S=2)
    elif maker == "gg_pileup":
        d = tiny_gg(T=12, N=10)
        d.pu_g, d.pu_frac = np.exp(-np.arange(4) / 2.0), 0.05
    else:
        d = synth.config3a()
    th = d.theta_true * (1 + 0.02 * np.random.default_rng(11).standard_normal(d.P))
    data = synth.load("c3a")[1] if d.multivariate else poisson_data(d, d.theta_true)
    got = oracle.grad_scale(d, data, th)
    want = _bruteforce_scale(d, data, th)
    np.testing.assert_allclose(got, want, rtol=1e-6)
    # it bounds the gradient, and the looser scale bounds it
    assert np.all(np.abs(oracle.grad(d, data, th)) <= got * (1 + 1e-12))
    assert np.all(got <= oracle.grad_scale_abs(d, data, th))

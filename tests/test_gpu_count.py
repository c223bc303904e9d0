"""GPU parity of the count estimator (one reco bin per count of fired PMTs,
negative binomial with mean L Q E and variance v0 + v1 m + v2 m^2) against
the FP64 oracle: NLL within 1e-9 relative, every gradient component within
1e-6 of its magnitude scale; pile-up, ragged sizes, the domain, server fits
and an Asimov fit."""
import numpy as np
import pytest

import oracle
from parity_util import check_nll_grad, grad_errors
import synth
from oracle import model as om

pytestmark = pytest.mark.gpu

F64 = 1


@pytest.fixture(scope="module")
def bx():
    import paper_1805_11125_amd as bx
    return bx


def small_count(T=600, N=700, pu=False):
    d = synth.count_config(T=T, N=N)
    if pu:
        d.pu_g = synth.pileup_spectrum()[:40]
        d.pu_frac = 0.02
    return d


def draw(d, th, seed=7):
    mu = om.forward(d, th).mu["energy"]
    return synth.Data(energy=np.random.default_rng(seed).poisson(mu).astype(float))


def check(bx, d, x, th, label):
    m = bx.Model(d, x, precision=F64)
    v, g = m.nll_grad(th)
    v0, g0 = oracle.nll_grad(d, x, th)
    check_nll_grad(label, d, x, th, v, g, v0, g0)
    assert m.nll(th) == v
    return m


@pytest.mark.parametrize("pu", [False, True])
def test_count_parity(bx, pu):
    d = small_count(pu=pu)
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    check(bx, d, x, th, f"count/pu={pu}")


@pytest.mark.parametrize("T,N", [(17, 31), (250, 151), (33, 1)])
def test_count_ragged(bx, T, N):
    d = synth.count_config(T=T, N=N)
    x = draw(d, d.theta_true)
    check(bx, d, x, d.theta_true * 1.003, f"count/T{T}/N{N}")


def test_count_domain_and_validation(bx):
    d = small_count()
    x = draw(d, d.theta_true)
    m = bx.Model(d, x, precision=F64)
    th = d.theta_true.copy()
    th[d.S + 1], th[d.S + 2], th[d.S + 3] = 0.0, 0.5, 0.0  # variance below the mean
    with pytest.raises(bx.DomainError):
        m.nll_grad(th)
    bad = d.copy()
    bad.reco_edges = bad.reco_edges * 2.0  # two counts per bin
    with pytest.raises(bx.BxError):
        bx.Model(bad, x, precision=F64)


def test_count_server_equals_plain(bx):
    d = small_count(T=300, N=500)
    models, starts = [], []
    for k in range(9):
        x = draw(d, d.theta_true, seed=200 + k)
        models.append(bx.Model(d, x, precision=F64))
        starts.append(d.theta_true * (1 + 0.03 * np.random.default_rng(k).standard_normal(d.P)))
    plain = [m.fit(th, float_mask=d.float_mask, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    s = bx.Server()
    tk = [s.submit(m, th, float_mask=d.float_mask, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    srv = [s.wait(t) for t in tk]
    s.close()
    for a, b in zip(plain, srv):
        assert a.status == b.status and a.nll == b.nll and np.array_equal(a.x, b.x)


def test_count_asimov_fit_recovers_truth(bx):
    d = small_count(T=300, N=500)
    mu = om.forward(d, d.theta_true).mu["energy"]
    m = bx.Model(d, synth.Data(energy=mu.copy()), precision=F64)
    th0 = d.theta_true * (1 + 0.02 * np.random.default_rng(9).standard_normal(d.P))
    th0[~d.float_mask] = d.theta_true[~d.float_mask]
    r = m.fit(th0, float_mask=d.float_mask, edm_tol=1e-12, max_iter=500)
    assert r.status == bx.BX_CONVERGED
    assert np.allclose(r.x, d.theta_true, rtol=1e-6)

"""GPU parity of the tabulated response (Monte Carlo matrices R_g at grid
points of one coordinate, interpolated linearly) against the FP64 oracle:
NLL within 1e-9 relative, every gradient component within 1e-6 of its
magnitude scale; with fixed and floated pile-up, multivariate terms, a
one-matrix table, the domain of the coordinate, server fits and an Asimov
fit."""
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


_cache = {}


def small_table(pu=None, mv=False, grid=(480.0, 490.0, 500.0, 510.0, 520.0)):
    """600 true bins (5 keV) x 300 reco bins (3 p.e.), the config-2 species,
    Monte Carlo tables at the light yields of grid (2000 events per column)."""
    key = (pu, mv, tuple(grid))
    if key not in _cache:
        g = synth.pileup_spectrum() if pu else None
        d = synth.table_config(grid_L=grid, true_step=0.005, reco_step=3.0, n_mc=2000, seed=23, pu_g=g)
        if pu == "float":
            d.pu_float = True
            d.theta_true = np.concatenate([d.theta_true, [d.pu_frac]])
            d.float_mask = np.ones(d.P, dtype=bool)
        if mv:
            d = synth._make_mv(d, [4], [8, 11])
        _cache[key] = d
    return _cache[key].copy()


def draw(d, th, seed=7):
    mu = om.forward(d, th).mu
    rng = np.random.default_rng(seed)
    pois = lambda k: rng.poisson(mu[k]).astype(float) if k in mu else None  # noqa
    j0, j1 = d.win
    full = lambda v: np.pad(v, [(j0, d.N - j1)] + [(0, 0)] * (v.ndim - 1))  # noqa
    if not d.multivariate:
        return synth.Data(energy=full(pois("energy")))
    return synth.Data(energy=full(pois("energy")), tagged=full(pois("tagged")),
                      radial=pois("radial"), ps=full(pois("ps")))


def check(bx, d, x, th, label):
    m = bx.Model(d, x, precision=F64)
    v, g = m.nll_grad(th)
    v0, g0 = oracle.nll_grad(d, x, th)
    check_nll_grad(label, d, x, th, v, g, v0, g0)
    assert m.nll(th) == v
    return m


@pytest.mark.parametrize("pu", [None, "fixed", "float"])
def test_table_parity(bx, pu):
    d = small_table(pu)
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    th[d.S] = 503.7  # inside the cell [500, 510]
    check(bx, d, x, th, f"table/pu={pu}")
    th[d.S] = 510.0  # an interior grid point: the slope of the cell above
    check(bx, d, x, th, f"table/pu={pu}/grid point")


def test_table_multivariate_parity(bx):
    d = small_table("fixed", mv=True)
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(4).standard_normal(d.P))
    th[d.S] = 487.2
    check(bx, d, x, th, "table/multivariate")


def test_table_one_matrix(bx):
    d = small_table(grid=(500.0,))
    assert d.P == d.S
    x = draw(d, d.theta_true)
    check(bx, d, x, d.theta_true * 1.01, "table/one matrix")


def test_table_domain(bx):
    d = small_table()
    x = draw(d, d.theta_true)
    m = bx.Model(d, x, precision=F64)
    for lam in (479.999, 520.001, np.nan):
        th = d.theta_true.copy()
        th[d.S] = lam
        with pytest.raises(bx.DomainError):
            m.nll_grad(th)
    th = d.theta_true.copy()
    th[d.S] = 520.0  # the top of the grid is inside
    v, g = m.nll_grad(th)
    assert np.isfinite(v) and np.all(np.isfinite(g))


def test_table_server_equals_plain(bx):
    d = small_table("fixed")
    models, starts = [], []
    for k in range(10):
        x = draw(d, d.theta_true, seed=100 + k)
        models.append(bx.Model(d, x, precision=F64))
        th = d.theta_true * (1 + 0.03 * np.random.default_rng(k).standard_normal(d.P))
        th[d.S] = 495.0 + k
        starts.append(th)
    plain = [m.fit(th, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    s = bx.Server()
    tk = [s.submit(m, th, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    srv = [s.wait(t) for t in tk]
    s.close()
    for a, b in zip(plain, srv):
        assert a.status == b.status and a.nll == b.nll and np.array_equal(a.x, b.x)


def test_table_asimov_fit_recovers_truth(bx):
    d = small_table("fixed")
    th_true = d.theta_true.copy()
    th_true[d.S] = 506.3
    mu = om.forward(d, th_true).mu["energy"]
    x = synth.Data(energy=mu.copy())  # Asimov data: the expectation itself
    m = bx.Model(d, x, precision=F64)
    th0 = th_true * (1 + 0.02 * np.random.default_rng(9).standard_normal(d.P))
    th0[d.S] = 501.0
    r = m.fit(th0, edm_tol=1e-12, max_iter=500)
    assert r.status == bx.BX_CONVERGED
    assert abs(r.x[d.S] - 506.3) < 1e-5
    assert np.allclose(r.x[: d.S], th_true[: d.S], rtol=1e-6)

"""GPU parity of the joint energy x radius x pulse-shape term (the vetoed
events in one 3D histogram instead of three additive terms) against the FP64
oracle: NLL within 1e-9 relative, every gradient component within 1e-6 of
its magnitude scale; with the Gaussian and generalized-gamma responses, a
floated pile-up fraction, a tabulated response, the one-bin reduction to the
energy term, and server fits."""
import numpy as np
import pytest

import oracle
from parity_util import check_nll_grad, grad_errors
import synth
from oracle import model as om

pytestmark = pytest.mark.gpu

F32, F64 = 0, 1


@pytest.fixture(scope="module")
def bx():
    import paper_1805_11125_amd as bx
    return bx


def to_joint(d):
    d = d.copy()
    d.joint = True
    return d


def draw(d, th, seed=11):
    mu = om.forward(d, th).mu
    rng = np.random.default_rng(seed)
    j0, j1 = d.win
    pad = lambda v: np.pad(v, [(j0, d.N - j1)] + [(0, 0)] * (v.ndim - 1))  # noqa
    return synth.Data(energy=None, tagged=pad(rng.poisson(mu["tagged"]).astype(float)),
                      joint=pad(rng.poisson(mu["joint"]).astype(float)))


def check(bx, d, x, th, prec, label):
    m = bx.Model(d, x, precision=prec)
    v, g = m.nll_grad(th)
    v0, g0 = oracle.nll_grad(d, x, th)
    check_nll_grad(label, d, x, th, v, g, v0, g0)
    assert m.nll(th) == v
    return m, v, g


@pytest.mark.parametrize("prec", [F64, F32])
def test_joint_gauss_parity(bx, prec):
    d = to_joint(synth.config3a())
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
    check(bx, d, x, th, prec, f"joint/c3a/prec{prec}")


def coarse(t, n):
    """Templates rebinned to n bins (keeps the oracle's 3D histogram small)."""
    t = np.asarray(t, np.float64)
    return t.reshape(t.shape[0], n, -1).sum(axis=2)


def test_joint_gg_pileup_float_parity(bx):
    d = to_joint(synth.config3b(synth.pileup_spectrum()))
    d.rad_tmpl, d.ps_tmpl = coarse(d.rad_tmpl, 20), coarse(d.ps_tmpl, 10)
    d.pu_float = True
    d.theta_true = np.concatenate([d.theta_true, [d.pu_frac]])
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(4).standard_normal(d.P))
    check(bx, d, x, th, F32, "joint/c3b/pu float")


def test_joint_table_parity(bx):
    d = synth.table_config(true_step=0.005, reco_step=3.0, n_mc=2000, seed=23)
    d = synth._make_mv(d, [4], [8, 11])
    d.joint = True
    x = draw(d, d.theta_true)
    th = d.theta_true * (1 + 0.01 * np.random.default_rng(5).standard_normal(d.P))
    th[d.S] = 496.3
    check(bx, d, x, th, F64, "joint/table")


def test_joint_one_bin_equals_energy_and_tagged_terms(bx):
    d = to_joint(synth.config3a())
    d.rad_tmpl = np.ones((d.S, 1))
    d.ps_tmpl = np.ones((d.S, 1))
    x = draw(d, d.theta_true)
    flat = d.copy()
    flat.joint = False
    flat.rad_tmpl = flat.ps_tmpl = None
    xf = synth.Data(energy=x.joint[:, 0, 0].copy(), tagged=x.tagged)
    th = d.theta_true * 1.01
    v1, g1 = bx.Model(d, x, precision=F64).nll_grad(th)
    v2, g2 = bx.Model(flat, xf, precision=F64).nll_grad(th)
    assert v1 == pytest.approx(v2, rel=1e-13)
    assert np.allclose(g1, g2, rtol=1e-10, atol=1e-8)


def test_joint_server_equals_plain(bx):
    d = to_joint(synth.config3a())
    models, starts = [], []
    for k in range(9):
        x = draw(d, d.theta_true, seed=300 + k)
        models.append(bx.Model(d, x, precision=F64))
        starts.append(d.theta_true * (1 + 0.03 * np.random.default_rng(k).standard_normal(d.P)))
    plain = [m.fit(th, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    s = bx.Server()
    tk = [s.submit(m, th, edm_tol=1e-10, max_iter=300) for m, th in zip(models, starts)]
    srv = [s.wait(t) for t in tk]
    s.close()
    for a, b in zip(plain, srv):
        assert a.status == b.status and a.nll == b.nll and np.array_equal(a.x, b.x)


def test_joint_negative_rate_domain(bx):
    # A negative rate makes some coefficients c_s < 0.  The kernel handles
    # the bins with counts one by one, and the empty ones only through the
    # closed-form sum, so a row with c_s < 0 is scanned bin by bin for
    # lambda >= 0.  Two cases: lambda stays >= 0 everywhere (parity holds),
    # and lambda < 0 only in empty bins (a domain error, as in the oracle).
    d = to_joint(synth.config3a())
    x = draw(d, d.theta_true)
    ok = d.theta_true.copy()
    ok[2] = -1e-3 * ok[2]
    lam = om.forward(d, ok).mu["joint"]
    assert lam.min() >= 0.0
    check(bx, d, x, ok, F64, "joint/negative rate, lambda >= 0")
    bad = d.theta_true.copy()
    bad[0] = -1e-3 * bad[0]
    lam = om.forward(d, bad).mu["joint"]
    j0, j1 = d.win
    neg = lam < 0
    assert neg.any() and not np.any(x.joint[j0:j1][neg] > 0)  # negative only where empty
    m = bx.Model(d, x, precision=F64)
    with pytest.raises(bx.DomainError):
        m.nll(bad)
    with pytest.raises(bx.DomainError):
        m.nll_grad(bad)
    assert np.isfinite(m.nll(d.theta_true))


def test_joint_set_data_rebuilds_the_bin_lists(bx):
    # The non-zero bins are listed again on new data: from a sparse
    # histogram to one with counts in every bin and back, each against the
    # oracle and against a model built on that data.
    d = to_joint(synth.config3a())
    th = d.theta_true * 1.002
    sparse = draw(d, d.theta_true, seed=21)
    full = synth.Data(energy=None, tagged=sparse.tagged.copy(), joint=sparse.joint + 1.0)
    assert np.all(full.joint > 0) and np.mean(sparse.joint > 0) < 0.2
    m = bx.Model(d, sparse, precision=F64)
    v1, g1 = m.nll_grad(th)
    for x in (full, sparse):
        m.set_data(x)
        v, g = m.nll_grad(th)
        v0, g0 = oracle.nll_grad(d, x, th)
        check_nll_grad("joint set_data", d, x, th, v, g, v0, g0)
        fresh = bx.Model(d, x, precision=F64)
        assert fresh.nll_grad(th)[0] == v
        fresh.close()
    assert v == v1 and np.array_equal(g, g1)

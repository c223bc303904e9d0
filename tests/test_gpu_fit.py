"""GPU fits: the plain quasi-Newton path against the oracle's minimum, the
autograd entry point, and the fit server (batched = plain, isolation in a
mix, admission under a small memory budget)."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import model as om

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F32, F64 = 0, 1


@pytest.fixture(scope="module")
def bx():
    import paper_1805_11125_amd as bx
    return bx


def fit_fixture(name):
    p = os.path.join(GOLDEN, f"fit_{name}.npz")
    if not os.path.exists(p):
        pytest.skip(f"{p} not generated")
    return np.load(p)


# MIX: FP32 cells for the bulk of the iterations, then the FP64 model of the
# same fit from EDM < 1e-8 (mixed precision); held to the FP64 bounds.
MIX = 2


@pytest.mark.parametrize("name,prec,tol", [("c1", F64, 1e-14), ("c3a", F64, 1e-14), ("c2", F64, 1e-14),
                                           ("c1", MIX, 1e-14), ("c2", MIX, 1e-14), ("c3a", MIX, 1e-14),
                                           ("c3b", MIX, 1e-12),
                                           ("c1", F32, 1e-8), ("c2", F32, 1e-8)])
def test_plain_fit_matches_oracle_minimum(bx, name, prec, tol):
    z = fit_fixture(name)
    d, x = synth.load(name)
    m = bx.Model(d, x, precision=F64 if prec == F64 else F32)
    pm = bx.Model(d, x, precision=F64) if prec == MIX else None
    r = m.fit(z["theta0"], float_mask=z["mask"], edm_tol=tol, max_iter=1000, polish=pm)
    err = np.where(np.isfinite(z["err"]), z["err"], 0.0)
    scale = np.maximum(np.abs(z["theta"]), err)
    dev = np.abs(r.x - z["theta"]) / scale
    dsig = np.abs(r.x - z["theta"]) / np.where(err > 0, err, np.inf)
    print(f"{name}/p{prec}: status {r.status} iters {r.n_iter} evals {r.n_eval} edm {r.edm:.2e} "
          f"nll {r.nll:.10g} oracle {float(z['nll']):.10g}; rates max |d|/max(|r|,sigma) "
          f"{dev[:d.S].max():.2e}; response params max |d|/sigma {dsig[d.S:].max():.2e}")
    assert r.status == bx.BX_CONVERGED
    if prec in (F64, MIX):
        # fitted rates: |r - r*| <= 1e-6 max(|r*|, sigma*); response parameters within 1e-6 sigma
        assert np.all(dev[: d.S] <= 1e-6), dev
        assert np.all(dsig[d.S:] <= 1e-6), dsig
    else:
        # FP32 cells alone: their rounding (~1e-7 relative per cell) biases the
        # gradient a little and EDM stops at 1e-8; the minimum moves by ~3e-6
        # sigma on the 3000 x 900 grid; every parameter within 1e-4 sigma
        dall = np.abs(r.x - z["theta"]) / np.where(err > 0, err, np.inf)
        assert np.all(dall <= 1e-4), dall
    assert abs(r.nll - float(z["nll"])) <= 1e-9 * abs(float(z["nll"]))


def test_asimov_fit_recovers_truth(bx):
    d = synth.config1()
    mu = om.forward(d, d.theta_true).mu["energy"]
    m = bx.Model(d, synth.Data(energy=mu), precision=F64)
    th0 = d.theta_true * np.array([1.1, 0.9, 1.05, 0.95, 1.2, 0.8])
    r = m.fit(th0, edm_tol=1e-16, max_iter=1000)
    np.testing.assert_allclose(r.x, d.theta_true, rtol=1e-7)


def test_asimov_fit_recovers_pileup_fraction(bx):
    # the pile-up fraction floated with the rates and the response: an Asimov
    # data set (the oracle's expected counts) gives back the truth
    d, _ = synth.load("c2")
    d = d.copy()
    d.pu_float = True
    d.theta_true = np.concatenate([d.theta_true, [d.pu_frac]])
    d.float_mask = np.concatenate([d.float_mask, [True]])
    mu = om.forward(d, d.theta_true).mu["energy"]
    m = bx.Model(d, synth.Data(energy=mu), precision=F64)
    th0 = d.theta_true.copy()
    th0[-1] = 0.035
    th0[: d.S] *= 1.01
    r = m.fit(th0, float_mask=d.float_mask, edm_tol=1e-12, max_iter=2000)
    assert r.status == bx.BX_CONVERGED
    assert abs(r.x[-1] - d.pu_frac) <= 1e-6 * d.pu_frac
    np.testing.assert_allclose(r.x[: d.S], d.theta_true[: d.S], rtol=1e-6)


def test_autograd_function(bx):
    import torch
    d, x = synth.load("c2")
    m = bx.Model(d, x, precision=F32)
    th = d.theta_true * 1.01
    v, g = m.nll_grad(th)
    t = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = bx.NLLFunction.apply(m, t)
    (2.5 * loss).backward()
    assert loss.item() == v
    np.testing.assert_array_equal(t.grad.cpu().numpy(), 2.5 * g)


def test_autograd_then_host_path_are_ordered(bx):
    # an evaluation enqueued on torch's stream (autograd) and a host-path
    # evaluation at another point issued right after it share the model's
    # workspace: each must equal its isolated result bit for bit
    import torch
    d, x = synth.load("c2")
    m = bx.Model(d, x, precision=F32)
    th_a = d.theta_true * 1.01
    th_b = d.theta_true * (1 + 0.01 * np.random.default_rng(4).standard_normal(d.P))
    va, ga = m.nll_grad(th_a)
    vb, gb = m.nll_grad(th_b)
    side = torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(side):
            t = torch.tensor(th_a, dtype=torch.float64, device="cuda", requires_grad=True)
            loss = bx.NLLFunction.apply(m, t)
        v2, g2 = m.nll_grad(th_b)          # no synchronisation in between
        with torch.cuda.stream(side):
            loss.backward()
        torch.cuda.synchronize()
        assert loss.item() == va and np.array_equal(t.grad.cpu().numpy(), ga)
        assert v2 == vb and np.array_equal(g2, gb)


def _toys(n, first=0):
    base, per_species, theta = synth.catalogue()
    out = []
    for b in range(first, first + n):
        t = synth.toy(b, per_species, theta)
        d = synth.toy_desc(base, t)
        out.append((d, synth.Data(energy=t.counts), t))
    return out


def test_server_eval_grad_equals_plain(bx):
    d, x = synth.load("c2")
    m = bx.Model(d, x, precision=F32)
    th = d.theta_true * 0.99
    v, g = m.nll_grad(th)
    s = bx.Server()
    r = s.wait(s.submit(m, th, kind=bx.BX_EVAL_GRAD))
    assert r.nll == v and np.array_equal(r.grad, g)
    s.close()


def test_server_multivariate_in_a_mixed_batch(bx):
    # multivariate fits (radial and pulse-shape terms) batched together with
    # single-histogram fits of the same kind and precision: every result
    # equals the plain path's
    cases = [("c3a", F64), ("c1", F64), ("c3b", F32), ("c2", F32)]
    models, pts, ref = [], [], []
    for name, prec in cases:
        d, x = synth.load(name)
        m = bx.Model(d, x, precision=prec)
        th = d.theta_true * (1 + 0.01 * np.random.default_rng(7).standard_normal(d.P))
        models.append(m)
        pts.append(th)
        ref.append(m.nll_grad(th))
    s = bx.Server()
    tickets = [s.submit(m, th, kind=bx.BX_EVAL_GRAD) for m, th in zip(models, pts)]
    res = [s.wait(tk) for tk in tickets]
    s.close()
    for (name, _), (v, g), r in zip(cases, ref, res):
        assert r.nll == v and np.array_equal(r.grad, g), name


def test_batched_fits_equal_plain_and_isolated(bx):
    toys = _toys(6)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]
    plain = [m.fit(t.theta0, float_mask=d.float_mask, edm_tol=1e-9, max_iter=300)
             for m, (d, x, t) in zip(models, toys)]
    s = bx.Server()
    tickets = [s.submit(m, t.theta0, float_mask=d.float_mask, edm_tol=1e-9, max_iter=300)
               for m, (d, x, t) in zip(models, toys)]
    batched = [s.wait(tk) for tk in tickets]
    # one fit alone, then inside a different mix with staggered arrivals
    alone = s.wait(s.submit(models[2], toys[2][2].theta0, float_mask=toys[2][0].float_mask,
                            edm_tol=1e-9, max_iter=300))
    mix = []
    for k in [4, 2, 0]:
        mix.append(s.submit(models[k], toys[k][2].theta0, float_mask=toys[k][0].float_mask,
                            edm_tol=1e-9, max_iter=300))
    mixed = [s.wait(tk) for tk in mix]
    s.close()
    for p, b in zip(plain, batched):
        assert p.n_eval == b.n_eval and p.nll == b.nll and np.array_equal(p.x, b.x)
    assert np.array_equal(alone.x, mixed[1].x) and alone.nll == mixed[1].nll
    print("toy fits:", [(r.status, r.n_iter, r.n_eval, f"{r.edm:.1e}") for r in batched])


def test_mixed_precision_fits_batched_equal_plain(bx):
    # FP32 cells until EDM < 1e-8, then the FP64 model of the same toy: the
    # server moves each fit to its FP64 placement at that point, and every
    # result equals the plain path's bit for bit
    toys = _toys(4, first=20)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]
    pol = [bx.Model(d, x, precision=F64) for d, x, _ in toys]
    plain = [m.fit(t.theta0, float_mask=d.float_mask, edm_tol=1e-12, max_iter=500, polish=p)
             for m, p, (d, x, t) in zip(models, pol, toys)]
    s = bx.Server()
    tickets = [s.submit(m, t.theta0, float_mask=d.float_mask, edm_tol=1e-12, max_iter=500, polish=p)
               for m, p, (d, x, t) in zip(models, pol, toys)]
    batched = [s.wait(tk) for tk in tickets]
    s.close()
    for p, b in zip(plain, batched):
        assert p.status == bx.BX_CONVERGED and p.edm < 1e-12
        assert p.n_eval == b.n_eval and p.nll == b.nll and np.array_equal(p.x, b.x)
    # the FP64 model's point: its own NLL there
    for m64, r in zip(pol, plain):
        assert m64.nll(r.x) == r.nll
    print("mixed toy fits:", [(r.n_iter, r.n_eval, f"{r.edm:.1e}") for r in plain])


def test_device_minimised_batch_equals_plain(bx):
    # the minimisers on the device, one iteration of all the fits replayed as
    # a graph: every fit ends exactly as on the plain path (FP32 fits, then
    # mixed-precision fits that move to their FP64 placement mid-way)
    toys = _toys(6, first=30)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]
    pol = [bx.Model(d, x, precision=F64) for d, x, _ in toys]
    x0s = [t.theta0 for _, _, t in toys]
    masks = [d.float_mask for d, _, _ in toys]
    for polish, tol in ((None, 1e-9), (pol, 1e-12)):
        plain = [m.fit(x0, float_mask=mk, edm_tol=tol, max_iter=500, polish=None if polish is None else polish[i])
                 for i, (m, x0, mk) in enumerate(zip(models, x0s, masks))]
        bat = bx.fit_batch(models, x0s, masks, edm_tol=tol, max_iter=500, polish=polish, check_every=3)
        for p, b in zip(plain, bat):
            assert p.status == b.status and p.n_iter == b.n_iter and p.n_eval == b.n_eval
            assert p.nll == b.nll and p.edm == b.edm and np.array_equal(p.x, b.x) and np.array_equal(p.grad, b.grad)
        print("device-minimised:", [(b.status, b.n_eval, f"{b.edm:.1e}") for b in bat])


def test_toy_fits_converge_at_the_bounds(bx):
    # 256 toy fits (FP32 cells, then FP64): the minimiser holds a rate whose
    # Newton step would cross zero on its bound and solves again for the
    # rest, so fits with rates at zero converge in few evaluations; toy 172
    # is one whose variance coefficient v2 runs to the domain wall.  Every
    # converged fit meets the bound conditions: a rate on its bound has a
    # gradient pushing it out of the box.
    toys = _toys(256)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]
    pol = [bx.Model(d, x, precision=F64) for d, x, _ in toys]
    res = bx.fit_batch(models, [t.theta0 for _, _, t in toys], [d.float_mask for d, _, _ in toys],
                       edm_tol=1e-12, max_iter=500, polish=pol)
    conv = [r for r in res if r.status == bx.BX_CONVERGED]
    ev = np.array([r.n_eval for r in res])
    print(f"toy fits: {len(conv)} of {len(res)} converged, evaluations median {np.median(ev):.0f} "
          f"mean {ev.mean():.1f}; not converged: {[i for i, r in enumerate(res) if r.status != bx.BX_CONVERGED]}")
    assert len(conv) >= 254
    assert np.median(ev) <= 50
    at_bound = 0
    for (d, _, _), r in zip(toys, res):
        if r.status != bx.BX_CONVERGED:
            continue
        assert r.edm < 1e-12
        for s in range(d.S):
            if d.float_mask[s] and r.x[s] == 0.0:
                at_bound += 1
                assert r.grad[s] >= -1e-6
    assert at_bound > 0  # the sample exercises the bounds


def test_device_minimised_batch_of_mixed_kinds(bx):
    # fits of several launch groups (Gaussian FP64, multivariate, generalized
    # gamma FP32) in one batch
    cases = [("c1", F64), ("c3a", F64), ("c2", F32), ("c1", F32)]
    models, x0s, masks, ref = [], [], [], []
    for name, prec in cases:
        d, x = synth.load(name)
        m = bx.Model(d, x, precision=prec)
        z = np.random.default_rng(11).standard_normal(d.P)
        x0 = d.theta_true * (1 + 0.03 * z)
        mk = d.float_mask if d.float_mask is not None else np.ones(d.P, bool)
        x0[~mk] = d.theta_true[~mk]
        models.append(m)
        x0s.append(x0)
        masks.append(mk)
        ref.append(m.fit(x0, float_mask=mk, edm_tol=1e-10, max_iter=500))
    bat = bx.fit_batch(models, x0s, masks, edm_tol=1e-10, max_iter=500)
    for (name, _), p, b in zip(cases, ref, bat):
        assert p.n_eval == b.n_eval and p.nll == b.nll and np.array_equal(p.x, b.x), name


def test_polish_model_must_match(bx):
    d, x = synth.load("c1")
    m = bx.Model(d, x, precision=F32)
    with pytest.raises(bx.BxError):  # the polishing model is not FP64
        m.fit(d.theta_true, polish=bx.Model(d, x, precision=F32))
    d2, x2 = synth.load("c3a")
    with pytest.raises(bx.BxError):  # other shapes
        m.fit(d.theta_true, polish=bx.Model(d2, x2, precision=F64))


def test_admission_under_small_budget(bx):
    toys = _toys(4, first=10)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]
    ref = [m.fit(t.theta0, float_mask=d.float_mask, edm_tol=1e-9, max_iter=200)
           for m, (d, x, t) in zip(models, toys)]
    # room for one or two of these fits (10-26 MB each) and two slots: requests
    # queue and are admitted as fits leave
    from paper_1805_11125_amd import _abi
    import ctypes as C
    s = bx.Server(hbm_budget_bytes=40 << 20, max_slots=2)
    tickets = [s.submit(m, t.theta0, float_mask=d.float_mask, edm_tol=1e-9, max_iter=200)
               for m, (d, x, t) in zip(models, toys)]
    res = [s.wait(tk) for tk in tickets]
    for a, b in zip(ref, res):
        assert np.array_equal(a.x, b.x)
    # admission order: each fit admitted after the previous one finished or in parallel
    assert all(r.t_admit_ns >= r.t_submit_ns for r in res)
    # a request that can never fit is rejected
    s2 = bx.Server(hbm_budget_bytes=1 << 16)
    with pytest.raises(bx.BxError):
        s2.submit(models[0], toys[0][2].theta0)
    s.close()
    s2.close()
    del _abi, C


def test_plain_results_never_stale(bx):
    # Alternating two points on the plain path: every result must be the one
    # of its own point, bit for bit.  A CPU cache line of the result block
    # fetched while the device was still writing it once returned the previous
    # point's NLL and first gradient entries (the line before the mark's).
    toys = _toys(4, first=12)
    rng = np.random.default_rng(5)
    bad = []
    for i, (d, x, t) in enumerate(toys):
        m = bx.Model(d, x, precision=F32)
        A = np.asarray(t.theta0, dtype=np.float64)
        B = A * (1 + 1e-3 * rng.standard_normal(A.size))
        ref = [m.nll_grad(A), m.nll_grad(B)]
        for k in range(8000):
            v, g = m.nll_grad(B if k & 1 else A)
            r = ref[k & 1]
            if v != r[0] or not np.array_equal(g, r[1]):
                bad.append((i, k, v, r[0]))
        m.close()
    assert not bad, bad[:5]


def test_plain_fits_reproducible_around_server_runs(bx):
    # The plain path exchanges theta and results with the kernels through one
    # pinned buffer; host-written and device-written values must never share
    # a cache line (a stale host copy written back over a fresh NLL changed
    # the path of some fits from run to run).
    toys = _toys(16)
    models = [bx.Model(d, x, precision=F32) for d, x, _ in toys]

    def plain():
        return [m.fit(t.theta0, float_mask=d.float_mask, edm_tol=1e-8, max_iter=500)
                for m, (d, x, t) in zip(models, toys)]

    first = plain()
    for _ in range(2):
        s = bx.Server()
        tickets = [s.submit(m, t.theta0, float_mask=d.float_mask, edm_tol=1e-8, max_iter=500)
                   for m, (d, x, t) in zip(models, toys)]
        batched = [s.wait(tk) for tk in tickets]
        s.close()
        again = plain()
        for a, b, c in zip(first, again, batched):
            assert a.nll == b.nll and np.array_equal(a.x, b.x) and a.n_eval == b.n_eval
            assert np.array_equal(a.x, c.x)

"""The allocation-free entry point (bx_nll_grad_dev_noalloc) against the
device-pointer entry point it mirrors (bx_nll_grad_dev): the same results bit
for bit, on two calls in a row (the second on a smaller model), and within
the parity tolerances of the FP64 oracle; a model too large for the fixed
array is rejected."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import check_nll_grad

pytestmark = pytest.mark.gpu


def _pair(bx, m, th):
    import torch
    st = torch.cuda.current_stream().cuda_stream
    t = torch.tensor(th, dtype=torch.float64, device="cuda")
    ref = torch.full((m.P + 1,), np.nan, dtype=torch.float64, device="cuda")
    out = torch.full((m.P + 1,), np.nan, dtype=torch.float64, device="cuda")
    m.nll_grad_dev(t.data_ptr(), ref.data_ptr(), st)
    m.nll_grad_dev_noalloc(t.data_ptr(), out.data_ptr(), st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_equals_dev_path_on_two_calls():
    import paper_1805_11125_amd as bx
    # config 2 (3000 x 900, 12 species, FP32 cells), then config 1 (400 x 200)
    for name, prec in (("c2", bx.BX_PREC_F32), ("c1", bx.BX_PREC_F64)):
        d, x = synth.load(name)
        th = d.theta_true * (1 + 0.01 * np.random.default_rng(3).standard_normal(d.P))
        m = bx.Model(d, x, precision=prec)
        ref, out = _pair(bx, m, th)
        print(f"{name}: noalloc {out[0]!r} dev {ref[0]!r}", flush=True)
        assert np.array_equal(out, ref), (name, out - ref)
        check_nll_grad(f"noalloc {name}", d, x, th, out[0], out[1:])
        m.close()


def test_noalloc_multivariate_then_single():
    import paper_1805_11125_amd as bx
    for name in ("c3b", "c1"):
        d, x = synth.load(name)
        th = d.theta_true * (1 + 0.01 * np.random.default_rng(5).standard_normal(d.P))
        m = bx.Model(d, x, precision=bx.BX_PREC_F32)
        ref, out = _pair(bx, m, th)
        assert np.array_equal(out, ref), name
        m.close()


def test_noalloc_rejects_a_workspace_beyond_the_array():
    import paper_1805_11125_amd as bx
    T, N = 90000, 40            # about 18 MB of column parameters alone
    te = np.linspace(0.0, 2.0, T + 1)
    re = np.linspace(0.0, 2.0, N + 1)
    F = np.ones((1, T))
    d = synth.ModelDesc(kind="gauss", true_edges=te, reco_edges=re, spectra=F, species=["flat"],
                        win=(0, N), theta_true=np.array([1e4, 0.05, 0.001]))
    x = synth.Data(energy=np.full(N, 250.0))
    m = bx.Model(d, x, precision=bx.BX_PREC_F64)
    import torch
    t = torch.tensor(d.theta_true, dtype=torch.float64, device="cuda")
    out = torch.zeros(m.P + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(bx.BxError, match="scratch"):
        m.nll_grad_dev_noalloc(t.data_ptr(), out.data_ptr())
    m.close()

"""MI355X spectral-fit likelihood (Ding et al., arXiv:1805.11125, Secs. 3-4).

Thin Python layer over libbx.so (include/bx.h): argument marshalling, a
torch.autograd.Function around the device-pointer NLL+gradient entry point,
and wrappers of the fitter and the fit server.  All arithmetic runs in the
HIP library; if it is not built, importing the model classes raises.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _abi
from ._abi import (BX_CONVERGED, BX_EVAL_GRAD, BX_FAILED, BX_FIT, BX_MAXITER, BX_OK,
                   BX_PENDING, BX_PREC_F32, BX_PREC_F64, BxError, DomainError, check, dptr)

__all__ = ["Model", "Server", "NLLFunction", "BxError", "DomainError", "FitResult",
           "BX_PREC_F32", "BX_PREC_F64", "BX_FIT", "BX_EVAL_GRAD", "BX_CONVERGED",
           "BX_MAXITER", "BX_FAILED"]


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class FitResult:
    def __init__(self, r: _abi.bx_fit_result, P: int):
        self.status = int(r.status)
        self.nll = float(r.nll)
        self.x = np.array(r.x[:P])
        self.grad = np.array(r.grad[:P])
        self.edm = float(r.edm)
        self.n_iter = int(r.n_iter)
        self.n_eval = int(r.n_eval)
        self.t_submit_ns = int(r.t_submit_ns)
        self.t_admit_ns = int(r.t_admit_ns)
        self.t_done_ns = int(r.t_done_ns)

    @property
    def latency_s(self):
        return (self.t_done_ns - self.t_submit_ns) * 1e-9


def _fit_opts(P, x0, float_mask=None, lo=None, hi=None, edm_tol=0.0, max_iter=0, kind=BX_FIT,
              max_eval=0, polish=None, polish_edm=0.0):
    keep = []
    x0 = _f64(x0)
    keep.append(x0)
    o = _abi.bx_fit_opts()
    o.kind = kind
    o.x0 = dptr(x0)
    if float_mask is not None:
        m = np.ascontiguousarray(np.asarray(float_mask, dtype=np.uint8))
        keep.append(m)
        o.float_mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
    if lo is not None:
        lo = _f64(lo)
        keep.append(lo)
        o.lo = dptr(lo)
    if hi is not None:
        hi = _f64(hi)
        keep.append(hi)
        o.hi = dptr(hi)
    o.edm_tol = float(edm_tol)
    o.max_iter = int(max_iter)
    o.max_eval = int(max_eval)
    if polish is not None:  # mixed precision: the FP64 model of the same fit
        o.polish = polish.handle
        o.polish_edm = float(polish_edm)
    return o, keep


class Model:
    """A spectral model plus its observed histograms, resident on the GPU.

    desc: object with the fields of a model description: kind ("gauss",
    "gg", "table" or "count"), true_edges, reco_edges, spectra[S, T],
    exposure, gg_p, quench, pu_frac, pu_g, pu_float, win; optionally the
    multivariate fields tag_frac, rad_tmpl, rad_win, ps_tmpl and joint; and
    for kind "table" the grid table_grid[G] and matrices table_R[G, N, T].
    data: object with energy (and tagged, radial, ps, or joint[N, n_rad,
    n_ps] for the joint term).  The parameter vector is the rates, then the
    response parameters (Gaussian a, b; generalized gamma and count
    estimator L, v0, v1, v2; table: the grid coordinate when G > 1), then
    the pile-up fraction when it floats."""

    def __init__(self, desc, data, precision=BX_PREC_F32, stream=None):
        self._lib = _abi.load()
        self._keep = []
        d = _abi.bx_model_desc()
        arr = self._arr
        te, re = arr(desc.true_edges), arr(desc.reco_edges)
        sp = arr(np.asarray(desc.spectra, dtype=np.float64).reshape(-1))
        S = int(np.asarray(desc.spectra).shape[0])
        d.T, d.N, d.S = len(te) - 1, len(re) - 1, S
        d.true_edges, d.reco_edges, d.spectra = dptr(te), dptr(re), dptr(sp)
        d.response = {"gauss": _abi.BX_RESP_GAUSS, "gg": _abi.BX_RESP_GG,
                      "table": _abi.BX_RESP_TABLE, "count": _abi.BX_RESP_COUNT}[desc.kind]
        if desc.kind == "table":
            grid = arr(desc.table_grid)
            rtab = arr(np.asarray(desc.table_R, np.float64))
            d.n_grid, d.grid, d.rtab = len(grid), dptr(grid), dptr(rtab)
        d.gg_p = float(getattr(desc, "gg_p", 1.0))
        q = getattr(desc, "quench", None)
        d.quench = dptr(arr(q)) if q is not None else None
        d.exposure = float(desc.exposure)
        g = getattr(desc, "pu_g", None)
        pf = float(getattr(desc, "pu_frac", 0.0) or 0.0)
        d.pu_float = 1 if getattr(desc, "pu_float", False) else 0
        if g is not None and (pf != 0.0 or d.pu_float):
            g = arr(g)
            d.pu_K, d.pu_g, d.pu_frac = len(g), dptr(g), pf
        d.win_lo, d.win_hi = int(desc.win[0]), int(desc.win[1])
        d.precision = int(precision)
        tag = getattr(desc, "tag_frac", None)
        self.multivariate = tag is not None
        if self.multivariate:
            d.multivariate = 1
            d.joint = 1 if getattr(desc, "joint", False) else 0
            d.tag_frac = dptr(arr(tag))
            rt = getattr(desc, "rad_tmpl", None)
            if rt is not None:
                rt = np.asarray(rt, np.float64)
                d.n_rad = rt.shape[1]
                d.rad_tmpl = dptr(arr(rt.reshape(-1)))
                d.rad_lo, d.rad_hi = int(desc.rad_win[0]), int(desc.rad_win[1])
            pt = getattr(desc, "ps_tmpl", None)
            if pt is not None:
                pt = np.asarray(pt, np.float64)
                d.n_ps = pt.shape[1]
                d.ps_tmpl = dptr(arr(pt.reshape(-1)))
        self.N, self.T, self.S = d.N, d.T, S
        self.n_rad, self.n_ps = d.n_rad, d.n_ps
        xd = self._data_struct(data)
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else None
        check(self._lib.bx_model_build(C.byref(d), C.byref(xd), st, C.byref(h)))
        self._h = h
        self.P = int(self._lib.bx_model_nparams(h))
        self._keep = []   # everything was copied by the library
        self._theta = np.zeros(self.P)
        self._grad = np.zeros(self.P)
        self._v = C.c_double()
        self._vaddr = C.addressof(self._v)

    def _arr(self, a):
        a = _f64(np.asarray(a).reshape(-1))
        self._keep.append(a)
        return a

    def _data_struct(self, data):
        x = _abi.bx_data()
        if getattr(data, "energy", None) is not None:
            x.energy = dptr(self._arr(data.energy))
        for name in ("tagged", "radial", "ps", "joint"):
            v = getattr(data, name, None)
            if v is not None:
                setattr(x, name, dptr(self._arr(np.asarray(v).reshape(-1))))
        return x

    @property
    def handle(self):
        return self._h

    def set_data(self, data):
        xd = self._data_struct(data)
        check(self._lib.bx_model_set_data(self._h, C.byref(xd)))
        self._keep = []

    def lnfact(self):
        v = C.c_double()
        check(self._lib.bx_model_lnfact(self._h, C.byref(v)))
        return v.value

    def _theta_addr(self, theta):
        t = theta if (isinstance(theta, np.ndarray) and theta.dtype == np.float64
                      and theta.flags.c_contiguous) else np.ascontiguousarray(theta, dtype=np.float64)
        if t.shape != (self.P,):
            raise ValueError(f"theta must have {self.P} entries")
        return t, t.ctypes.data

    def nll(self, theta):
        t, ta = self._theta_addr(theta)
        check(self._lib.bx_nll_eval(self._h, ta, self._vaddr))
        return self._v.value

    def nll_grad(self, theta):
        t, ta = self._theta_addr(theta)
        check(self._lib.bx_nll_grad(self._h, ta, self._vaddr, self._grad.ctypes.data))
        return self._v.value, self._grad.copy()

    def expected(self, theta):
        """Expected counts of every term over the full reco range."""
        t = _f64(theta)
        n = int(self._lib.bx_model_expected_size(self._h))
        out = np.zeros(n)
        check(self._lib.bx_model_expected(self._h, dptr(t), dptr(out)))
        if not self.multivariate:
            return {"energy": out}
        N, nr, nps = self.N, self.n_rad, self.n_ps
        return {"energy": out[:N], "tagged": out[N:2 * N], "radial": out[2 * N:2 * N + nr],
                "ps": out[2 * N + nr:].reshape(N, nps)}

    STAGES = ["colparams", "cells_fwd", "reduce_M", "rowterms", "radial", "adjoint",
              "cells_bwd", "final", "total", "cells_fwd_main", "cells_bwd_main"]

    def stage_times(self, theta, reps=20):
        """Average ms per evaluation stage (HIP events, each stage's kernel
        launched back to back on its own).  For a tabulated response stage
        "colparams" is the table interpolation; "radial" also holds the
        joint term's kernel."""
        t = _f64(theta)
        ms = np.zeros(len(self.STAGES))
        check(self._lib.bx_model_stage_times(self._h, dptr(t), int(reps), dptr(ms)))
        return dict(zip(self.STAGES, ms))

    def batch_times(self, theta, copies, reps=10):
        """Average ms per batched launch of each stage for `copies` fits of
        this model evaluated together (bx_model_batch_times)."""
        t = _f64(theta)
        ms = np.zeros(len(self.STAGES))
        check(self._lib.bx_model_batch_times(self._h, dptr(t), int(copies), int(reps), dptr(ms)))
        return dict(zip(self.STAGES, ms))

    def cell_ceiling(self, theta, reps=64):
        """Cells per second the response's backward cell arithmetic (value and
        two derivatives) reaches on its own at theta (bx_model_cell_ceiling):
        the measured ceiling of the cell sweeps."""
        t = _f64(theta)
        v = C.c_double()
        check(self._lib.bx_model_cell_ceiling(self._h, dptr(t), int(reps), C.byref(v)))
        return v.value

    def nll_grad_dev(self, theta_dev, out_dev, stream=None):
        """Stream-ordered: theta_dev, out_dev are device addresses (ints)."""
        check(self._lib.bx_nll_grad_dev(self._h, C.c_void_p(theta_dev), C.c_void_p(out_dev),
                                        C.c_void_p(stream) if stream else None))

    def nll_grad_dev_noalloc(self, theta_dev, out_dev, stream=None):
        """As nll_grad_dev, with the workspace in the library's fixed device
        array (bx_nll_grad_dev_noalloc): no device memory is allocated."""
        check(self._lib.bx_nll_grad_dev_noalloc(self._h, C.c_void_p(theta_dev), C.c_void_p(out_dev),
                                                C.c_void_p(stream) if stream else None))

    def fit(self, x0, float_mask=None, lo=None, hi=None, edm_tol=0.0, max_iter=0, max_eval=0,
            polish=None, polish_edm=0.0):
        """Fit on the calling thread (bx_fit).  polish: an FP64 Model of the
        same fit that takes over at EDM < polish_edm (mixed precision)."""
        o, keep = _fit_opts(self.P, x0, float_mask, lo, hi, edm_tol, max_iter, max_eval=max_eval,
                            polish=polish, polish_edm=polish_edm)
        r = _abi.bx_fit_result()
        check(self._lib.bx_fit(self._h, C.byref(o), C.byref(r)))
        del keep
        return FitResult(r, self.P)

    def close(self):
        if getattr(self, "_h", None):
            check(self._lib.bx_model_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching fit server (bx_server_*)."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, stream=None):
        self._lib = _abi.load()
        h = C.c_void_p()
        check(self._lib.bx_server_create(C.c_size_t(hbm_budget_bytes), int(max_slots),
                                         C.c_void_p(stream) if stream else None, C.byref(h)))
        self._h = h
        self._P = {}

    def submit(self, model: Model, x0, float_mask=None, lo=None, hi=None, edm_tol=0.0,
               max_iter=0, kind=BX_FIT, max_eval=0, polish=None, polish_edm=0.0):
        o, keep = _fit_opts(model.P, x0, float_mask, lo, hi, edm_tol, max_iter, kind, max_eval,
                            polish=polish, polish_edm=polish_edm)
        t = C.c_uint64()
        check(self._lib.bx_fit_submit(self._h, model.handle, C.byref(o), C.byref(t)))
        self._P[t.value] = model.P
        return t.value

    def poll(self, ticket):
        r = _abi.bx_fit_result()
        st = check(self._lib.bx_fit_poll(self._h, C.c_uint64(ticket), C.byref(r)),
                   allow=(BX_OK, BX_PENDING))
        if st == BX_PENDING:
            return None
        return FitResult(r, self._P.pop(ticket))

    def wait(self, ticket, sleep=1e-4):
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(sleep)

    def drain(self):
        check(self._lib.bx_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None):
            check(self._lib.bx_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit_batch(models, x0s, float_masks=None, edm_tol=0.0, max_iter=0, max_eval=0, polish=None,
              polish_edm=0.0, check_every=0):
    """Fit models[i] from x0s[i] together, with the minimisers on the device
    and one iteration of all the fits replayed as a HIP graph
    (bx_fit_batch).  polish: FP64 models of the same fits (mixed precision),
    or None.  Returns one FitResult per fit, equal to Model.fit's."""
    n = len(models)
    if n == 0:
        return []
    lib = models[0]._lib
    arr = (_abi.bx_fit_opts * n)()
    keep = []
    for i, m in enumerate(models):
        o, k = _fit_opts(m.P, x0s[i], None if float_masks is None else float_masks[i], None, None, edm_tol,
                         max_iter, BX_FIT, max_eval, None if polish is None else polish[i], polish_edm)
        arr[i] = o
        keep.append(k)
    hs = (C.c_void_p * n)(*[m.handle for m in models])
    res = (_abi.bx_fit_result * n)()
    check(lib.bx_fit_batch(hs, arr, n, res, int(check_every)))
    del keep
    return [FitResult(res[i], models[i].P) for i in range(n)]


def _make_nll_function():
    import torch

    class NLLFunction(torch.autograd.Function):
        """loss = NLLFunction.apply(model, theta): theta is a float64 CUDA
        tensor [P]; the forward pass runs the HIP NLL+gradient on torch's
        current stream and keeps the gradient; backward scales it."""

        @staticmethod
        def forward(ctx, model, theta):
            if not theta.is_cuda or theta.dtype != torch.float64:
                raise TypeError("theta must be a float64 tensor on the GPU")
            theta = theta.contiguous()
            out = torch.empty(model.P + 1, dtype=torch.float64, device=theta.device)
            stream = torch.cuda.current_stream(theta.device).cuda_stream
            model.nll_grad_dev(theta.data_ptr(), out.data_ptr(), stream)
            ctx.save_for_backward(out[1:])
            return out[0]

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return None, grad_out * g

    return NLLFunction


class _Lazy:
    def __init__(self):
        self._f = None

    def apply(self, *a):
        if self._f is None:
            self._f = _make_nll_function()
        return self._f.apply(*a)


NLLFunction = _Lazy()

"""ctypes binding of libbx.so (include/bx.h).  Argument marshalling only:
every step of the likelihood runs in the HIP library."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbx.so")
# tile table measured on MI355X by paper_1805_11125_amd.tune (read by the
# library at model build and server admission unless BX_TUNE_CACHE is set)
TILE_TABLE = os.path.join(HERE, "tiles_mi355x.txt")

BX_OK, BX_PENDING = 0, 1
BX_E_INVAL, BX_E_NOMEM, BX_E_DEVICE, BX_E_DOMAIN, BX_E_BUSY, BX_E_NOTFOUND = -1, -2, -3, -4, -5, -6
BX_RESP_GAUSS, BX_RESP_GG, BX_RESP_TABLE, BX_RESP_COUNT = 0, 1, 2, 3
BX_PREC_F32, BX_PREC_F64 = 0, 1
BX_FIT, BX_EVAL_GRAD = 0, 1
BX_CONVERGED, BX_MAXITER, BX_FAILED = 0, 1, 2

_dp = C.POINTER(C.c_double)


class bx_model_desc(C.Structure):
    _fields_ = [("T", C.c_int32), ("N", C.c_int32), ("S", C.c_int32),
                ("true_edges", _dp), ("reco_edges", _dp), ("spectra", _dp),
                ("response", C.c_int32), ("gg_p", C.c_double), ("quench", _dp),
                ("exposure", C.c_double), ("pu_K", C.c_int32), ("pu_g", _dp),
                ("pu_frac", C.c_double), ("win_lo", C.c_int32), ("win_hi", C.c_int32),
                ("precision", C.c_int32), ("multivariate", C.c_int32), ("tag_frac", _dp),
                ("n_rad", C.c_int32), ("rad_tmpl", _dp), ("rad_lo", C.c_int32),
                ("rad_hi", C.c_int32), ("n_ps", C.c_int32), ("ps_tmpl", _dp),
                ("pu_float", C.c_int32), ("n_grid", C.c_int32), ("grid", _dp), ("rtab", _dp),
                ("joint", C.c_int32)]


class bx_data(C.Structure):
    _fields_ = [("energy", _dp), ("tagged", _dp), ("radial", _dp), ("ps", _dp), ("joint", _dp)]


class bx_fit_opts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("x0", _dp), ("float_mask", C.POINTER(C.c_uint8)),
                ("lo", _dp), ("hi", _dp), ("edm_tol", C.c_double), ("max_iter", C.c_int32),
                ("max_eval", C.c_int32), ("polish", C.c_void_p), ("polish_edm", C.c_double)]


class bx_fit_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("nll", C.c_double), ("x", C.c_double * 32),
                ("grad", C.c_double * 32), ("edm", C.c_double), ("n_iter", C.c_int32),
                ("n_eval", C.c_int32), ("t_submit_ns", C.c_int64), ("t_admit_ns", C.c_int64),
                ("t_done_ns", C.c_int64)]


# every exported entry point: name -> (restype, argtypes)
SIGNATURES = {
    "bx_model_build": (C.c_int, [C.POINTER(bx_model_desc), C.POINTER(bx_data), C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    "bx_model_set_data": (C.c_int, [C.c_void_p, C.POINTER(bx_data)]),
    "bx_model_free": (C.c_int, [C.c_void_p]),
    "bx_model_nparams": (C.c_int32, [C.c_void_p]),
    "bx_model_lnfact": (C.c_int, [C.c_void_p, _dp]),
    # raw addresses (ints) for the per-evaluation calls: cheaper to marshal
    "bx_nll_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bx_nll_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bx_nll_grad_dev": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bx_nll_grad_dev_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bx_model_expected_size": (C.c_int64, [C.c_void_p]),
    "bx_model_expected": (C.c_int, [C.c_void_p, _dp, _dp]),
    "bx_model_stage_times": (C.c_int, [C.c_void_p, _dp, C.c_int32, _dp]),
    "bx_model_batch_times": (C.c_int, [C.c_void_p, _dp, C.c_int32, C.c_int32, _dp]),
    "bx_model_cell_ceiling": (C.c_int, [C.c_void_p, _dp, C.c_int32, _dp]),
    "bx_fit_batch": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(bx_fit_opts), C.c_int32,
                               C.POINTER(bx_fit_result), C.c_int32]),
    "bx_fit": (C.c_int, [C.c_void_p, C.POINTER(bx_fit_opts), C.POINTER(bx_fit_result)]),
    "bx_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "bx_server_destroy": (C.c_int, [C.c_void_p]),
    "bx_fit_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(bx_fit_opts),
                                C.POINTER(C.c_uint64)]),
    "bx_fit_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(bx_fit_result)]),
    "bx_server_drain": (C.c_int, [C.c_void_p]),
    "bx_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libbx.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1805_11125_amd.build` (HIP, gfx950)")
        # PyTorch (device memory and streams for the autograd path) ships its
        # own HIP runtime; it has to claim the GPU before this library's does.
        try:
            import torch
            torch.cuda.is_available()
        except Exception:
            pass
        if "BX_TUNE_CACHE" not in os.environ and os.path.exists(TILE_TABLE):
            os.environ["BX_TUNE_CACHE"] = TILE_TABLE
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class BxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bx status {status}: {msg}")
        self.status = status


class DomainError(BxError):
    pass


def check(status, allow=(BX_OK,)):
    if status in allow:
        return status
    msg = load().bx_last_error().decode(errors="replace")
    if status == BX_E_DOMAIN:
        raise DomainError(status, msg)
    raise BxError(status, msg)


def dptr(a):
    """Pointer to a C-contiguous float64 numpy array (None -> NULL)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)

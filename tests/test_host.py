"""Host-side checks that need no GPU: the C ABI library loads and exports
every function include/bx.h declares, argument validation returns the
documented status codes, and the quasi-Newton core passes its C++ unit test."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_1805_11125_amd import _abi
    return _abi


def test_library_exports_every_declared_symbol(abi):
    lib = abi.load()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in abi.SIGNATURES, f"binding lacks {n}"


def _desc(abi, d, precision=0, **over):
    keep = []

    def arr(a):
        a = np.ascontiguousarray(np.asarray(a, np.float64).reshape(-1))
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    s = abi.bx_model_desc()
    s.T, s.N, s.S = d.T, d.N, d.S
    s.true_edges, s.reco_edges, s.spectra = arr(d.true_edges), arr(d.reco_edges), arr(d.spectra)
    s.response = 0 if d.kind == "gauss" else 1
    s.gg_p = d.gg_p
    if d.quench is not None:
        s.quench = arr(d.quench)
    s.exposure = d.exposure
    s.win_lo, s.win_hi = d.win
    s.precision = precision
    for k, v in over.items():
        setattr(s, k, arr(v) if isinstance(v, np.ndarray) else v)
    x = abi.bx_data()
    x.energy = arr(np.ones(d.N))
    return s, x, keep


@pytest.mark.parametrize("field,value", [
    ("T", 0), ("N", 0), ("S", 17), ("precision", 7), ("response", 5), ("exposure", 0.0),
    ("win_lo", 150), ("win_hi", 500), ("pu_K", 300),
    ("pu_float", 1),  # a floated pile-up fraction without a random-trigger spectrum
])
def test_build_rejects_invalid_descriptions(abi, field, value):
    d = synth.config1()
    s, x, keep = _desc(abi, d)
    if field == "win_lo":
        s.win_lo, s.win_hi = 150, 100
    else:
        setattr(s, field, value)
    h = C.c_void_p()
    st = abi.load().bx_model_build(C.byref(s), C.byref(x), None, C.byref(h))
    assert st == abi.BX_E_INVAL, (field, st)
    assert not h.value
    assert len(abi.load().bx_last_error()) > 0


def test_build_rejects_bad_arrays(abi):
    lib = abi.load()
    d = synth.config1()
    bad = d.reco_edges.copy()
    bad[5] = bad[4]
    s, x, keep = _desc(abi, d, reco_edges=bad)
    h = C.c_void_p()
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL
    sp = d.spectra.copy()
    sp[1] = 0.0
    s, x, keep = _desc(abi, d, spectra=sp)
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL
    s, x, keep = _desc(abi, d)
    x.energy = None
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL
    # pile-up on non-uniform reco bins
    d2 = synth.config1()
    d2.reco_edges = np.concatenate([d2.reco_edges[:-1], [d2.reco_edges[-1] + 0.5]])
    s, x, keep = _desc(abi, d2, pu_K=3, pu_g=np.ones(3), pu_frac=0.1)
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL


def test_build_rejects_invalid_tables(abi):
    # tabulated response: grid size, order, and matrices
    lib = abi.load()
    d = synth.config1()
    G = 3
    R = np.full((G, d.N, d.T), 1.0 / d.N)
    for n_grid, grid, rtab in [(0, [1.0], R), (65, [1.0], R), (G, [1.0, 3.0, 2.0], R),
                               (G, [1.0, 2.0, 3.0], -R), (G, [1.0, 2.0, np.nan], R)]:
        s, x, keep = _desc(abi, d, grid=np.asarray(grid, np.float64), rtab=np.asarray(rtab))
        s.response, s.n_grid = abi.BX_RESP_TABLE, n_grid
        h = C.c_void_p()
        assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL, (n_grid, grid)


def test_build_rejects_invalid_count_estimator(abi):
    # one count per reco bin, integer edges from >= 0, and the quenching table
    lib = abi.load()
    d = synth.count_config(T=20, N=30)
    for edges in (np.arange(31) * 2.0, np.arange(31) + 0.5, np.arange(31) - 1.0):
        s, x, keep = _desc(abi, d, reco_edges=edges, quench=d.quench)
        s.response = abi.BX_RESP_COUNT
        h = C.c_void_p()
        assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL, edges[:3]
    s, x, keep = _desc(abi, d)
    s.response = abi.BX_RESP_COUNT
    s.quench = None
    h = C.c_void_p()
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL


def test_build_rejects_joint_without_templates_or_histogram(abi):
    lib = abi.load()
    d = synth.config3a()
    S = d.S
    # the joint term needs both templates
    s, x, keep = _desc(abi, d, tag_frac=d.tag_frac, rad_tmpl=d.rad_tmpl)
    s.multivariate, s.joint, s.n_rad, s.n_ps = 1, 1, d.rad_tmpl.shape[1], 0
    h = C.c_void_p()
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL
    # and its histogram
    s, x, keep = _desc(abi, d, tag_frac=d.tag_frac, rad_tmpl=d.rad_tmpl, ps_tmpl=d.ps_tmpl)
    s.multivariate, s.joint, s.n_rad, s.n_ps = 1, 1, d.rad_tmpl.shape[1], d.ps_tmpl.shape[1]
    t = np.ones(d.N)
    x.tagged = t.ctypes.data_as(C.POINTER(C.c_double))
    assert S == d.rad_tmpl.shape[0]
    assert lib.bx_model_build(C.byref(s), C.byref(x), None, C.byref(h)) == abi.BX_E_INVAL
    assert b"joint" in lib.bx_last_error()


def test_null_arguments(abi):
    lib = abi.load()
    v = C.c_double()
    assert lib.bx_nll_eval(None, None, C.byref(v)) == abi.BX_E_INVAL
    assert lib.bx_model_nparams(None) == -1
    assert lib.bx_model_free(None) == abi.BX_OK
    assert lib.bx_model_build(None, None, None, None) == abi.BX_E_INVAL


def test_fitcore_unit(tmp_path):
    exe = tmp_path / "test_fitcore"
    src = os.path.join(ROOT, "tests", "host", "test_fitcore.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-o", str(exe), src], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "OK" in out.stdout

"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects invalid arguments on the host before touching a
device."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1408_3048_amd as pkg
from paper_1408_3048_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.EXPORTED)


def test_default_opts():
    lib = pkg.load()
    o = L.mm_opts()
    lib.mm_default_opts(ctypes.byref(o))
    assert o.n_stokes == 3 and o.lambda_ == 1024 and o.f_samp == 200.0
    assert o.rank_tol == 1e-10 and o.window == L.MM_WIN_GAUSS


def _plan_call(n=100, offsets=(0, 50, 100), psd=((1, 1, 1), (1, 1, 1)), n_stokes=1, lam=8,
               pix_ptr=1, n_pix=10, weights=None):
    lib = pkg.load()
    o = L.mm_opts()
    lib.mm_default_opts(ctypes.byref(o))
    o.n_stokes = n_stokes
    o.lambda_ = lam
    off = np.array(offsets, dtype=np.int64)
    ps = np.array(psd, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.mm_plan(ctypes.byref(h), n, ctypes.c_void_p(pix_ptr), weights, L.MM_F64, n_pix,
                     len(off) - 1, off.ctypes.data_as(ctypes.c_void_p),
                     ps.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o))
    return st, h, L.last_error()


@pytest.mark.parametrize("kw,frag", [
    (dict(offsets=(0, 60, 50)), "offsets"),
    (dict(offsets=(0, 50, 99)), "end at n_samples"),
    (dict(psd=((1, 1, 1), (0, 1, 1))), "PSD"),
    (dict(psd=((1, -1, 1), (1, 1, 1))), "PSD"),
    (dict(n=0, offsets=(0, 0)), "n_samples"),
    (dict(n_stokes=2), "n_stokes"),
    (dict(n_stokes=3, weights=None), "weights"),
    (dict(lam=-1), "mm_opts"),
    (dict(n_pix=0), "n_pix"),
])
def test_plan_rejects_bad_arguments_on_host(kw, frag):
    st, h, msg = _plan_call(**kw)
    assert st == L.MM_ERR_ARG
    assert h.value is None
    assert frag in msg


def test_null_plan_calls_are_errors():
    lib = pkg.load()
    assert lib.mm_n_obs(None) == -1
    assert lib.mm_apply_A(None, None, None, 0) == L.MM_ERR_ARG
    assert lib.mm_coarse_rank(None) == L.MM_ERR_ARG
    lib.mm_destroy(None)
    assert lib.mm_gemm_tn_f64(None, None, None, 3, 16, 16, None) == L.MM_ERR_ARG

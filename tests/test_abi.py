"""C-ABI checks that need no GPU: the library loads, exports every symbol of
include/bse.h, and validates arguments before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "bse.h")


def _header_symbols():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^(?:const char\*|bse_status)\s+(bse_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2607_05853_amd import bse
    return bse.lib()


def test_exports_every_declared_symbol(L):
    syms = _header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    from paper_2607_05853_amd import bse
    assert sorted(bse.EXPORTS) == syms


def test_status_strings(L):
    assert L.bse_status_string(0) == b"ok"
    assert b"invalid" in L.bse_status_string(1)
    assert b"breakdown" in L.bse_status_string(100).lower()
    assert L.bse_version().startswith(b"bse-gfx950")


def test_interpolate_validation_before_hip(L):
    R = np.zeros((1, 3), np.int32)
    w = np.ones(1)
    q = np.zeros((1, 3))
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert L.bse_interpolate_W(0, 1, dummy, R.ctypes.data, w.ctypes.data, 1, q.ctypes.data, dummy, 0, None) == 1
    assert L.bse_interpolate_W(4, 1, None, R.ctypes.data, w.ctypes.data, 1, q.ctypes.data, dummy, 0, None) == 1
    assert L.bse_interpolate_W(4, 1, dummy, R.ctypes.data, w.ctypes.data, 1, q.ctypes.data, dummy, 7, None) == 1
    assert b"precision" in L.bse_last_error()
    assert L.bse_interpolate_W_adjoint(4, 1, None, w.ctypes.data, 1, q.ctypes.data, dummy, dummy, None) == 1
    # the allocation-free variant: same validation, and sizes beyond its static workspace are refused
    # (BSE_ESHAPE) before any HIP call
    assert L.bse_interpolate_W_noalloc(0, 1, dummy, R.ctypes.data, w.ctypes.data, 1, q.ctypes.data, dummy, 0,
                                       None) == 1
    assert L.bse_interpolate_W_noalloc(4, 1, None, R.ctypes.data, w.ctypes.data, 1, q.ctypes.data, dummy, 0,
                                       None) == 1
    Rb, wb, qb = np.zeros((1000, 3), np.int32), np.ones(1000), np.zeros((2000, 3))
    assert L.bse_interpolate_W_noalloc(4, 1000, dummy, Rb.ctypes.data, wb.ctypes.data, 2000, qb.ctypes.data,
                                       dummy, 0, None) == 2
    assert b"static scratch" in L.bse_last_error()


def _dims(**kw):
    from paper_2607_05853_amd.bse import _Dims
    d = dict(nk=(2, 2, 2), n_ao=8, nv=2, nc=2, n_aux=12, alpha=2.0)
    d.update(kw)
    return _Dims((ctypes.c_int32 * 3)(*d["nk"]), d["n_ao"], d["nv"], d["nc"], d["n_aux"], d["alpha"])


def test_plan_create_validation_before_hip(L):
    dummy = ctypes.c_void_p(16)
    out = ctypes.c_void_p()
    args = lambda d, prec=0, nb=4, flags=0, ptr=dummy: L.bse_plan_create(
        ctypes.byref(d), ptr, dummy, dummy, dummy, dummy, prec, nb, flags, None, ctypes.byref(out))
    assert args(_dims(nk=(0, 2, 2))) == 1
    assert args(_dims(nv=0)) == 1
    assert args(_dims(alpha=float("nan"))) == 1
    assert args(_dims(), ptr=None) == 1
    assert args(_dims(), prec=5) == 1
    assert args(_dims(), nb=0) == 1
    assert args(_dims(), flags=16) == 1                  # unknown flag
    assert args(_dims(), prec=2, flags=4 | 8) == 1       # both conduction routes
    assert args(_dims(), prec=0, flags=8) == 1           # the B_c contraction is a BF16x3 route
    assert args(_dims(nv=12), prec=2, flags=8) == 2      # nv^2 > 128
    assert args(_dims(n_ao=136), prec=2, flags=8) == 2   # n_ao > 128
    assert args(_dims(nv=32, nc=32), nb=4) == 2          # nv*nc*max_nb above the limit
    assert args(_dims(nk=(2048, 2048, 2))) == 2          # too many k points
    assert L.bse_plan_create(None, dummy, dummy, dummy, dummy, dummy, 0, 4, 0, None, ctypes.byref(out)) == 1
    assert out.value is None


def test_plan_create_2c_validation_before_hip(L):
    dummy = ctypes.c_void_p(16)
    out = ctypes.c_void_p()
    RC = np.zeros((1, 3), np.int32)
    kf = np.zeros((2, 8, 3))
    args = lambda d=None, nR=1, rc=RC.ctypes.data, cr=dummy, k=kf.ctypes.data, prec=0, flags=0: \
        L.bse_plan_create_2c(ctypes.byref(d or _dims()), dummy, dummy, nR, rc, cr, k, dummy, dummy, prec, 4, flags,
                             None, ctypes.byref(out))
    assert args(nR=0) == 1
    assert args(rc=None) == 1
    assert args(cr=None) == 1
    assert args(k=None) == 1
    assert args(d=_dims(nv=0)) == 1
    assert args(prec=2, flags=8) == 1                    # no B_c(k) contraction with two centres
    assert b"k-independent" in L.bse_last_error()
    assert args(flags=32) == 1
    assert out.value is None


def test_null_plan_calls(L):
    dummy = ctypes.c_void_p(16)
    assert L.bse_apply(None, dummy, dummy, 1, None) == 1
    assert L.bse_apply_adjoint(None, dummy, dummy, 1, None, None, None, None) == 1
    assert L.bse_haydock_spectrum(None, dummy, 1, 1, dummy, 1, 0.1, dummy, dummy, dummy, dummy, None, None) == 1
    assert L.bse_plan_set_R(None, 1, dummy, dummy) == 1
    assert L.bse_plan_destroy(None) == 0
    assert L.bse_lowest_excitons(None, 4, 10, 1e-8, None, dummy, None, None, None) == 1
    assert L.bse_velocity_start(None, dummy, dummy, 1, dummy, dummy, None) == 1
    a, b = ctypes.c_int64(), ctypes.c_int64()
    assert L.bse_plan_pairs(None, ctypes.byref(a), ctypes.byref(b)) == 1
    c = ctypes.c_int32()
    assert L.bse_plan_conduction(None, ctypes.byref(c)) == 1
    assert L.bse_plan_fused(None, ctypes.byref(c)) == 1
    assert L.bse_plan_frag(None, ctypes.byref(c)) == 1
    # offset averaging: NULL arrays and empty offset lists are rejected before any HIP call
    w = (ctypes.c_double * 1)(1.0)
    om = (ctypes.c_double * 1)(2.0)
    S = (ctypes.c_double * 1)()
    assert L.bse_offset_spectrum(None, None, w, 1, 1, 1, om, 1, 0.1, S, None, None) == 1
    plans = (ctypes.c_void_p * 1)(None)
    Ps = (ctypes.c_void_p * 1)(dummy)
    assert L.bse_offset_spectrum(plans, Ps, w, 1, 1, 1, om, 1, 0.1, S, None, None) == 1
    assert L.bse_offset_spectrum(plans, Ps, w, 0, 1, 1, om, 1, 0.1, S, None, None) == 1
    assert L.bse_offset_set(None, None, None) == 1
    # full BSE
    assert L.bse_apply_coupling(None, dummy, dummy, 1, None) == 1
    assert L.bse_apply_full(None, dummy, dummy, 1, None) == 1
    assert L.bse_full_spectrum(None, dummy, 1, 2, om, 1, 0.1, S, S, S, None, None) == 1
    assert L.bse_full_lowest(None, 1, 10, 1e-8, None, om, None, None, None) == 1


def test_offset_set_is_the_papers(L):
    n = ctypes.c_int32()
    off = (ctypes.c_double * 12)()
    w = (ctypes.c_double * 4)()
    assert L.bse_offset_set(ctypes.byref(n), off, w) == 0
    assert n.value == 4
    assert [round(27 * w[j]) for j in range(4)] == [1, 8, 6, 12]
    assert [round(3 * off[i]) for i in range(12)] == [0, 0, 0, 1, 0, 0, 1, 1, 0, 2, 1, 0]


def test_binding_rejects_cpu_tensors():
    import torch
    from paper_2607_05853_amd import bse
    with pytest.raises(TypeError):
        bse.interpolate_W(torch.zeros((1, 2, 2), dtype=torch.complex128), np.zeros((1, 3)), np.ones(1),
                          np.zeros((1, 3)))


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as strict C99 with no C++ or torch types
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "h.c"
    src.write_text('#include "bse.h"\nint main(void) { return 0; }\n')
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

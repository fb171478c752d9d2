"""The C ABI on the CPU: libxf.so loads, exports every function include/xf.h
declares, and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xf.h")
LIB = os.path.join(ROOT, "paper_2403_05910_amd", "libxf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libxf.so not built")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("xf_rhs", "xf_rk3_step", "xf_rhs_vjp", "xf_create", "xf_status"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_the_abi():
    from paper_2403_05910_amd import xf
    assert sorted(xf.EXPORTED) == declared()
    for n in declared():
        assert callable(getattr(xf, n))


def test_strerror_and_argument_errors_without_device():
    from paper_2403_05910_amd import xf
    assert xf.xf_strerror(0) == "success"
    assert "invalid" in xf.xf_strerror(xf.XF_EINVAL)
    W = (ctypes.c_double * 2)(0.028, 0.004)
    a = (ctypes.c_double * 12)(*([3.5, 0, 0, 0, 0, 0] * 2))
    th = xf.xf_thermo(2, ctypes.cast(W, xf._dp), ctypes.cast(a, xf._dp), 0.0, 0.0)
    h = ctypes.c_void_p()
    bad_grids = [
        xf.xf_grid(2, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0)),    # active dim with n < 3
        xf.xf_grid(8, 1, 1, -0.1, 1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0)),   # dx <= 0
        xf.xf_grid(8, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(0, 1, 0, 0, 0, 0)),    # unpaired periodic side
        xf.xf_grid(8, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(7, 7, 0, 0, 0, 0)),    # unknown bc
        xf.xf_grid(0, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0)),    # n < 1
        xf.xf_grid(8, 70000, 1, 0.1, 0.1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0)),  # n > 65535
    ]
    for g in bad_grids:
        assert xf._create(ctypes.byref(g), ctypes.byref(th), 0, ctypes.byref(h)) == xf.XF_EINVAL
        assert not h.value
    good = xf.xf_grid(8, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0))
    assert xf._create(ctypes.byref(good), ctypes.byref(th), 7, ctypes.byref(h)) == xf.XF_EINVAL
    th10 = xf.xf_thermo(10, ctypes.cast(W, xf._dp), ctypes.cast(a, xf._dp), 0.0, 0.0)
    assert xf._create(ctypes.byref(good), ctypes.byref(th10), 0, ctypes.byref(h)) == xf.XF_EUNSUPPORTED
    thb = xf.xf_thermo(2, ctypes.cast(W, xf._dp), ctypes.cast(a, xf._dp), 500.0, 400.0)
    assert xf._create(ctypes.byref(good), ctypes.byref(thb), 0, ctypes.byref(h)) == xf.XF_EINVAL
    assert xf._create(None, ctypes.byref(th), 0, ctypes.byref(h)) == xf.XF_EINVAL
    # ghost width: 3 or 4 only, and an active dimension needs at least that many cells
    for ng in (0, 2, 5):
        assert xf._create_ghosts(ctypes.byref(good), ctypes.byref(th), 0, ng, ctypes.byref(h)) == xf.XF_EINVAL
        assert not h.value
    three = xf.xf_grid(3, 1, 1, 0.1, 1, 1, (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0))
    assert xf._create_ghosts(ctypes.byref(three), ctypes.byref(th), 0, 4, ctypes.byref(h)) == xf.XF_EINVAL
    assert xf._create_ghosts(None, ctypes.byref(th), 0, 4, ctypes.byref(h)) == xf.XF_EINVAL
    # null contexts and buffers are refused before any device work
    assert xf._rhs(None, None, None, None, None) == xf.XF_EINVAL
    assert xf._rk3(None, None, 0.1, None, None, None) == xf.XF_EINVAL
    assert xf._rhs_vjp(None, None, None, None, None, None) == xf.XF_EINVAL
    assert xf._rk3_vjp(None, None, 0.1, None, None, None) == xf.XF_EINVAL
    assert xf._fill(None, None, None) == xf.XF_EINVAL
    assert xf._set_pp(None, 1) == xf.XF_EINVAL
    assert xf._set_visc(None, 1) == xf.XF_EINVAL
    assert xf._set_recon(None, 1) == xf.XF_EINVAL
    assert xf._set_viscous(None, None, 7) == xf.XF_EINVAL
    assert xf._set_reactions(None, None, 4, 0) == xf.XF_EINVAL
    assert xf._react(None, None, 1e-6, None, None) == xf.XF_EINVAL
    assert xf._state_elems(None) == 0
    assert xf._ws_bytes(None, 0) == 0

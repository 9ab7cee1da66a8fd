"""Host-side checks of the C ABI (no GPU needed): exports, argument validation, error codes."""
import ctypes
import os

import pytest

from paper_2403_20135_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="library not built (run __graft_entry__.build())")


def _cfg(**kw):
    base = dict(T=31, nlat=48, nlon=96, radius=6.371e6, gravity=9.81, omega=7.292e-5, mean_depth=1e4,
                M=3, K=2, nodes=0, qdelta=0, precision=0, batch=1)
    base.update(kw)
    return _lib.SdcConfig(**base)


def test_every_declared_function_is_exported():
    lib = _lib.load()
    names = _lib.header_functions()
    assert "sdc_init" in names and "sdc_step" in names and "sht_forward" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


@pytest.mark.parametrize("kw,code", [
    (dict(T=0), _lib.SDC_EINVAL),
    (dict(T=31, nlat=30), _lib.SDC_EINVAL),            # nlat < T+1
    (dict(nlat=49), _lib.SDC_EINVAL),                   # odd nlat
    (dict(nlon=62), _lib.SDC_EINVAL),                   # nlon < 2T+1
    (dict(M=0), _lib.SDC_EINVAL),
    (dict(M=9), _lib.SDC_EINVAL),
    (dict(K=0), _lib.SDC_EINVAL),
    (dict(nodes=1), _lib.SDC_EINVAL),
    (dict(qdelta=3), _lib.SDC_EINVAL),
    (dict(precision=7), _lib.SDC_EINVAL),
    (dict(batch=0), _lib.SDC_EINVAL),
    (dict(radius=-1.0), _lib.SDC_EINVAL),
    (dict(mean_depth=0.0), _lib.SDC_EINVAL),
    (dict(nlon=100), _lib.SDC_EUNSUPPORTED),            # not 2^p or 3*2^p
    (dict(nlon=4096, T=31), _lib.SDC_EUNSUPPORTED),
    (dict(precision=2), _lib.SDC_EUNSUPPORTED),         # BF16x3 not implemented
])
def test_init_rejects_invalid_config_on_host(kw, code):
    lib = _lib.load()
    h = ctypes.c_void_p(123)
    cfg = _cfg(**kw)
    rc = lib.sdc_init(ctypes.byref(cfg), None, ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert lib.sdc_last_error()


def test_null_arguments():
    lib = _lib.load()
    cfg = _cfg()
    assert lib.sdc_init(ctypes.byref(cfg), None, None) == _lib.SDC_EINVAL
    assert lib.sdc_init(None, None, ctypes.byref(ctypes.c_void_p())) == _lib.SDC_EINVAL
    assert lib.sdc_free(None) == _lib.SDC_OK
    assert lib.sdc_step(None, None, 1.0, 1, 1) == _lib.SDC_EINVAL
    assert lib.sdc_sync(None) == _lib.SDC_EINVAL
    assert lib.sht_forward(None, None, None) == _lib.SDC_EINVAL
    assert lib.eval_explicit(None, None, None) == _lib.SDC_EINVAL
    assert lib.imex2_step(None, None, 1.0) == _lib.SDC_EINVAL
    assert lib.sdc_tape_size(None, 1, 1, ctypes.byref(ctypes.c_longlong())) == _lib.SDC_EINVAL
    assert lib.sdc_step_taped(None, None, 1.0, 1, 1, None) == _lib.SDC_EINVAL
    assert lib.sdc_step_adjoint_taped(None, None, None, None, 1.0, 1, 1) == _lib.SDC_EINVAL
    assert lib.sdc_step_sequential(None, None, 1.0, 1, 1) == _lib.SDC_EINVAL
    assert lib.sdc_step_sequential_graph(None, None, 1.0, 1, 1) == _lib.SDC_EINVAL
    assert lib.imex2_step_graph(None, None, 1.0) == _lib.SDC_EINVAL
    pl = _lib.SdcPlan(1, 8, 4, 1)
    assert lib.sdc_get_plan(None, ctypes.byref(pl)) == _lib.SDC_EINVAL
    assert lib.sdc_set_plan(None, ctypes.byref(pl)) == _lib.SDC_EINVAL
    assert lib.sdc_autotune(None, 3, ctypes.byref(pl)) == _lib.SDC_EINVAL
    assert b"NULL" in lib.sdc_last_error()


def test_error_wrapper():
    with pytest.raises(_lib.SDCError) as ei:
        _lib.check(_lib.load().sdc_step(None, None, 1.0, 1, 1))
    assert ei.value.code == _lib.SDC_EINVAL

"""Host-side C ABI checks shared by test_abi.py (the built library) and test_abi_sanitized.py (the
library with AddressSanitizer and UndefinedBehaviorSanitizer on its host code, run in a child
process that preloads the sanitizer runtime).  Every call here fails validation on the host, so
no GPU is touched."""
import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2403_20135_amd import _lib  # noqa: E402

BASE = dict(T=31, nlat=48, nlon=96, radius=6.371e6, gravity=9.81, omega=7.292e-5, mean_depth=1e4,
            M=3, K=2, nodes=0, qdelta=0, precision=0, batch=1, implicit_coriolis=0)

INVALID_CONFIGS = [
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
    (dict(implicit_coriolis=2), _lib.SDC_EINVAL),
    (dict(nlon=100), _lib.SDC_EUNSUPPORTED),            # not 2^p or 3*2^p
    (dict(nlon=4096, T=31), _lib.SDC_EUNSUPPORTED),
    (dict(precision=-1), _lib.SDC_EINVAL),
]


def cfg(**kw):
    base = dict(BASE)
    base.update(kw)
    return _lib.SdcConfig(**base)


def load(path=None):
    """The library at path (default: the built one) with the binding's signatures."""
    if path is None:
        return _lib.load()
    lib = ctypes.CDLL(path)
    for name, (res, args) in _lib._SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def check_invalid_configs(lib):
    for kw, code in INVALID_CONFIGS:
        h = ctypes.c_void_p(123)
        c = cfg(**kw)
        rc = lib.sdc_init(ctypes.byref(c), None, ctypes.byref(h))
        assert rc == code, (kw, rc)
        assert h.value is None, kw
        assert lib.sdc_last_error(), kw


def check_null_arguments(lib):
    c = cfg()
    dp = ctypes.c_void_p()
    ll = ctypes.c_longlong()
    assert lib.sdc_init(ctypes.byref(c), None, None) == _lib.SDC_EINVAL
    assert lib.sdc_init(None, None, ctypes.byref(dp)) == _lib.SDC_EINVAL
    assert lib.sdc_free(None) == _lib.SDC_OK
    E = _lib.SDC_EINVAL
    calls = [
        lib.sdc_step(None, None, 1.0, 1, 1), lib.sdc_step_graph(None, None, 1.0, 1, 1),
        lib.sdc_step_adjoint(None, None, None, None, 1.0, 1, 1), lib.sdc_sync(None),
        lib.sht_forward(None, None, None), lib.sht_inverse(None, None, None),
        lib.sht_inverse_adjoint(None, None, None), lib.imex_solve(None, 1.0, None, None),
        lib.eval_explicit(None, None, None), lib.eval_implicit(None, None, None),
        lib.imex2_step(None, None, 1.0), lib.imex2_step_graph(None, None, 1.0),
        lib.imex2_step_noalloc(None, None, 1.0), lib.sdc_tape_size(None, 1, 1, ctypes.byref(ll)),
        lib.sdc_step_taped(None, None, 1.0, 1, 1, None),
        lib.sdc_step_adjoint_taped(None, None, None, None, 1.0, 1, 1),
        lib.sdc_step_sequential(None, None, 1.0, 1, 1), lib.sdc_step_sequential_graph(None, None, 1.0, 1, 1),
        lib.sdc_timing_enable(None, 1), lib.sdc_get_info(None, None),
        lib.sdc_group_step(None, None, None, 1, 1), lib.sdc_group_set_mode(None, 1),
        lib.sdc_group_sync(None),
    ]
    assert all(rc == E for rc in calls), calls
    assert lib.sdc_group_free(None) == _lib.SDC_OK
    assert lib.sdc_group_create(None, 0, None, None) == E
    pl = _lib.SdcPlan(1, 8, 4, 1)
    assert lib.sdc_get_plan(None, ctypes.byref(pl)) == E
    assert lib.sdc_set_plan(None, ctypes.byref(pl)) == E
    assert lib.sdc_get_plan_for(None, 1, ctypes.byref(pl)) == E
    assert lib.sdc_set_plan_for(None, 1, ctypes.byref(pl)) == E
    assert lib.sdc_autotune(None, 3, ctypes.byref(pl)) == E
    assert b"NULL" in lib.sdc_last_error()
    # long messages are truncated to the message buffer, not overrun
    long_cfg = cfg(T=-12345678)
    assert lib.sdc_init(ctypes.byref(long_cfg), None, ctypes.byref(dp)) == E
    assert len(lib.sdc_last_error()) < 512


def run_all(path=None):
    lib = load(path)
    check_invalid_configs(lib)
    check_null_arguments(lib)


if __name__ == "__main__":
    run_all(sys.argv[1] if len(sys.argv) > 1 else None)
    print("abi checks passed")

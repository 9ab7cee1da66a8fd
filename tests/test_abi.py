"""Host-side checks of the C ABI (no GPU needed): exports, argument validation, error codes."""
import os

import pytest

import abi_checks
from paper_2403_20135_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="library not built (run __graft_entry__.build())")


def test_every_declared_function_is_exported():
    lib = _lib.load()
    names = _lib.header_functions()
    assert "sdc_init" in names and "sdc_step" in names and "sht_forward" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


def test_init_rejects_invalid_config_on_host():
    abi_checks.check_invalid_configs(_lib.load())


def test_null_arguments():
    abi_checks.check_null_arguments(_lib.load())


def test_error_wrapper():
    with pytest.raises(_lib.SDCError) as ei:
        _lib.check(_lib.load().sdc_step(None, None, 1.0, 1, 1))
    assert ei.value.code == _lib.SDC_EINVAL

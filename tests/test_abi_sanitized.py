"""The host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library is rebuilt with both sanitizers on its host code (device code unchanged) and every
host-side check of abi_checks runs in a child process that preloads the sanitizer runtime; any
report (heap or stack overflow, use after free, undefined behaviour) fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc not available")


def test_host_abi_under_address_and_ub_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2403_20135_amd import build
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.sanitizer_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = os.pathsep.join([HERE, ROOT])
    r = subprocess.run([sys.executable, os.path.join(HERE, "abi_checks.py"), lib], env=env,
                       capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "abi checks passed" in r.stdout

"""Read-before-write check of the step (the Jacobi sweeps read only the previous sweep's values):
with sdc_debug_poison on, every workspace a launch of the step writes is filled with NaN bit
patterns just before that launch, so a kernel reading a value of its own sweep before it is
written, a padding row it does not clear, or a value left from an earlier sweep would turn the
step's result into NaN.  The poisoned steps must equal the plain ones bit for bit."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _sdc, _states

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,nlat,nlon,M,K,batch,prec,plan", [
    (31, 48, 96, 4, 4, 2, "fp64", None),                  # node update fused in the analysis
    (31, 48, 96, 3, 3, 1, "fp64", None),                  # separate update kernel
    (21, 34, 64, 2, 4, 1, "fp64", None),                  # K > M, ragged latitude tile
    (31, 48, 96, 4, 3, 2, "fp32", None),                  # FP32 columns (half-size layouts)
    (63, 96, 192, 4, 4, 1, "fp64", (4, 2, 2, 1, 1, 1, 1)),   # regenerating Legendre variants
    (31, 48, 96, 4, 4, 1, "fp64", (2, 2, 2, 1, 1, 0, 0, 1)),  # one node per launch
])
def test_poisoned_steps_equal_plain_steps(T, nlat, nlon, M, K, batch, prec, plan):
    sdc = _sdc(T, nlat, nlon, M, K, batch, precision=prec)
    if plan:
        sdc.set_plan(*plan)
    x0 = _states(T, batch, 951)
    dt = 600.0
    plain, poisoned, graph = _dev(x0), _dev(x0), _dev(x0)
    for _ in range(2):
        sdc.step(plain, dt)
    sdc.debug_poison(True)
    for _ in range(2):
        sdc.step(poisoned, dt)
        sdc.step_graph(graph, dt)
    tape = sdc.new_tape()
    taped = _dev(x0)
    sdc.step_taped(taped, dt, tape)
    sdc.debug_poison(False)
    sdc.sync()
    a, b, g = _host(plain), _host(poisoned), _host(graph)
    print(f"[gpu] poison T{T} M={M} K={K} x{batch} {prec} {plan}: finite {np.isfinite(b).all()}, "
          f"max |diff| {np.nanmax(np.abs(a - b)):.3e}", flush=True)
    assert np.isfinite(b).all() and np.isfinite(g).all()
    assert np.array_equal(a, b) and np.array_equal(a, g)
    one = _dev(x0)
    sdc.step(one, dt)
    assert np.array_equal(_host(taped), _host(one))
    sdc.close()


def test_roctx_phase_ranges_leave_results_unchanged(monkeypatch):
    """A handle created with SDC_ROCTX set marks its phases with roctx ranges (host side only):
    the same states bit for bit as a handle without them."""
    T, nlat, nlon, M, K = 31, 48, 96, 4, 4
    x0 = _states(T, 1, 961)
    plain = _sdc(T, nlat, nlon, M, K, 1)
    monkeypatch.setenv("SDC_ROCTX", "1")
    marked = _sdc(T, nlat, nlon, M, K, 1)
    a, b = _dev(x0), _dev(x0)
    for _ in range(2):
        plain.step(a, 600.0)
        marked.step(b, 600.0)
        marked.step_graph(_dev(x0), 600.0)
    plain.sync()
    marked.sync()
    assert np.array_equal(_host(a), _host(b))
    plain.close()
    marked.close()

"""The allocation-free IMEX-o2 entry point (imex2_step_noalloc) against imex2_step, through the
C ABI: bitwise the same states on two handles in a row (the second with a smaller input: fewer
members of a lower truncation), each over several steps, reusing the library's one device scratch
array; the oracle's IMEX-o2 on the smaller case (<= 1e-11 relative L2); and the size limit."""
import numpy as np
import pytest

import workloads as W
from oracle.sdc import Oracle

from test_gpu_parity import _dev, _host, _sdc, _states, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_imex2_matches_imex2_on_two_handles(precision):
    cases = [(63, 96, 192, 3, 480.0), (31, 48, 96, 1, 600.0)]     # second: smaller input
    for T, nlat, nlon, batch, dt in cases:
        sdc = _sdc(T, nlat, nlon, 2, 2, batch, precision)
        x0 = _states(T, batch, 70 + T)
        a, b = _dev(x0), _dev(x0)
        for k in range(3):
            sdc.imex2_step_noalloc(b, dt)
            sdc.imex2_step(a, dt)
            sdc.sync()
            ga, gb = _host(a), _host(b)
            print(f"[gpu] T{T} x{batch} {precision} step {k + 1}: noalloc equal to imex2_step: "
                  f"{np.array_equal(ga, gb)}", flush=True)
            assert np.array_equal(ga, gb)
        if T == 31 and precision == "fp64":
            o = Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
            ref = np.stack([o.imex2(x0[i], dt, steps=3) for i in range(batch)])
            err = rel_l2(gb, ref, T)
            print(f"[gpu] T31 noalloc IMEX-o2 3 steps vs oracle: rel L2 {err:.3e}", flush=True)
            assert err <= 1e-11
        sdc.close()


def test_noalloc_imex2_rejects_inputs_beyond_its_scratch():
    from paper_2403_20135_amd._lib import SDC_EINVAL, SDCError
    T, nlat, nlon, batch = 31, 48, 96, 1400        # 3 * 1400 * 3 * 528 * 16 B > 64 MiB
    sdc = _sdc(T, nlat, nlon, 1, 1, batch)
    x = _dev(np.zeros((batch, 3, (T + 1) * (T + 2) // 2, 2)))
    with pytest.raises(SDCError) as e:
        sdc.imex2_step_noalloc(x, 600.0)
    assert e.value.code == SDC_EINVAL and "scratch" in str(e.value)
    assert not _host(x).any()                      # nothing was enqueued
    sdc.close()

"""GPU parity of the method variants beside the paper's choices, against the oracle through the
C ABI: MIN-SR-NS diagonal coefficients (tau_m / M in every sweep) for the step and its adjoint."""
import numpy as np
import pytest

import workloads as W
from oracle.sdc import Oracle

from test_gpu_parity import _dev, _host, _states, rel_l2

pytestmark = pytest.mark.gpu


def _sdc_ns(T, nlat, nlon, M, K, batch):
    from paper_2403_20135_amd.api import SDC
    print(f"\n[gpu] SDC(T={T}, {nlat}x{nlon}, M={M}, K={K}, batch={batch}, MIN-SR-NS)", flush=True)
    return SDC(T, nlat, nlon, M, K, batch, "fp64", W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH,
               qdelta="ns")


def _oracle_ns(T, nlat, nlon):
    return Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH, qdelta="ns")


@pytest.mark.parametrize("T,nlat,nlon,M,K,dt,steps,batch", [
    (31, 48, 96, 3, 3, 600.0, 5, 1),
    (63, 96, 192, 4, 4, 480.0, 2, 2),
    (21, 34, 64, 2, 5, 900.0, 3, 1),        # K > M
])
def test_min_sr_ns_step_matches_oracle(T, nlat, nlon, M, K, dt, steps, batch):
    sdc = _sdc_ns(T, nlat, nlon, M, K, batch)
    o = _oracle_ns(T, nlat, nlon)
    u0 = _states(T, batch, 501)
    x = _dev(u0)
    for _ in range(steps):
        sdc.step(x, dt)
    sdc.sync()
    ref = np.stack([o.step(u0[b], dt, M, K, steps=steps) for b in range(batch)])
    err = rel_l2(_host(x), ref, T)
    # the variant really differs from MIN-SR-FLEX
    flex = np.stack([Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
                     .step(u0[b], dt, M, K, steps=steps) for b in range(batch)])
    print(f"[gpu] MIN-SR-NS T{T} M{M}K{K}: rel L2 {err:.3e} (FLEX differs by {rel_l2(flex, ref, T):.2e})",
          flush=True)
    assert err <= 1e-11
    assert rel_l2(flex, ref, T) > 1e-9


def test_min_sr_ns_adjoint_matches_oracle_vjp():
    T, nlat, nlon, M, K, dt = 31, 48, 96, 3, 3, 600.0
    sdc = _sdc_ns(T, nlat, nlon, M, K, 1)
    o = _oracle_ns(T, nlat, nlon)
    x = _states(T, 1, 502)
    lam = W.random_state(T, 503)[None]
    lam[..., :T + 1, 1] = 0.0
    out = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), out, dt)
    ref = o.step_vjp(x[0], lam[0], dt, M, K)[None]
    err = rel_l2(_host(out), ref, T)
    print(f"[gpu] MIN-SR-NS adjoint: rel L2 {err:.3e}", flush=True)
    assert err <= 1e-10

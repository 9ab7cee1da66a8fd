"""GPU checks of the FP32 precision mode (Legendre contractions with FP32 tables, FP32 operands and
FP32 accumulation on MFMA; every other step FP64) against the FP64 oracle, and its error next to
the plain FP64 path on the plain-vs-compensated workload (T127 jet, M=3, K=3, dt=240 s).

Tolerances (FP32 unit roundoff u = 2^-24): one tendency evaluation sums at most T+1 products per
output, so its relative error is bounded by about (T+1) u; the tests allow 2 (T+1) u for f_E and
the adjoint.  A step mixes f_E into the state with weight dt, so the state error after k steps is
bounded by k times the tendency error relative to the state change; the step tests allow
2 (T+1) u k (checked on the state change, not the state).
"""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, _torch, rel_l2

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.mark.parametrize("T,nlat,nlon,batch", [(31, 48, 96, 3), (63, 96, 192, 1), (21, 34, 64, 2)])
def test_fp32_explicit_tendency_vs_oracle(T, nlat, nlon, batch):
    sdc = _sdc(T, nlat, nlon, 2, 2, batch, precision="fp32")
    ref64 = _sdc(T, nlat, nlon, 2, 2, batch)
    o = _oracle(T, nlat, nlon)
    x = _states(T, batch, 71)
    f32 = _dev(np.zeros_like(x))
    f64 = _dev(np.zeros_like(x))
    sdc.eval_explicit(_dev(x), f32)
    ref64.eval_explicit(_dev(x), f64)
    ref = np.stack([o.f_explicit(x[b]) for b in range(batch)])
    e32, e64 = rel_l2(_host(f32), ref, T), rel_l2(_host(f64), ref, T)
    print(f"[gpu] f_E T{T}: fp32 rel L2 {e32:.3e}, fp64 {e64:.3e}, bound {2 * (T + 1) * U32:.2e}",
          flush=True)
    assert e64 <= 1e-11
    assert e32 <= 2 * (T + 1) * U32
    assert e32 > 10 * e64          # the FP32 tables are really in use


def test_fp32_steps_vs_oracle():
    """The plain-method shape (T31, M=3, K=2, dt=600 s), 10 steps."""
    T, nlat, nlon, M, K, dt, steps = 31, 48, 96, 3, 2, 600.0, 10
    sdc = _sdc(T, nlat, nlon, M, K, 2, precision="fp32")
    o = _oracle(T, nlat, nlon)
    x0 = _states(T, 2, 81)
    x = _dev(x0)
    for _ in range(steps):
        sdc.step(x, dt)
    sdc.sync()
    got = _host(x)
    ref = np.stack([o.step(x0[b], dt, M, K, steps=steps) for b in range(2)])
    # error relative to the change of the state over the run
    err = rel_l2(got - x0, ref - x0, T)
    print(f"[gpu] fp32 {steps} steps: rel L2 of the state change {err:.3e}", flush=True)
    assert err <= 2 * (T + 1) * U32 * steps


def test_fp32_adjoint_vs_oracle_vjp():
    T, nlat, nlon, M, K, dt = 31, 48, 96, 3, 2, 600.0
    sdc = _sdc(T, nlat, nlon, M, K, 1, precision="fp32")
    o = _oracle(T, nlat, nlon)
    x = _states(T, 1, 91)
    lam = np.stack([W.random_state(T, 92)])
    lam[..., :T + 1, 1] = 0.0
    out = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), out, dt, M, K)
    got = _host(out)
    ref = o.step_vjp(x[0], lam[0], dt, M, K)[None]
    # the adjoint maps lam to lam_n = lam + (terms through f_E); compare the f_E part
    err = rel_l2(got - lam, ref - lam, T)
    print(f"[gpu] fp32 adjoint: rel L2 of the f_E part {err:.3e}", flush=True)
    assert err <= 2 * (T + 1) * U32 * 4


def _zeta_history(sdc, x0, dt, steps, every):
    x = _dev(x0)
    out = []
    for k in range(1, steps + 1):
        sdc.step(x, dt)
        if k % every == 0:
            out.append(_host(x)[:, 1].copy())
    sdc.sync()
    return out


def test_equal_error_plain_vs_fp32_t127_jet():
    """E = max over output times of the relative L2 error of zeta against the FP64 path at dt/8;
    FP32 is at equal error when E_fp32 <= 1.1 E_fp64 (recorded either way, asserted to stay
    within a factor 10 so that a broken FP32 path fails)."""
    wl = W.WORKLOADS["t127_m3k3_jet"]
    mb = wl.members[0]
    T = mb.T
    x0 = W.initial_state(wl)[None]
    steps, every = 20, 5
    ref = _zeta_history(_sdc(T, mb.nlat, mb.nlon, wl.M, wl.K), x0, mb.dt / 8, 8 * steps, 8 * every)
    h64 = _zeta_history(_sdc(T, mb.nlat, mb.nlon, wl.M, wl.K), x0, mb.dt, steps, every)
    h32 = _zeta_history(_sdc(T, mb.nlat, mb.nlon, wl.M, wl.K, precision="fp32"), x0, mb.dt, steps, every)
    e64 = max(rel_l2(a, r, T) for a, r in zip(h64, ref))
    e32 = max(rel_l2(a, r, T) for a, r in zip(h32, ref))
    print(f"[gpu] T127 jet, {steps} steps of dt={mb.dt}: E_fp64 {e64:.3e}, E_fp32 {e32:.3e}, "
          f"ratio {e32 / e64:.3f} ({'equal' if e32 <= 1.1 * e64 else 'NOT equal'} error)", flush=True)
    assert e32 <= 10 * e64

"""GPU checks of the BF16x3 precision mode (the FP32 mode's FP32 tables and columns, each MFMA
operand split exactly into three BF16 terms, the products formed from all cross terms but the
smallest on BF16 MFMA, FP32 accumulation; every other step FP64) against the FP64 oracle and
against the FP32 mode.

Tolerances (FP32 unit roundoff u = 2^-24), as for the FP32 mode: the operands are the FP32 mode's
FP32 values, the products exact to 2^-32 relative, the sums FP32, so the error is that of the FP32
mode: the tests allow 2 (T+1) u per step on the state change and for the adjoint's f_E part, and
hold f_E to 1.5 times the FP32 mode's own error on the same input (and 4 (T+1) u).  A split that
dropped its third term would leave products wrong by about 2^-16, one that kept a single term
(plain BF16) by 2^-8: hundreds of times the FP32 mode's error.
"""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, rel_l2

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.mark.parametrize("T,nlat,nlon,batch", [(31, 48, 96, 3), (63, 96, 192, 1), (21, 34, 64, 2)])
def test_bf16x3_explicit_tendency_vs_oracle_and_fp32(T, nlat, nlon, batch):
    sdc = {p: _sdc(T, nlat, nlon, 2, 2, batch, precision=p) for p in ("fp64", "fp32", "bf16x3")}
    o = _oracle(T, nlat, nlon)
    x = _states(T, batch, 171)
    f = {}
    for p, s in sdc.items():
        y = _dev(np.zeros_like(x))
        s.eval_explicit(_dev(x), y)
        f[p] = _host(y)
    ref = np.stack([o.f_explicit(x[b]) for b in range(batch)])
    e = {p: rel_l2(v, ref, T) for p, v in f.items()}
    d = rel_l2(f["bf16x3"], f["fp32"], T)
    print(f"[gpu] f_E T{T}: bf16x3 rel L2 {e['bf16x3']:.3e}, fp32 {e['fp32']:.3e}, fp64 {e['fp64']:.3e}, "
          f"bf16x3 vs fp32 {d:.3e}, bound {4 * (T + 1) * U32:.2e}", flush=True)
    assert e["fp64"] <= 1e-11
    assert e["bf16x3"] <= 1.5 * e["fp32"]
    assert e["bf16x3"] <= 4 * (T + 1) * U32
    assert e["bf16x3"] > 10 * e["fp64"]        # the FP32 operands are really in use
    assert not np.array_equal(f["bf16x3"], f["fp32"])   # and the BF16 products
    for s in sdc.values():
        s.close()


def test_bf16x3_sht_round_trip():
    """A band-limited field through sht_inverse and sht_forward (FP64 transforms in every mode:
    the precision modes change the step's contractions only) and the inverse against the FP32
    mode's: the same grid values."""
    T, nlat, nlon = 31, 48, 96
    s3 = _sdc(T, nlat, nlon, 2, 2, 1, precision="bf16x3")
    s64 = _sdc(T, nlat, nlon, 2, 2, 1)
    x = _states(T, 1, 181)
    spec = _dev(x[:, 1].copy())
    g3 = _dev(np.zeros((1, nlat, nlon)))
    g64 = _dev(np.zeros((1, nlat, nlon)))
    s3.sht_inverse(spec, g3)
    s64.sht_inverse(spec, g64)
    assert np.array_equal(_host(g3), _host(g64))
    back = _dev(np.zeros_like(x[:, 1]))
    s3.sht_forward(g3, back)
    err = np.max(np.abs(_host(back) - x[:, 1])) / np.max(np.abs(x[:, 1]))
    print(f"[gpu] bf16x3 handle SHT round trip: rel max {err:.3e}", flush=True)
    assert err <= 1e-13
    s3.close()
    s64.close()


def test_bf16x3_steps_vs_oracle_and_graph():
    """The plain-method shape (T31, M=3, K=2, dt=600 s), 10 steps, eager and graph-replayed."""
    T, nlat, nlon, M, K, dt, steps = 31, 48, 96, 3, 2, 600.0, 10
    sdc = _sdc(T, nlat, nlon, M, K, 2, precision="bf16x3")
    o = _oracle(T, nlat, nlon)
    x0 = _states(T, 2, 181)
    x, xg = _dev(x0), _dev(x0)
    for _ in range(steps):
        sdc.step(x, dt)
        sdc.step_graph(xg, dt)
    sdc.sync()
    got = _host(x)
    assert np.array_equal(got, _host(xg))
    ref = np.stack([o.step(x0[b], dt, M, K, steps=steps) for b in range(2)])
    err = rel_l2(got - x0, ref - x0, T)
    print(f"[gpu] bf16x3 {steps} steps: rel L2 of the state change {err:.3e} "
          f"(bar {2 * (T + 1) * U32 * steps:.2e})", flush=True)
    assert err <= 2 * (T + 1) * U32 * steps
    sdc.close()


@pytest.mark.parametrize("T,nlat,nlon,M,K", [(31, 48, 96, 3, 2), (63, 96, 192, 4, 4)])
def test_bf16x3_adjoint_vs_oracle_vjp_and_taped(T, nlat, nlon, M, K):
    dt = 600.0
    sdc = _sdc(T, nlat, nlon, M, K, 1, precision="bf16x3")
    o = _oracle(T, nlat, nlon)
    x = _states(T, 1, 191)
    lam = np.stack([W.random_state(T, 192)])
    lam[..., :T + 1, 1] = 0.0
    out = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), out, dt, M, K)
    got = _host(out)
    tape = sdc.new_tape()
    u = _dev(x)
    sdc.step_taped(u, dt, tape)
    gt = _dev(np.zeros_like(x))
    sdc.step_adjoint_taped(tape, _dev(lam), gt, dt)
    sdc.sync()
    assert np.array_equal(got, _host(gt))
    ref = o.step_vjp(x[0], lam[0], dt, M, K)[None]
    err = rel_l2(got - lam, ref - lam, T)
    print(f"[gpu] bf16x3 adjoint T{T} M={M} K={K}: rel L2 of the f_E part {err:.3e}", flush=True)
    assert err <= 2 * (T + 1) * U32 * M * K
    sdc.close()

"""Oracle parity of the full-size and full-length workloads, and of the non-zonal closed forms
through the GPU's explicit tendency.

* The non-zonal closed forms of the explicit tendency (Rossby-Haurwitz single-degree wave, solid-body
  advection of Phi', the Coriolis linear part with its n +- 1 couplings, cross terms with solid-body
  rotation; derived from the shallow-water equations of Section 3.2) evaluated with the GPU's
  eval_explicit: <= 1e-12 relative (max norm), the same bar the oracle meets.
* The headline step (T255 on 384 x 768, M = K = 4, dt = 120 s) with the autotuned plan: the adjoint
  step (recomputing and taped) against the oracle's autograd VJP, <= 1e-10 relative L2 (as at the
  small sizes), and in the FP32 mode on the f_E part of the adjoint, 2 (T+1) u_32 M K.
* FP32 steps at T255 against the oracle on the state change, 2 (T+1) u_32 per step (the bound
  derived in test_gpu_precision: a step adds dt-weighted tendencies, each within 2 (T+1) u_32).
* The plain-vs-compensated workload at full length (T127 jet, M = K = 3, dt = 240 s, 100 steps):
  FP64 <= 1e-11 relative L2 per field at every 10th step; FP32 error stated and held to
  2 (T+1) u_32 k on the state change.
* T511 (768 x 1536, M = K = 4, dt = 60 s): one FP64 adjoint step against the oracle's VJP.
"""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, rel_l2
from test_oracle_swe import _nonzonal_pin_errors

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


class _GpuTendency:
    """eval_explicit of the GPU library behind the oracle's f_explicit interface."""

    def __init__(self, sdc):
        self.sdc = sdc

    def f_explicit(self, st):
        x = _dev(np.asarray(st)[None])
        f = _dev(np.zeros((1,) + np.asarray(st).shape))
        self.sdc.eval_explicit(x, f)
        return _host(f)[0]


@pytest.mark.parametrize("plan", [None, (2, 2, 2, 1, 1, 1, 1)])
def test_nonzonal_closed_forms_gpu_explicit_tendency(plan):
    sdc = _sdc(31, 48, 96, 2, 2, 1)
    if plan:
        sdc.set_plan(*plan)
    errs = _nonzonal_pin_errors(_GpuTendency(sdc))
    names = ("Rossby-Haurwitz zeta", "solid-body Phi'", "Coriolis zeta", "Coriolis delta",
             "rotation cross zeta", "rotation cross delta")
    for n, e in zip(names, errs):
        print(f"[gpu] closed form {n}: rel max err {e:.3e}", flush=True)
    assert max(errs) <= 1e-12
    sdc.close()


def _lam(T, seed):
    lam = W.random_state(T, seed)[None]
    lam[..., :T + 1, 1] = 0.0
    return lam


@pytest.fixture(scope="module")
def t255():
    mb = W.WORKLOADS["t255_m4k4"].members[0]
    return mb, _oracle(mb.T, mb.nlat, mb.nlon)


def test_t255_headline_adjoint_vs_oracle_vjp(t255):
    mb, o = t255
    T, M, K, dt = mb.T, 4, 4, mb.dt
    x = W.initial_state(W.WORKLOADS["t255_m4k4"])[None]
    lam = _lam(T, 255)
    ref = o.step_vjp(x[0], lam[0], dt, M, K)[None]
    for prec in ("fp64", "fp32", "bf16x3"):
        sdc = _sdc(T, mb.nlat, mb.nlon, M, K, 1, precision=prec)
        print(f"[gpu] T255 {prec} autotuned plan {sdc.autotune(5)}", flush=True)
        g = _dev(np.zeros_like(x))
        sdc.step_adjoint(_dev(x), _dev(lam), g, dt)
        got = _host(g)
        tape = sdc.new_tape()
        u = _dev(x)
        sdc.step_taped(u, dt, tape)
        gt = _dev(np.zeros_like(x))
        sdc.step_adjoint_taped(tape, _dev(lam), gt, dt)
        got_t = _host(gt)
        sdc.sync()
        err = rel_l2(got, ref, T)
        err_fe = rel_l2(got - lam, ref - lam, T)
        print(f"[gpu] T255 M=K=4 {prec} adjoint vs oracle VJP: rel L2 {err:.3e} (f_E part "
              f"{err_fe:.3e}); taped equal: {np.array_equal(got, got_t)}", flush=True)
        assert np.array_equal(got, got_t)
        if prec == "fp64":
            assert err <= 1e-10
        else:
            assert err_fe <= 2 * (T + 1) * U32 * M * K
        sdc.close()


def test_t255_reduced_precision_steps_vs_oracle(t255):
    mb, o = t255
    T, M, K, dt, steps = mb.T, 4, 4, mb.dt, 3
    x0 = W.initial_state(W.WORKLOADS["t255_m4k4"])[None]
    ref = o.step(x0[0], dt, M, K, steps=steps)[None]
    for prec in ("fp64", "fp32", "bf16x3"):
        sdc = _sdc(T, mb.nlat, mb.nlon, M, K, 1, precision=prec)
        sdc.autotune(5)
        x = _dev(x0)
        for _ in range(steps):
            sdc.step_graph(x, dt)
        sdc.sync()
        got = _host(x)
        err = max(rel_l2(got[:, k], ref[:, k], T) for k in range(3))
        err_d = rel_l2(got - x0, ref - x0, T)
        print(f"[gpu] T255 M=K=4 {prec} {steps} graph steps vs oracle: rel L2 {err:.3e}, "
              f"of the state change {err_d:.3e}", flush=True)
        if prec == "fp64":
            assert err <= 1e-11
        else:
            assert err_d <= 2 * (T + 1) * U32 * steps
        sdc.close()


def test_t127_jet_full_run_fp64_fp32_bf16x3():
    wl = W.WORKLOADS["t127_m3k3_jet"]
    mb = wl.members[0]
    T = mb.T
    o = _oracle(T, mb.nlat, mb.nlon)
    x0 = W.initial_state(wl)[None]
    every = 10
    refs = []
    u = x0[0]
    for k in range(0, wl.steps, every):
        u = o.step(u, mb.dt, wl.M, wl.K, steps=every)
        refs.append(u[None].copy())
    for prec in ("fp64", "fp32", "bf16x3"):
        sdc = _sdc(T, mb.nlat, mb.nlon, wl.M, wl.K, 1, precision=prec)
        x = _dev(x0)
        worst, worst_d = 0.0, 0.0
        for i, ref in enumerate(refs):
            for _ in range(every):
                sdc.step_graph(x, mb.dt)
            got = _host(x)
            e = max(rel_l2(got[:, k], ref[:, k], T) for k in range(3))
            ed = rel_l2(got - x0, ref - x0, T)
            worst, worst_d = max(worst, e), max(worst_d, ed)
            if prec != "fp64":
                assert ed <= 2 * (T + 1) * U32 * (i + 1) * every
        sdc.sync()
        print(f"[gpu] T127 jet {wl.steps} steps {prec}: max over output times of the rel L2 vs the "
              f"oracle {worst:.3e} (of the state change {worst_d:.3e})", flush=True)
        if prec == "fp64":
            assert worst <= 1e-11
        sdc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_t127_reduced_precision_adjoint_vs_oracle_vjp(prec):
    wl = W.WORKLOADS["t127_adjoint"]
    mb = wl.members[0]
    T = mb.T
    o = _oracle(T, mb.nlat, mb.nlon)
    x = W.initial_state(wl)[None]
    lam = _lam(T, 127)
    ref = o.step_vjp(x[0], lam[0], mb.dt, wl.M, wl.K)[None]
    sdc = _sdc(T, mb.nlat, mb.nlon, wl.M, wl.K, 1, precision=prec)
    g = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), g, mb.dt)
    got = _host(g)
    err_fe = rel_l2(got - lam, ref - lam, T)
    print(f"[gpu] T127 M=K=3 {prec} adjoint vs oracle VJP: f_E part rel L2 {err_fe:.3e} "
          f"(bar {2 * (T + 1) * U32 * wl.M * wl.K:.2e})", flush=True)
    assert err_fe <= 2 * (T + 1) * U32 * wl.M * wl.K
    sdc.close()


def test_t511_adjoint_vs_oracle_vjp():
    """One FP64 adjoint step at T511 (768 x 1536, M = K = 4, dt = 60 s), autotuned plan (the
    regenerating Legendre variants), against the oracle's autograd VJP: <= 1e-10 relative L2."""
    wl = W.WORKLOADS["t511_m4k4"]
    mb = wl.members[0]
    T = mb.T
    o = _oracle(T, mb.nlat, mb.nlon)
    x = W.initial_state(wl)[None]
    lam = _lam(T, 511)
    sdc = _sdc(T, mb.nlat, mb.nlon, wl.M, wl.K, 1)
    print(f"[gpu] T511 autotuned plan {sdc.autotune(3)}", flush=True)
    g = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), g, mb.dt)
    got = _host(g)
    sdc.close()
    ref = o.step_vjp(x[0], lam[0], mb.dt, wl.M, wl.K)[None]
    err = rel_l2(got, ref, T)
    err_fe = rel_l2(got - lam, ref - lam, T)
    print(f"[gpu] T511 M=K=4 fp64 adjoint vs oracle VJP: rel L2 {err:.3e} (f_E part {err_fe:.3e})",
          flush=True)
    assert err <= 1e-10

"""Pins of the oracle's split with the linear Coriolis term on the implicit side (the outlook of
Section 6: changing which terms are integrated implicitly), f_I = L_g + L_c, f_E = N_a + N_r:

* L_c by the transform route equals the closed form of the linear Coriolis term (degree
  couplings n +- 1 through mu and H = (1 - mu^2) d/dmu, derived from -div(f V), curl(f V)) and
  equals the per-order matrix the solve uses (a second route: Legendre parts of one order only);
* the solve's residual u - alpha (L_g + L_c)(u) - beta vanishes through the transform route, and
  with Omega = 0 the solve is the closed-form gravity-wave solve;
* the total right-hand side is unchanged by the split; the steady balanced jet stays a fixed
  point of a dSDC step; a step converges with order K;
* planted sign slips in L_c fail the pins.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.sdc import Oracle
from oracle.sht import CT, DT, to_complex, to_real

from test_oracle_swe import T_NZ, _apply_h, _mul_mu, _nm, _to_c


def _oracles(T=T_NZ, nlat=48, nlon=96, omega=W.OMEGA):
    args = (T, nlat, nlon, W.RADIUS, W.GRAVITY, omega, W.MEAN_DEPTH)
    return Oracle(*args), Oracle(*args, coriolis_implicit=True)


def _c(st):
    return to_complex(torch.as_tensor(st, dtype=DT))


def _rel(got, want):
    got, want = np.asarray(got), np.asarray(want)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def test_coriolis_term_matches_closed_form():
    _, oc = _oracles()
    st = W.random_state(T_NZ, 51, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6))
    lc = oc.swe.coriolis_term(_c(st)).numpy()
    _, m, nn1, inv = _nm()
    z, d = _to_c(st[W.FIELD_ZETA]), _to_c(st[W.FIELD_DIV])
    beta = 2j * W.OMEGA * m / np.where(nn1 > 0, nn1, 1.0)
    a2 = W.RADIUS ** 2
    want_z = beta * z - 2 * W.OMEGA * (_mul_mu(d) + _apply_h(inv * d) / a2)
    want_d = beta * d + 2 * W.OMEGA * (_mul_mu(z) + _apply_h(inv * z) / a2)
    assert _rel(lc[W.FIELD_ZETA], want_z) <= 1e-12
    assert _rel(lc[W.FIELD_DIV], want_d) <= 1e-12
    assert np.max(np.abs(lc[W.FIELD_PHI])) == 0.0


def test_per_order_matrix_is_the_transform_route():
    _, oc = _oracles()
    st = W.random_state(T_NZ, 52, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6))
    u = _c(st)
    want = oc.swe.f_implicit(u).numpy()
    sp = oc.sphere
    got = np.zeros_like(want)
    for m, A in enumerate(oc.swe.blocks()):
        L = sp.T + 1 - m
        sl = slice(sp.off[m], sp.off[m + 1])
        got[:, sl] = (A @ u[:, sl].reshape(3 * L)).reshape(3, L).numpy()
    for f in range(3):
        assert _rel(got[f], want[f]) <= 1e-12, f


@pytest.mark.parametrize("alpha", [30.0, 450.0])
def test_solve_residual_through_transforms(alpha):
    _, oc = _oracles()
    beta = _c(W.random_state(T_NZ, 53, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6)))
    beta[..., 0, :] = beta[..., 0, :]
    x = oc.swe.solve(alpha, beta)
    res = x - alpha * oc.swe.f_implicit(x) - beta
    for f in range(3):
        assert float(res[f].abs().max()) <= 1e-12 * float(beta[f].abs().max()), f
    # m = 0 stays real, (0, 0) of zeta and delta stays 0
    assert float(x[:, :T_NZ + 1].imag.abs().max()) <= 1e-25 * float(x.abs().max())


def test_solve_without_rotation_is_the_closed_form():
    o0, oc0 = _oracles(omega=0.0)
    beta = _c(W.random_state(T_NZ, 54, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6)))
    for alpha in (60.0, 300.0):
        a = oc0.swe.solve(alpha, beta)
        b = o0.swe.solve(alpha, beta)
        assert float((a - b).abs().max()) <= 1e-13 * float(b.abs().max())


def test_split_keeps_the_right_hand_side():
    o, oc = _oracles()
    u = _c(W.random_state(T_NZ, 55, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6)))
    tot = (o.swe.f_explicit(u) + o.swe.f_implicit(u)).numpy()
    tot_c = (oc.swe.f_explicit(u) + oc.swe.f_implicit(u)).numpy()
    for f in range(3):
        assert _rel(tot_c[f], tot[f]) <= 1e-12, f
    # the nonlinear part is quadratic: f_E(2u) = 4 f_E(u)
    assert _rel(oc.swe.f_explicit(2 * u).numpy(), 4 * oc.swe.f_explicit(u).numpy()) <= 1e-12


@pytest.mark.parametrize("u0", [20.0, -35.0])
def test_balanced_jet_is_a_fixed_point(u0):
    _, oc = _oracles()
    st = W.balanced_jet(T_NZ, u0)
    u = _c(st)
    fe, fi = oc.swe.f_explicit(u), oc.swe.f_implicit(u)
    # delta: the Coriolis and gravity terms (now both implicit) balance the kinetic-energy and
    # relative-vorticity terms (explicit); every term is O(1e-11)
    assert float(fi[2].abs().max()) > 1e-11 and float(fe[2].abs().max()) > 1e-12
    assert float((fe[2] + fi[2]).abs().max()) < 1e-12 * float(fi[2].abs().max())
    scale_phi = abs(st[0]).max() * abs(u0) / W.RADIUS
    assert float((fe[0] + fi[0]).abs().max()) < 1e-13 * scale_phi
    assert float((fe[1] + fi[1]).abs().max()) < 1e-20
    out = oc.step(st, 600.0, 3, 3)
    for f in range(3):
        if np.any(st[f]):
            assert _rel(out[f], st[f]) <= 1e-13, f
        else:                           # divergence: zero up to rounding of the vorticity scale
            assert np.max(np.abs(out[f])) <= 1e-13 * np.max(np.abs(st[W.FIELD_ZETA])), f


def test_step_converges_with_order_k():
    T = 10
    _, oc = _oracles(T, 16, 32)
    st = W.random_state(T, 56, scales=(0.01 * W.PHI_BAR, 2e-5, 2e-6))
    Tend, M, K = 3600.0, 3, 3
    ref = oc.step(st, Tend / 64, M, K, steps=64)
    errs = []
    for div in (4, 8):
        s = oc.step(st, Tend / div, M, K, steps=div)
        errs.append(np.linalg.norm(s - ref) / np.linalg.norm(ref))
    slope = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert slope >= K - 0.4, (errs, slope)


@pytest.mark.parametrize("mutant", ["curl_sign", "div_sign", "f_sign", "im_sign"])
def test_planted_coriolis_slips_fail_the_pins(monkeypatch, mutant):
    """Sign slips planted in the per-order matrix or in the transform route (on the CPU) break
    the agreement of the two routes or the closed form."""
    from oracle import sht as sht_mod
    _, oc = _oracles()
    Sph = sht_mod.Sphere
    if mutant == "curl_sign":
        dc = Sph.div_curl
        monkeypatch.setattr(Sph, "div_curl", lambda self, X, Y: (lambda r: (r[0], -r[1]))(dc(self, X, Y)))
    elif mutant == "div_sign":
        dc = Sph.div_curl
        monkeypatch.setattr(Sph, "div_curl", lambda self, X, Y: (lambda r: (-r[0], r[1]))(dc(self, X, Y)))
    elif mutant == "f_sign":
        oc.swe.coriolis = -oc.swe.coriolis
    else:
        wi = Sph.winds
        monkeypatch.setattr(Sph, "winds", lambda self, z, d: wi(self, z.conj(), d.conj()))
    caught = False
    try:
        st = W.random_state(T_NZ, 51, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6))
        lc = oc.swe.coriolis_term(_c(st)).numpy()
        _, m, nn1, inv = _nm()
        z, d = _to_c(st[W.FIELD_ZETA]), _to_c(st[W.FIELD_DIV])
        beta = 2j * W.OMEGA * m / np.where(nn1 > 0, nn1, 1.0)
        a2 = W.RADIUS ** 2
        want_z = beta * z - 2 * W.OMEGA * (_mul_mu(d) + _apply_h(inv * d) / a2)
        want_d = beta * d + 2 * W.OMEGA * (_mul_mu(z) + _apply_h(inv * z) / a2)
        caught = _rel(lc[W.FIELD_ZETA], want_z) > 1e-6 or _rel(lc[W.FIELD_DIV], want_d) > 1e-6
    except AssertionError:
        caught = True
    assert caught, mutant

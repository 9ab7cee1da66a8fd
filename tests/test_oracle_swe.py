"""Pins of the oracle's shallow-water right-hand side and implicit solve (CPU)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.sdc import Oracle
from oracle.sht import to_complex


def _oracle(T=31, nlat=48, nlon=96):
    return Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)


@pytest.mark.parametrize("u0", [20.0, -35.0])
def test_balanced_zonal_flow_is_steady(u0):
    """The gradient-wind balanced jet has f_E + f_I = 0 (signs of every term, Coriolis, KE)."""
    o = _oracle()
    u = to_complex(torch.tensor(W.balanced_jet(31, u0)))
    fe = o.swe.f_explicit(u)
    fi = o.swe.f_implicit(u)
    # individual terms are O(1e-10) (delta) and O(1e-2) (flux of Phi'); the sum must vanish
    assert torch.max(torch.abs(fi[2])).item() > 1e-10
    assert torch.max(torch.abs(fe[2] + fi[2])).item() < 1e-13 * torch.max(torch.abs(fi[2])).item() * 10
    scale_phi = abs(W.balanced_jet(31, u0)[0]).max() * abs(u0) / W.RADIUS
    assert torch.max(torch.abs(fe[0] + fi[0])).item() < 1e-13 * scale_phi
    assert torch.max(torch.abs(fe[1])).item() < 1e-20


def test_jet_broken_balance_is_not_steady():
    """A jet with the wrong Phi' sign is far from steady (the steady pin is not vacuous)."""
    o = _oracle()
    st = W.balanced_jet(31, 20.0)
    st[0] *= -1
    u = to_complex(torch.tensor(st))
    r = o.swe.f_explicit(u) + o.swe.f_implicit(u)
    assert torch.max(torch.abs(r[2])).item() > 1e-10


def test_mass_and_global_modes():
    """The (0,0) tendencies vanish identically: global mass Phi'_00 is invariant."""
    o = _oracle()
    st = W.random_state(31, 5)
    st[0, 0, 0] = 123.0
    u = to_complex(torch.tensor(st))
    fe = o.swe.f_explicit(u)
    fi = o.swe.f_implicit(u)
    for f in range(3):
        assert fe[f, 0].item() == 0          # H_0^0 = 0 and n(n+1) = 0 at n = 0
        assert fi[f, 0].item() == 0
    s1 = o.step(st, 600.0, 3, 3, steps=3)
    assert abs(s1[0, 0, 0] - 123.0) <= 1e-15 * W.PHI_BAR
    assert s1[1, 0, 0] == 0.0 and s1[2, 0, 0] == 0.0


def test_solve_residual_and_special_cases():
    o = _oracle()
    beta = to_complex(torch.tensor(W.random_state(31, 6)))
    for alpha in (0.0, 37.5, 600.0):
        u = o.swe.solve(alpha, beta)
        r = u - alpha * o.swe.f_implicit(u) - beta
        for f in range(3):
            assert torch.max(torch.abs(r[f])).item() <= 1e-13 * torch.max(torch.abs(beta[f])).item() + 1e-300
    assert torch.equal(o.swe.solve(0.0, beta), beta)


def test_f_implicit_is_gravity_wave_operator():
    """A single degree-n mode of L_g oscillates with frequency sqrt(Phi_bar n(n+1))/a."""
    o = _oracle()
    n = 7
    st = np.zeros((3, W.ncoef(31), 2))
    st[0, W.coef_index(31, 3, n)] = [1.0, 0.0]
    u = to_complex(torch.tensor(st))
    LL = o.swe.f_implicit(o.swe.f_implicit(u))
    lam2 = -W.PHI_BAR * n * (n + 1) / W.RADIUS ** 2
    assert torch.max(torch.abs(LL - lam2 * u)).item() < 1e-14 * abs(lam2)


# ---------------------------------------------------------------------------------------------
# Non-zonal explicit tendencies (Section 3.2: L_c + N_a + N_r in vorticity/divergence form),
# pinned by closed forms derived from the equations themselves, independent of the transforms:
#   zeta_t  = -div((zeta + f) V),   delta_t = curl((zeta + f) V) - lap(|V|^2 / 2),
#   Phi'_t  = -div(Phi' V),         f = 2 Omega mu.
# Spectral operators used below (orthonormal Pbar, eps_n^m = sqrt((n^2 - m^2)/(4 n^2 - 1))):
#   mu Pbar_n = eps_{n+1} Pbar_{n+1} + eps_n Pbar_{n-1},
#   (1 - mu^2) dPbar_n/dmu = (n+1) eps_n Pbar_{n-1} - n eps_{n+1} Pbar_{n+1}.
# f_E is a polynomial of degree two in the state, so (f_E(u) - f_E(-u)) / 2 is exactly its
# linear part and f_E(a + b) - f_E(a - b) = 2 (linear part of b + cross terms of a and b).
# ---------------------------------------------------------------------------------------------
T_NZ = 31


def _eps(n, m):
    n = float(n)
    return math.sqrt(max(n * n - m * m, 0.0) / (4.0 * n * n - 1.0)) if n > 0 else 0.0


def _to_c(field):
    return field[:, 0] + 1j * field[:, 1]


def _mul_mu(c, T=T_NZ):
    """Coefficients of mu * f (truncated at T) for the coefficients c of f."""
    out = np.zeros_like(c)
    for m in range(T + 1):
        for n in range(m, T + 1):
            v = c[W.coef_index(T, m, n)]
            if n + 1 <= T:
                out[W.coef_index(T, m, n + 1)] += _eps(n + 1, m) * v
            if n - 1 >= m:
                out[W.coef_index(T, m, n - 1)] += _eps(n, m) * v
    return out


def _apply_h(c, T=T_NZ):
    """Coefficients of (1 - mu^2) df/dmu (truncated at T)."""
    out = np.zeros_like(c)
    for m in range(T + 1):
        for n in range(m, T + 1):
            v = c[W.coef_index(T, m, n)]
            if n + 1 <= T:
                out[W.coef_index(T, m, n + 1)] += -n * _eps(n + 1, m) * v
            if n - 1 >= m:
                out[W.coef_index(T, m, n - 1)] += (n + 1) * _eps(n, m) * v
    return out


def _nm(T=T_NZ):
    n, m = W.degree_order_arrays(T)
    nn1 = (n * (n + 1.0)).astype(float)
    inv = np.zeros_like(nn1)
    inv[n > 0] = -W.RADIUS ** 2 / nn1[n > 0]      # inverse Laplacian
    return n, m, nn1, inv


def _fe(o, st):
    return o.f_explicit(st)            # [3, ncoef, 2] real


def _close(got, want, rel=1e-12):
    scale = np.max(np.abs(want))
    assert scale > 0
    err = np.max(np.abs(got - want))
    assert err <= rel * scale, (err, scale)


def test_rossby_haurwitz_single_degree():
    """A vorticity field of one degree n (all orders m), no divergence, no Phi': the advection
    J(psi, zeta) vanishes (zeta is proportional to psi), leaving the beta term
    zeta_t,nm = 2 i Omega m / (n (n+1)) zeta_nm exactly; Phi'_t = 0."""
    o = _oracle()
    n_deg = 9
    n, m, nn1, _ = _nm()
    st = np.zeros((3, W.ncoef(T_NZ), 2))
    sel = n == n_deg
    st[W.FIELD_ZETA] = W.red_spectrum_field(T_NZ, 1e-5, 77, 1)
    st[W.FIELD_ZETA][~sel] = 0.0
    st[W.FIELD_ZETA][m == 0, 1] = 0.0
    fe = _fe(o, st)
    z = _to_c(st[W.FIELD_ZETA])
    want = 2j * W.OMEGA * m / np.where(nn1 > 0, nn1, 1.0) * z
    _close(_to_c(fe[W.FIELD_ZETA]), want)
    assert np.max(np.abs(fe[W.FIELD_PHI])) <= 1e-30


def test_solid_body_advection_of_geopotential():
    """Solid-body flow u = u0 cos(lat) (zeta of degree 1) with any band-limited Phi':
    Phi'_t = -div(Phi' V) = -i m (u0 / a) Phi'_nm exactly (non-zonal Phi')."""
    o = _oracle()
    u0 = 30.0
    _, m, _, _ = _nm()
    st = np.zeros((3, W.ncoef(T_NZ), 2))
    st[W.FIELD_ZETA] = W.balanced_jet(T_NZ, u0)[W.FIELD_ZETA]
    st[W.FIELD_PHI] = W.red_spectrum_field(T_NZ, 0.01 * W.PHI_BAR, 78, 0)
    fe = _fe(o, st)
    want = -1j * m * (u0 / W.RADIUS) * _to_c(st[W.FIELD_PHI])
    _close(_to_c(fe[W.FIELD_PHI]), want)


def test_coriolis_linear_part():
    """The linear part of f_E is the Coriolis term L_c (Phi_bar's terms sit in f_I):
    per degree, zeta_t = 2 i Omega m/(n(n+1)) zeta - 2 Omega (mu delta + H(chi)/a^2),
      delta_t = 2 i Omega m/(n(n+1)) delta + 2 Omega (mu zeta + H(psi)/a^2),  Phi'_t = 0,
    with psi, chi the inverse Laplacians of zeta, delta and H = (1-mu^2) d/dmu."""
    o = _oracle()
    _, m, nn1, inv = _nm()
    st = W.random_state(T_NZ, 41, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6))
    lin = 0.5 * (_fe(o, st) - _fe(o, -st))
    z, d = _to_c(st[W.FIELD_ZETA]), _to_c(st[W.FIELD_DIV])
    beta = 2j * W.OMEGA * m / np.where(nn1 > 0, nn1, 1.0)
    a2 = W.RADIUS ** 2
    want_z = beta * z - 2 * W.OMEGA * (_mul_mu(d) + _apply_h(inv * d) / a2)
    want_d = beta * d + 2 * W.OMEGA * (_mul_mu(z) + _apply_h(inv * z) / a2)
    _close(_to_c(lin[W.FIELD_ZETA]), want_z)
    _close(_to_c(lin[W.FIELD_DIV]), want_d)
    assert np.max(np.abs(lin[W.FIELD_PHI])) <= 1e-12 * W.PHI_BAR * 1e-5


def test_advection_by_solid_body_rotation():
    """Cross terms of solid-body flow (zeta_sb = 2 (u0/a) mu, u_sb = u0 cos(lat)) and a
    non-divergent perturbation zeta' (stream function psi'):
      zeta_t  = [2 i Omega m/(n(n+1)) - i m (u0/a) (1 - 2/(n(n+1)))] zeta'   (Rossby-Haurwitz
                 phase speed: advection by the rotation plus its own beta term),
      delta_t = L_c part + 2 (u0/a)(mu zeta' + H(psi')/a^2) - (u0/a)(H(zeta') - 2 mu zeta')
                 - (u0/a) n(n+1)/a^2 H(psi')   (curl of zeta_sb V' and zeta' V_sb, minus the
                 Laplacian of u_sb u' = -(u0/a) H(psi'); the last two cancel, as they must: a
                 solid-body rotation only shifts the frame's rotation rate by u0/a),
      Phi'_t  = -i m (u0/a) Phi'  (zero here, Phi' = 0 in both states)."""
    o = _oracle()
    u0 = 25.0
    _, m, nn1, inv = _nm()
    base = np.zeros((3, W.ncoef(T_NZ), 2))
    base[W.FIELD_ZETA] = W.balanced_jet(T_NZ, u0)[W.FIELD_ZETA]
    pert = np.zeros_like(base)
    pert[W.FIELD_ZETA] = W.red_spectrum_field(T_NZ, 1e-5, 79, 1)
    diff = 0.5 * (_fe(o, base + pert) - _fe(o, base - pert))
    zp = _to_c(pert[W.FIELD_ZETA])
    om = u0 / W.RADIUS
    a2 = W.RADIUS ** 2
    nn1s = np.where(nn1 > 0, nn1, 1.0)
    want_z = (2j * W.OMEGA * m / nn1s - 1j * m * om * (1.0 - 2.0 / nn1s)) * zp
    want_z[nn1 == 0] = 0.0
    psi = inv * zp
    coriolis_d = 2 * W.OMEGA * (_mul_mu(zp) + _apply_h(psi) / a2)
    cross_d = (2 * om * (_mul_mu(zp) + _apply_h(psi) / a2)
               - om * (_apply_h(zp) - 2 * _mul_mu(zp))
               - om * (nn1 / a2) * _apply_h(psi))
    _close(_to_c(diff[W.FIELD_ZETA]), want_z)
    _close(_to_c(diff[W.FIELD_DIV]), coriolis_d + cross_d)
    # the frame-shift identity itself: the delta cross terms are the Coriolis term of 2 u0/a
    _close(_to_c(diff[W.FIELD_DIV]), coriolis_d * (1.0 + om / W.OMEGA))
    assert np.max(np.abs(diff[W.FIELD_PHI])) <= 1e-30


def _nonzonal_pin_errors(o):
    """Relative errors of the four non-zonal closed forms above for the oracle `o`."""
    errs = []
    n, m, nn1, inv = _nm()
    a2 = W.RADIUS ** 2
    nn1s = np.where(nn1 > 0, nn1, 1.0)
    rel = lambda got, want: float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    # Rossby-Haurwitz single degree
    st = np.zeros((3, W.ncoef(T_NZ), 2))
    st[W.FIELD_ZETA] = W.red_spectrum_field(T_NZ, 1e-5, 77, 1)
    st[W.FIELD_ZETA][n != 9] = 0.0
    z = _to_c(st[W.FIELD_ZETA])
    errs.append(rel(_to_c(_fe(o, st)[W.FIELD_ZETA]), 2j * W.OMEGA * m / nn1s * z))
    # solid-body advection of Phi'
    st = np.zeros((3, W.ncoef(T_NZ), 2))
    st[W.FIELD_ZETA] = W.balanced_jet(T_NZ, 30.0)[W.FIELD_ZETA]
    st[W.FIELD_PHI] = W.red_spectrum_field(T_NZ, 0.01 * W.PHI_BAR, 78, 0)
    errs.append(rel(_to_c(_fe(o, st)[W.FIELD_PHI]), -1j * m * (30.0 / W.RADIUS) * _to_c(st[W.FIELD_PHI])))
    # Coriolis linear part
    st = W.random_state(T_NZ, 41, scales=(0.01 * W.PHI_BAR, 1e-5, 3e-6))
    lin = 0.5 * (_fe(o, st) - _fe(o, -st))
    z, d = _to_c(st[W.FIELD_ZETA]), _to_c(st[W.FIELD_DIV])
    beta = 2j * W.OMEGA * m / nn1s
    errs.append(rel(_to_c(lin[W.FIELD_ZETA]), beta * z - 2 * W.OMEGA * (_mul_mu(d) + _apply_h(inv * d) / a2)))
    errs.append(rel(_to_c(lin[W.FIELD_DIV]), beta * d + 2 * W.OMEGA * (_mul_mu(z) + _apply_h(inv * z) / a2)))
    # advection by solid-body rotation
    base = np.zeros((3, W.ncoef(T_NZ), 2))
    base[W.FIELD_ZETA] = W.balanced_jet(T_NZ, 25.0)[W.FIELD_ZETA]
    pert = np.zeros_like(base)
    pert[W.FIELD_ZETA] = W.red_spectrum_field(T_NZ, 1e-5, 79, 1)
    diff = 0.5 * (_fe(o, base + pert) - _fe(o, base - pert))
    zp = _to_c(pert[W.FIELD_ZETA])
    om = 25.0 / W.RADIUS
    wz = (2j * W.OMEGA * m / nn1s - 1j * m * om * (1.0 - 2.0 / nn1s)) * zp
    wz[nn1 == 0] = 0.0
    errs.append(rel(_to_c(diff[W.FIELD_ZETA]), wz))
    errs.append(rel(_to_c(diff[W.FIELD_DIV]),
                    2 * (W.OMEGA + om) * (_mul_mu(zp) + _apply_h(inv * zp) / a2)))
    return errs


def test_nonzonal_pins_all_hold():
    assert max(_nonzonal_pin_errors(_oracle())) <= 1e-12


@pytest.mark.parametrize("mutant", ["V_sign", "curl_sign", "div_sign", "dphi_sign", "dzeta_sign",
                                    "coriolis_sign", "psi_H_sign", "im_sign"])
def test_nonzonal_pins_catch_planted_mistakes(monkeypatch, mutant):
    """Plausible slips planted in the oracle's f_E (on the CPU) each fail a non-zonal pin, so the
    pins fix the sign of B = q V, D = Phi' V, d zeta = -div(A, B), d Phi' = -div(C, D), the curl,
    the Coriolis parameter, the H part of the winds and the i m longitude derivative; the balanced
    zonal jet alone cannot see most of them (V = 0, m = 0)."""
    from oracle import sht as sht_mod
    from oracle import swe as swe_mod
    o = _oracle()
    Sph = sht_mod.Sphere
    winds, div_curl, lsyn = Sph.winds, Sph.div_curl, Sph.legendre_synthesis
    orig_stack = torch.stack
    if mutant == "V_sign":
        monkeypatch.setattr(Sph, "winds", lambda self, z, d: (lambda UV: (UV[0], -UV[1]))(winds(self, z, d)))
    elif mutant == "curl_sign":
        monkeypatch.setattr(Sph, "div_curl", lambda self, X, Y: (lambda dc: (dc[0], -dc[1]))(div_curl(self, X, Y)))
    elif mutant == "div_sign":
        monkeypatch.setattr(Sph, "div_curl", lambda self, X, Y: (lambda dc: (-dc[0], dc[1]))(div_curl(self, X, Y)))
    elif mutant in ("dphi_sign", "dzeta_sign"):
        idx = 0 if mutant == "dphi_sign" else 1

        def stacked(ts, dim=0):
            if len(ts) == 3 and dim == -2:
                ts = list(ts)
                ts[idx] = -ts[idx]
            return orig_stack(ts, dim=dim)
        monkeypatch.setattr(swe_mod.torch, "stack", stacked)
    elif mutant == "coriolis_sign":
        o.swe.coriolis = -o.swe.coriolis
    elif mutant == "psi_H_sign":
        # H tables entering the winds with the wrong sign
        def lsyn_bad(self, c, table="P"):
            out = lsyn(self, c, table)
            return -out if table == "H" else out
        monkeypatch.setattr(Sph, "legendre_synthesis", lsyn_bad)
    elif mutant == "im_sign":
        def winds_bad(self, z, d):
            return winds(self, torch.conj(z), torch.conj(d))
        monkeypatch.setattr(Sph, "winds", winds_bad)
    errs = _nonzonal_pin_errors(o)
    assert max(errs) > 1e-6, (mutant, errs)

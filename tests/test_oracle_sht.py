"""Pins of the oracle's spherical-harmonic transforms (CPU)."""
import math

import numpy as np
import pytest
import torch
from scipy.special import lpmv

import workloads as W
from oracle.sht import Sphere, to_complex

A = W.RADIUS


def _pbar_scipy(n, m, x):
    norm = math.sqrt((2 * n + 1) / 2.0 * math.factorial(n - m) / math.factorial(n + m))
    return (-1) ** m * norm * lpmv(m, n, x)


def _direct_eval(T, c, lam, mu):
    """Brute-force f(lam, mu) = sum_{n,m} s_m Re(c_nm Pbar_n^m(mu) e^{i m lam}) at given points."""
    f = np.zeros(np.broadcast(lam, mu).shape)
    for m in range(T + 1):
        for n in range(m, T + 1):
            cc = c[W.coef_index(T, m, n)]
            s = 1.0 if m == 0 else 2.0
            f = f + s * np.real(cc * _pbar_scipy(n, m, mu) * np.exp(1j * m * lam))
    return f


def _rand_c(T, seed):
    st = W.random_state(T, seed)
    return to_complex(torch.tensor(st[0] / np.abs(st[0]).max()))


@pytest.mark.parametrize("T,nlat,nlon", [(31, 48, 96), (63, 96, 192), (20, 32, 64)])
def test_round_trip_band_limited(T, nlat, nlon):
    sp = Sphere(T, nlat, nlon, A)
    c = _rand_c(T, 1)
    c2 = sp.analysis(sp.synthesis(c))
    assert torch.max(torch.abs(c2 - c)).item() < 1e-13


def test_synthesis_against_brute_force():
    T, nlat, nlon = 3, 6, 8
    sp = Sphere(T, nlat, nlon, A)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(W.ncoef(T)) + 1j * rng.standard_normal(W.ncoef(T))
    c[:T + 1] = c[:T + 1].real
    g = sp.synthesis(torch.tensor(c)).numpy()
    lam = 2 * math.pi * np.arange(nlon) / nlon
    ref = _direct_eval(T, c, lam[None, :], sp.mu_np[:, None])
    np.testing.assert_allclose(g, ref, atol=1e-13)


def test_longitude_transform_against_rfft():
    sp = Sphere(31, 48, 96, A)
    f = W.random_grid(48, 96, 0)[0]
    F = sp.grid_to_fourier(torch.tensor(f)).numpy()            # [m, j]
    ref = np.fft.rfft(f, axis=1)[:, :32].T / 96
    np.testing.assert_allclose(F, ref, atol=1e-14)


def test_winds_closed_forms():
    T = 15
    sp = Sphere(T, 24, 48, A)
    u0 = 20.0
    jet = torch.tensor(W.balanced_jet(T, u0))
    z = to_complex(jet[1])
    d = torch.zeros_like(z)
    U, V = sp.winds(z, d)
    mu = sp.mu_np[:, None]
    np.testing.assert_allclose(U.numpy(), np.broadcast_to(u0 * (1 - mu ** 2), U.shape), atol=1e-13)
    assert np.max(np.abs(V.numpy())) < 1e-13
    # pure divergence in degree 1: chi = -a^2/2 * d10 * sqrt(3/2) mu,  V = (1-mu^2) dchi/dmu / a
    dd = np.zeros(W.ncoef(T), dtype=complex)
    d10 = 3e-6
    dd[W.coef_index(T, 0, 1)] = d10
    U, V = sp.winds(torch.zeros_like(z), torch.tensor(dd))
    np.testing.assert_allclose(V.numpy(), np.broadcast_to(-0.5 * A * d10 * math.sqrt(1.5) * (1 - mu ** 2), V.shape),
                               atol=1e-13)
    assert np.max(np.abs(U.numpy())) < 1e-13


def test_winds_against_finite_differences():
    """U = (dchi/dlam - (1-mu^2) dpsi/dmu)/a, V = (dpsi/dlam + (1-mu^2) dchi/dmu)/a by brute force."""
    T, nlat, nlon = 5, 8, 16
    sp = Sphere(T, nlat, nlon, A)
    rng = np.random.default_rng(11)
    zeta = rng.standard_normal(W.ncoef(T)) + 1j * rng.standard_normal(W.ncoef(T))
    delta = rng.standard_normal(W.ncoef(T)) + 1j * rng.standard_normal(W.ncoef(T))
    zeta[:T + 1] = zeta[:T + 1].real
    delta[:T + 1] = delta[:T + 1].real
    zeta[0] = delta[0] = 0
    U, V = sp.winds(torch.tensor(zeta), torch.tensor(delta))
    n = np.array([n for m in range(T + 1) for n in range(m, T + 1)], dtype=float)
    inv = np.where(n > 0, -A * A / np.maximum(n * (n + 1), 1), 0.0)
    psi, chi = zeta * inv, delta * inv
    lam = 2 * math.pi * np.arange(nlon) / nlon
    L, MU = np.meshgrid(lam, sp.mu_np)
    h = 1e-5

    def d_lam(c):
        return (_direct_eval(T, c, L + h, MU) - _direct_eval(T, c, L - h, MU)) / (2 * h)

    def d_mu(c):
        return (_direct_eval(T, c, L, MU + h) - _direct_eval(T, c, L, MU - h)) / (2 * h)

    Uref = (d_lam(chi) - (1 - MU ** 2) * d_mu(psi)) / A
    Vref = (d_lam(psi) + (1 - MU ** 2) * d_mu(chi)) / A
    scale = max(np.abs(Uref).max(), np.abs(Vref).max())
    np.testing.assert_allclose(U.numpy(), Uref, atol=1e-8 * scale)
    np.testing.assert_allclose(V.numpy(), Vref, atol=1e-8 * scale)


@pytest.mark.parametrize("T,nlat,nlon", [(31, 48, 96), (63, 96, 192)])
def test_vector_round_trip(T, nlat, nlon):
    sp = Sphere(T, nlat, nlon, A)
    st = W.random_state(T, 2)
    z = to_complex(torch.tensor(st[1]))
    d = to_complex(torch.tensor(st[2]))
    U, V = sp.winds(z, d)
    div, curl = sp.div_curl(U, V)
    assert torch.max(torch.abs(curl - z)).item() < 1e-13 * torch.max(torch.abs(z)).item() * 10
    assert torch.max(torch.abs(div - d)).item() < 1e-13 * torch.max(torch.abs(d)).item() * 10


def test_solid_body_advection():
    """-div(Phi' U, Phi' V) with U = u0 (1-mu^2), V = 0 equals -i m (u0/a) Phi'_nm exactly."""
    T, nlat, nlon = 31, 48, 96
    sp = Sphere(T, nlat, nlon, A)
    u0 = 35.0
    phi = _rand_c(T, 4) * 1000.0
    phig = sp.synthesis(phi)
    U = u0 * (1 - sp.mu ** 2)[:, None] * torch.ones(nlat, nlon, dtype=torch.float64)
    div, _ = sp.div_curl(phig * U, torch.zeros_like(U))
    ref = -1j * sp.m_of.to(torch.complex128) * (u0 / A) * phi
    err = torch.max(torch.abs(-div - ref)).item()
    assert err < 1e-13 * torch.max(torch.abs(ref)).item()

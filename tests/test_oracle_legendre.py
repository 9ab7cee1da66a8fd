"""Pins of the oracle's associated Legendre tables (CPU)."""
import math

import numpy as np
import pytest
from scipy.special import lpmv

from oracle import legendre, quadrature


def _pbar_scipy(n, m, x):
    # lpmv carries the Condon-Shortley phase (-1)^m; orthonormal on [-1,1]
    norm = math.sqrt((2 * n + 1) / 2.0 * math.factorial(n - m) / math.factorial(n + m))
    return (-1) ** m * norm * lpmv(m, n, x)


def test_pbar_against_scipy():
    x = np.linspace(-0.999, 0.999, 41)
    for m in range(0, 21):
        P = legendre.pbar_m(m, 20, x)
        for n in range(m, 21):
            ref = _pbar_scipy(n, m, x)
            np.testing.assert_allclose(P[n - m], ref, atol=1e-13 * max(1.0, np.max(np.abs(ref))))


@pytest.mark.parametrize("T,nlat", [(31, 48), (127, 192)])
def test_orthonormal_under_gauss_quadrature(T, nlat):
    mu, w = quadrature.gauss_legendre(nlat)
    P, _ = legendre.tables(T, mu)
    for m in (0, 1, 7, T // 2, T - 1, T):
        G = (P[m] * w) @ P[m].T
        np.testing.assert_allclose(G, np.eye(T - m + 1), atol=2e-13)


def test_h_is_meridional_derivative():
    x = np.linspace(-0.95, 0.95, 23)
    h = 1e-6
    for m in (0, 1, 3, 10):
        H = legendre.h_m(m, 24, x)
        Pp = legendre.pbar_m(m, 24, x + h)
        Pm = legendre.pbar_m(m, 24, x - h)
        fd = (1.0 - x * x) * (Pp - Pm) / (2 * h)
        np.testing.assert_allclose(H, fd, atol=5e-8)


def test_parity_symmetry():
    mu, _ = quadrature.gauss_legendre(48)
    P, H = legendre.tables(31, mu)
    for m in (0, 2, 5):
        for n in range(m, 32):
            s = (-1) ** (n + m)
            np.testing.assert_allclose(P[m][n - m][::-1], s * P[m][n - m], atol=1e-14)
            np.testing.assert_allclose(H[m][n - m][::-1], -s * H[m][n - m], atol=1e-13)

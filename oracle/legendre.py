"""Orthonormal associated Legendre functions on the Gaussian grid (oracle; test infrastructure).

Normalisation: integral_{-1}^{1} Pbar_n^m(mu)^2 dmu = 1, no Condon-Shortley phase, m >= 0.
Recurrences (standard, written from the definitions):
  Pbar_0^0 = 1/sqrt(2)
  Pbar_m^m = sqrt((2m+1)/(2m)) * sqrt(1-mu^2) * Pbar_{m-1}^{m-1}
  Pbar_n^m = (mu * Pbar_{n-1}^m - eps_{n-1}^m * Pbar_{n-2}^m) / eps_n^m,
      eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1))
and the meridional derivative used by the vector transforms
  H_n^m = (1-mu^2) dPbar_n^m/dmu = (n+1) eps_n^m Pbar_{n-1}^m - n eps_{n+1}^m Pbar_{n+1}^m.

Pins: tests/test_oracle_legendre.py (orthonormality under Gauss quadrature, scipy's lpmv after
normalisation, H against central differences of Pbar).
"""
from __future__ import annotations

import math
from typing import List

import numpy as np


def eps(n: int, m: int) -> float:
    if n <= m:
        return 0.0
    return math.sqrt((n * n - m * m) / (4.0 * n * n - 1.0))


def pbar_m(m: int, nmax: int, mu: np.ndarray) -> np.ndarray:
    """Pbar_n^m(mu) for n = m..nmax as an array [nmax-m+1, len(mu)]."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    p = np.full_like(mu, 1.0 / math.sqrt(2.0))
    for k in range(1, m + 1):
        p = p * math.sqrt((2.0 * k + 1.0) / (2.0 * k)) * s
    out = np.zeros((nmax - m + 1, mu.size))
    out[0] = p
    if nmax >= m + 1:
        out[1] = math.sqrt(2.0 * m + 3.0) * mu * p
    for n in range(m + 2, nmax + 1):
        out[n - m] = (mu * out[n - m - 1] - eps(n - 1, m) * out[n - m - 2]) / eps(n, m)
    return out


def h_m(m: int, nmax: int, mu: np.ndarray) -> np.ndarray:
    """H_n^m(mu) = (1-mu^2) dPbar_n^m/dmu for n = m..nmax, array [nmax-m+1, len(mu)]."""
    p = pbar_m(m, nmax + 1, mu)            # rows n = m..nmax+1
    out = np.zeros((nmax - m + 1, np.asarray(mu).size))
    for n in range(m, nmax + 1):
        below = p[n - m - 1] if n - 1 >= m else 0.0
        out[n - m] = (n + 1) * eps(n, m) * below - n * eps(n + 1, m) * p[n - m + 1]
    return out


def tables(T: int, mu: np.ndarray):
    """Lists P[m], H[m] of arrays [T-m+1, nlat] holding Pbar_n^m(mu_j), H_n^m(mu_j), n = m..T."""
    P: List[np.ndarray] = []
    H: List[np.ndarray] = []
    for m in range(T + 1):
        P.append(pbar_m(m, T, mu))
        H.append(h_m(m, T, mu))
    return P, H

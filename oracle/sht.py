"""Spherical-harmonic transforms written as direct sums (oracle; test infrastructure only).

Conventions (the paper relies on SHTns for this step, Section 3.2, without fixing them; the
readings are listed with the oracle's other readings in the design notes):

* Coefficients c_nm, 0 <= m <= n <= T, complex, m-major triangular storage; m = 0 real.
* Synthesis: f(lambda, mu) = sum_m s_m Re[ F_m(mu) e^{i m lambda} ],
  F_m(mu) = sum_n c_nm Pbar_n^m(mu),  s_0 = 1, s_m = 2 (m > 0).
* Analysis: F_m(mu_j) = (1/nlon) sum_i f(lambda_i, mu_j) e^{-i m lambda_i},
  c_nm = sum_j w_j Pbar_n^m(mu_j) F_m(mu_j)   (Gauss weights w_j).
* Winds U = u cos(lat), V = v cos(lat) from vorticity zeta and divergence delta through the
  streamfunction psi and velocity potential chi (psi_nm = -a^2 zeta_nm / (n(n+1)), chi alike,
  zero at n = 0):
  U_m = (1/a) sum_n [ i m chi_nm Pbar - psi_nm H ],  V_m = (1/a) sum_n [ i m psi_nm Pbar + chi_nm H ].
* Divergence and curl of a vector given as (X, Y) = (x cos(lat), y cos(lat)) on the grid:
  div_nm  = (1/a) sum_j w_j/(1-mu_j^2) [ i m X_m Pbar - Y_m H ],
  curl_nm = (1/a) sum_j w_j/(1-mu_j^2) [ i m Y_m Pbar + X_m H ].

The longitude sums are explicit DFT sums (a matrix product with e^{i m lambda}); no FFT.
Pins: tests/test_oracle_sht.py (round trip on band-limited fields, brute-force evaluation with
scipy's Legendre functions, numpy's rfft, closed-form winds, solid-body advection).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import legendre, quadrature

DT = torch.float64
CT = torch.complex128


class Sphere:
    """Gaussian grid, Legendre tables and DFT matrices for truncation T on nlat x nlon."""

    def __init__(self, T: int, nlat: int, nlon: int, radius: float, grid=None):
        """grid: optional (mu, w) replacing the Gauss-Legendre nodes and weights (used by the
        tests to measure how much a result moves when the nodes move by one ulp)."""
        if nlat < T + 1 or nlon < 2 * T + 1:
            raise ValueError("grid too small for truncation")
        self.T, self.nlat, self.nlon, self.radius = T, nlat, nlon, radius
        mu, w = quadrature.gauss_legendre(nlat) if grid is None else grid
        self.mu_np, self.w_np = mu, w
        self.mu = torch.tensor(mu, dtype=DT)
        self.w = torch.tensor(w, dtype=DT)
        P, H = legendre.tables(T, mu)
        self.P = [torch.tensor(p, dtype=DT).to(CT) for p in P]
        self.H = [torch.tensor(h, dtype=DT).to(CT) for h in H]
        self.off = [m * (2 * T + 3 - m) // 2 for m in range(T + 2)]
        lam = 2.0 * math.pi * np.arange(nlon) / nlon
        mm = np.arange(T + 1)
        self.E = torch.tensor(np.exp(1j * np.outer(mm, lam)), dtype=CT)      # [T+1, nlon]
        self.s = torch.tensor(np.where(mm == 0, 1.0, 2.0), dtype=DT)
        n_of = np.concatenate([np.arange(m, T + 1) for m in range(T + 1)])
        m_of = np.concatenate([np.full(T + 1 - m, m) for m in range(T + 1)])
        self.n_of = torch.tensor(n_of, dtype=DT)
        self.m_of = torch.tensor(m_of, dtype=DT)
        nn1 = n_of * (n_of + 1.0)
        # -a^2/(n(n+1)) (inverse Laplacian), 0 at n = 0;  n(n+1)/a^2 (minus the Laplacian)
        inv = np.zeros_like(nn1)
        inv[n_of > 0] = -radius ** 2 / nn1[n_of > 0]
        self.inv_lap = torch.tensor(inv, dtype=DT)
        self.neg_lap = torch.tensor(nn1 / radius ** 2, dtype=DT)
        self.ncoef = len(n_of)

    # ---- coefficient slices --------------------------------------------------------------
    def _slice(self, c, m):
        return c[..., self.off[m]:self.off[m + 1]]

    # ---- Legendre part ---------------------------------------------------------------------
    def legendre_synthesis(self, c, table="P"):
        """F[..., m, j] = sum_n c_nm X_n^m(mu_j) with X = Pbar or H."""
        tab = self.P if table == "P" else self.H
        return torch.stack([self._slice(c, m) @ tab[m] for m in range(self.T + 1)], dim=-2)

    def legendre_analysis(self, F, weight, table="P"):
        """c_nm = sum_j weight_j X_n^m(mu_j) F[..., m, j]."""
        tab = self.P if table == "P" else self.H
        Fw = F * weight.to(CT)
        return torch.cat([Fw[..., m, :] @ tab[m].transpose(0, 1) for m in range(self.T + 1)], dim=-1)

    # ---- longitude part --------------------------------------------------------------------
    def fourier_to_grid(self, F):
        """f[..., j, i] = sum_m s_m Re(F[..., m, j] e^{i m lambda_i})."""
        Fs = F * self.s.to(CT)[:, None]
        return torch.real(torch.matmul(Fs.transpose(-1, -2), self.E))

    def grid_to_fourier(self, f):
        """F[..., m, j] = (1/nlon) sum_i f[..., j, i] e^{-i m lambda_i}."""
        return torch.matmul(f.to(CT), torch.conj(self.E).transpose(0, 1)).transpose(-1, -2) / self.nlon

    # ---- scalar transforms -----------------------------------------------------------------
    def synthesis(self, c):
        return self.fourier_to_grid(self.legendre_synthesis(c, "P"))

    def analysis(self, f):
        return self.legendre_analysis(self.grid_to_fourier(f), self.w, "P")

    # ---- vector transforms -----------------------------------------------------------------
    def winds(self, zeta, delta):
        """Grid U = u cos(lat), V = v cos(lat) from vorticity and divergence coefficients."""
        psi = zeta * self.inv_lap.to(CT)
        chi = delta * self.inv_lap.to(CT)
        im = (1j * torch.arange(self.T + 1, dtype=DT)).to(CT)[:, None]
        Pchi = self.legendre_synthesis(chi, "P")
        Ppsi = self.legendre_synthesis(psi, "P")
        Hchi = self.legendre_synthesis(chi, "H")
        Hpsi = self.legendre_synthesis(psi, "H")
        Uf = (im * Pchi - Hpsi) / self.radius
        Vf = (im * Ppsi + Hchi) / self.radius
        return self.fourier_to_grid(Uf), self.fourier_to_grid(Vf)

    def div_curl(self, X, Y):
        """Spectral divergence and curl of the vector field (X, Y) = (x cos, y cos) on the grid."""
        Xf = self.grid_to_fourier(X)
        Yf = self.grid_to_fourier(Y)
        g = self.w / (1.0 - self.mu * self.mu) / self.radius
        im = (1j * torch.arange(self.T + 1, dtype=DT)).to(CT)[:, None]
        div = self.legendre_analysis(im * Xf, g, "P") - self.legendre_analysis(Yf, g, "H")
        curl = self.legendre_analysis(im * Yf, g, "P") + self.legendre_analysis(Xf, g, "H")
        return div, curl


def to_complex(x):
    """[..., ncoef, 2] float64 -> [..., ncoef] complex128."""
    x = torch.as_tensor(x, dtype=DT)
    return torch.view_as_complex(x.contiguous())


def to_real(c):
    """[..., ncoef] complex128 -> [..., ncoef, 2] float64."""
    return torch.view_as_real(c).contiguous()

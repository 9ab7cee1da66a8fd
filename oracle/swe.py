"""Split right-hand side of the rotating shallow-water equations (oracle; test infrastructure).

The prognostic state is (Phi', zeta, delta) in spherical-harmonic space (Section 3.2).  The
right-hand side L_g + L_c + N_a + N_r of the shallow-water system in Section 3.2 is split as the
paper does for its spectral code:

* f_I = L_g, the linear gravity-wave part, treated implicitly:
      d Phi'/dt = -Phi_bar delta,   d zeta/dt = 0,   d delta/dt = -lap(Phi') = n(n+1)/a^2 Phi'_nm
  (Phi_bar = g H is the constant mean geopotential, so only Phi' has a gradient).
* f_E = L_c + N_a + N_r, Coriolis plus nonlinear terms, treated explicitly by a transform round
  trip.  In vorticity/divergence form with q = zeta + f, f = 2 Omega mu, on the grid
      A = q U, B = q V, C = Phi' U, D = Phi' V, E = (U^2 + V^2) / (2 (1 - mu^2))
  and back in spectral space
      d zeta/dt  = -div(A, B)
      d delta/dt =  curl(A, B) - lap(E)
      d Phi'/dt  = -div(C, D)
  (the momentum equation written as -q k x V - grad(KE + Phi'), the continuity equation in flux
  form; the gravity part -Phi_bar delta and -lap(Phi') sit in f_I).
* The implicit solve of u - alpha f_I(u) = beta (Section 4.2, third required routine) is closed
  form per coefficient:  zeta = beta_zeta,
      Phi' = (beta_Phi - alpha Phi_bar beta_delta) / (1 + alpha^2 Phi_bar n(n+1)/a^2),
      delta = beta_delta + alpha n(n+1)/a^2 Phi'.

States are complex tensors [..., 3, ncoef] in the field order (Phi', zeta, delta).
Pins: tests/test_oracle_swe.py (steady balanced zonal flow, mass conservation, solve residual;
non-zonal flow: the Rossby-Haurwitz single-degree wave, solid-body advection of Phi', the
Coriolis linear part with its n +- 1 couplings, and the cross terms of a perturbation with
solid-body rotation -- each of these closed forms derived from the equations above, and each
shown to fail for planted sign slips).
"""
from __future__ import annotations

import torch

from .sht import CT, DT, Sphere

PHI, ZETA, DIV = 0, 1, 2


class SWE:
    def __init__(self, sphere: Sphere, gravity: float, omega: float, mean_depth: float):
        self.sp = sphere
        self.phi_bar = gravity * mean_depth
        self.omega = omega
        self.gravity = gravity
        self.coriolis = (2.0 * omega * sphere.mu)[:, None]          # f on the grid [nlat, 1]
        self.nf_eval = 0                                             # number of f_E evaluations

    def f_explicit(self, u):
        """f_E(u) = L_c + N_a + N_r in spectral space."""
        self.nf_eval += 1
        sp = self.sp
        zeta_g = sp.synthesis(u[..., ZETA, :])
        phi_g = sp.synthesis(u[..., PHI, :])
        U, V = sp.winds(u[..., ZETA, :], u[..., DIV, :])
        q = zeta_g + self.coriolis
        A, B = q * U, q * V
        C, D = phi_g * U, phi_g * V
        E = (U * U + V * V) / (2.0 * (1.0 - sp.mu * sp.mu))[:, None]
        div_ab, curl_ab = sp.div_curl(A, B)
        div_cd, _ = sp.div_curl(C, D)
        e_c = sp.analysis(E)
        d_zeta = -div_ab
        d_delta = curl_ab + sp.neg_lap.to(CT) * e_c
        d_phi = -div_cd
        return torch.stack([d_phi, d_zeta, d_delta], dim=-2)

    def f_implicit(self, u):
        """f_I(u) = L_g(u)."""
        nl = self.sp.neg_lap.to(CT)
        return torch.stack([-self.phi_bar * u[..., DIV, :],
                            torch.zeros_like(u[..., ZETA, :]),
                            nl * u[..., PHI, :]], dim=-2)

    def solve(self, alpha, beta):
        """The u with u - alpha f_I(u) = beta; alpha is a scalar or has shape beta.shape[:-2]."""
        a = torch.as_tensor(alpha, dtype=DT).to(CT)
        if a.dim() > 0:
            a = a[..., None]
        nl = self.sp.neg_lap.to(CT)
        bphi, bzeta, bdiv = beta[..., PHI, :], beta[..., ZETA, :], beta[..., DIV, :]
        phi = (bphi - a * self.phi_bar * bdiv) / (1.0 + a * a * self.phi_bar * nl)
        div = bdiv + a * nl * phi
        return torch.stack([phi, bzeta, div], dim=-2)

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

`SWECoriolisImplicit` is the variant the paper's outlook (Section 6) names, changing which terms
are integrated implicitly: the linear Coriolis term moves to the implicit side,
    f_I = L_g + L_c,   L_c(u) = (0, -div(f U, f V), curl(f U, f V)),
    f_E = N_a + N_r    (the products above with q = zeta instead of zeta + f),
and the solve of u - alpha f_I(u) = beta couples the degrees n +- 1 of one order m through L_c:
it is done per order m as a dense linear solve with the matrix of L_g + L_c on that order, the
L_c block formed from the per-order Legendre parts of the same definition (f is zonal, so f U
keeps the order of U).  Pins: tests/test_oracle_coriolis.py (L_c against the closed form of the
linear part of f_E and against its per-order matrix, the solve's residual through the transform
route, Omega = 0 reducing to the closed-form solve, the unchanged total right-hand side, the
steady jet as a fixed point of a step, order K, planted sign slips).
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


class SWECoriolisImplicit(SWE):
    """The shallow-water split with the linear Coriolis term on the implicit side (see the
    module docstring): f_I = L_g + L_c, f_E = N_a + N_r."""

    def __init__(self, sphere: Sphere, gravity: float, omega: float, mean_depth: float):
        super().__init__(sphere, gravity, omega, mean_depth)
        self._blocks = None

    def coriolis_term(self, u):
        """L_c(u) = (0, -div(f U, f V), curl(f U, f V)) by a transform round trip."""
        sp = self.sp
        U, V = sp.winds(u[..., ZETA, :], u[..., DIV, :])
        div, curl = sp.div_curl(self.coriolis * U, self.coriolis * V)
        return torch.stack([torch.zeros_like(div), -div, curl], dim=-2)

    def f_explicit(self, u):
        """f_E(u) = N_a + N_r: the transform round trip of SWE.f_explicit with q = zeta."""
        self.nf_eval += 1
        sp = self.sp
        zeta_g = sp.synthesis(u[..., ZETA, :])
        phi_g = sp.synthesis(u[..., PHI, :])
        U, V = sp.winds(u[..., ZETA, :], u[..., DIV, :])
        A, B = zeta_g * U, zeta_g * V
        C, D = phi_g * U, phi_g * V
        E = (U * U + V * V) / (2.0 * (1.0 - sp.mu * sp.mu))[:, None]
        div_ab, curl_ab = sp.div_curl(A, B)
        div_cd, _ = sp.div_curl(C, D)
        e_c = sp.analysis(E)
        return torch.stack([-div_cd, -div_ab, curl_ab + sp.neg_lap.to(CT) * e_c], dim=-2)

    def f_implicit(self, u):
        """f_I(u) = L_g(u) + L_c(u)."""
        return SWE.f_implicit(self, u) + self.coriolis_term(u)

    def blocks(self):
        """Per order m, the matrix of L_g + L_c acting on (Phi', zeta, delta) of that order
        (3 L x 3 L complex, L = T + 1 - m, unknowns field-major then degree).  The L_c part is the
        definition restricted to one order: winds of the order from psi, chi (Pbar and H rows of
        the order), multiplied by f at every latitude, then the order's divergence and curl by
        Gauss quadrature."""
        if self._blocks is not None:
            return self._blocks
        sp = self.sp
        a = sp.radius
        f = self.coriolis[:, 0].to(CT)                        # [nlat]
        g = (sp.w / (1.0 - sp.mu * sp.mu) / a).to(CT)           # quadrature weight of div / curl
        blocks = []
        for m in range(sp.T + 1):
            L = sp.T + 1 - m
            P, H = sp.P[m], sp.H[m]                            # [L, nlat]
            il = sp._slice(sp.inv_lap.to(CT), m)               # inverse Laplacian of the order
            nl = sp._slice(sp.neg_lap.to(CT), m)
            im = 1j * m
            # rows: unit inputs (zeta_n or delta_n); columns: latitudes
            U_z = -(il[:, None] * H) / a
            V_z = im * (il[:, None] * P) / a
            U_d = im * (il[:, None] * P) / a
            V_d = (il[:, None] * H) / a

            def div_curl(X, Y):
                Xf, Yf = X * f, Y * f
                div = (im * Xf * g) @ P.T - (Yf * g) @ H.T
                curl = (im * Yf * g) @ P.T + (Xf * g) @ H.T
                return div, curl                               # [inputs, outputs]
            dz, cz = div_curl(U_z, V_z)
            dd, cd = div_curl(U_d, V_d)
            A = torch.zeros((3 * L, 3 * L), dtype=CT)
            # L_g: d Phi' = -Phi_bar delta, d delta = n(n+1)/a^2 Phi'
            A[0:L, 2 * L:3 * L] = -self.phi_bar * torch.eye(L, dtype=CT)
            A[2 * L:3 * L, 0:L] = torch.diag(nl)
            # L_c: d zeta = -div, d delta = curl (output rows, input columns)
            A[L:2 * L, L:2 * L] = -dz.T
            A[L:2 * L, 2 * L:3 * L] = -dd.T
            A[2 * L:3 * L, L:2 * L] += cz.T
            A[2 * L:3 * L, 2 * L:3 * L] += cd.T
            blocks.append(A)
        self._blocks = blocks
        return blocks

    def solve(self, alpha, beta):
        """The u with u - alpha f_I(u) = beta (alpha a scalar): per order m a dense solve of
        (I - alpha (L_g + L_c)) x = beta restricted to the order."""
        sp = self.sp
        a = complex(float(alpha))
        out = torch.zeros_like(beta)
        for m, A in enumerate(self.blocks()):
            L = sp.T + 1 - m
            sl = slice(sp.off[m], sp.off[m + 1])
            b = beta[..., :, sl].reshape(beta.shape[:-2] + (3 * L,))
            Mx = torch.eye(3 * L, dtype=CT) - a * A
            x = torch.linalg.solve(Mx, b.unsqueeze(-1)).squeeze(-1)
            out[..., :, sl] = x.reshape(beta.shape[:-2] + (3, L))
        return out

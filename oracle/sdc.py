"""Diagonal IMEX SDC time step (oracle; test infrastructure only).

`dsdc_step` follows Algorithm 2 of the paper with the node update of Section 4.2:

    u_m^{k+1} - dt q^D_{m,m} f_I(u_m^{k+1})
        = u_n + dt sum_j q_{m,j} [f_I(u_j^k) + f_E(u_j^k)] - dt q^D_{m,m} f_I(u_m^k)

solved with the routine for u - alpha f_I(u) = beta, alpha = dt q^D_{m,m}.  The first K-1
sweeps update every node from the previous sweep's values (the loop the paper runs in
parallel); the K-th sweep updates only the last node, whose value is the new state
(tau_M = 1 for Radau-right nodes).  f_E and f_I are not evaluated at that final iterate.
MIN-SR-FLEX: q^D_{m,m} = tau_m / min(s, M) in sweep s = 1..K (readings: the sweep index in
the coefficient is the 1-based sweep count; the paper defines the coefficients for sweeps 1..M
only, and sweeps beyond M -- K > M, used by tests only -- keep tau_m / M; the initial guess is
the state at the start of the step; f_I of a new iterate is evaluated, not recovered from the
solve).

`imex_sdc_step` is the sequential IMEX SDC of Algorithm 1 (the method dSDC parallelises).

Pins: tests/test_oracle_sdc.py (steady balanced flow, IMEX Euler special case, brute-force
linear stage matrices, order of accuracy, collocation limit against the Pade approximant,
operation count 1 + (K-1) M of f_E per step, performance-model speedup 3.25 of Section 4.7;
for Algorithm 1: IMEX Euler at M = K = 1, block lower-triangular stage matrices, collocation
limit, order K).
"""
from __future__ import annotations

from typing import Callable

import numpy as np
import torch

from . import quadrature
from .imex2 import imex2_step
from .sht import CT, DT, Sphere, to_complex, to_real
from .swe import SWE, SWECoriolisImplicit


def dsdc_step(u_n, dt: float, tau: np.ndarray, Q: np.ndarray, K: int,
              f_explicit: Callable, f_implicit: Callable, solve: Callable,
              qdelta: Callable = quadrature.min_sr_flex):
    """One dSDC step u_n -> u_{n+1} for any state tensor u_n (node axis added in front);
    qdelta(tau, s) is the diagonal of Q_Delta in sweep s (MIN-SR-FLEX unless given)."""
    M = len(tau)
    E0 = f_explicit(u_n)
    I0 = f_implicit(u_n)
    shape = (M,) + tuple(u_n.shape)
    U = u_n.unsqueeze(0).expand(shape)
    E = E0.unsqueeze(0).expand(shape)
    I = I0.unsqueeze(0).expand(shape)
    Qt = torch.as_tensor(Q, dtype=DT).to(u_n.dtype)
    flat = (M, -1)

    def rhs(m_rows, alpha):
        # u_n + dt sum_j q_{m,j}(I_j + E_j) - alpha_m I_m for the node rows m_rows
        F = (I + E).reshape(flat)
        quad = (Qt[m_rows] @ F).reshape((len(m_rows),) + tuple(u_n.shape))
        a = torch.as_tensor(alpha, dtype=DT).to(u_n.dtype).reshape((-1,) + (1,) * u_n.dim())
        return u_n.unsqueeze(0) + dt * quad - a * I[m_rows]

    all_m = list(range(M))
    for s in range(1, K):
        alpha = dt * qdelta(tau, s)
        beta = rhs(all_m, alpha)
        U = torch.stack([solve(float(alpha[m]), beta[m]) for m in all_m])
        E = torch.stack([f_explicit(U[m]) for m in all_m])
        I = torch.stack([f_implicit(U[m]) for m in all_m])
    alpha_last = dt * qdelta(tau, K)[M - 1]
    beta = rhs([M - 1], np.array([alpha_last]))
    return solve(float(alpha_last), beta[0])


def imex_sdc_step(u_n, dt: float, tau: np.ndarray, Q: np.ndarray, K: int,
                  f_explicit: Callable, f_implicit: Callable, solve: Callable):
    """One sequential IMEX SDC step (Algorithm 1 with the node update of Section 4.1): K sweeps,
    each updating the nodes one after another; node m of sweep k+1 uses the new values of nodes
    j < m through forward-Euler differences of f_E (weights dtau_{j+1}) and backward-Euler
    differences of f_I (weights dtau_j, j <= m; the j = m term is the implicit solve), with
    dtau_1 = tau_1 and dtau_j = tau_j - tau_{j-1}.  The initial guess is u_n at every node;
    f_E of the final iterate is not evaluated."""
    M = len(tau)
    dtau = np.diff(np.concatenate([[0.0], tau]))
    E0, I0 = f_explicit(u_n), f_implicit(u_n)
    U, E, I = [u_n] * M, [E0] * M, [I0] * M
    for k in range(K):
        Un, En, In = [], [], []
        for m in range(M):
            beta = u_n + dt * sum(Q[m, j] * (I[j] + E[j]) for j in range(M))
            for j in range(m):
                beta = beta + dt * dtau[j + 1] * (En[j] - E[j]) + dt * dtau[j] * (In[j] - I[j])
            beta = beta - dt * dtau[m] * I[m]
            um = solve(float(dt * dtau[m]), beta)
            Un.append(um)
            if k == K - 1 and m == M - 1:
                break
            En.append(f_explicit(um))
            In.append(f_implicit(um))
        U, E, I = Un, En, In
    return U[M - 1]


class Oracle:
    """Sphere + shallow-water right-hand side + collocation coefficients for one truncation."""

    def __init__(self, T: int, nlat: int, nlon: int, radius: float, gravity: float,
                 omega: float, mean_depth: float, grid=None, qdelta: str = "flex",
                 coriolis_implicit: bool = False):
        """coriolis_implicit: the split with the linear Coriolis term on the implicit side
        (SWECoriolisImplicit) instead of the paper's spectral-code split."""
        self.sphere = Sphere(T, nlat, nlon, radius, grid)
        self.qdelta = quadrature.QDELTA[qdelta]
        cls = SWECoriolisImplicit if coriolis_implicit else SWE
        self.swe = cls(self.sphere, gravity, omega, mean_depth)
        self.gravity = gravity
        self.mean_depth = mean_depth

    def coefficients(self, M: int):
        tau = quadrature.radau_right_nodes(M)
        return tau, quadrature.collocation_matrix(tau)

    # complex-state API
    def step_c(self, u, dt: float, M: int, K: int):
        tau, Q = self.coefficients(M)
        return dsdc_step(u, dt, tau, Q, K, self.swe.f_explicit, self.swe.f_implicit, self.swe.solve,
                         self.qdelta)

    def seq_step_c(self, u, dt: float, M: int, K: int):
        tau, Q = self.coefficients(M)
        return imex_sdc_step(u, dt, tau, Q, K, self.swe.f_explicit, self.swe.f_implicit, self.swe.solve)

    def seq_step(self, state, dt: float, M: int, K: int, steps: int = 1):
        """Sequential IMEX SDC steps (Algorithm 1) on a real state [3, ncoef, 2]."""
        u = to_complex(torch.as_tensor(np.asarray(state), dtype=DT))
        for _ in range(steps):
            u = self.seq_step_c(u, dt, M, K)
        return to_real(u).numpy()

    # real-state API: [3, ncoef, 2] float64 arrays / tensors (the device layout)
    def step(self, state, dt: float, M: int, K: int, steps: int = 1):
        u = to_complex(torch.as_tensor(np.asarray(state), dtype=DT))
        for _ in range(steps):
            u = self.step_c(u, dt, M, K)
        return to_real(u).numpy()

    def imex2_c(self, u, dt: float):
        return imex2_step(u, dt, self.swe.f_explicit, self.swe.f_implicit, self.swe.solve)

    def imex2(self, state, dt: float, steps: int = 1):
        """IMEX-o2 steps (the paper's reference integrator) on a real state [3, ncoef, 2]."""
        u = to_complex(torch.as_tensor(np.asarray(state), dtype=DT))
        for _ in range(steps):
            u = self.imex2_c(u, dt)
        return to_real(u).numpy()

    def f_explicit(self, state):
        return to_real(self.swe.f_explicit(to_complex(torch.as_tensor(np.asarray(state))))).numpy()

    def f_implicit(self, state):
        return to_real(self.swe.f_implicit(to_complex(torch.as_tensor(np.asarray(state))))).numpy()

    def solve(self, alpha, beta):
        return to_real(self.swe.solve(alpha, to_complex(torch.as_tensor(np.asarray(beta))))).numpy()

    def synthesis(self, spec):
        """spec [..., ncoef, 2] -> grid [..., nlat, nlon]."""
        return self.sphere.synthesis(to_complex(torch.as_tensor(np.asarray(spec)))).numpy()

    def analysis(self, grid):
        """grid [..., nlat, nlon] -> spec [..., ncoef, 2]."""
        return to_real(self.sphere.analysis(torch.as_tensor(np.asarray(grid), dtype=DT))).numpy()

    # loss of the gradient workload: 0.5 * sum over grid points of (h - h_target)^2,
    # h = (Phi_bar + Phi')/g, h_target = H + Phi'_target/g.
    def loss_c(self, u, phi_target_c):
        diff = self.sphere.synthesis(u[..., 0, :] - phi_target_c) / self.gravity
        return 0.5 * torch.sum(diff * diff)

    def loss_and_grad(self, state, phi_target, dt: float, M: int, K: int, steps: int):
        """Loss after `steps` dSDC steps and its gradient w.r.t. the real state (torch autograd).

        The gradient is taken w.r.t. (Re, Im) of every coefficient; the imaginary parts of
        m = 0 coefficients are held at zero (their gradient entries are set to 0).
        """
        x = torch.tensor(np.asarray(state), dtype=DT, requires_grad=True)
        u = to_complex(x)
        for _ in range(steps):
            u = self.step_c(u, dt, M, K)
        tgt = to_complex(torch.as_tensor(np.asarray(phi_target), dtype=DT))
        L = self.loss_c(u, tgt)
        L.backward()
        g = x.grad.detach().clone()
        g[..., 0:self.sphere.T + 1, 1] = 0.0
        return float(L.detach()), g.numpy()

    def step_vjp(self, state, lam, dt: float, M: int, K: int):
        """(d u_{n+1}/d u_n)^T lam by torch autograd through one oracle step (real inner product
        over (Re, Im) of every coefficient; m = 0 imaginary entries of the result set to 0)."""
        x = torch.tensor(np.asarray(state), dtype=DT, requires_grad=True)
        y = to_real(self.step_c(to_complex(x), dt, M, K))
        (g,) = torch.autograd.grad(y, x, torch.as_tensor(np.asarray(lam), dtype=DT))
        g = g.detach().clone()
        g[..., 0:self.sphere.T + 1, 1] = 0.0
        return g.numpy()

    def synthesis_vjp(self, grid):
        """Transpose of the scalar synthesis (grid [..., nlat, nlon] -> spec [..., ncoef, 2])."""
        c0 = torch.zeros(np.asarray(grid).shape[:-2] + (self.sphere.ncoef, 2), dtype=DT, requires_grad=True)
        y = self.sphere.synthesis(to_complex(c0))
        (g,) = torch.autograd.grad(y, c0, torch.as_tensor(np.asarray(grid), dtype=DT))
        g = g.detach().clone()
        g[..., 0:self.sphere.T + 1, 1] = 0.0
        return g.numpy()

    def loss(self, state, phi_target, dt: float, M: int, K: int, steps: int) -> float:
        with torch.no_grad():
            u = to_complex(torch.as_tensor(np.asarray(state), dtype=DT))
            for _ in range(steps):
                u = self.step_c(u, dt, M, K)
            tgt = to_complex(torch.as_tensor(np.asarray(phi_target), dtype=DT))
            return float(self.loss_c(u, tgt))


def make_oracle(member, radius, gravity, omega, mean_depth) -> Oracle:
    return Oracle(member.T, member.nlat, member.nlon, radius, gravity, omega, mean_depth)

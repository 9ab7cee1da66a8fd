"""IMEX-o2, the paper's reference integrator for the spectral shallow-water model (oracle; test
infrastructure only).

Section 3.2 describes it as a second-order Strang splitting that integrates the gravity part L_g
(here f_I) with Crank-Nicolson and the rest, L_c + N_a + N_r (here f_E), with Heun's explicit
second-order Runge-Kutta method.  The paper does not say which part takes the half steps.
Reading: two Crank-Nicolson half steps of f_I around one full Heun step of f_E (two f_E
evaluations per step):

    u*      = C(dt/2) u_n,   C(h) = (I - h/2 f_I)^{-1} (I + h/2 f_I)
    k1      = f_E(u*),   k2 = f_E(u* + dt k1)
    u**     = u* + dt/2 (k1 + k2)
    u_{n+1} = C(dt/2) u**

C(h) u is formed with the solver routine of Section 4.2: solve(h/2, u + h/2 f_I(u)).

Pins: tests/test_oracle_imex2.py (order two against matrix exponentials of linear systems,
for the whole split step and for each part alone; the phase of the Crank-Nicolson half steps on a
gravity-wave mode against the closed form 2 atan(omega h / 2) per step of length h and their
exact energy conservation; second-order convergence on the shallow-water jet against a
high-order dSDC reference).
"""
from __future__ import annotations

from typing import Callable


def imex2_step(u_n, dt: float, f_explicit: Callable, f_implicit: Callable, solve: Callable):
    """One IMEX-o2 step u_n -> u_{n+1}."""
    a = 0.25 * dt                              # C(dt/2): h/2 = dt/4

    def cn_half(u):
        return solve(a, u + a * f_implicit(u))

    us = cn_half(u_n)
    k1 = f_explicit(us)
    k2 = f_explicit(us + dt * k1)
    return cn_half(us + 0.5 * dt * (k1 + k2))

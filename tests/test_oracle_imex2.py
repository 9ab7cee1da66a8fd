"""Pins of the oracle's IMEX-o2 step (CPU): the paper's reference integrator of Section 3.2."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle.imex2 import imex2_step
from oracle.sdc import Oracle


def _linear_problem(seed, d=4, implicit=True, explicit=True):
    rng = np.random.default_rng(seed)
    # implicit part: a stiff-ish oscillator block (skew) plus mild damping; explicit: O(1) mixing
    S = rng.standard_normal((d, d))
    A = 3.0 * (S - S.T) - 0.2 * np.eye(d) if implicit else np.zeros((d, d))
    B = 0.5 * rng.standard_normal((d, d)) if explicit else np.zeros((d, d))
    I = np.eye(d)
    return (A, B, lambda u: B @ u, lambda u: A @ u,
            lambda a, beta: np.linalg.solve(I - a * A, beta))


def _global_error(prob, u0, t_end, n):
    A, B, fe, fi, solve = prob
    u = u0.copy()
    for _ in range(n):
        u = imex2_step(u, t_end / n, fe, fi, solve)
    exact = scipy.linalg.expm((A + B) * t_end) @ u0
    return np.linalg.norm(u - exact) / np.linalg.norm(exact)


@pytest.mark.parametrize("implicit,explicit", [(True, True), (True, False), (False, True)])
def test_second_order_against_matrix_exponential(implicit, explicit):
    """u' = (A + B) u: the split step, Crank-Nicolson alone and Heun alone converge to
    expm((A + B) t) u0 with order two (error ratio 4 per halving of dt)."""
    prob = _linear_problem(3, implicit=implicit, explicit=explicit)
    u0 = np.random.default_rng(4).standard_normal(4)
    errs = [_global_error(prob, u0, 1.0, n) for n in (40, 80, 160)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)
    assert errs[2] < 1e-2


def test_crank_nicolson_phase_and_energy_on_a_gravity_wave():
    """With f_E = 0 a step is two Crank-Nicolson half steps of the gravity-wave operator.  For one
    coefficient (n, m) the pair (Phi', delta) rotates in the energy coordinates (sqrt(c_n) Phi',
    sqrt(Phi_bar) delta) with frequency omega = sqrt(Phi_bar c_n); Crank-Nicolson over a step of
    length h rotates by exactly 2 atan(omega h / 2) and keeps the radius (the energy)."""
    import torch
    T = 21
    o = Oracle(T, 34, 64, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    sw = o.swe
    n_of, m_of = W.degree_order_arrays(T)
    k = int(np.flatnonzero((n_of == 7) & (m_of == 3))[0])
    u = torch.zeros((3, len(n_of)), dtype=torch.complex128)
    u[0, k] = 1.0e3 + 0.0j           # Phi'
    u[2, k] = 2.0e-6 + 0.0j          # delta
    c = 7 * 8 / W.RADIUS ** 2
    pb = W.GRAVITY * W.MEAN_DEPTH
    om = math.sqrt(pb * c)
    dt = 3600.0
    out = imex2_step(u, dt, lambda x: torch.zeros_like(x), sw.f_implicit, sw.solve)

    def polar(v):
        x, y = math.sqrt(c) * v[0, k].real, math.sqrt(pb) * v[2, k].real
        return math.hypot(x, y), math.atan2(y, x)

    r0, a0 = polar(u)
    r1, a1 = polar(out)
    assert abs(r1 - r0) <= 1e-14 * r0
    assert abs((a1 - a0) - 4.0 * math.atan(om * dt / 4.0)) <= 1e-13
    others = out.clone()
    others[:, k] = 0
    assert float(others.abs().max()) == 0.0


def test_second_order_on_the_shallow_water_jet():
    """T15 jet plus a random perturbation over two hours: IMEX-o2 converges with order two to a
    dSDC(M=4, K=4) reference at a 16 times smaller step."""
    T, nlat, nlon = 15, 24, 48
    o = Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    st = W.random_state(T, 0) + W.balanced_jet(T, 20.0)
    t_end = 7200.0
    ref = o.step(st, t_end / 256, 4, 4, steps=256)
    errs = []
    for n in (16, 32, 64):
        s = o.imex2(st, t_end / n, steps=n)
        errs.append(np.linalg.norm(s - ref) / np.linalg.norm(ref))
    slopes = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert all(1.8 < sl < 2.2 for sl in slopes), (errs, slopes)

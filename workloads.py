"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds only input data: the workload table (truncations, grids, node and sweep
counts, step sizes) and seeded random spectral fields.  It contains none of the method's
arithmetic (no transform, no tendency, no time step), so both sides of a parity test can use
it without sharing code.

State layout (used by every caller): a float64 array of shape [batch, 3, ncoef, 2] holding the
spherical-harmonic coefficients of the three prognostic fields in the order
(geopotential perturbation Phi', vorticity zeta, divergence delta) -- the state vector of the
vorticity/divergence formulation in Section 3.2 of the paper.  The last axis is (Re, Im).
Coefficients are stored m-major and triangular: index(m, n) = m*(2T+3-m)/2 + (n-m) for
0 <= m <= n <= T.  Coefficients with m = 0 are real (Im = 0).

Synthetic fields stand in for the paper's Galewsky test case (Section 5.1), whose analytic
constants are not reproduced here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Physical constants used for every workload (Earth-like values; the paper does not list them).
RADIUS = 6.371e6        # a [m]
GRAVITY = 9.81          # g [m/s^2]
OMEGA = 7.292e-5        # Omega [1/s]
MEAN_DEPTH = 1.0e4      # H [m]; mean geopotential Phi_bar = g*H
PHI_BAR = GRAVITY * MEAN_DEPTH

FIELD_PHI, FIELD_ZETA, FIELD_DIV = 0, 1, 2
SEED_ROOT = 2403


def ncoef(T: int) -> int:
    return (T + 1) * (T + 2) // 2


def coef_index(T: int, m: int, n: int) -> int:
    return m * (2 * T + 3 - m) // 2 + (n - m)


def degree_order_arrays(T: int):
    """Arrays (n, m) of length ncoef(T) in storage order."""
    ns, ms = [], []
    for m in range(T + 1):
        for n in range(m, T + 1):
            ns.append(n)
            ms.append(m)
    return np.asarray(ns, dtype=np.int64), np.asarray(ms, dtype=np.int64)


@dataclasses.dataclass(frozen=True)
class Member:
    """One ensemble member: a truncation with its Gaussian grid and step size."""
    T: int
    nlat: int
    nlon: int
    dt: float


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    members: List[Member]
    M: int
    K: int
    steps: int
    zeta_rms: float = 1.0e-5          # area-weighted RMS of the vorticity [1/s]
    phi_rms_frac: float = 0.01        # RMS of Phi' as a fraction of Phi_bar
    jet_u0: float = 0.0               # amplitude of the balanced zonal jet [m/s] (0 = none)

    @property
    def T(self) -> int:
        return self.members[0].T


def _grid(T: int) -> Member:
    nlon = 3 * (T + 1)
    return Member(T=T, nlat=nlon // 2, nlon=nlon, dt=0.0)


def _m(T: int, dt: float) -> Member:
    g = _grid(T)
    return Member(T=T, nlat=g.nlat, nlon=g.nlon, dt=dt)


WORKLOADS = {
    # T31 on 48x96, M=3 Radau-right nodes, K=2 sweeps, dt=600 s, 10 steps.
    "t31_m3k2": Workload("t31_m3k2", [_m(31, 600.0)], M=3, K=2, steps=10),
    # T127 on 192x384, M=3, K=3, dt=240 s, 100 steps, n^-3 spectrum plus a 20 m/s jet.
    "t127_m3k3_jet": Workload("t127_m3k3_jet", [_m(127, 240.0)], M=3, K=3, steps=100, jet_u0=20.0),
    # 32 members of mixed truncation, M=4, K=3, 50 steps.
    "mixed32_m4k3": Workload("mixed32_m4k3",
                             [_m(63, 480.0)] * 16 + [_m(127, 240.0)] * 12 + [_m(255, 120.0)] * 4,
                             M=4, K=3, steps=50),
    # Gradient of a grid loss after 20 steps at T127, M=3, K=3.
    "t127_adjoint": Workload("t127_adjoint", [_m(127, 240.0)], M=3, K=3, steps=20),
    # T511 on 768x1536, M=4, K=4, dt=60 s, 200 steps, vorticity amplitude 2e-5.
    "t511_m4k4": Workload("t511_m4k4", [_m(511, 60.0)], M=4, K=4, steps=200, zeta_rms=2.0e-5),
    # T255 on 384x768, M=4 nodes, K=M sweeps (the paper's choice), dt=120 s, 50 steps.
    "t255_m4k4": Workload("t255_m4k4", [_m(255, 120.0)], M=4, K=4, steps=50),
}


def _rng(member: int, field_id: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, member, field_id]))


def red_spectrum_field(T: int, rms: float, member: int, field_id: int) -> np.ndarray:
    """Seeded coefficients [ncoef, 2] with per-coefficient variance proportional to n^-3.

    n = 0 is zero.  For m = 0 only the real part is drawn; for m > 0 the real and imaginary
    parts each carry half of the variance.  The field is rescaled so that its area-weighted
    RMS on the sphere equals `rms`; for orthonormal Legendre functions that RMS is
    sqrt(0.5 * sum_m s_m |c_nm|^2) with s_0 = 1, s_m = 2 (Parseval).
    """
    n, m = degree_order_arrays(T)
    z = _rng(member, field_id).standard_normal((ncoef(T), 2))
    sigma = np.zeros(ncoef(T))
    pos = n >= 1
    sigma[pos] = n[pos].astype(np.float64) ** -1.5
    c = np.zeros((ncoef(T), 2))
    zonal = m == 0
    c[zonal, 0] = sigma[zonal] * z[zonal, 0]
    c[~zonal, 0] = sigma[~zonal] * z[~zonal, 0] / math.sqrt(2.0)
    c[~zonal, 1] = sigma[~zonal] * z[~zonal, 1] / math.sqrt(2.0)
    s = np.where(m == 0, 1.0, 2.0)
    cur = math.sqrt(0.5 * float(np.sum(s * (c[:, 0] ** 2 + c[:, 1] ** 2))))
    if cur > 0:
        c *= rms / cur
    return c


def balanced_jet(T: int, u0: float) -> np.ndarray:
    """Coefficients [3, ncoef, 2] of the steady zonal flow u = u0*cos(lat), v = 0.

    Vorticity 2*u0*mu/a lies in degree 1: zeta_{1,0} = 2*u0/(a*sqrt(3/2)).  Gradient-wind
    balance (f + u*tan(lat)/a)*u = -(1/a) dPhi/dlat gives, with zero global mean,
    Phi' = -(a*Omega*u0 + u0^2/2)(mu^2 - 1/3), which is degree 2:
    Phi'_{2,0} = -(a*Omega*u0 + u0^2/2) * (2/3) / sqrt(5/2).
    (Orthonormal P_1^0 = sqrt(3/2) mu and P_2^0 = sqrt(5/2)(3 mu^2 - 1)/2.)
    """
    out = np.zeros((3, ncoef(T), 2))
    if T >= 1:
        out[FIELD_ZETA, coef_index(T, 0, 1), 0] = 2.0 * u0 / (RADIUS * math.sqrt(1.5))
    if T >= 2:
        out[FIELD_PHI, coef_index(T, 0, 2), 0] = (-(RADIUS * OMEGA * u0 + 0.5 * u0 * u0)
                                                  * (2.0 / 3.0) / math.sqrt(2.5))
    return out


def initial_state(wl: Workload, member: int = 0, T: Optional[int] = None) -> np.ndarray:
    """Initial state [3, ncoef, 2] of one member of a workload."""
    T = wl.members[member].T if T is None else T
    st = np.zeros((3, ncoef(T), 2))
    st[FIELD_ZETA] = red_spectrum_field(T, wl.zeta_rms, member, FIELD_ZETA)
    st[FIELD_PHI] = red_spectrum_field(T, wl.phi_rms_frac * PHI_BAR, member, FIELD_PHI)
    # divergence starts at zero
    if wl.jet_u0 != 0.0:
        st += balanced_jet(T, wl.jet_u0)
    return st


def loss_target_phi(T: int, member: int = 0, rms_frac: float = 0.01) -> np.ndarray:
    """Seeded Phi' coefficients [ncoef, 2] of the loss target h_target = H + Phi'_tgt/g."""
    return red_spectrum_field(T, rms_frac * PHI_BAR, member, 7)


def random_state(T: int, seed: int, scales=(PHI_BAR * 0.01, 1e-5, 1e-6)) -> np.ndarray:
    """Generic seeded state [3, ncoef, 2] for unit tests (n^-3 spectra in every field)."""
    st = np.zeros((3, ncoef(T), 2))
    for f in range(3):
        st[f] = red_spectrum_field(T, scales[f], 1000 + seed, f)
    return st


def random_grid(nlat: int, nlon: int, seed: int, count: int = 1) -> np.ndarray:
    """Seeded white-noise grid fields [count, nlat, nlon] (not band-limited)."""
    return _rng(5000 + seed, 0).standard_normal((count, nlat, nlon))


def random_directions(shape, seed: int, count: int) -> np.ndarray:
    """Seeded Gaussian directions [count, *shape] for finite-difference checks."""
    return _rng(9000 + seed, 0).standard_normal((count,) + tuple(shape))

"""How far the FP64 oracle itself moves when its Gauss nodes move by one ulp: the floor under any
FP64 parity bar at large truncations (the weights near the poles, and the divergence tendency
with its n(n+1) factor, amplify a one-ulp node change to ~1e-11 .. 1e-10 relative)."""
import numpy as np

import workloads as W
from oracle import quadrature
from oracle.sdc import Oracle


def grid_one_ulp(nlat, seed):
    """Gauss nodes moved by one ulp each (seeded directions, mirror-symmetric), weights recomputed
    by the oracle's own formula."""
    mu, _ = quadrature.gauss_legendre(nlat)
    h = nlat // 2
    s = np.random.default_rng(seed).choice([-1.0, 1.0], size=h)
    mun = np.nextafter(mu[:h], mu[:h] + s)
    mu2 = np.concatenate([mun, -mun[::-1]])
    return mu2, quadrature.gauss_weights(nlat, mu2)


def oracle_one_ulp(T, nlat, nlon, seed=1, coriolis_implicit=False):
    return Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH, grid_one_ulp(nlat, seed),
                  coriolis_implicit=coriolis_implicit)

"""Quadrature and collocation coefficients (oracle; test infrastructure only).

* Gaussian latitudes: the roots of the Legendre polynomial P_nlat, found by Newton's method in
  FP64, ordered north to south, with Gauss weights.  (The spherical-harmonic transform of
  Section 3.2 integrates over Gauss latitudes.)
* Radau-right nodes on [0, 1] (Section 4.2: the last node coincides with the end of the step):
  the roots of P_M(2t-1) - P_{M-1}(2t-1).
* Collocation matrix Q (Section 4.1): q_{m,j} = integral from 0 to tau_m of the j-th Lagrange
  polynomial on the nodes.
* MIN-SR-FLEX diagonal coefficients (Section 4.2): q^Delta_{m,m} = tau_m / s in the s-th sweep
  (s counted from 1; sweeps beyond M reuse s = M).

Pins: tests/test_oracle_quadrature.py (library Gauss rule, exact moments, textbook Radau IIA
closed forms, exactness of Q on monomials, stiff-limit nilpotency of MIN-SR-FLEX).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def _legendre_and_derivative(n: int, x: np.ndarray):
    """P_n(x) and P_n'(x) by the three-term recurrence (k+1)P_{k+1} = (2k+1)x P_k - k P_{k-1}."""
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return p1, dp


def gauss_legendre(nlat: int):
    """Gauss-Legendre nodes mu (descending: north to south) and weights w, sum(w) = 2."""
    j = np.arange(nlat, dtype=np.float64)
    x = np.cos(math.pi * (j + 0.75) / (nlat + 0.5))
    for _ in range(100):
        p, dp = _legendre_and_derivative(nlat, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    # one more Newton step at convergence so that the weights use the polished nodes
    p, dp = _legendre_and_derivative(nlat, x)
    x = x - p / dp
    return x, gauss_weights(nlat, x)


def gauss_weights(nlat: int, x: np.ndarray) -> np.ndarray:
    """Gauss-Legendre weights w = 2 / ((1 - x^2) P_nlat'(x)^2) at the nodes x."""
    _, dp = _legendre_and_derivative(nlat, x)
    return 2.0 / ((1.0 - x * x) * dp * dp)


def radau_right_nodes(M: int) -> np.ndarray:
    """Radau-right collocation nodes tau_1 < ... < tau_M = 1 on [0, 1]."""
    if M == 1:
        return np.array([1.0])
    c = np.zeros(M + 1)
    c[M] = 1.0
    c[M - 1] = -1.0          # P_M - P_{M-1} in the Legendre basis
    x = np.sort(np.real(npleg.legroots(c)))
    dc = npleg.legder(c)
    for _ in range(5):       # polish the roots with Newton's method
        x = x - npleg.legval(x, c) / npleg.legval(x, dc)
    x[-1] = 1.0
    return 0.5 * (x + 1.0)


def collocation_matrix(tau: np.ndarray) -> np.ndarray:
    """Q[m, j] = integral_0^{tau_m} l_j(s) ds with l_j the Lagrange polynomials on tau."""
    M = len(tau)
    Q = np.zeros((M, M))
    for j in range(M):
        others = np.delete(tau, j)
        coef = nppoly.polyfromroots(others) / np.prod(tau[j] - others)
        integ = nppoly.polyint(coef)
        for m in range(M):
            Q[m, j] = nppoly.polyval(tau[m], integ) - nppoly.polyval(0.0, integ)
    return Q


def min_sr_flex(tau: np.ndarray, sweep: int) -> np.ndarray:
    """Diagonal of Q_Delta in sweep `sweep` (1-based): tau_m / min(sweep, M)."""
    M = len(tau)
    return tau / float(min(sweep, M))


def min_sr_ns(tau: np.ndarray, sweep: int) -> np.ndarray:
    """MIN-SR-NS, the sweep-independent diagonal of the same family (a variant beside the paper's
    MIN-SR-FLEX; the sweep argument is ignored): tau_m / M, for which Q - Q_Delta is nilpotent
    (the non-stiff limit of the iteration matrix vanishes after M sweeps)."""
    return tau / float(len(tau))


def ie_par(tau: np.ndarray, sweep: int) -> np.ndarray:
    """Parallel implicit Euler: q_mm = tau_m in every sweep (the sweep argument is ignored), i.e.
    each node's implicit correction is an implicit Euler step from t_n to its own node; one of
    the nonzero diagonals the node update of Section 4.2 admits, and MIN-SR-FLEX's first sweep."""
    return np.array(tau, dtype=float)


QDELTA = {"flex": min_sr_flex, "ns": min_sr_ns, "iepar": ie_par}

"""Pins of the oracle's quadrature and collocation coefficients (CPU)."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import quadrature as q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("nlat", [6, 24, 48, 96, 192, 384, 768])
def test_gauss_against_library_and_moments(nlat):
    mu, w = q.gauss_legendre(nlat)
    assert np.all(np.diff(mu) < 0), "nodes must run north to south"
    x, wl = leggauss(nlat)
    np.testing.assert_allclose(mu, x[::-1], atol=2e-15, rtol=0)
    # numpy's weights carry ~1e-11 relative error near the poles; ours are checked tighter below
    np.testing.assert_allclose(w, wl[::-1], rtol=2e-9, atol=0)
    assert abs(w.sum() - 2.0) < 1e-13
    # exact for polynomials of degree <= 2 nlat - 1 (checked on low and top monomials)
    for p in list(range(0, 12)) + [2 * nlat - 2, 2 * nlat - 1]:
        exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert abs(np.sum(w * mu ** p) - exact) < 1e-13


@pytest.mark.parametrize("nlat", [48, 192, 768])
def test_gauss_against_multiprecision(nlat):
    """Nodes and weights against 40-digit Newton iterates (mpmath) on P_nlat."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    mu, w = q.gauss_legendre(nlat)
    for j in [0, 1, nlat // 3, nlat // 2 - 1]:
        t = mp.mpf(mu[j])
        for _ in range(6):
            p0, p1 = mp.mpf(1), t
            for k in range(1, nlat):
                p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
            dp = nlat * (t * p1 - p0) / (t * t - 1)
            t = t - p1 / dp
        wt = 2 / ((1 - t * t) * dp * dp)
        assert abs(float(t) - mu[j]) <= 1.2e-16
        # a 1-ulp node error moves a polar weight by ~1/(1-mu) ulps: 1e-11 relative at nlat = 768
        assert abs(float((wt - w[j]) / wt)) < 2e-11


def _golden_radau():
    rows = {}
    with open(os.path.join(GOLDEN, "radau_iia.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows[(int(parts[0]), parts[1])] = np.array([float(v) for v in parts[2:]])
    return rows


def test_radau_textbook_closed_forms():
    g = _golden_radau()
    for M in (2, 3):
        tau = q.radau_right_nodes(M)
        np.testing.assert_allclose(tau, g[(M, "nodes")], atol=1e-15, rtol=0)
        Q = q.collocation_matrix(tau)
        np.testing.assert_allclose(Q[-1], g[(M, "weights")], atol=2e-15, rtol=0)
    assert q.radau_right_nodes(1)[0] == 1.0


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6])
def test_collocation_matrix_exact_on_polynomials(M):
    tau = q.radau_right_nodes(M)
    assert tau[-1] == 1.0 and np.all(np.diff(tau) > 0) and tau[0] > 0
    Q = q.collocation_matrix(tau)
    np.testing.assert_allclose(Q.sum(axis=1), tau, atol=1e-14 if M <= 4 else 1e-13)
    for p in range(M):
        np.testing.assert_allclose(Q @ tau ** p, tau ** (p + 1) / (p + 1), atol=1e-14)
    # the last row is a Radau quadrature on [0,1]: exact to degree 2M-2
    for p in range(2 * M - 1):
        assert abs(Q[-1] @ tau ** p - 1.0 / (p + 1)) < (1e-14 if M <= 4 else 1e-13)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_min_sr_flex_stiff_limit_nilpotent(M):
    """Stiff limit of the sweep error propagator: prod_s (I - QDelta_s^{-1} Q) = 0 for s = 1..M."""
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    prod = np.eye(M)
    for s in range(1, M + 1):
        d = q.min_sr_flex(tau, s)
        prod = (np.eye(M) - np.diag(1.0 / d) @ Q) @ prod
    assert np.max(np.abs(prod)) < 1e-12
    # one sweep short of M does not annihilate it (the pin would pass for a wrong sweep index)
    prod = np.eye(M)
    for s in range(1, M):
        d = q.min_sr_flex(tau, s)
        prod = (np.eye(M) - np.diag(1.0 / d) @ Q) @ prod
    assert np.max(np.abs(prod)) > 1e-3


def test_min_sr_flex_values():
    tau = q.radau_right_nodes(4)
    np.testing.assert_allclose(q.min_sr_flex(tau, 1), tau)
    np.testing.assert_allclose(q.min_sr_flex(tau, 3), tau / 3)
    np.testing.assert_allclose(q.min_sr_flex(tau, 9), tau / 4)   # beyond M: reuse s = M
    assert math.isclose(q.min_sr_flex(tau, 2)[-1], 0.5)


@pytest.mark.parametrize("M", [2, 3, 4, 5, 6])
def test_min_sr_ns_makes_q_minus_qdelta_nilpotent(M):
    """MIN-SR-NS: (Q - diag(tau / M))^M = 0 (the non-stiff limit of the sweep iteration matrix
    vanishes after M sweeps), and no smaller power does for M >= 2."""
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    A = Q - np.diag(q.min_sr_ns(tau, 1))
    assert np.abs(np.linalg.matrix_power(A, M)).max() < 1e-13
    assert np.abs(np.linalg.matrix_power(A, M - 1)).max() > 1e-6
    np.testing.assert_array_equal(q.min_sr_ns(tau, 1), q.min_sr_ns(tau, 7))


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
def test_parallel_implicit_euler_diagonal(M):
    """q_mm = tau_m (implicit Euler from t_n to each node) in every sweep; it is MIN-SR-FLEX's
    first sweep, and for M = 1 (tau = 1) all three diagonals coincide with the implicit Euler step."""
    tau = q.radau_right_nodes(M)
    for s in (1, 2, 7):
        np.testing.assert_array_equal(q.ie_par(tau, s), tau)
    np.testing.assert_array_equal(q.ie_par(tau, 3), q.min_sr_flex(tau, 1))
    if M == 1:
        assert q.ie_par(tau, 5)[0] == q.min_sr_ns(tau, 5)[0] == q.min_sr_flex(tau, 5)[0] == 1.0

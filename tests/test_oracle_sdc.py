"""Pins of the oracle's dSDC step (CPU)."""
import math
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import quadrature as q
from oracle.sdc import Oracle, dsdc_step
from oracle.sht import to_complex, to_real

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oracle(T=31, nlat=48, nlon=96):
    return Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)


@pytest.mark.parametrize("M,K", [(3, 2), (4, 4)])
def test_steady_flow_step_is_identity(M, K):
    o = _oracle()
    st = W.balanced_jet(31, 20.0)
    s1 = o.step(st, 900.0, M, K, steps=2)
    for f in range(3):
        scale = np.abs(st[f]).max()
        if scale:
            assert np.abs(s1[f] - st[f]).max() < 1e-13 * scale
        else:
            # delta starts at 0; the cancelling terms dt*f_I, dt*f_E are ~5e-7 per step here
            assert np.abs(s1[f]).max() < 1e-13 * 5e-7


@pytest.mark.parametrize("M", [1, 3])
def test_single_sweep_is_imex_euler(M):
    """K = 1 (any Radau-right M, since tau_M = 1 and the last row of Q sums to 1):
    u1 - dt f_I(u1) = u0 + dt f_E(u0)."""
    o = _oracle()
    st = W.initial_state(W.WORKLOADS["t31_m3k2"])
    dt = 600.0
    u0 = to_complex(torch.tensor(st))
    u1 = to_complex(torch.tensor(o.step(st, dt, M, 1)))
    fi1, fe0 = dt * o.swe.f_implicit(u1), dt * o.swe.f_explicit(u0)
    r = u1 - fi1 - u0 - fe0
    for f in range(3):
        scale = max(torch.max(torch.abs(x[f])).item() for x in (u0, u1, fi1, fe0))
        assert torch.max(torch.abs(r[f])).item() <= 1e-13 * scale


@pytest.mark.parametrize("qd", ["flex", "ns", "iepar"])
@pytest.mark.parametrize("M,K", [(2, 2), (3, 3), (4, 4), (3, 5)])
def test_linear_mode_against_stage_matrices(M, K, qd):
    """With f_E = 0 one (n,m) mode evolves by the product of the sweep matrices built from
    Q, QDelta and the 3x3 gravity-wave operator (Kronecker form of the node update)."""
    qfun = q.QDELTA[qd]
    T = 7
    o = _oracle(T, 12, 24)
    n, m = 5, 2
    c = n * (n + 1) / W.RADIUS ** 2
    L = np.array([[0.0, 0.0, -W.PHI_BAR], [0.0, 0.0, 0.0], [c, 0.0, 0.0]])
    u_mode = np.array([3.0 + 1.0j, 2e-6 - 1e-6j, 1e-6 + 4e-7j])
    st = np.zeros((3, W.ncoef(T)), dtype=complex)
    st[:, W.coef_index(T, m, n)] = u_mode
    dt = 700.0
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    out = dsdc_step(torch.tensor(st), dt, tau, Q, K,
                    lambda u: torch.zeros_like(u), o.swe.f_implicit, o.swe.solve, qfun).numpy()
    # brute force with Kronecker products
    I3 = np.eye(3)
    X = np.kron(np.ones(M), u_mode)
    one_un = np.kron(np.ones(M), u_mode)
    for s in range(1, K):
        a = dt * qfun(tau, s)
        D = np.eye(3 * M) - np.kron(np.diag(a), L)
        R = one_un + (dt * np.kron(Q, L) - np.kron(np.diag(a), L)) @ X
        X = np.linalg.solve(D, R)
    aM = dt * qfun(tau, K)[-1]
    rhs = u_mode + dt * np.kron(Q[-1], L) @ X - aM * L @ X[3 * (M - 1):]
    ref = np.linalg.solve(I3 - aM * L, rhs)
    got = out[:, W.coef_index(T, m, n)]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)
    mask = np.ones(W.ncoef(T), bool)
    mask[W.coef_index(T, m, n)] = False
    assert np.all(out[:, mask] == 0)


def _pade(k, l, z):
    P = sum(math.factorial(k + l - j) * math.factorial(k) /
            (math.factorial(k + l) * math.factorial(j) * math.factorial(k - j)) * z ** j for j in range(k + 1))
    Qd = sum(math.factorial(k + l - j) * math.factorial(l) /
             (math.factorial(k + l) * math.factorial(j) * math.factorial(l - j)) * (-z) ** j for j in range(l + 1))
    return P / Qd


@pytest.mark.parametrize("M", [2, 3, 4])
def test_collocation_limit_is_radau_iia(M):
    """Many sweeps on u' = lI u + lE u converge to the M-stage Radau IIA solution, whose stability
    function is the (M-1, M) Pade approximant of exp (textbook)."""
    lI, lE, dt = -1.0, 0.6j, 1.0
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    u0 = torch.tensor([1.0 + 0.0j], dtype=torch.complex128)
    out = dsdc_step(u0, dt, tau, Q, 80, lambda u: lE * u, lambda u: lI * u,
                    lambda a, b: b / (1.0 - a * lI)).numpy()[0]
    ref = _pade(M - 1, M, (lI + lE) * dt)
    assert abs(out - ref) < 1e-12
    assert abs(out - np.exp((lI + lE) * dt)) > 1e-7          # not just the exact exponential


def test_order_of_accuracy():
    """Order in dt on a smooth nonlinear flow: slope >= K - 0.3 (min(K, 2M-1) = K here)."""
    T, nlat, nlon = 15, 24, 48
    o = _oracle(T, nlat, nlon)
    st = W.random_state(T, 0) + W.balanced_jet(T, 20.0)
    Tend = 7200.0
    for (M, K) in [(3, 2), (3, 3), (4, 4)]:
        ref = o.step(st, Tend / 128, M, K, steps=128)
        errs = []
        for div in (16, 32):
            s = o.step(st, Tend / div, M, K, steps=div)
            errs.append(np.linalg.norm(s[1] - ref[1]) / np.linalg.norm(ref[1]))
        slope = math.log(errs[0] / errs[1]) / math.log(2.0)
        assert slope >= K - 0.3, (M, K, errs, slope)


def _read_perf_golden():
    rows = []
    with open(os.path.join(GOLDEN, "perf_model_speedup.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                M, r, S, digits = line.split()
                rows.append((int(M), float(r), float(S), int(digits)))
    return rows


def test_operation_counts_reproduce_performance_model():
    """The oracle's f_E and solve counts per step give the printed model speedups (Section 4.7)."""
    o = _oracle(7, 12, 24)
    st = W.random_state(7, 1)
    for M, r, S_printed, digits in _read_perf_golden():
        K = M
        nsolve = [0]
        solve = o.swe.solve

        def counting_solve(a, b):
            nsolve[0] += 1
            return solve(a, b)
        tau = q.radau_right_nodes(M)
        Q = q.collocation_matrix(tau)
        before = o.swe.nf_eval
        dsdc_step(to_complex(torch.tensor(st)), 100.0, tau, Q, K, o.swe.f_explicit, o.swe.f_implicit,
                  counting_solve)
        n_fe = o.swe.nf_eval - before
        assert n_fe == 1 + (K - 1) * M
        assert nsolve[0] == (K - 1) * M + 1
        # serial cost: every f_E and solve in sequence plus the extra explicit cost r(c_E+c_S)
        # per node update; parallel cost: one node update per sweep.  Units c_E + c_S = 1.
        node_updates = nsolve[0] - 1
        sweeps = K - 1
        c_seq = 1.0 + node_updates * (1.0 + r)
        c_par = 1.0 + sweeps * (1.0 + r)
        assert round(c_seq / c_par, digits) == S_printed


# ---------------------------------------------------------------- sequential IMEX SDC (Algorithm 1)
from oracle.sdc import imex_sdc_step  # noqa: E402


def _seq_matrices(tau):
    """Lower-triangular sweep matrices of Algorithm 1: implicit (backward Euler) Q_I[m][j] =
    dtau_j for j <= m, explicit (forward Euler) Q_E[m][j] = dtau_{j+1} for j < m (0-based)."""
    M = len(tau)
    dtau = np.diff(np.concatenate([[0.0], tau]))
    QI = np.zeros((M, M))
    QE = np.zeros((M, M))
    for m in range(M):
        for j in range(m + 1):
            QI[m, j] = dtau[j]
        for j in range(m):
            QE[m, j] = dtau[j + 1]
    return QI, QE


def test_seq_single_node_single_sweep_is_imex_euler():
    o = _oracle()
    st = W.initial_state(W.WORKLOADS["t31_m3k2"])
    dt = 600.0
    u0 = to_complex(torch.tensor(st))
    tau, Q = o.coefficients(1)
    u1 = imex_sdc_step(u0, dt, tau, Q, 1, o.swe.f_explicit, o.swe.f_implicit, o.swe.solve)
    fi1, fe0 = dt * o.swe.f_implicit(u1), dt * o.swe.f_explicit(u0)
    r = u1 - fi1 - u0 - fe0
    for f in range(3):
        scale = max(torch.max(torch.abs(x[f])).item() for x in (u0, u1, fi1, fe0))
        assert torch.max(torch.abs(r[f])).item() <= 1e-13 * scale


@pytest.mark.parametrize("M,K", [(2, 2), (3, 3), (4, 2), (3, 6)])
def test_seq_scalar_against_preconditioned_iteration(M, K):
    """u' = lI u + lE u: K sweeps of Algorithm 1 equal K steps of the matrix iteration
    (I - dt lI Q_I - dt lE Q_E) X+ = u_n + dt (lI (Q - Q_I) + lE (Q - Q_E)) X from X = u_n."""
    lI, lE, dt = -2.0 + 0.5j, 0.3j, 0.7
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    QI, QE = _seq_matrices(tau)
    u0 = 1.0 + 0.25j
    out = imex_sdc_step(u0, dt, tau, Q, K, lambda u: lE * u, lambda u: lI * u,
                        lambda a, b: b / (1.0 - a * lI))
    X = np.full(M, u0, dtype=complex)
    A = np.eye(M) - dt * lI * QI - dt * lE * QE
    B = dt * (lI * (Q - QI) + lE * (Q - QE))
    for _ in range(K):
        X = np.linalg.solve(A, u0 + B @ X)
    assert abs(out - X[-1]) <= 1e-14 * abs(X[-1])


@pytest.mark.parametrize("M", [2, 3, 4])
def test_seq_collocation_limit_is_radau_iia(M):
    lI, lE, dt = -1.0, 0.6j, 1.0
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    out = imex_sdc_step(1.0 + 0.0j, dt, tau, Q, 40, lambda u: lE * u, lambda u: lI * u,
                        lambda a, b: b / (1.0 - a * lI))
    assert abs(out - _pade(M - 1, M, (lI + lE) * dt)) < 1e-12


def test_seq_linear_mode_against_stage_matrices():
    """f_E = 0, one (n, m) mode of the gravity-wave operator: Kronecker form with Q_I."""
    T, M, K = 7, 3, 3
    o = _oracle(T, 12, 24)
    n, m = 5, 2
    c = n * (n + 1) / W.RADIUS ** 2
    L = np.array([[0.0, 0.0, -W.PHI_BAR], [0.0, 0.0, 0.0], [c, 0.0, 0.0]])
    u_mode = np.array([3.0 + 1.0j, 2e-6 - 1e-6j, 1e-6 + 4e-7j])
    st = np.zeros((3, W.ncoef(T)), dtype=complex)
    st[:, W.coef_index(T, m, n)] = u_mode
    dt = 700.0
    tau = q.radau_right_nodes(M)
    Q = q.collocation_matrix(tau)
    QI, _ = _seq_matrices(tau)
    out = imex_sdc_step(torch.tensor(st), dt, tau, Q, K, lambda u: torch.zeros_like(u),
                        o.swe.f_implicit, o.swe.solve).numpy()
    X = np.kron(np.ones(M), u_mode)
    A = np.eye(3 * M) - dt * np.kron(QI, L)
    B = dt * np.kron(Q - QI, L)
    for _ in range(K):
        X = np.linalg.solve(A, np.kron(np.ones(M), u_mode) + B @ X)
    np.testing.assert_allclose(out[:, W.coef_index(T, m, n)], X[3 * (M - 1):], rtol=1e-12, atol=0)


def test_seq_order_of_accuracy():
    """Order K (K <= 2M - 1) on the smooth nonlinear flow of test_order_of_accuracy."""
    T, nlat, nlon = 15, 24, 48
    o = _oracle(T, nlat, nlon)
    st = W.random_state(T, 0) + W.balanced_jet(T, 20.0)
    Tend = 7200.0
    u0 = to_complex(torch.tensor(st))
    for (M, K) in [(3, 2), (3, 3)]:
        ref = o.step(st, Tend / 128, 4, 4, steps=128)
        errs = []
        for div in (16, 32):
            u = u0
            for _ in range(div):
                u = o.seq_step_c(u, Tend / div, M, K)
            s = to_real(u).numpy()
            errs.append(np.linalg.norm(s[1] - ref[1]) / np.linalg.norm(ref[1]))
        slope = math.log(errs[0] / errs[1]) / math.log(2.0)
        assert slope >= K - 0.3, (M, K, errs, slope)

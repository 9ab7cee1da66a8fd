"""Pin of the oracle's reference gradient: central finite differences in seeded directions (CPU)."""
import numpy as np

import workloads as W
from oracle.sdc import Oracle


def _directions(x, T, count, seed):
    """Seeded directions with each field block scaled to that field's norm in x; m=0 Im = 0."""
    v = W.random_directions(x.shape, seed, count)
    v[..., :T + 1, 1] = 0.0
    for f in range(3):
        nx = np.linalg.norm(x[f])
        v[:, f] *= nx / np.linalg.norm(v[:, f], axis=(1, 2))[:, None, None]
    return v


def test_gradient_matches_central_differences():
    T, nlat, nlon = 15, 24, 48
    o = Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    x = W.random_state(T, 3) + W.balanced_jet(T, 20.0)
    tgt = W.loss_target_phi(T)
    dt, M, K, steps = 240.0, 3, 3, 3
    L0, g = o.loss_and_grad(x, tgt, dt, M, K, steps)
    assert L0 > 0
    eps = 1e-6
    for v in _directions(x, T, 8, 0):
        fd = (o.loss(x + eps * v, tgt, dt, M, K, steps) - o.loss(x - eps * v, tgt, dt, M, K, steps)) / (2 * eps)
        ad = float(np.sum(g * v))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_step_vjp_dot_product_with_finite_differences():
    """<J v, lam> (central differences of the oracle step) = <v, J^T lam> (autograd VJP)."""
    T, nlat, nlon = 15, 24, 48
    o = Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    x = W.random_state(T, 4) + W.balanced_jet(T, 15.0)
    lam = W.random_state(T, 5)
    lam[..., :T + 1, 1] = 0.0
    dt, M, K = 600.0, 3, 3
    g = o.step_vjp(x, lam, dt, M, K)
    eps = 1e-6
    for v in _directions(x, T, 3, 1):
        jv = (o.step(x + eps * v, dt, M, K) - o.step(x - eps * v, dt, M, K)) / (2 * eps)
        lhs = float(np.sum(jv * lam))
        rhs = float(np.sum(v * g))
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)


def test_synthesis_vjp_is_transpose():
    """<S c, g> = <c, S^T g> with S the scalar synthesis (m = 0 imaginary parts excluded)."""
    T, nlat, nlon = 15, 24, 48
    o = Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    c = W.random_state(T, 6)[0] / 100.0
    c[:T + 1, 1] = 0.0
    gr = W.random_grid(nlat, nlon, 7)[0]
    lhs = float(np.sum(o.synthesis(c) * gr))
    rhs = float(np.sum(c * o.synthesis_vjp(gr)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)

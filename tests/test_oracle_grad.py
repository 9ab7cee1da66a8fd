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

"""Pins of the oracle's shallow-water right-hand side and implicit solve (CPU)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.sdc import Oracle
from oracle.sht import to_complex


def _oracle(T=31, nlat=48, nlon=96):
    return Oracle(T, nlat, nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)


@pytest.mark.parametrize("u0", [20.0, -35.0])
def test_balanced_zonal_flow_is_steady(u0):
    """The gradient-wind balanced jet has f_E + f_I = 0 (signs of every term, Coriolis, KE)."""
    o = _oracle()
    u = to_complex(torch.tensor(W.balanced_jet(31, u0)))
    fe = o.swe.f_explicit(u)
    fi = o.swe.f_implicit(u)
    # individual terms are O(1e-10) (delta) and O(1e-2) (flux of Phi'); the sum must vanish
    assert torch.max(torch.abs(fi[2])).item() > 1e-10
    assert torch.max(torch.abs(fe[2] + fi[2])).item() < 1e-13 * torch.max(torch.abs(fi[2])).item() * 10
    scale_phi = abs(W.balanced_jet(31, u0)[0]).max() * abs(u0) / W.RADIUS
    assert torch.max(torch.abs(fe[0] + fi[0])).item() < 1e-13 * scale_phi
    assert torch.max(torch.abs(fe[1])).item() < 1e-20


def test_jet_broken_balance_is_not_steady():
    """A jet with the wrong Phi' sign is far from steady (the steady pin is not vacuous)."""
    o = _oracle()
    st = W.balanced_jet(31, 20.0)
    st[0] *= -1
    u = to_complex(torch.tensor(st))
    r = o.swe.f_explicit(u) + o.swe.f_implicit(u)
    assert torch.max(torch.abs(r[2])).item() > 1e-10


def test_mass_and_global_modes():
    """The (0,0) tendencies vanish identically: global mass Phi'_00 is invariant."""
    o = _oracle()
    st = W.random_state(31, 5)
    st[0, 0, 0] = 123.0
    u = to_complex(torch.tensor(st))
    fe = o.swe.f_explicit(u)
    fi = o.swe.f_implicit(u)
    for f in range(3):
        assert fe[f, 0].item() == 0          # H_0^0 = 0 and n(n+1) = 0 at n = 0
        assert fi[f, 0].item() == 0
    s1 = o.step(st, 600.0, 3, 3, steps=3)
    assert abs(s1[0, 0, 0] - 123.0) <= 1e-15 * W.PHI_BAR
    assert s1[1, 0, 0] == 0.0 and s1[2, 0, 0] == 0.0


def test_solve_residual_and_special_cases():
    o = _oracle()
    beta = to_complex(torch.tensor(W.random_state(31, 6)))
    for alpha in (0.0, 37.5, 600.0):
        u = o.swe.solve(alpha, beta)
        r = u - alpha * o.swe.f_implicit(u) - beta
        for f in range(3):
            assert torch.max(torch.abs(r[f])).item() <= 1e-13 * torch.max(torch.abs(beta[f])).item() + 1e-300
    assert torch.equal(o.swe.solve(0.0, beta), beta)


def test_f_implicit_is_gravity_wave_operator():
    """A single degree-n mode of L_g oscillates with frequency sqrt(Phi_bar n(n+1))/a."""
    o = _oracle()
    n = 7
    st = np.zeros((3, W.ncoef(31), 2))
    st[0, W.coef_index(31, 3, n)] = [1.0, 0.0]
    u = to_complex(torch.tensor(st))
    LL = o.swe.f_implicit(o.swe.f_implicit(u))
    lam2 = -W.PHI_BAR * n * (n + 1) / W.RADIUS ** 2
    assert torch.max(torch.abs(LL - lam2 * u)).item() < 1e-14 * abs(lam2)

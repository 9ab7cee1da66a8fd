"""Edge cases of the supported grid range, through the C ABI.

* The smallest grids the library accepts (nlon = 16, 24 or 32; one to eight latitude pairs; T down
  to 1: FFTs of one or two butterflies per stage, 16-latitude tiles that are almost all padding,
  orders with a single row per parity) against the oracle: f_E <= 1e-12 relative L2, steps
  <= 1e-11, the adjoint step <= 1e-10 against the oracle's VJP, graph replays bitwise equal to
  eager steps.
* The largest truncation the library accepts (T = 1023 on 1024 x 2048, 4.3 GB of FP64 tables),
  where the oracle's direct sums are out of reach, by properties that hold at any size: the
  spectral round trip of a band-limited field (<= 1e-11 relative L2), the balanced jet a fixed
  point of a step (<= 1e-12 of the field scale), and the Rossby-Haurwitz closed form of the
  explicit tendency (zeta_t = 2 i Omega m / (n (n+1)) zeta_nm, Phi'_t = 0; <= 1e-11 relative, the
  max norm) at degree 300: this grid is the linear one (nlat = T + 1, nlon = 2 T + 2), which
  resolves the quadratic products of a degree-n field exactly only while their degree 2n + 1 plus
  the analysis degree stays within the Gauss rule's 2 nlat - 1 and their orders 2n stay below
  nlon - T (n <= 511); past that the flux terms alias and the closed form holds only up to the
  aliasing error, as it would in any transform method.
"""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,nlat,nlon", [(1, 2, 16), (2, 4, 16), (5, 6, 16), (7, 8, 24), (11, 12, 24),
                                         (15, 16, 32)])
def test_smallest_grids_match_oracle(T, nlat, nlon):
    M, K, dt, batch = 2, 3, 600.0, 2
    sdc = _sdc(T, nlat, nlon, M, K, batch)
    o = _oracle(T, nlat, nlon)
    x0 = _states(T, batch, 961, jet=False)
    f = _dev(np.zeros_like(x0))
    sdc.eval_explicit(_dev(x0), f)
    ref_f = np.stack([o.f_explicit(x0[b]) for b in range(batch)])
    ef = rel_l2(_host(f), ref_f, T)
    x, xg = _dev(x0), _dev(x0)
    for _ in range(2):
        sdc.step(x, dt)
        sdc.step_graph(xg, dt)
    sdc.sync()
    got = _host(x)
    assert np.array_equal(got, _host(xg))
    ref = np.stack([o.step(x0[b], dt, M, K, steps=2) for b in range(batch)])
    es = max(rel_l2(got[:, k], ref[:, k], T) for k in range(3))
    lam = np.stack([W.random_state(T, 962 + b) for b in range(batch)])
    lam[..., :T + 1, 1] = 0.0
    g = _dev(np.zeros_like(x0))
    sdc.step_adjoint(_dev(x0), _dev(lam), g, dt)
    ref_g = np.stack([o.step_vjp(x0[b], lam[b], dt, M, K) for b in range(batch)])
    ea = rel_l2(_host(g), ref_g, T)
    print(f"[gpu] T{T} {nlat}x{nlon}: f_E {ef:.3e}, 2 steps {es:.3e}, adjoint {ea:.3e}", flush=True)
    assert ef <= 1e-12
    assert es <= 1e-11
    assert ea <= 1e-10
    sdc.close()


def test_maximum_truncation_properties():
    T, nlat, nlon = 1023, 1024, 2048
    sdc = _sdc(T, nlat, nlon, 2, 2, 1)
    # spectral round trip of a band-limited field
    spec = W.random_state(T, 971)[W.FIELD_ZETA][None].copy()
    grid = _dev(np.zeros((1, nlat, nlon)))
    sdc.sht_inverse(_dev(spec), grid)
    back = _dev(np.zeros_like(spec))
    sdc.sht_forward(grid, back)
    e_rt = rel_l2(_host(back), spec, T)
    # the balanced jet is a fixed point of a step
    jet = W.balanced_jet(T, 20.0)[None]
    xj = _dev(jet)
    sdc.step(xj, 60.0)
    sdc.sync()
    jh = _host(xj)
    e_jet = max(float(np.max(np.abs(jh[0, f] - jet[0, f])) /
                      np.max(np.abs(jet[0, W.FIELD_ZETA if f == W.FIELD_DIV else f]))) for f in range(3))
    # Rossby-Haurwitz: one degree of vorticity, no divergence, no Phi'
    n, m = W.degree_order_arrays(T)
    n_deg = 300
    st = np.zeros((1, 3, W.ncoef(T), 2))
    z = W.red_spectrum_field(T, 1e-5, 973, 1)
    z[n != n_deg] = 0.0
    z[m == 0, 1] = 0.0
    st[0, W.FIELD_ZETA] = z
    f = _dev(np.zeros_like(st))
    sdc.eval_explicit(_dev(st), f)
    fh = _host(f)[0]
    zc = z[:, 0] + 1j * z[:, 1]
    want = 2j * W.OMEGA * m / (n_deg * (n_deg + 1.0)) * zc
    got = fh[W.FIELD_ZETA, :, 0] + 1j * fh[W.FIELD_ZETA, :, 1]
    e_rh = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    e_phi = float(np.max(np.abs(fh[W.FIELD_PHI])))
    print(f"[gpu] T1023 1024x2048: round trip {e_rt:.3e}, jet step {e_jet:.3e}, Rossby-Haurwitz n={n_deg} "
          f"{e_rh:.3e} (|Phi'_t| {e_phi:.1e})", flush=True)
    assert e_rt <= 1e-11
    assert e_jet <= 1e-12
    assert e_rh <= 1e-11
    assert e_phi <= 1e-30                     # no Phi': its fluxes vanish exactly
    sdc.close()


def test_grid_kernel_high_order_lines():
    """With T + 1 > nlon / 3 the grid kernel writes the analysis lines of the higher orders in two
    parts (A..D before E is transformed).  A field band-limited to degree 460 on 900 latitudes has
    alias-free products at nlon = 1536 and 2048, so f_E at T = 600 (orders >= 512 written in parts
    at nlon = 1536, whole at 2048) agrees to rounding: <= 1e-10 relative L2 (2e-12 measured; the
    divergence tendency's cancellation between the vorticity-flux curl and the kinetic-energy
    Laplacian sets the rounding level, as in the smaller grids), the small values of orders above
    511 on their own <= 1e-8 (1e-10 measured); a misplaced line value would be O(1)."""
    T, nlat, L = 600, 900, 460
    a = _sdc(T, nlat, 1536, 2, 2, 1)
    b = _sdc(T, nlat, 2048, 2, 2, 1)
    x = W.random_state(T, 991)[None].copy()
    n, m = W.degree_order_arrays(T)
    x[:, :, n > L] = 0.0
    fa, fb = _dev(np.zeros_like(x)), _dev(np.zeros_like(x))
    a.eval_explicit(_dev(x), fa)
    b.eval_explicit(_dev(x), fb)
    ha, hb = _host(fa), _host(fb)
    err = rel_l2(ha, hb, T)
    hi = m >= 512
    err_hi = float(np.linalg.norm(ha[..., hi, :] - hb[..., hi, :]) / np.linalg.norm(hb[..., hi, :]))
    print(f"[gpu] T600 f_E nlon 1536 vs 2048: rel L2 {err:.3e}, orders >= 512 {err_hi:.3e}", flush=True)
    assert np.linalg.norm(hb[..., hi, :]) > 0
    assert err <= 1e-10
    assert err_hi <= 1e-8
    a.close()
    b.close()

"""Launch variants of the Legendre kernels and the autotuner (GPU, through the C ABI).

Every variant forms the same sums in the same order, so f_E, a step and an adjoint step must agree
bitwise with the default variants; the grids include an odd number of 16-latitude tiles (T63:
three tiles, so two-, four- and six-tile synthesis tasks have tiles past the end) and batched
node states.
"""
import numpy as np
import pytest

import workloads as W
from paper_2403_20135_amd import _lib

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, _torch, rel_l2

pytestmark = pytest.mark.gpu

DEFAULT = dict(syn_lat_tiles=2, syn_depth=2, ana_depth=2, ana_interleave=1, fuse_update=1, syn_recur=0,
               ana_recur=0, node_launch=0)
# (syn_lat_tiles, syn_depth, ana_depth, ana_interleave[, fuse_update, syn_recur]); syn_recur = 1
# regenerates the tables in the synthesis by the recurrence that wrote them
VARIANTS = [(1, 8, 4, 1), (1, 4, 4, 1), (2, 4, 4, 1), (2, 2, 4, 1), (3, 2, 4, 1), (4, 2, 4, 1),
            (4, 1, 4, 1), (6, 1, 4, 1), (1, 8, 2, 1), (1, 8, 4, 0), (2, 4, 2, 0),
            (4, 2, 2, 1, 1, 1), (4, 1, 2, 1, 1, 1), (4, 2, 4, 0, 0, 1), (2, 2, 2, 1, 1, 1),
            (2, 4, 2, 1, 1, 1), (1, 4, 2, 1, 1, 1), (1, 8, 4, 1, 1, 1), (2, 2, 2, 1, 1, 0, 1),
            (2, 2, 4, 0, 1, 0, 1), (4, 2, 2, 1, 1, 1, 1), (2, 2, 2, 1, 0, 0, 1)]


def _outputs(sdc, x, lam, dt):
    f = _dev(np.zeros_like(x))
    sdc.eval_explicit(_dev(x), f)
    u = _dev(x)
    sdc.step(u, dt)
    g = _dev(np.zeros_like(x))
    sdc.step_adjoint(_dev(x), _dev(lam), g, dt)
    sdc.sync()
    return _host(f), _host(u), _host(g)


@pytest.mark.parametrize("T,nlat,nlon,batch,prec", [(63, 96, 192, 2, "fp64"), (31, 48, 96, 3, "fp32"),
                                                    (21, 34, 64, 1, "fp64"), (10, 12, 24, 2, "fp64"),
                                                    (31, 48, 96, 2, "bf16x3")])
def test_variants_agree_bitwise(T, nlat, nlon, batch, prec):
    sdc = _sdc(T, nlat, nlon, 3, 3, batch, precision=prec)
    x = _states(T, batch, 301)
    lam = np.stack([W.random_state(T, 302 + b) for b in range(batch)])
    lam[..., :T + 1, 1] = 0.0
    dt = 600.0
    assert sdc.plan() == DEFAULT
    ref = _outputs(sdc, x, lam, dt)
    for v in VARIANTS:
        sdc.set_plan(*v)
        got = _outputs(sdc, x, lam, dt)
        for name, a, b in zip(("f_E", "step", "adjoint"), got, ref):
            print(f"[gpu] T{T} {prec} variant {v} {name}: max |diff| {np.max(np.abs(a - b)):.3e}", flush=True)
            assert np.array_equal(a, b), (v, name)


SPLIT = [((2, 2, 2, 1), (4, 2, 2, 1, 1, 1, 1)), ((2, 2, 2, 1), (1, 8, 4, 0, 1, 1, 0)),
         ((4, 2, 2, 1, 1, 1, 1), (2, 2, 4, 1)), ((6, 1, 4, 0), (2, 4, 2, 1, 1, 1, 1))]


@pytest.mark.parametrize("T,nlat,nlon,batch,prec", [(63, 96, 192, 2, "fp64"), (31, 48, 96, 3, "fp32"),
                                                    (21, 34, 64, 2, "bf16x3")])
def test_split_plans_agree_bitwise(T, nlat, nlon, batch, prec):
    """Different variants for the launches over one state per member (the first f_E, eval_explicit,
    the adjoint's first stage; the first synthesis reading the states in place, also when it
    regenerates its tables) and over the node states: the same f_E, step, graph step and adjoint
    bit for bit."""
    sdc = _sdc(T, nlat, nlon, 3, 3, batch, precision=prec)
    x = _states(T, batch, 321)
    lam = np.stack([W.random_state(T, 322 + b) for b in range(batch)])
    lam[..., :T + 1, 1] = 0.0
    dt = 600.0
    ref = _outputs(sdc, x, lam, dt)
    for main, one in SPLIT:
        sdc.set_plan(*main)
        sdc.set_plan_for(1, *one)
        assert sdc.plan_for(3) == sdc.plan()
        p1 = sdc.plan_for(1)
        assert (p1["syn_lat_tiles"], p1["syn_depth"], p1["ana_depth"], p1["ana_interleave"]) == one[:4]
        got = _outputs(sdc, x, lam, dt)
        xg = _dev(x)
        sdc.step_graph(xg, dt)
        sdc.sync()
        for name, a, b in zip(("f_E", "step", "adjoint", "graph step"), got + (_host(xg),), ref + (ref[1],)):
            print(f"[gpu] T{T} {prec} split {main} / {one} {name}: max |diff| {np.max(np.abs(a - b)):.3e}",
                  flush=True)
            assert np.array_equal(a, b), (main, one, name)
    with pytest.raises(_lib.SDCError) as ei:
        sdc.set_plan_for(2, *DEFAULT.values())
    assert ei.value.code == _lib.SDC_EINVAL
    sdc.close()


def test_set_plan_rejects_variants_not_built():
    sdc = _sdc(21, 34, 64, 2, 2, 1)
    for bad in [(2, 8, 4, 1), (4, 4, 4, 1), (3, 4, 4, 1), (5, 2, 4, 1), (6, 2, 4, 1), (1, 6, 4, 1),
                (1, 8, 3, 1), (1, 8, 4, 2), (2, 2, 2, 1, 2), (2, 2, 2, 1, 1, 2), (3, 2, 2, 1, 1, 1),
                (6, 1, 2, 1, 1, 1), (2, 2, 2, 1, 1, 0, 2)]:
        with pytest.raises(_lib.SDCError) as ei:
            sdc.set_plan(*bad)
        assert ei.value.code == _lib.SDC_EINVAL
    assert sdc.plan() == DEFAULT


def test_autotune_keeps_results_and_graphs():
    T, nlat, nlon, M, K, dt = 63, 96, 192, 3, 2, 480.0
    sdc = _sdc(T, nlat, nlon, M, K, 4)
    o = _oracle(T, nlat, nlon)
    x0 = _states(T, 4, 311)
    x = _dev(x0)
    sdc.step_graph(x, dt)                 # a cached graph from before tuning
    chosen = sdc.autotune(5)
    one = sdc.plan_for(1)
    print(f"[gpu] autotune T{T} x4: {chosen}; one state per member: {one}", flush=True)
    assert chosen == sdc.plan()
    assert (one["syn_lat_tiles"], one["syn_depth"]) in [(1, 8), (1, 4), (2, 4), (2, 2), (3, 2),
                                                        (4, 2), (4, 1), (6, 1)]
    assert one["fuse_update"] == chosen["fuse_update"] and one["node_launch"] == 0
    assert (chosen["syn_lat_tiles"], chosen["syn_depth"]) in [(1, 8), (1, 4), (2, 4), (2, 2), (3, 2),
                                                                (4, 2), (4, 1), (6, 1)]
    assert chosen["syn_recur"] in (0, 1) and chosen["ana_recur"] in (0, 1) and chosen["fuse_update"] == 1
    assert chosen["ana_depth"] in (2, 4) and chosen["ana_interleave"] in (0, 1)
    for _ in range(2):
        sdc.step_graph(x, dt)             # recaptured with the chosen variants
    sdc.sync()
    ref = np.stack([o.step(x0[b], dt, M, K, steps=3) for b in range(4)])
    err = rel_l2(_host(x), ref, T)
    print(f"[gpu] after autotune: 3 steps rel L2 {err:.3e}", flush=True)
    assert err <= 1e-11
    with pytest.raises(_lib.SDCError):
        sdc.autotune(0)


@pytest.mark.parametrize("T,nlat,nlon,M,K,batch,prec,qd", [
    (31, 48, 96, 4, 3, 2, "fp64", "flex"),
    (21, 34, 64, 2, 4, 3, "fp64", "ns"),      # ragged tile, K > M, MIN-SR-NS, odd member count
    (31, 48, 96, 1, 2, 5, "fp32", "flex"),    # one node: every state of a group is a member
    (63, 96, 192, 4, 1, 1, "fp64", "flex"),   # one sweep: the first f_E's analysis writes the state
    (31, 48, 96, 3, 3, 2, "fp64", "flex"),    # M = 3: the separate update kernel either way
])
def test_fused_update_is_bitwise_the_separate_one(T, nlat, nlon, M, K, batch, prec, qd):
    """The node updates inside the analysis epilogues (forward and adjoint) give bitwise the same
    steps (eager and graph), taped steps and adjoints as the separate update kernels, also with
    both Legendre kernels regenerating their tables."""
    from paper_2403_20135_amd.api import SDC
    torch = _torch()
    sdc = SDC(T, nlat, nlon, M, K, batch, prec, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH, qdelta=qd)
    x0 = _states(T, batch, 701)
    lam = np.stack([W.random_state(T, 702 + b) for b in range(batch)])
    lam[..., :T + 1, 1] = 0.0
    dt = 600.0
    res = {}
    # plans: separate update kernels (the reference), fused updates, fused updates with both
    # Legendre kernels regenerating their tables
    for key, plan in ((0, (2, 2, 2, 1, 0)), (1, (2, 2, 2, 1, 1)), (2, (4, 2, 2, 1, 1, 1, 1))):
        sdc.set_plan(*plan)
        x, xg = _dev(x0), _dev(x0)
        for _ in range(3):
            sdc.step(x, dt)
            sdc.step_graph(xg, dt)
        tape = sdc.new_tape()
        xt = _dev(x0)
        sdc.step_taped(xt, dt, tape)
        ga, gb = _dev(np.zeros_like(x0)), _dev(np.zeros_like(x0))
        sdc.step_adjoint(_dev(x0), _dev(lam), ga, dt)
        sdc.step_adjoint_taped(tape, _dev(lam), gb, dt)
        sdc.sync()
        torch.cuda.synchronize()
        res[key] = [_host(v) for v in (x, xg, xt, ga, gb)]
    for key in (1, 2):
        for name, a, b in zip(("step", "graph step", "taped step", "adjoint", "taped adjoint"), res[key], res[0]):
            print(f"[gpu] {'fused' if key == 1 else 'fused+regenerated'} T{T} M{M}K{K} x{batch} {prec} {name}: "
                  f"max |diff| {np.max(np.abs(a - b)):.3e}", flush=True)
            assert np.array_equal(a, b), (key, name)
    assert np.array_equal(res[1][0], res[1][1])


@pytest.mark.parametrize("T,nlat,nlon,M,K,prec", [(63, 96, 192, 4, 4, "fp64"), (31, 48, 96, 3, 3, "fp32"),
                                                  (21, 34, 64, 2, 4, "fp64")])
def test_node_launch_agrees_bitwise(T, nlat, nlon, M, K, prec):
    """One node per launch (the sequential counterpart of the batched nodes): the same step, taped
    step and adjoint step bit for bit, eager and as a graph, with the fused update of the batched
    plan as the reference."""
    sdc = _sdc(T, nlat, nlon, M, K, 1, precision=prec)
    x = _states(T, 1, 311)
    lam = W.random_state(T, 312)[None]
    lam[..., :T + 1, 1] = 0.0
    dt = 480.0
    ref = _outputs(sdc, x, lam, dt)
    tape_ref = sdc.new_tape()
    u = _dev(x)
    sdc.step_taped(u, dt, tape_ref)
    sdc.set_plan(**dict(DEFAULT, node_launch=1))
    assert sdc.plan()["node_launch"] == 1
    got = _outputs(sdc, x, lam, dt)
    for name, a, b in zip(("f_E", "step", "adjoint"), got, ref):
        print(f"[gpu] T{T} M={M} K={K} {prec} node_launch {name}: max |diff| {np.max(np.abs(a - b)):.3e}",
              flush=True)
        assert np.array_equal(a, b), name
    ug = _dev(x)
    for _ in range(2):
        sdc.step_graph(ug, dt)
    ue = _dev(x)
    for _ in range(2):
        sdc.step(ue, dt)
    tape = sdc.new_tape()
    ut = _dev(x)
    sdc.step_taped(ut, dt, tape)
    sdc.sync()
    assert np.array_equal(_host(ug), _host(ue))
    assert np.array_equal(_host(ut), ref[1])
    assert np.array_equal(_host(tape), _host(tape_ref))       # the same stage fields, same places
    sdc.close()


def test_node_launch_needs_one_member():
    sdc = _sdc(21, 34, 64, 2, 2, 2)
    with pytest.raises(_lib.SDCError) as e:
        sdc.set_plan(**dict(DEFAULT, node_launch=1))
    assert e.value.code == _lib.SDC_EINVAL
    assert sdc.plan() == DEFAULT
    sdc.close()


@pytest.mark.parametrize("prec,M", [("fp64", 2), ("fp64", 3), ("fp32", 2), ("bf16x3", 3)])
def test_member_alone_and_in_a_batch_agree_bitwise(prec, M):
    """Members evaluated alone or two at a time (the one- and two-state launches: the synthesis
    forms both Pbar tiles in one product, the analysis contracts one column tile) and inside a
    batch of three (separate tiles, two column tiles): f_E, a step and an adjoint step bit for
    bit, for several variants, with the node update fused into the analysis (M = 2) and separate
    (M = 3)."""
    T, nlat, nlon, batch, dt = 63, 96, 192, 3, 600.0
    x = _states(T, batch, 331)
    lam = np.stack([W.random_state(T, 332 + b) for b in range(batch)])
    lam[..., :T + 1, 1] = 0.0
    together = _sdc(T, nlat, nlon, M, 3, batch, precision=prec)
    alone = _sdc(T, nlat, nlon, M, 3, 1, precision=prec)
    pair = _sdc(T, nlat, nlon, M, 3, 2, precision=prec)
    for v in [(2, 2, 2, 1), (1, 4, 4, 0), (6, 1, 2, 1), (4, 2, 2, 1, 1, 1, 1)]:
        for h in (together, alone, pair):
            h.set_plan(*v)
        ref = _outputs(together, x, lam, dt)
        parts = [(b, b + 1, alone) for b in range(batch)] + [(1, 3, pair)]
        for b0, b1, h in parts:
            got = _outputs(h, x[b0:b1], lam[b0:b1], dt)
            for name, a, r in zip(("f_E", "step", "adjoint"), got, ref):
                d = np.max(np.abs(a - r[b0:b1]))
                print(f"[gpu] T{T} {prec} {v} members {b0}..{b1 - 1} {name}: max |diff| {d:.3e}", flush=True)
                assert np.array_equal(a, r[b0:b1]), (v, b0, name)
    for h in (together, alone, pair):
        h.close()

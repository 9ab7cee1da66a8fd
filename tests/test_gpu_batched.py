"""GPU checks of graph-captured steps and of ensembles with mixed truncations (one graph launch
per step for all members), against eager steps (bitwise) and against the FP64 oracle (1e-11)."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _dev, _host, _oracle, _sdc, _states, _torch, rel_l2

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager_bitwise():
    """Replays with eager work and synchronisations in between; every replay checked."""
    T, nlat, nlon = 31, 48, 96
    sdc = _sdc(T, nlat, nlon, 4, 3, 2)
    u0 = _states(T, 2, 13)
    ref = _dev(u0)
    x = _dev(u0)
    for r in range(4):
        sdc.step(ref, 600.0)
        sdc.step_graph(x, 600.0)
        _torch().cuda.synchronize()
        junk = _dev(np.ones((3, 5)))            # unrelated eager work between replays
        junk.mul_(2.0)
        assert np.array_equal(_host(x), _host(ref)), f"replay {r} differs"
    sdc.sync()
    # a different key (dt) captures a new graph; the old one still replays correctly
    y = _dev(u0)
    sdc.step_graph(y, 300.0)
    z = _dev(u0)
    sdc.step(z, 300.0)
    assert np.array_equal(_host(y), _host(z))


def _group(configs):
    from paper_2403_20135_amd.api import SDCGroup
    handles = [_sdc(T, nlat, nlon, M, K, b) for (T, nlat, nlon, M, K, b) in configs]
    return handles, SDCGroup(handles)


def test_group_of_mixed_truncations_matches_oracle():
    configs = [(10, 12, 24, 3, 3, 2), (21, 34, 64, 3, 3, 3), (31, 48, 96, 3, 3, 1)]
    dts = [1200.0, 900.0, 600.0]
    handles, grp = _group(configs)
    u0 = [_states(c[0], c[5], 50 + k) for k, c in enumerate(configs)]
    xs = [_dev(u) for u in u0]
    for _ in range(3):
        grp.step(xs, dts, 3, 3)
    grp.sync()
    for k, (T, nlat, nlon, M, K, b) in enumerate(configs):
        o = _oracle(T, nlat, nlon)
        ref = np.stack([o.step(u0[k][i], dts[k], M, K, steps=3) for i in range(b)])
        assert rel_l2(_host(xs[k]), ref, T) <= 1e-11


def test_mixed32_workload_one_graph_per_step():
    """The 32-member ensemble (16 x T63, 12 x T127, 4 x T255; M=4, K=3; dt 480/240/120 s), two steps
    as one graph launch each; members sampled per truncation against the oracle."""
    wl = W.WORKLOADS["mixed32_m4k3"]
    groups = {}
    for k, mb in enumerate(wl.members):
        groups.setdefault(mb.T, []).append((k, mb))
    configs, u0, dts = [], [], []
    for T, lst in sorted(groups.items()):
        mb = lst[0][1]
        configs.append((T, mb.nlat, mb.nlon, wl.M, wl.K, len(lst)))
        u0.append(np.stack([W.initial_state(wl, member=k) for k, _ in lst]))
        dts.append(mb.dt)
    handles, grp = _group(configs)
    xs = [_dev(u) for u in u0]
    for _ in range(2):
        grp.step(xs, dts, wl.M, wl.K)
    grp.sync()
    for g, (T, nlat, nlon, M, K, b) in enumerate(configs):
        got = _host(xs[g])
        assert np.all(np.isfinite(got))
        o = _oracle(T, nlat, nlon)
        for i in sorted({0, b - 1}):
            ref = o.step(u0[g][i], dts[g], M, K, steps=2)
            err = rel_l2(got[i], ref, T)
            print(f"[gpu] mixed32 T{T} member {i}: rel L2 {err:.3e}", flush=True)
            assert err <= 1e-11


def _mixed32_handles(precision="fp64"):
    from paper_2403_20135_amd.api import SDC, SDCGroup
    wl = W.WORKLOADS["mixed32_m4k3"]
    groups = {}
    for k, mb in enumerate(wl.members):
        groups.setdefault(mb.T, []).append((k, mb))
    handles, u0, dts, cfgs = [], [], [], []
    for T, lst in sorted(groups.items()):
        mb = lst[0][1]
        handles.append(SDC(T, mb.nlat, mb.nlon, wl.M, wl.K, len(lst), precision, W.RADIUS, W.GRAVITY,
                           W.OMEGA, W.MEAN_DEPTH))
        u0.append(np.stack([W.initial_state(wl, member=k) for k, _ in lst]))
        dts.append(mb.dt)
        cfgs.append((T, mb.nlat, mb.nlon, len(lst)))
    return wl, handles, SDCGroup(handles), u0, dts, cfgs


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_mixed32_one_launch_per_phase_is_bitwise_the_branches(precision):
    """Mode 1 (one synthesis, grid and analysis launch per sweep over all 32 members of three
    truncations) against mode 0 (one graph branch per truncation): the same states bit for bit,
    over graph replays."""
    wl, handles, grp, u0, dts, _ = _mixed32_handles(precision)
    assert grp.mode == 1
    x1 = [_dev(u) for u in u0]
    for _ in range(3):
        grp.step(x1, dts, wl.M, wl.K)
    grp.sync()
    grp.set_mode(0)
    assert grp.mode == 0
    x0 = [_dev(u) for u in u0]
    for _ in range(3):
        grp.step(x0, dts, wl.M, wl.K)
    grp.sync()
    for a, b in zip(x1, x0):
        ha, hb = _host(a), _host(b)
        print(f"[gpu] mixed32 {precision} merged vs branches: max |diff| {np.max(np.abs(ha - hb)):.3e}", flush=True)
        assert np.array_equal(ha, hb)


def test_mixed32_one_launch_per_phase_matches_oracle():
    """The 32-member ensemble in mode 1, with the merged launches' variants chosen by the group
    autotuner (which restores the states it times on): after 6 steps the first and last member of
    every truncation against the oracle, and after the workload's full 50 steps those of the T63
    and T127 truncations (the oracle's T255 steps are too slow for 50), <= 1e-11 relative L2."""
    wl, handles, grp, u0, dts, cfgs = _mixed32_handles()
    xs = [_dev(u) for u in u0]
    mode = grp.autotune(xs, dts, wl.M, wl.K, 2)
    print(f"[gpu] mixed32 group autotune chose mode {mode}", flush=True)
    for x, u in zip(xs, u0):
        assert np.array_equal(_host(x), u)              # states restored
    grp.set_mode(1)
    steps = 6
    for _ in range(steps):
        grp.step(xs, dts, wl.M, wl.K)
    grp.sync()
    refs = {}
    for g, (T, nlat, nlon, b) in enumerate(cfgs):
        got = _host(xs[g])
        o = _oracle(T, nlat, nlon)
        for i in sorted({0, b - 1}):
            ref = o.step(u0[g][i], dts[g], wl.M, wl.K, steps=steps)
            refs[(g, i)] = ref
            err = rel_l2(got[i], ref, T)
            print(f"[gpu] mixed32 one launch per phase, T{T} member {i}, {steps} steps: rel L2 {err:.3e}",
                  flush=True)
            assert err <= 1e-11
    for _ in range(steps, wl.steps):
        grp.step(xs, dts, wl.M, wl.K)
    grp.sync()
    for g, (T, nlat, nlon, b) in enumerate(cfgs):
        if T > 127:
            continue
        got = _host(xs[g])
        o = _oracle(T, nlat, nlon)
        for i in sorted({0, b - 1}):
            ref = o.step(refs[(g, i)], dts[g], wl.M, wl.K, steps=wl.steps - steps)
            err = rel_l2(got[i], ref, T)
            print(f"[gpu] mixed32 one launch per phase, T{T} member {i}, {wl.steps} steps: rel L2 {err:.3e}",
                  flush=True)
            assert err <= 1e-11


def test_merged_group_with_separate_updates():
    """M = 3 (the separate node-update kernel, also one launch over the members), T31 x 2 and
    T63 x 1: mode 1 bitwise mode 0 and against the oracle; a group whose members cannot share
    launches refuses mode 1."""
    from paper_2403_20135_amd import _lib
    configs = [(31, 48, 96, 3, 3, 2), (63, 96, 192, 3, 3, 1)]
    dts = [600.0, 480.0]
    handles, grp = _group(configs)
    assert grp.mode == 1
    u0 = [_states(c[0], c[5], 60 + k) for k, c in enumerate(configs)]
    x1 = [_dev(u) for u in u0]
    for _ in range(2):
        grp.step(x1, dts, 3, 3)
    grp.set_mode(0)
    x0 = [_dev(u) for u in u0]
    for _ in range(2):
        grp.step(x0, dts, 3, 3)
    grp.sync()
    for k, (T, nlat, nlon, M, K, b) in enumerate(configs):
        assert np.array_equal(_host(x1[k]), _host(x0[k]))
        o = _oracle(T, nlat, nlon)
        ref = np.stack([o.step(u0[k][i], dts[k], M, K, steps=2) for i in range(b)])
        assert rel_l2(_host(x1[k]), ref, T) <= 1e-11
    # nlon = 64 is not a length of the merged grid kernel
    h2, g2 = _group([(21, 34, 64, 3, 3, 1), (31, 48, 96, 3, 3, 1)])
    assert g2.mode == 0
    g2.set_mode(1)
    with pytest.raises(_lib.SDCError) as e:
        g2.step([_dev(_states(21, 1, 70)), _dev(_states(31, 1, 71))], [900.0, 600.0], 3, 3)
    assert e.value.code == _lib.SDC_EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_merged_group_of_single_members_with_fused_updates(precision):
    """M = 4 (the node update fused into the analysis, every synthesis reading its states in
    place) with members of one and two states (the one- and two-state launches form both Pbar
    tiles in one product): mode 1 bitwise mode 0, after the group autotuner, and FP64 against the
    oracle (1e-11)."""
    from paper_2403_20135_amd.api import SDCGroup
    configs = [(31, 48, 96, 4, 3, 1), (63, 96, 192, 4, 3, 2)]
    dts = [600.0, 480.0]
    handles = [_sdc(T, nlat, nlon, M, K, b, precision=precision) for (T, nlat, nlon, M, K, b) in configs]
    grp = SDCGroup(handles)
    u0 = [_states(c[0], c[5], 80 + k) for k, c in enumerate(configs)]
    grp.autotune([_dev(u) for u in u0], dts, 4, 3)
    res = {}
    for mode in (1, 0):
        grp.set_mode(mode)
        xs = [_dev(u) for u in u0]
        for _ in range(2):
            grp.step(xs, dts, 4, 3)
        grp.sync()
        res[mode] = [_host(x) for x in xs]
    for k in range(len(configs)):
        assert np.array_equal(res[1][k], res[0][k]), k
    if precision == "fp64":
        for k, (T, nlat, nlon, M, K, b) in enumerate(configs):
            o = _oracle(T, nlat, nlon)
            ref = np.stack([o.step(u0[k][i], dts[k], M, K, steps=2) for i in range(b)])
            err = rel_l2(res[1][k], ref, T)
            print(f"[gpu] group member T{T} x{b}: rel L2 vs oracle {err:.3e}", flush=True)
            assert err <= 1e-11
    grp.close()
    for h in handles:
        h.close()

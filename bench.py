#!/usr/bin/env python
"""Benchmark: dSDC steps/s of the T255, M=4, K=4 shallow-water workload on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload t255_m4k4] [--no-cpu-baseline]
                    [--no-fp32] [--no-adjoint] [--no-work-precision]
                    [--plan TILES,DEPTH,ANA_DEPTH,INTERLEAVE]
    python bench.py --summarize-pmc FETCH.csv WRITE.csv COPY_MIB OUT.json FETCH.log WRITE.log [COMMAND]
                                                                            (counter summary)

Prints ONE JSON line.  Every handle first runs the library's autotuner (untimed; it picks the
Legendre launch variants, reported as `legendre_plan`).  `value` is the plain FP64 path: exactly
K steps (after W warm-up steps and one graph capture) on synthetic seeded fields already resident in device memory, bracketed by
torch.cuda.synchronize(); each step is one replay of the step's captured hipGraph (four more
regions of K replays follow: `steps_per_s_median_of_5` and `steps_per_s_range_of_5` report the
median and spread of the five, `value` stays the first).  A second
region of K eager steps brackets every launch with HIP events on the library's stream; the
dominant kernel class (largest summed time) is reported against its roofline.  A third region
times K forward steps with one checkpoint each followed by K adjoint steps (forward+adjoint, each
adjoint step recomputing its forward stages), and a fourth the same with every step's stages
taped in HBM (forward+adjoint taped: no recomputation).
The same three regions are measured for the FP32 precision mode (Legendre contractions in FP32
on MFMA), whose error is compared with the plain path's at equal step size against the FP64
path at dt/8 ("equal error": E_fp32 <= 1.1 E_fp64, E = max over output times of the relative
L2 error of vorticity).  Two further workloads are reported beside the headline: the 32-member
ensemble of mixed truncations (one graph launch per step) and T511 (FP64 and FP32, forward and
forward+adjoint), the steps/s of dSDC next to the sequential IMEX SDC it parallelises and to the
reference integrator IMEX-o2, and a work-precision comparison of dSDC with IMEX-o2 over one
simulated day (errors against IMEX-o2 at dt = 1.5 s, wall time per run, dSDC's
speedup at equal error).  The CPU baseline is the FP64 oracle timed on the host cores on a bounded
sample.

Rooflines: the Legendre kernels are priced at min(MFMA peak, AI x HBM peak) with AI = useful
flops / algorithmic bytes (tables read once per launch, spectral and Fourier I/O); when the
bandwidth term is the smaller one they are reported in GB/s against 8 TB/s.  Grid and update
kernels are HBM-bound (minimal bytes).  `traffic` comes from a committed counter summary
(FETCH_SIZE, WRITE_SIZE scaled by a copy kernel of known size) and is reported only when that
summary was taken from the current kernel sources.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "SDC steps/s (fwd, fwd+adjoint) at T255 M=4 vs plain FP64 GPU at equal error"
PEAK_HBM_GBS = 8000.0
# MFMA ceilings of the algorithmic contraction flops: FP64 and FP32 MFMA peaks; BF16x3 forms each
# product from 8 BF16 slot products (16x16x32 for one 16x16x4 step), so its ceiling is the BF16
# MFMA peak over 8
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 8}
TABLE_BYTES = {"fp64": 8, "fp32": 4, "bf16x3": 4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_t255_m4k4.json")


# the sources of the kernels a counter summary covers (synthesis, grid, analysis, node update)
PROFILED_SOURCES = ("legendre.hip", "grid.hip", "update.hip")


def source_hash() -> str:
    """Hash of the device sources of the profiled kernel classes (their .hip files and every shared
    header): a counter summary is valid only for the kernels it measured.  The Legendre launch
    variants, the only host-side choice that changes what those kernels do per launch, are checked
    separately (the plan)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_20135_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in PROFILED_SOURCES] + glob.glob(os.path.join(csrc, "*.h"))
    for p in sorted(srcs):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + f.read())
    return h.hexdigest()[:16]


def algorithmic_work(T, nlat, M, K, batch, precision, fused=False, syn_recur=False, ana_recur=False,
                     syn_recur1=None, ana_recur1=None):
    """Algorithmic work of every kernel class over one step: {class: (flops, bytes)}.  Bytes are
    the minimum each class must move, independent of the layouts the kernels use.

    Legendre: one scalar-equivalent complex transform with equatorial symmetry costs
    2*ncoef*nlat flops; synthesis does 6 per state (zeta, Phi', psi and chi with Pbar, psi and chi
    with H), analysis 7 (div/curl pairs of (A,B), (C,D), and KE).  Bytes per launch: both tables
    (Pbar, H: ncoef x nlat/2 entries each) once; per state the synthesis reads the state in place
    (3 complex FP64 per coefficient; the FP32 mode rounds them to FP32 in registers) and writes 4
    Fourier fields (nlat x (T+1) complex FP64); the analysis reads 5 Fourier
    fields (A..E, nlat x (T+1) complex at the column precision) and writes 3 complex per
    coefficient.  Grid: reads 4 Fourier fields (FP64), writes 5 (column precision).
    Update (separate kernel): per coefficient and member, each full sweep reads u_n (3 complex)
    and per node j the Phi', delta of u_j (2) and E_j (3), and writes node m (3); the last sweep
    writes node M only.
    fused (the node update in the analysis epilogue, M in {1, 2, 4}): the tendencies never reach
    HBM, so the analysis loses its spectral output and gains per coefficient and member
    (K-1)(3 + 5M) + (6 + 2M) complex (u_n, Phi' and delta of the nodes, the new nodes).
    syn_recur (the synthesis regenerates its tables): it reads the recurrence coefficients
    (4 FP64 per (m, n), n < T + 16) and the sectoral values (FP64 per m and northern latitude)
    instead of the tables.  ana_recur (the analysis restarts the recurrence): a quarter of the
    table bytes.  syn_recur1 / ana_recur1: the same for the step's first launch (one state per
    member), whose plan may differ (default: the node launches').
    """
    syn_recur1 = syn_recur if syn_recur1 is None else syn_recur1
    ana_recur1 = ana_recur if ana_recur1 is None else ana_recur1
    ncoef = (T + 1) * (T + 2) // 2
    transform = 2.0 * ncoef * nlat
    states = batch * (1 + (K - 1) * M)          # states transformed per step
    tables = 2.0 * ncoef * (nlat // 2) * TABLE_BYTES[precision]   # per launch
    nhp = (nlat // 2 + 15) // 16 * 16
    rec_data = 32.0 * (T + 1) * (T + 16) + 8.0 * (T + 1) * nhp
    col = 2.0 * TABLE_BYTES[precision]          # one complex value at the column precision
    four = nlat * (T + 1)                        # Fourier coefficients of one field
    syn_tab = (rec_data if syn_recur1 else tables) + (K - 1) * (rec_data if syn_recur else tables)
    ana_tab = (tables / 4 if ana_recur1 else tables) + (K - 1) * (tables / 4 if ana_recur else tables)
    syn_bytes = syn_tab + states * (3 * 16.0 * ncoef + 4 * 16.0 * four)
    ana_bytes = ana_tab + states * (5 * col * four + 3 * 16.0 * ncoef)
    grid_bytes = (4 * 16.0 + 5 * col) * four * states
    upd_bytes = batch * ncoef * 16.0 * ((K - 1) * (3 + 8 * M) + (6 + 5 * M))
    if fused:
        ana_bytes += batch * ncoef * 16.0 * ((K - 1) * (3 + 5 * M) + (6 + 2 * M)) \
            - states * 3 * 16.0 * ncoef
        upd_bytes = 0.0
    return {"synthesis": (6 * transform * states, syn_bytes),
            "analysis": (7 * transform * states, ana_bytes),
            "grid": (0.0, grid_bytes), "update": (0.0, upd_bytes)}


def roofline_entry(flops, nbytes, secs, launches, precision):
    """Achieved rate against min(MFMA peak, AI x HBM peak) (bytes only: HBM)."""
    if flops > 0:
        ai = flops / nbytes
        if ai * PEAK_HBM_GBS * 1e9 < PEAK_TFLOPS[precision] * 1e12:
            bound, ach, peak, unit = "hbm", nbytes / secs / 1e9, PEAK_HBM_GBS, "GB/s"
        else:
            bound, ach, peak, unit = "mfma", flops / secs / 1e12, PEAK_TFLOPS[precision], "TFLOP/s"
        extra = {"ai_flop_per_byte": round(ai, 3), "tflops": round(flops / secs / 1e12, 3)}
    else:
        bound, ach, peak, unit = "hbm", nbytes / secs / 1e9, PEAK_HBM_GBS, "GB/s"
        extra = {}
    e = {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
         "frac": round(ach / peak, 4), "avg_us": round(secs * 1e6 / max(launches, 1), 2),
         "launches": launches, "algorithmic_bytes_per_launch": round(nbytes / max(launches, 1))}
    e.update(extra)
    return e


FORCED_PLAN = None          # --plan: Legendre variants set instead of tuned
FORCED_PLAN1 = None         # --plan1: those of the launches over one state per member


def measure(wl, precision, steps, warmup, with_kernels=True, with_adjoint=True):
    """Graph-replay steps/s, per-kernel HIP-event timing over eager steps, fwd+adj steps/s."""
    import torch
    from paper_2403_20135_amd.api import SDC
    mb = wl.members[0]
    batch = 1
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, batch, precision, W.RADIUS, W.GRAVITY,
              W.OMEGA, W.MEAN_DEPTH)
    x = torch.tensor(W.initial_state(wl)[None], dtype=torch.float64, device="cuda")
    if FORCED_PLAN is not None:                       # fixed variants (profiling runs)
        sdc.set_plan(*FORCED_PLAN)
        if FORCED_PLAN1 is not None:
            sdc.set_plan_for(1, *FORCED_PLAN1)
        plan = sdc.plan()
    else:
        plan = sdc.autotune(10)                       # Legendre launch variants (untimed setup)
    for _ in range(warmup):
        sdc.step(x, mb.dt)
    sdc.sync()

    # timed region: K steps, each one replay of the step's captured hipGraph
    sdc.step_graph(x, mb.dt)                          # capture (untimed)
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sdc.step_graph(x, mb.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sdc.sync()
    out = {"steps_per_s": steps / elapsed, "ms_per_step": elapsed / steps * 1e3, "plan": plan,
           "plan1": sdc.plan_for(1)}
    # four more timed regions of K replays after the contract one (not part of `value`): the
    # median of five and their spread
    rates = [steps / elapsed]
    for _ in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sdc.step_graph(x, mb.dt)
        torch.cuda.synchronize()
        rates.append(steps / (time.perf_counter() - t0))
    out["repeats"] = sorted(rates)

    if with_kernels:
        # per-kernel HIP events (on the library's stream) over K eager steps of the same kernels
        sdc.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sdc.step(x, mb.dt)
        torch.cuda.synchronize()
        out["eager_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        sdc.sync()
        kt = sdc.timing_read()
        sdc.timing(False)
        fused = bool(plan["fuse_update"]) and wl.M in (1, 2, 4)
        work = algorithmic_work(mb.T, mb.nlat, wl.M, wl.K, batch, precision, fused,
                                bool(plan["syn_recur"]), bool(plan["ana_recur"]),
                                bool(out["plan1"]["syn_recur"]), bool(out["plan1"]["ana_recur"]))
        out["kernels"] = {name: roofline_entry(work[name][0] * steps, work[name][1] * steps, ms / 1e3,
                                               launches, precision)
                          for name, (ms, launches) in kt.items() if launches > 0}
        out["kernel_ms"] = {name: ms for name, (ms, _) in kt.items()}

    if not with_adjoint:
        sdc.close()
        return out
    # forward + adjoint: every forward step keeps its input (one checkpoint per step), then the
    # adjoint steps run in reverse, each recomputing its step's stages from the checkpoint
    ckpt = torch.empty((steps,) + tuple(x.shape), dtype=torch.float64, device="cuda")
    lam = torch.ones_like(x)
    lam_out = torch.empty_like(x)
    sdc.step_adjoint(x, lam, lam_out, mb.dt)          # allocates the adjoint workspaces once
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ckpt[k].copy_(x)
        sdc.step(x, mb.dt)
    for k in range(steps - 1, -1, -1):
        sdc.step_adjoint(ckpt[k], lam, lam, mb.dt)
    torch.cuda.synchronize()
    elapsed_fa = time.perf_counter() - t0
    sdc.sync()
    if not bool(torch.isfinite(lam).all()) or not bool(torch.isfinite(x).all()):
        raise RuntimeError(f"non-finite state or adjoint ({precision})")
    out["fwd_adj_steps_per_s"] = steps / elapsed_fa
    out["fwd_adj_ms_per_step"] = elapsed_fa / steps * 1e3
    # forward + adjoint with every step's stages taped in HBM (no recomputation in the adjoint)
    tapes = [sdc.new_tape() for _ in range(steps)]
    lam.fill_(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        sdc.step_taped(x, mb.dt, tapes[k])
    for k in range(steps - 1, -1, -1):
        sdc.step_adjoint_taped(tapes[k], lam, lam, mb.dt)
    torch.cuda.synchronize()
    elapsed_ft = time.perf_counter() - t0
    sdc.sync()
    if not bool(torch.isfinite(lam).all()):
        raise RuntimeError(f"non-finite taped adjoint ({precision})")
    out["fwd_adj_taped_steps_per_s"] = steps / elapsed_ft
    out["tape_bytes_per_step"] = tapes[0].numel()
    del tapes
    sdc.close()
    return out


def equal_error(wl, steps=40, every=10):
    """E_fp64, E_fp32, E_bf16x3 against the FP64 path at dt/8: max over output times of the
    relative L2 error (sphere norm) of vorticity."""
    import numpy as np
    import torch
    from paper_2403_20135_amd.api import SDC
    mb = wl.members[0]
    _, m = W.degree_order_arrays(mb.T)
    sm = np.where(m == 0, 1.0, 2.0)[:, None]

    def history(precision, dt, n, ev):
        sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, precision, W.RADIUS, W.GRAVITY,
                  W.OMEGA, W.MEAN_DEPTH)
        x = torch.tensor(W.initial_state(wl)[None], dtype=torch.float64, device="cuda")
        out = []
        for k in range(1, n + 1):
            sdc.step(x, dt)
            if k % ev == 0:
                out.append(x[0, 1].cpu().numpy())
        sdc.sync()
        sdc.close()
        return out

    ref = history("fp64", mb.dt / 8, 8 * steps, 8 * every)

    def err(h):
        return max(math.sqrt(np.sum(sm * (a - r) ** 2) / np.sum(sm * r ** 2)) for a, r in zip(h, ref))

    e64, e32 = err(history("fp64", mb.dt, steps, every)), err(history("fp32", mb.dt, steps, every))
    e3 = err(history("bf16x3", mb.dt, steps, every))
    return {"E_fp64": e64, "E_fp32": e32, "ratio": e32 / e64, "equal": bool(e32 <= 1.1 * e64),
            "E_bf16x3": e3, "ratio_bf16x3": e3 / e64, "equal_bf16x3": bool(e3 <= 1.1 * e64),
            "quantity": f"max over t = {every}..{steps} steps (every {every}) of rel. L2 of zeta",
            "reference": f"FP64 GPU path at dt/8 ({8 * steps} steps of {mb.dt / 8} s)"}


def measure_mixed(steps=20, warmup=3):
    """The 32-member ensemble of mixed truncations (16 x T63, 12 x T127, 4 x T255; M=4, K=3):
    one graph launch per step advances every member (FP64)."""
    import torch
    from paper_2403_20135_amd.api import SDC, SDCGroup
    wl = W.WORKLOADS["mixed32_m4k3"]
    groups = {}
    for k, mb in enumerate(wl.members):
        groups.setdefault(mb.T, []).append((k, mb))
    handles, xs, dts = [], [], []
    for T, lst in sorted(groups.items()):
        mb = lst[0][1]
        handles.append(SDC(T, mb.nlat, mb.nlon, wl.M, wl.K, len(lst), "fp64", W.RADIUS, W.GRAVITY,
                           W.OMEGA, W.MEAN_DEPTH))
        handles[-1].autotune(10)
        xs.append(torch.tensor(__import__("numpy").stack([W.initial_state(wl, member=k) for k, _ in lst]),
                               dtype=torch.float64, device="cuda"))
        dts.append(mb.dt)
    grp = SDCGroup(handles)
    chosen = grp.autotune(xs, dts, wl.M, wl.K, 5)
    res = {}
    for mode in (1, 0):
        grp.set_mode(mode)
        for _ in range(warmup):
            grp.step(xs, dts, wl.M, wl.K)
        grp.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            grp.step(xs, dts, wl.M, wl.K)
        torch.cuda.synchronize()
        res[mode] = time.perf_counter() - t0
        grp.sync()
    if not all(bool(torch.isfinite(x).all()) for x in xs):
        raise RuntimeError("non-finite ensemble state")
    grp.close()
    for h in handles:
        h.close()
    el = res[chosen]
    return {"workload": wl.name, "members": len(wl.members), "steps": steps,
            "steps_per_s": round(steps / el, 3), "member_steps_per_s": round(len(wl.members) * steps / el, 1),
            "ms_per_step": round(el / steps * 1e3, 4), "precision": "fp64",
            "mode_chosen_by_group_autotuner": chosen,
            "member_steps_per_s_one_launch_per_phase": round(len(wl.members) * steps / res[1], 1),
            "member_steps_per_s_graph_branches": round(len(wl.members) * steps / res[0], 1),
            "launch": "one hipGraph per step; mode 1: every phase one launch over all 32 members, "
                      "mode 0: one graph branch per truncation"}


def speedup_at_equal_error(rows):
    """dSDC's speedup over IMEX-o2 at equal error: for every dSDC row whose error lies inside the
    IMEX-o2 errors, the IMEX-o2 time interpolated linearly in (log error, log time) between the
    two bracketing IMEX-o2 rows, divided by the dSDC time."""
    imex = sorted([(r["error"], r["seconds"]) for r in rows if r["method"] == "IMEX-o2"])
    speed = []
    for r in rows:
        if r["method"] != "dSDC":
            continue
        for (e0, t0), (e1, t1) in zip(imex, imex[1:]):
            if 0 < e0 <= r["error"] <= e1 and e1 > e0:
                f = math.log(r["error"] / e0) / math.log(e1 / e0)
                t_imex = math.exp(math.log(t0) + f * (math.log(t1) - math.log(t0)))
                speed.append({"dt_dSDC": r["dt"], "error": r["error"],
                              "speedup_vs_IMEX_o2": round(t_imex / r["seconds"], 3)})
                break
    return speed


JET_U0 = 20.0     # the work-precision study's jet [m/s]


def work_precision(wl, t_end=86400.0, out_every=21600.0):
    """Work against precision over one simulated day (the comparison of Section 5: dSDC against
    the IMEX-o2 reference integrator, both on this GPU) from the workload's field on a balanced
    zonal jet (the synthetic counterpart of the paper's perturbed jet): absolute L-infinity-in-time, L2-in-space
    error of vorticity at the output times against IMEX-o2 at dt = 1.5 s, and the wall time of each
    run (graph replays, output copies on the device).  The absolute L2 norm is the area-weighted
    RMS over the sphere, sqrt(1/2 sum_m s_m |c|^2) by Parseval."""
    import numpy as np
    import torch
    from paper_2403_20135_amd.api import SDC
    mb = wl.members[0]
    _, m = W.degree_order_arrays(mb.T)
    sm = torch.tensor(np.where(m == 0, 1.0, 2.0)[:, None], dtype=torch.float64, device="cuda")
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, "fp64", W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    plan = sdc.autotune(10)
    # the synthetic jet: the workload's n^-3 field on the balanced 20 m/s zonal jet
    x0 = torch.tensor((W.initial_state(wl) + W.balanced_jet(mb.T, JET_U0))[None], dtype=torch.float64,
                      device="cuda")
    nout = int(round(t_end / out_every))

    def run(method, dt):
        n = int(round(t_end / dt))
        per = int(round(out_every / dt))
        assert n * dt == t_end and per * dt == out_every
        x = x0.clone()
        outs = torch.empty((nout,) + tuple(x[0, 1].shape), dtype=torch.float64, device="cuda")
        stepf = (lambda: sdc.step_graph(x, dt)) if method == "dSDC" else (lambda: sdc.imex2_step_graph(x, dt))
        stepf()                                        # capture (untimed): restart from x0
        x.copy_(x0)
        sdc.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, n + 1):
            stepf()
            if k % per == 0:
                outs[k // per - 1].copy_(x[0, 1])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        sdc.sync()
        return n, secs, outs

    # dSDC against itself at a small step: the observed order per halving of dt shows where the
    # asymptotic order K begins (stiff gravity waves: omega dt < 1 below ~80 s at T255)
    _, _, ref_self = run("dSDC", 3.75)
    conv = []
    for dt in (480.0, 240.0, 120.0, 60.0, 30.0, 15.0):
        _, _, outs = run("dSDC", dt)
        d = outs - ref_self
        conv.append({"dt": dt, "error": float(torch.sqrt(0.5 * (sm * d * d).sum(dim=(-2, -1))).max())})
    for a, b in zip(conv, conv[1:]):
        b["order_vs_previous"] = round(math.log(a["error"] / b["error"]) / math.log(a["dt"] / b["dt"]), 2)
    _, _, ref = run("IMEX-o2", 1.5)
    rows = []
    for method, dts in (("dSDC", (450.0, 360.0, 240.0, 180.0, 120.0, 60.0)),
                        ("IMEX-o2", (60.0, 30.0, 15.0, 7.5, 3.75))):
        for dt in dts:
            n, secs, outs = run(method, dt)
            d = outs - ref
            err = float(torch.sqrt(0.5 * (sm * d * d).sum(dim=(-2, -1))).max())
            rows.append({"method": method, "dt": dt, "steps": n, "seconds": round(secs, 5),
                         "error": err})
    sdc.close()
    speed = speedup_at_equal_error(rows)
    return {"workload": wl.name, "initial_state": f"n^-3 spectrum on the balanced {JET_U0:g} m/s zonal jet",
            "t_end_s": t_end, "output_every_s": out_every, "M": wl.M, "K": wl.K,
            "precision": "fp64", "reference": "IMEX-o2 at dt = 1.5 s",
            "error": "max over output times of the area-weighted RMS of the vorticity difference [1/s]",
            "legendre_plan": plan, "rows": rows, "speedup_at_equal_error": speed,
            "dSDC_self_convergence": {"reference": "dSDC at dt = 3.75 s", "rows": conv}}


def integrators(wl, steps=100, warmup=3):
    """Steps/s of the three integrators on the headline workload (FP64, graph replays): dSDC
    (Algorithm 2, the nodes of a sweep batched), the sequential IMEX SDC it parallelises
    (Algorithm 1, one node at a time) and the reference integrator IMEX-o2."""
    import torch
    from paper_2403_20135_amd.api import SDC
    mb = wl.members[0]
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, "fp64", W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    sdc.autotune(10)
    x0 = torch.tensor(W.initial_state(wl)[None], dtype=torch.float64, device="cuda")
    out = {}
    for name, f in (("dSDC", sdc.step_graph), ("sequential_IMEX_SDC", sdc.step_sequential_graph),
                    ("IMEX_o2", sdc.imex2_step_graph)):
        x = x0.clone()
        for _ in range(warmup):
            f(x, mb.dt)
        sdc.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f(x, mb.dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sdc.sync()
        out[name] = {"steps_per_s": round(steps / el, 2), "ms_per_step": round(el / steps * 1e3, 4)}
    # the same dSDC step with the f_E of the nodes of a sweep one node per launch (bitwise the same
    # states): the sequential counterpart of evaluating the nodes together
    sdc.set_plan(**dict(sdc.plan(), node_launch=1))
    x = x0.clone()
    for _ in range(warmup):
        sdc.step_graph(x, mb.dt)
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sdc.step_graph(x, mb.dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sdc.sync()
    out["dSDC_one_node_per_launch"] = {"steps_per_s": round(steps / el, 2), "ms_per_step": round(el / steps * 1e3, 4)}
    sdc.close()
    # the variant with the linear Coriolis term implicit (f_I = L_g + L_c: two tridiagonal chain
    # solves per order in every node update)
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, "fp64", W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH,
              implicit_coriolis=True)
    sdc.autotune(10)
    x = x0.clone()
    for _ in range(warmup):
        sdc.step_graph(x, mb.dt)
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sdc.step_graph(x, mb.dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sdc.sync()
    out["dSDC_implicit_coriolis"] = {"steps_per_s": round(steps / el, 2), "ms_per_step": round(el / steps * 1e3, 4)}
    sdc.close()
    out["f_E_evaluations_per_step"] = {"dSDC": 1 + (wl.K - 1) * wl.M, "sequential_IMEX_SDC": wl.K * wl.M,
                                       "IMEX_o2": 2}
    out["dSDC_speedup_vs_sequential"] = round(out["dSDC"]["steps_per_s"] /
                                              out["sequential_IMEX_SDC"]["steps_per_s"], 3)
    # speedup of evaluating the M nodes of each sweep together over one node per launch, beside
    # the paper's performance model (Section 4.7: S = (1 + (K-1) M) / (1 + (K-1)) for free node
    # parallelism, 3.25 at M = K = 4) and its measured speedup of the time-parallel dSDC (2.9)
    model = (1 + (wl.K - 1) * wl.M) / (1 + (wl.K - 1))
    out["pint_speedup"] = {"measured": round(out["dSDC"]["steps_per_s"] /
                                             out["dSDC_one_node_per_launch"]["steps_per_s"], 3),
                           "model_S": round(model, 3), "paper_measured": 2.9,
                           "meaning": "dSDC steps/s with the nodes of a sweep batched in one launch per "
                                      "kernel class, over one node per launch (same step, bitwise)"}
    return out


def traffic_for(kernel, plan, plan1=None):
    """Measured HBM bytes per launch of `kernel` from the committed counter summary, or None when
    the summary is missing, was taken from other kernel sources or (for the Legendre classes)
    from other launch variants than `plan`."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != source_hash() or kernel not in t.get("kernels", {}):
        return None
    # the plan fields that change what each Legendre kernel does per launch
    fields = {"synthesis": ("syn_lat_tiles", "syn_depth", "syn_recur"),
              "analysis": ("ana_depth", "ana_interleave", "ana_recur", "fuse_update")}.get(kernel, ())
    profiled = t.get("legendre_plan") or {}
    if any(profiled.get(f) != plan.get(f) for f in fields):
        return None
    if plan1 is not None and kernel in ("synthesis", "analysis"):
        profiled1 = t.get("legendre_plan_one_state") or profiled
        if any(profiled1.get(f) != plan1.get(f) for f in fields):
            return None
    k = t["kernels"][kernel]
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def summarize_pmc(fetch_csv, write_csv, copy_mib, out_json, bench_logs, command=None):
    """Counter summary: mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel class, scaled
    so that the device-to-device copy of copy_mib MiB reads and writes exactly that many bytes.
    The Legendre classes take the launch variants the profiled bench runs used (their JSON lines in
    bench_logs name them; both runs must agree); the autotuner's trial launches of other variants
    are left out."""
    import csv
    plans = []
    for log in bench_logs:
        found = [json.loads(line) for line in open(log) if line.startswith('{"metric"')]
        if not found:
            raise RuntimeError(f"no bench result line in {log}")
        plans.append((found[-1]["legendre_plan"], found[-1].get("legendre_plan_one_state")))
    if any(p != plans[0] for p in plans):
        raise RuntimeError(f"the counter runs tuned different Legendre variants: {plans}")
    plan, plan1 = plans[0]
    # forward FP64 kernels of the bench workload (names as rocprofv3 prints them): the variants of
    # both launch shapes (the first f_E's synthesis reads the state in place: a second flag)
    classes = {}
    for pl, first in ((plan, "false"), (plan1 or plan, "true")):
        rec = "true" if pl.get("syn_recur") else "false"
        classes[f"void k_synthesis<0, double, {pl['syn_lat_tiles']}, {pl['syn_depth']}, {rec}, {first}>"] = \
            "synthesis"
        classes[f"void k_analysis_swe<0, double, {pl['ana_depth']}, "
                f"{'true' if pl.get('ana_recur') else 'false'}>"] = "analysis"
    classes.update({"void k_grid_swe<": "grid", "void k_update<": "update"})

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
        return acc

    out = {"source_sha": source_hash(), "copy_mib": copy_mib, "kernels": {}}
    if command:
        out["commands"] = command
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = copy_mib * (1 << 20)
    cf = [v for k, vs in fetch.items() if "copyBuffer" in k for v in vs]
    cw = [v for k, vs in write.items() if "copyBuffer" in k for v in vs]
    f_scale = copy_bytes / (max(cf) * 1024.0)
    w_scale = copy_bytes / (max(cw) * 1024.0)
    out["fetch_scale"], out["write_scale"] = f_scale, w_scale
    out["legendre_plan"] = plan
    out["legendre_plan_one_state"] = plan1
    acc = {}                        # per class: every dispatch of every kernel of the class
    for name, vals in fetch.items():
        cls = next((c for key, c in classes.items() if name.startswith(key)), None)
        if cls is None:
            continue
        a = acc.setdefault(cls, {"names": set(), "fetch": [], "write": []})
        a["names"].add(name.split("(")[0])
        a["fetch"] += vals
        a["write"] += write.get(name, [])
    for cls, a in acc.items():
        wv = a["write"] or [0.0]
        out["kernels"][cls] = {
            "kernel_name": " + ".join(sorted(a["names"])),
            "dispatches": len(a["fetch"]),
            "fetch_bytes_per_launch": sum(a["fetch"]) / len(a["fetch"]) * 1024.0 * f_scale,
            "write_bytes_per_launch": sum(wv) / len(wv) * 1024.0 * w_scale}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


MFMA_PEAK_TFLOPS = {"F64": 78.6, "F32": 157.3, "BF16": 2500.0}


def _kernel_key(name):
    """A kernel's template name as rocprofv3 prints it, without the argument list."""
    return name.split("(")[0].strip()


def read_kernel_stats(stats_csv):
    """Per kernel: calls and average duration [us] from a rocprofv3 --stats kernel summary."""
    import csv
    out = {}
    for r in csv.DictReader(open(stats_csv)):
        out[_kernel_key(r["Name"])] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                                       "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                                       "pct": float(r["Percentage"])}
    return out


def summarize_trace(stats_csv, out_md, title, command):
    """Markdown table of a rocprofv3 --kernel-trace --stats summary (kernels above 0.5 % of the
    GPU time)."""
    st = read_kernel_stats(stats_csv)
    lines = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp, repository at /root/repo):", "",
             "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for k, v in sorted(st.items(), key=lambda kv: -kv[1]["pct"]):
        if v["pct"] < 0.5:
            continue
        lines.append(f"| `{k}` | {v['calls']} | {v['avg_us']:.1f} | {v['min_us']:.1f} | {v['max_us']:.1f} | "
                     f"{v['pct']:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_mfma(counter_csv, stats_csv, out_md, title, command):
    """MFMA evidence of the Legendre kernels from one rocprofv3 --pmc pass (SQ_INSTS_VALU_MFMA_*,
    SQ_INSTS_VALU_MFMA_MOPS_* in units of 512 flops, SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE)
    and the kernel-trace durations of the same command without counters.  Per kernel: MFMA
    instructions and issued MFMA flops per dispatch, the issued rate over the traced average
    duration against the peak of the instruction's type, and the MFMA-busy share of the SIMD
    cycles, SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 32 CUs x 4 SIMDs x 8 XCDs):
    GRBM_GUI_ACTIVE adds up the busy cycles of the 8 XCDs (a 35.8 us dispatch reads 7.6e5)."""
    import csv
    st = read_kernel_stats(stats_csv)
    acc = {}
    for r in csv.DictReader(open(counter_csv)):
        k = _kernel_key(r["Kernel_Name"])
        if not (k.startswith("void k_synthesis") or k.startswith("void k_analysis")):
            continue
        a = acc.setdefault(k, {"ids": set()})
        a["ids"].add(r["Dispatch_Id"])
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# {title}", "", "Commands (run from /tmp with TMPDIR=/tmp, repository at /root/repo):", "",
             "```", command, "```", "",
             "Issued flops = SQ_INSTS_VALU_MFMA_MOPS_{F64,F32,BF16} x 512 per dispatch (padding columns and "
             "rows included); rate = issued flops / the traced average duration; busy = "
             "SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 256 CUs x 4 SIMDs), GRBM_GUI_ACTIVE being the "
             "sum over the 8 XCDs. The useful (algorithmic) flops of the same launches are in the "
             "bench line's kernels entries (tflops).", "",
             "| kernel | dispatches | MFMA instr / dispatch | issued GFLOP / dispatch | avg us (trace) | "
             "issued TFLOP/s | of MFMA peak | MFMA busy |", "|---|---|---|---|---|---|---|---|"]
    summary = {}
    for k, a in sorted(acc.items()):
        n = len(a["ids"])
        typ = next((t for t in ("F64", "F32", "BF16") if a.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) > 0), "F32")
        mops = a.get(f"SQ_INSTS_VALU_MFMA_MOPS_{typ}", 0.0) / n
        instr = a.get(f"SQ_INSTS_VALU_MFMA_{typ}", 0.0) / n
        flop = mops * 512.0
        busy = a.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / n
        gui = a.get("GRBM_GUI_ACTIVE", 0.0) / n
        util = busy / (gui / 8 * 256 * 4) if gui > 0 else float("nan")
        t = st.get(k, {}).get("avg_us")
        rate = flop / (t * 1e-6) / 1e12 if t else float("nan")
        frac = rate / MFMA_PEAK_TFLOPS[typ]
        summary[k] = {"dispatches": n, "type": typ, "mfma_instr": instr, "issued_flop": flop, "avg_us": t,
                      "issued_tflops": rate, "of_peak": frac, "mfma_busy": util}
        lines.append(f"| `{k}` | {n} | {instr:.0f} | {flop / 1e9:.3f} | "
                     f"{t if t is not None else float('nan'):.1f} | {rate:.1f} | {frac:.3f} ({typ} "
                     f"{MFMA_PEAK_TFLOPS[typ]}) | {util:.3f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return summary


def summarize_counters(counter_csv, stats_csv, out_md, title, command, prefixes):
    """Per-dispatch averages of every counter of one rocprofv3 --pmc pass for the kernels whose
    template names start with one of the comma-separated prefixes, with the traced average
    duration and derived shares: VALU instructions per wave, SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES
    (the share of a wave's life issuing VALU), SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES and
    SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE."""
    import csv
    st = read_kernel_stats(stats_csv)
    pre = [p.strip() for p in prefixes.split(",")]
    acc = {}
    for r in csv.DictReader(open(counter_csv)):
        k = _kernel_key(r["Kernel_Name"])
        if not any(k.startswith(p) for p in pre):
            continue
        grid = int(r["Grid_Size"])
        a = acc.setdefault((k, grid), {"ids": set()})
        a["ids"].add(r["Dispatch_Id"])
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    counters = sorted({c for a in acc.values() for c in a if c != "ids"})
    lines = [f"# {title}", "", "Commands (run from /tmp with TMPDIR=/tmp, repository at /root/repo):", "",
             "```", command, "```", "",
             "Per dispatch (mean over the dispatches of one kernel and grid size); avg us from the "
             "kernel trace of the same kernel over all its grid sizes.", "",
             "| kernel | grid (threads) | dispatches | avg us | " + " | ".join(counters)
             + " | VALU / wave | VALU-issue share | wait share | LDS conflict share |",
             "|" + "---|" * (len(counters) + 8)]
    summary = {}
    for (k, grid), a in sorted(acc.items()):
        n = len(a["ids"])
        v = {c: a.get(c, 0.0) / n for c in counters}
        waves = v.get("SQ_WAVES", 0.0)
        cyc = v.get("SQ_WAVE_CYCLES", 0.0)
        d = {"valu_per_wave": v.get("SQ_INSTS_VALU", 0.0) / waves if waves else float("nan"),
             "valu_issue_share": v.get("SQ_ACTIVE_INST_VALU", 0.0) / cyc if cyc else float("nan"),
             "wait_share": v.get("SQ_WAIT_INST_ANY", 0.0) / cyc if cyc else float("nan"),
             "lds_conflict_share": (v.get("SQ_LDS_BANK_CONFLICT", 0.0) / v["SQ_LDS_IDX_ACTIVE"]
                                    if v.get("SQ_LDS_IDX_ACTIVE") else float("nan"))}
        t = st.get(k, {}).get("avg_us", float("nan"))
        summary[f"{k} [{grid}]"] = {"dispatches": n, "avg_us": t, **v, **d}
        lines.append(f"| `{k}` | {grid} | {n} | {t:.1f} | " + " | ".join(f"{v[c]:.4g}" for c in counters)
                     + f" | {d['valu_per_wave']:.0f} | {d['valu_issue_share']:.3f} | {d['wait_share']:.3f} | "
                       f"{d['lds_conflict_share']:.3f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return summary


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def sphere_rel_l2(got, ref, T):
    """Relative L2 (sphere norm, sqrt(sum_m s_m |c|^2) by Parseval) per field (Phi', zeta, delta),
    maximised over members; got, ref [members][3][ncoef][2]."""
    import numpy as np
    _, m = W.degree_order_arrays(T)
    s = np.where(m == 0, 1.0, 2.0)[:, None]
    got = np.asarray(got).reshape(-1, 3, len(m), 2)
    ref = np.asarray(ref).reshape(-1, 3, len(m), 2)
    out = {}
    for f, name in enumerate(("phi", "zeta", "delta")):
        worst = 0.0
        for a, b in zip(got[:, f], ref[:, f]):
            num, den = float(np.sum(s * (a - b) ** 2)), float(np.sum(s * b ** 2))
            worst = max(worst, math.sqrt(num / den) if den > 0 else math.sqrt(num))
        out[name] = worst
    out["max"] = max(out.values())
    return out


def cpu_baseline(wl, state0, budget_s=15.0):
    """The CPU-baseline leg: the FP64 oracle timed on the host cores (all threads torch uses over
    n steps, n sized to about budget_s, then one step on one thread), and, untimed, the oracle's
    references for the error of every GPU result the line reports: the headline state after 1 and
    1 + n steps from state0, the VJP of one headline step, one member of each truncation of the
    mixed ensemble after 2 steps, and one T511 step."""
    import torch
    from oracle.sdc import Oracle
    mb = wl.members[0]
    o = Oracle(mb.T, mb.nlat, mb.nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    t0 = time.perf_counter()
    x1 = o.step(state0, mb.dt, wl.M, wl.K, steps=1)
    t1 = time.perf_counter() - t0
    n = max(1, min(20, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    xn = o.step(x1, mb.dt, wl.M, wl.K, steps=n)
    dt_all = time.perf_counter() - t0
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        o.step(x1, mb.dt, wl.M, wl.K, steps=1)
        dt_one = time.perf_counter() - t0
    finally:
        torch.set_num_threads(threads)
    base = {"value": n / dt_all, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} dSDC steps of {wl.name} (T{mb.T} {mb.nlat}x{mb.nlon}, M={wl.M}, K={wl.K}) "
                      f"after 1 untimed step, torch-CPU float64 oracle, {threads} threads",
            "single_thread": {"value": 1.0 / dt_one, "unit": "steps/s", "cores": 1,
                              "sample": "1 step of the same workload on one thread"},
            "host": host_cpu()}
    refs = {"after": {1: x1, 1 + n: xn}}
    if wl.name != "t255_m4k4":
        return base, refs
    lam = W.random_state(mb.T, 255)
    lam[:, :mb.T + 1, 1] = 0.0                       # m = 0 imaginary parts are held at 0
    refs["lam"] = lam
    refs["vjp"] = o.step_vjp(state0, lam, mb.dt, wl.M, wl.K)
    mix = W.WORKLOADS["mixed32_m4k3"]
    refs["mixed"] = {}
    for k, m0 in enumerate(mix.members):
        if any(m0.T == mm.T for mm in mix.members[:k]):
            continue                                 # the first member of each truncation
        om = Oracle(m0.T, m0.nlat, m0.nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
        refs["mixed"][k] = om.step(W.initial_state(mix, member=k), m0.dt, mix.M, mix.K, steps=2)
    big = W.WORKLOADS["t511_m4k4"]
    bm = big.members[0]
    ob = Oracle(bm.T, bm.nlat, bm.nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    refs["t511"] = ob.step(W.initial_state(big), bm.dt, big.M, big.K, steps=1)
    oc = Oracle(mb.T, mb.nlat, mb.nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH, coriolis_implicit=True)
    refs["implicit_coriolis"] = oc.step(state0, mb.dt, wl.M, wl.K, steps=1)
    return base, refs


def oracle_errors(wl, refs):
    """Error against the FP64 oracle (references from the CPU-baseline leg) of every result the
    line reports: the headline step in FP64, FP32 and BF16x3 after 1 and 1 + n steps, one adjoint step of
    each precision, the first member of each truncation of the mixed ensemble after 2 group steps,
    and one T511 step in FP64, FP32 and BF16x3.  Relative L2 per field (sphere norm), max over members."""
    import numpy as np
    import torch
    from paper_2403_20135_amd.api import SDC, SDCGroup
    mb = wl.members[0]
    x0 = W.initial_state(wl)[None]
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    out = {"metric": "relative L2 per field (sphere norm) against the FP64 oracle, max over members"}
    for prec in ("fp64", "fp32", "bf16x3"):
        sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, prec, W.RADIUS, W.GRAVITY, W.OMEGA,
                  W.MEAN_DEPTH)
        sdc.autotune(5)
        x = dev(x0)
        done, res = 0, {}
        for k in sorted(refs["after"]):
            while done < k:
                sdc.step_graph(x, mb.dt)
                done += 1
            sdc.sync()
            res[f"after_{k}_steps"] = sphere_rel_l2(x.cpu().numpy(), refs["after"][k][None], mb.T)
        g = torch.zeros_like(x)
        sdc.step_adjoint(dev(x0), dev(refs["lam"][None]), g, mb.dt)
        sdc.sync()
        res["adjoint_step"] = sphere_rel_l2(g.cpu().numpy(), refs["vjp"][None], mb.T)
        sdc.close()
        out[f"{wl.name}_{prec}"] = res

    mix = W.WORKLOADS["mixed32_m4k3"]
    groups = {}
    for k, m in enumerate(mix.members):
        groups.setdefault(m.T, []).append(k)
    handles, xs, dts = [], [], []
    for T, ks in sorted(groups.items()):
        m0 = mix.members[ks[0]]
        handles.append(SDC(T, m0.nlat, m0.nlon, mix.M, mix.K, len(ks), "fp64", W.RADIUS,
                           W.GRAVITY, W.OMEGA, W.MEAN_DEPTH))
        xs.append(dev(np.stack([W.initial_state(mix, member=k) for k in ks])))
        dts.append(m0.dt)
    grp = SDCGroup(handles)
    for _ in range(2):
        grp.step(xs, dts, mix.M, mix.K)
    grp.sync()
    mres = {}
    for (T, ks), x in zip(sorted(groups.items()), xs):
        mres[f"member_{ks[0]}_T{T}"] = sphere_rel_l2(x[0].cpu().numpy()[None], refs["mixed"][ks[0]][None], T)
    grp.close()
    for h in handles:
        h.close()
    out["mixed32_m4k3_fp64_2_steps"] = mres

    big = W.WORKLOADS["t511_m4k4"]
    bm = big.members[0]
    for prec in ("fp64", "fp32", "bf16x3"):
        sdc = SDC(bm.T, bm.nlat, bm.nlon, big.M, big.K, 1, prec, W.RADIUS, W.GRAVITY, W.OMEGA,
                  W.MEAN_DEPTH)
        sdc.autotune(3)
        x = dev(W.initial_state(big)[None])
        sdc.step(x, bm.dt)
        sdc.sync()
        out[f"t511_m4k4_{prec}_1_step"] = sphere_rel_l2(x.cpu().numpy(), refs["t511"][None], bm.T)
        sdc.close()
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, 1, "fp64", W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH,
              implicit_coriolis=True)
    x = dev(x0)
    sdc.step(x, mb.dt)
    sdc.sync()
    out[f"{wl.name}_implicit_coriolis_fp64_1_step"] = sphere_rel_l2(x.cpu().numpy(), refs["implicit_coriolis"][None],
                                                                    mb.T)
    sdc.close()
    return out


# The paper's own single-node CPU results, context only (other hardware, the Galewsky workload,
# unstated precision): SWEET on one JUSUF node (Section 5.3; s/DoF/step converted to steps/s at the
# stated DoF counts) and ICON-O on one JUWELS node (Section 5.2); the model speedup of Section 4.7.
PAPER_CONTEXT = {
    "note": "CPU results of the paper, not targets: Galewsky test case, dSDC M=4 K=4 MIN-SR-FLEX",
    "SWEET_JUSUF": {
        "node": "2x AMD EPYC 7742 (128 cores, 2.25 GHz)",
        "dofs_256^2_(~T255)": {"dSDC_PinT_best_steps_per_s": 16.3, "dSDC_space_only_best": 12.2,
                                "dSDC_1_thread": 1.15, "IMEX_o2_best": 99.1, "PinT_speedup_4_threads": 2.60},
        "dofs_512^2_(~T511)": {"dSDC_PinT_best_steps_per_s": 4.0, "dSDC_space_only_best": 4.13,
                                "dSDC_1_thread": 0.189, "IMEX_o2_best": 34.9, "PinT_speedup_4_threads": 2.90},
    },
    "ICON-O_JUWELS": {"node": "2x Intel Xeon Platinum 8168 (48 cores, 2.7 GHz)",
                      "PinT_speedup_4_threads": 3.37, "model_S": 3.39},
    "model_S_SWEET": 3.25,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="t255_m4k4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="measure the plain FP64 path only")
    ap.add_argument("--no-work-precision", action="store_true",
                    help="skip the dSDC / IMEX-o2 work-precision comparison")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward+adjoint region (counter runs of the forward kernels)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a reference kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--plan", default=None, metavar="TILES,DEPTH,ANA_DEPTH,INTERLEAVE[,FUSE,SREC,AREC]",
                    help="set these Legendre launch variants instead of running the autotuner "
                         "(profiling runs that must launch the same kernels)")
    ap.add_argument("--plan1", default=None, metavar="TILES,DEPTH,ANA_DEPTH,INTERLEAVE[,FUSE,SREC,AREC]",
                    help="with --plan: the variants of the launches over one state per member")
    ap.add_argument("--no-extras", action="store_true",
                    help="measure the FP64 and FP32 steps only (no integrators, work-precision "
                         "study, equal-error check, ensemble or T511 runs): counter runs")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("STATS_CSV", "OUT_MD", "TITLE", "COMMAND"))
    ap.add_argument("--summarize-mfma", nargs=5,
                    metavar=("COUNTER_CSV", "STATS_CSV", "OUT_MD", "TITLE", "COMMAND"))
    ap.add_argument("--summarize-counters", nargs=6,
                    metavar=("COUNTER_CSV", "STATS_CSV", "OUT_MD", "TITLE", "COMMAND", "KERNEL_PREFIXES"))
    ap.add_argument("--summarize-pmc", nargs="+",
                    metavar="FETCH_CSV WRITE_CSV COPY_MIB OUT FETCH_LOG WRITE_LOG [COMMAND]")
    args = ap.parse_args()
    global FORCED_PLAN, FORCED_PLAN1
    if args.plan:
        FORCED_PLAN = tuple(int(v) for v in args.plan.split(","))
        FORCED_PLAN1 = tuple(int(v) for v in args.plan1.split(",")) if args.plan1 else None
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_pmc:
        if len(args.summarize_pmc) not in (6, 7):
            ap.error("--summarize-pmc takes FETCH_CSV WRITE_CSV COPY_MIB OUT FETCH_LOG WRITE_LOG [COMMAND]")
        f, w, mib, outp, flog, wlog = args.summarize_pmc[:6]
        cmd = args.summarize_pmc[6] if len(args.summarize_pmc) == 7 else None
        summarize_pmc(f, w, float(mib), outp, [flog, wlog], cmd)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the step on a single MI355X "
              "(sharding across GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    wl = W.WORKLOADS[args.workload]
    mb = wl.members[0]
    r64 = measure(wl, "fp64", args.steps, args.warmup, with_adjoint=not args.no_adjoint)
    kernels = r64["kernels"]
    dom = max(r64["kernel_ms"], key=lambda k: r64["kernel_ms"][k])
    d = kernels[dom]
    tr = traffic_for(dom, r64["plan"], r64["plan1"])
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                "frac": d["frac"], "traffic": tr, "kernel": dom, "avg_launch_us": d["avg_us"],
                "timed_over": "eager steps with per-launch HIP events on the library's stream"}
    result = {
        "metric": METRIC,
        "value": round(r64["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "T": mb.T, "nlat": mb.nlat, "nlon": mb.nlon, "M": wl.M,
                   "K": wl.K, "dt": mb.dt, "batch": 1, "precision": "fp64"},
        "steps_per_s_median_of_5": round(r64["repeats"][2], 3),
        "steps_per_s_range_of_5": [round(r64["repeats"][0], 3), round(r64["repeats"][-1], 3)],
        "eager_ms_per_step": round(r64["eager_ms_per_step"], 4),
        "fwd_adj_steps_per_s": round(r64["fwd_adj_steps_per_s"], 3) if "fwd_adj_steps_per_s" in r64 else None,
        "fwd_adj_ms_per_step": round(r64["fwd_adj_ms_per_step"], 4) if "fwd_adj_ms_per_step" in r64 else None,
        "fwd_adj_taped_steps_per_s": (round(r64["fwd_adj_taped_steps_per_s"], 3)
                                      if "fwd_adj_taped_steps_per_s" in r64 else None),
        "tape_bytes_per_step": r64.get("tape_bytes_per_step"),
        "roofline": roofline,
        "kernels": kernels,
        "legendre_plan": r64["plan"],
        "legendre_plan_one_state": r64["plan1"],
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_fp32:
        r32 = measure(wl, "fp32", args.steps, args.warmup)
        ee = None if args.no_extras else equal_error(wl)
        result["fp32"] = {
            "value": round(r32["steps_per_s"], 3), "unit": "steps/s",
            "dtype": "f32 Legendre contractions (FP32 MFMA, FP32 accumulation); f64 elsewhere",
            "ms_per_step": round(r32["ms_per_step"], 4),
            "fwd_adj_steps_per_s": round(r32["fwd_adj_steps_per_s"], 3),
            "fwd_adj_taped_steps_per_s": round(r32["fwd_adj_taped_steps_per_s"], 3),
            "speedup_vs_fp64": round(r32["steps_per_s"] / r64["steps_per_s"], 4),
            "fwd_adj_speedup_vs_fp64": round(r32["fwd_adj_steps_per_s"] / r64["fwd_adj_steps_per_s"], 4),
            "equal_error": ee,
            "kernels": r32["kernels"],
            "legendre_plan": r32["plan"],
            "legendre_plan_one_state": r32["plan1"],
        }
    if not args.no_fp32:
        r3 = measure(wl, "bf16x3", args.steps, args.warmup)
        result["bf16x3"] = {
            "value": round(r3["steps_per_s"], 3), "unit": "steps/s",
            "dtype": "bf16x3 Legendre contractions (FP32 operands split into three BF16 terms, BF16 MFMA "
                     "products, FP32 accumulation); f64 elsewhere",
            "ms_per_step": round(r3["ms_per_step"], 4),
            "fwd_adj_steps_per_s": round(r3["fwd_adj_steps_per_s"], 3),
            "fwd_adj_taped_steps_per_s": round(r3["fwd_adj_taped_steps_per_s"], 3),
            "speedup_vs_fp64": round(r3["steps_per_s"] / r64["steps_per_s"], 4),
            "fwd_adj_speedup_vs_fp64": round(r3["fwd_adj_steps_per_s"] / r64["fwd_adj_steps_per_s"], 4),
            "kernels": r3["kernels"],
            "legendre_plan": r3["plan"],
            "legendre_plan_one_state": r3["plan1"],
        }
    if not args.no_fp32 and not args.no_work_precision and not args.no_extras and args.workload == "t255_m4k4":
        result["integrators"] = integrators(wl)
        result["work_precision"] = work_precision(wl)
    if not args.no_fp32 and not args.no_extras and args.workload == "t255_m4k4":
        result["mixed32_m4k3"] = measure_mixed()
        big = W.WORKLOADS["t511_m4k4"]
        r511 = {p: measure(big, p, 20, 3, with_kernels=False) for p in ("fp64", "fp32", "bf16x3")}
        result["t511_m4k4"] = {
            "config": {"T": 511, "nlat": 768, "nlon": 1536, "M": 4, "K": 4, "dt": 60.0, "steps": 20},
            **{p: {"steps_per_s": round(r["steps_per_s"], 3),
                   "fwd_adj_steps_per_s": round(r["fwd_adj_steps_per_s"], 3),
                   "fwd_adj_taped_steps_per_s": round(r["fwd_adj_taped_steps_per_s"], 3),
                   "legendre_plan": r["plan"], "legendre_plan_one_state": r["plan1"]}
                for p, r in r511.items()}}
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["calibration_copy_bytes"] = 2 * src.numel() * 8      # read + write
    if not args.no_cpu_baseline:
        base, refs = cpu_baseline(wl, W.initial_state(wl))
        result["cpu_baseline"] = base
        if "vjp" in refs:
            result["err_vs_oracle"] = oracle_errors(wl, refs)
    print(json.dumps(result))


if __name__ == "__main__":
    main()

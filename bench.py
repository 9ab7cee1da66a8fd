#!/usr/bin/env python
"""Benchmark: dSDC steps/s of the T255, M=4, K=4 shallow-water workload on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload t255_m4k4] [--no-cpu-baseline]

Prints ONE JSON line.  The timed region is exactly K steps (after W warm-up steps and one graph
capture) of the HIP library on synthetic seeded fields already resident in device memory,
bracketed by torch.cuda.synchronize(); each step is one replay of the step's captured hipGraph.
A second region of K eager steps of the same kernels brackets every launch with HIP events on the
library's stream; the dominant kernel class (largest summed time) is reported against its
roofline from algorithmic work per launch (flops of the useful Legendre contractions with
equatorial symmetry, or minimal HBM bytes of the grid/update kernels).  A third region times K
forward steps with one checkpoint each followed by K adjoint steps (forward+adjoint steps/s).
The CPU baseline is the FP64 oracle timed on this machine's host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "SDC steps/s (fwd, fwd+adjoint) at T255 M=4 vs plain FP64 GPU at equal error"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK = {"fp64": PEAK_FP64_TFLOPS, "fp32": 157.3, "bf16x3": 2500.0}


def algorithmic_work(T, nlat, M, K, batch):
    """Algorithmic work of every kernel class over one step.

    Legendre (flops): one scalar-equivalent complex transform with equatorial symmetry costs
    2*ncoef*nlat flops; synthesis does 6 per state (zeta, Phi', psi and chi with Pbar, psi and
    chi with H), analysis 7 (div/curl pairs of (A,B), (C,D), and KE).
    Grid (bytes): reads 4 Fourier fields and writes 5 (minimal), nlat*(T+1) complex each per state.
    Update (bytes): per coefficient and member, reads u_n (3 complex), per node j the Phi',
    delta of u_j (2) and E_j (3), writes the updated nodes (3 each) and their synthesis-layout
    copy (4 each: zeta, Phi', psi, chi); the last sweep writes node M only; the first f_E of a
    step converts u_n to the synthesis layout (reads 3, writes 4).
    """
    ncoef = (T + 1) * (T + 2) // 2
    transform = 2.0 * ncoef * nlat
    states = batch * (1 + (K - 1) * M)          # states transformed per step
    syn_flops = 6 * transform * states
    ana_flops = 7 * transform * states
    grid_bytes = 9.0 * nlat * (T + 1) * 16 * states
    upd_bytes = batch * ncoef * 16.0 * ((K - 1) * (3 + 12 * M) + (3 + 5 * M + 3) + 7)
    return {"synthesis": ("flops", syn_flops), "analysis": ("flops", ana_flops),
            "grid": ("bytes", grid_bytes), "update": ("bytes", upd_bytes)}


def cpu_baseline(wl, state0, budget_s=15.0):
    import torch
    from oracle.sdc import Oracle
    mb = wl.members[0]
    o = Oracle(mb.T, mb.nlat, mb.nlon, W.RADIUS, W.GRAVITY, W.OMEGA, W.MEAN_DEPTH)
    t0 = time.perf_counter()
    x = o.step(state0, mb.dt, wl.M, wl.K, steps=1)
    t1 = time.perf_counter() - t0
    n = max(1, min(20, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    o.step(x, mb.dt, wl.M, wl.K, steps=n)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{n} dSDC steps of {wl.name} (T{mb.T} {mb.nlat}x{mb.nlon}, M={wl.M}, K={wl.K}) "
                      f"after 1 untimed step, torch-CPU float64 oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="t255_m4k4")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (a reference kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the step on a single MI355X "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2403_20135_amd.api import SDC

    wl = W.WORKLOADS[args.workload]
    mb = wl.members[0]
    batch = 1
    sdc = SDC(mb.T, mb.nlat, mb.nlon, wl.M, wl.K, batch, args.precision, W.RADIUS, W.GRAVITY,
              W.OMEGA, W.MEAN_DEPTH)
    state0 = W.initial_state(wl)
    x = torch.tensor(state0[None], dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        sdc.step(x, mb.dt)
    sdc.sync()

    # timed region: K steps, each one replay of the step's captured hipGraph
    sdc.step_graph(x, mb.dt)                          # capture (untimed)
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sdc.step_graph(x, mb.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sdc.sync()

    # per-kernel HIP events (on the library's stream) over K eager steps of the same kernels
    sdc.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sdc.step(x, mb.dt)
    torch.cuda.synchronize()
    elapsed_eager = time.perf_counter() - t0
    sdc.sync()
    kt = sdc.timing_read()
    sdc.timing(False)

    work = algorithmic_work(mb.T, mb.nlat, wl.M, wl.K, batch)
    kernels = {}
    for name, (ms, launches) in kt.items():
        kind, per_step = work[name]
        total = per_step * args.steps
        secs = ms / 1e3
        if kind == "flops":
            ach, unit, peak, bound = total / secs / 1e12, "TFLOP/s", PEAK[args.precision], "mfma"
        else:
            ach, unit, peak, bound = total / secs / 1e9, "GB/s", PEAK_HBM_GBS, "hbm"
        kernels[name] = {"ms_total": round(ms, 3), "launches": launches,
                         "avg_us": round(ms * 1e3 / max(launches, 1), 2),
                         "achieved": round(ach, 3), "unit": unit, "peak": peak, "bound": bound,
                         "frac": round(ach / peak, 4),
                         "algorithmic_per_launch": total / max(launches, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    d = kernels[dom]
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                "frac": d["frac"], "traffic": None, "kernel": dom,
                "avg_launch_us": d["avg_us"], "timed_over": "eager steps with per-launch HIP events"}

    # forward + adjoint: every forward step keeps its input (one checkpoint per step), then the
    # adjoint steps run in reverse, each recomputing its step's stages from the checkpoint
    ckpt = torch.empty((args.steps,) + tuple(x.shape), dtype=torch.float64, device="cuda")
    lam = torch.ones_like(x)
    lam_out = torch.empty_like(x)
    sdc.step_adjoint(x, lam, lam_out, mb.dt)          # allocates the adjoint workspaces once
    sdc.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ckpt[k].copy_(x)
        sdc.step(x, mb.dt)
    for k in range(args.steps - 1, -1, -1):
        sdc.step_adjoint(ckpt[k], lam, lam, mb.dt)
    torch.cuda.synchronize()
    elapsed_fa = time.perf_counter() - t0
    sdc.sync()
    if not bool(torch.isfinite(lam).all()):
        raise RuntimeError("non-finite adjoint")
    del ckpt

    steps_s = args.steps / elapsed
    result = {
        "metric": METRIC,
        "value": round(steps_s, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "eager_ms_per_step": round(elapsed_eager / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {"workload": wl.name, "T": mb.T, "nlat": mb.nlat, "nlon": mb.nlon, "M": wl.M,
                   "K": wl.K, "dt": mb.dt, "batch": batch, "precision": args.precision},
        "fwd_adj_steps_per_s": round(args.steps / elapsed_fa, 3),
        "fwd_adj_ms_per_step": round(elapsed_fa / args.steps * 1e3, 4),
        "roofline": roofline,
        "kernels": kernels,
    }
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["calibration_copy_bytes"] = 2 * src.numel() * 8      # read + write
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, state0)
    if not np.all(np.isfinite(x.cpu().numpy())):
        raise RuntimeError("non-finite state after the timed steps")
    print(json.dumps(result))


if __name__ == "__main__":
    main()

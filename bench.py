#!/usr/bin/env python3
"""Throughput of the micropolar FFT-based solver on one MI355X.

Workload: the 128^3 random-sphere cell in FP64 (40 non-overlapping elastic
spheres, radii U[6, 12] voxels, contrast 10, E11 -> 0.02 with curvature
Gamma12 -> 0.002 over 50 steps, tolerance 1e-8, Eq. 38 error measure).
A bench step is one load step of Alg. 2: the first iterate, every
fixed-point iteration until convergence, and the commit.  W warm-up steps
(load steps 1..W) are run first, then K timed steps (W+1..W+K).

Prints one JSON line: value = voxel-iterations/s over the timed steps (inputs
resident in HBM), the roofline of the dominant kernel (timed live with HIP
events on the library's stream), and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

# algorithmic HBM bytes per voxel per launch, FP64 (8-byte words)
#   x pass : read 18 half spectra (18 w), e/gamma old (18 w), history base
#            (18 w), p_n, q_n (2 x 8 B), phase id (1 B); write e/gamma (18 w)
#            and 18 half spectra (18 w)
#   y passes, fused z pass (z forward + Green operator + z inverse):
#            read + write 18 half spectra (36 w)
BYTES_PER_VOXEL = {
    "x_pass": 90 * 8 + 16 + 1,
    "y_fwd": 36 * 8, "z_green": 36 * 8, "y_inv": 36 * 8,
    "err_reduce": 0,
}
BYTES_PER_VOXEL_ITER = sum(BYTES_PER_VOXEL.values())


def cpu_baseline(wl, iters=2):
    """The oracle, untuned, on a bounded sample: load step 1 of the same cell
    with a fixed schedule of `iters` loop iterations (setup excluded)."""
    from threadpoolctl import threadpool_limits
    from oracle import micropolar as O
    with threadpool_limits(limits=1):
        solver = O.Solver(wl.phase_map, wl.phases, h=wl.h, tol=wl.tol, norm=wl.err_norm)
        t0 = time.perf_counter()
        solver.solve(wl.times[:2], wl.E[:1], wl.G[:1], schedule=[iters])
        dt = time.perf_counter() - t0
    nvox = wl.phase_map.size
    return {"value": iters * nvox / dt, "unit": "voxel-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"load step 1 of the same 128^3 cell, {iters} fixed-point iterations "
                      f"(plus the first iterate and commit), {dt:.1f} s wall, 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_10774_amd import mp, workloads as W

    W_, K = args.warmup, args.steps
    wl = W.random_spheres_128(n_steps=W_ + K)
    nvox = wl.phase_map.size
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol)
    print(f"# workload {wl.name}: {wl.info}, warmup {W_} step(s), timed {K}", file=sys.stderr,
          flush=True)
    if W_ > 0:
        it_w = plan.solve(wl.times[: W_ + 1], wl.E[:W_], wl.G[:W_])
        print(f"# warmup iterations {it_w}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    plan.profile(not args.no_profile)
    t0 = time.perf_counter()
    iters = plan.solve(wl.times[W_: W_ + K + 1], wl.E[W_: W_ + K], wl.G[W_: W_ + K])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    print(f"# timed iterations {iters}, {dt:.3f} s", file=sys.stderr, flush=True)
    value = sum(iters) * nvox / dt

    kernels = {}
    for k, (ms, n) in prof.items():
        if n:
            avg = ms / n
            b = BYTES_PER_VOXEL[k] * nvox
            kernels[k] = {"avg_ms": round(avg, 4), "launches": n, "share": None,
                          "GBps": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
    tot = sum(prof[k][0] for k in prof)
    roof = None
    if kernels:
        for k in kernels:
            kernels[k]["share"] = round(prof[k][0] / tot, 4)
        dom = max(kernels, key=lambda k: prof[k][0])
        avg = kernels[dom]["avg_ms"] * 1e-3
        achieved = BYTES_PER_VOXEL[dom] * nvox / avg / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": BYTES_PER_VOXEL[dom] * nvox}

    line = {
        "metric": "voxel-iterations/s",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W_,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random-sphere microstructure)",
        "config": {"workload": "spheres128_fp64: 128^3 voxels, 40 random elastic spheres r~U[6,12], "
                               "contrast 10, E11->0.02 + Gamma12->0.002 over 50 steps, tol 1e-8 (Eq. 38)",
                   "timed_load_steps": [W_ + 1, W_ + K], "iterations": iters,
                   "parallelism": "single GPU"},
        "iteration_hbm_frac": round(BYTES_PER_VOXEL_ITER * value / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(wl),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

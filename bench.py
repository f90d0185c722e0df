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

# HBM bytes per voxel per launch that this design moves (w = bytes per bulk
# word: 8 FP64, 4 mixed; the strain state and p_n, q_n are FP64 in both)
#   x pass : read 18 half spectra (18 w), e/gamma old (18 x 8 B), history
#            base (18 w), p_n, q_n (2 x 8 B), phase id (1 B); write e/gamma
#            (18 x 8 B) and 18 half spectra (18 w); the stresses of the old
#            iterate are recomputed, not stored
#   y passes, fused z pass (z forward + Green operator + z inverse):
#            read + write 18 half spectra (36 w)
def bytes_per_voxel(w):
    return {"x_pass": 54 * w + 36 * 8 + 16 + 1, "y_fwd": 36 * w, "z_green": 36 * w, "y_inv": 36 * w,
            "err_reduce": 0}


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by a 1 GiB copy calibration: x2.000 and x1.000), valid
# only for the kernel sources they were taken on (SHA-1 of the two headers)
MEASURED_TRAFFIC = {
    "spheres128_fp64": {"kernel": "x_pass", "bytes": (941.9 + 619.7) * 1e6,
                        "src_sha1": "77dc9aeb6cc33d85a046e0fb0c06bf19e2851704"},
    "spheres256_mixed": {"kernel": "x_pass", "bytes": (5117.3 + 3687.2) * 1e6,
                         "src_sha1": "77dc9aeb6cc33d85a046e0fb0c06bf19e2851704"},
    "spheres256_fp64": {"kernel": "x_pass", "bytes": (7533.2 + 4897.1) * 1e6,
                        "src_sha1": "77dc9aeb6cc33d85a046e0fb0c06bf19e2851704"},
    "aniso128_fp64": {"kernel": "x_pass", "bytes": (942.1 + 619.7) * 1e6,
                      "src_sha1": "77dc9aeb6cc33d85a046e0fb0c06bf19e2851704"},
}


def algorithmic_x_bytes(w):
    """Algorithmic bytes per voxel of the x pass, the unit figure the
    roofline line reports: the half spectra, the strain state and the
    stresses read and written, the history base (126 w), p_n, q_n (16 B) and
    the phase id (1 B) -- the traffic of a pass that stores the stresses of
    the old iterate instead of recomputing them (1025 B FP64, 521 B mixed)."""
    return 126 * w + 16 + 1


def algorithmic_bytes_per_voxel(w):
    """The same model over one whole iteration: x pass plus three axis passes
    of 36 w (1889 B FP64, 953 B mixed)."""
    return {"x_pass": algorithmic_x_bytes(w), "y_fwd": 36 * w, "z_green": 36 * w, "y_inv": 36 * w, "err_reduce": 0}


def kernel_src_sha1():
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2409_10774_amd", "csrc")
    h = hashlib.sha1()
    for f in ("kernels.hpp", "device_math.hpp"):
        h.update(open(os.path.join(here, f), "rb").read())
    return h.hexdigest()


WORKLOADS = {
    "spheres128_fp64": dict(
        precision="fp64", dtype="f64",
        desc="spheres128_fp64: 128^3 voxels, 40 random elastic spheres r~U[6,12], contrast 10, "
             "E11->0.02 + Gamma12->0.002 over 50 steps, tol 1e-8 (Eq. 38)"),
    "spheres256_mixed": dict(
        precision="mixed", dtype="f32 bulk / f64 reductions",
        desc="spheres256_mixed: 256^3 voxels, random elastic spheres r~U[5,15] to volume fraction "
             "0.25, contrast 10, E11->0.01 over 20 steps, tol 1e-6 (Eq. 38), FP32 bulk arithmetic"),
    "spheres256_fp64": dict(
        precision="fp64", dtype="f64",
        desc="spheres256_fp64: the 256^3 cell of spheres256_mixed in FP64 (the reference of the "
             "mixed form), tol 1e-6 (Eq. 38)"),
    "aniso128_fp64": dict(
        precision="fp64", dtype="f64",
        desc="aniso128_fp64: the 128^3 cell of spheres128_fp64 with Eq. 5 anisotropic spheres "
             "(general tensors, mean eigenvalues 17 and 50) and the unweighted mean of the phases' "
             "tensors as reference medium (per-frequency factored Green operator); same load path"),
    "batch64_mixed": dict(
        precision="mixed", dtype="f32 bulk / f64 reductions",
        desc="batch64_mixed: 64 resident RVEs, edge U{32,64,96,128}, 1-60 spheres r~U[n/20,n/10], "
             "contrast U[2,20], l~U[0.5,4], tY~U[0.003,0.01], random symmetric strain to norm 0.01 "
             "over 20 steps, tol 1e-6, one batch, graph-captured iterations"),
    "serve_mixed": dict(
        precision="mixed", dtype="f32 bulk / f64 reductions",
        desc="serve_mixed: Poisson request trace, edge {32,64,128,256} with weights .4/.3/.2/.1, "
             "10-40 steps per request, continuous batching (mixed) against sequential FP64 plans"),
}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, iters=4):
    """The oracle, untuned, on a bounded sample: load step 1 of the same cell
    with a fixed schedule of `iters` loop iterations (one above 128^3), setup
    excluded; once with one thread, once with every host thread allowed to
    the numeric libraries (numpy's FFT itself stays on one thread)."""
    nvox = wl.phase_map.size
    if nvox > 128 ** 3:
        iters = 1
    from threadpoolctl import threadpool_limits
    from oracle import micropolar as O
    nproc = os.cpu_count() or 1

    def timed(threads):
        with threadpool_limits(limits=threads):
            solver = O.Solver(wl.phase_map, wl.phases, h=wl.h, tol=wl.tol, norm=wl.err_norm,
                              ref_mode=wl.ref_mode)
            t0 = time.perf_counter()
            solver.solve(wl.times[:2], wl.E[:1], wl.G[:1], schedule=[iters])
            return time.perf_counter() - t0

    dt = timed(1)
    dt_all = timed(nproc)
    return {"value": iters * nvox / dt, "unit": "voxel-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"load step 1 of the same cell, {iters} fixed-point iteration(s) "
                      f"(plus the first iterate and commit), {dt:.1f} s wall, 1 thread",
            "all_threads": {"value": iters * nvox / dt_all, "threads_allowed": nproc,
                            "seconds": round(dt_all, 2)},
            "nproc": nproc, "cpu_model": cpu_model()}


def field_errors(torch, a, b):
    """max_x |a - b| / max_x |b| per field (Frobenius norm over the nine
    components of a tensor field), on the device."""
    out = {}
    for k in a:
        x, y = a[k], b[k]
        if x.dim() == 4:
            d = ((x - y) ** 2).sum(0).sqrt().max()
            r = (y ** 2).sum(0).sqrt().max()
        else:
            d, r = (x - y).abs().max(), y.abs().max()
        out[k] = float(d / r) if float(r) > 0 else float(d)
    return out


def curve_errors(a, b, fields_ref):
    """Per-component relative error of the response columns whose average
    reaches 1 % of its field's scale, and the error of the smaller averages on
    their field's scale (columns: <t>, <m>, <e>, <gamma>, <p>, <q>, <t_eq>,
    <m_eq>)."""
    groups = [(range(0, 9), "t"), (range(9, 18), "m"), (range(18, 27), "e"), (range(27, 36), "g"),
              ([36], "p"), ([37], "q"), ([38], "t"), ([39], "m")]
    big = small = 0.0
    for cols, name in groups:
        scale = float(fields_ref[name].abs().max())
        if scale == 0:
            continue
        for c in cols:
            d = float(np.abs(a[:, c] - b[:, c]).max())
            ref = float(np.abs(b[:, c]).max())
            if ref >= 1e-2 * scale:
                big = max(big, d / ref)
            else:
                small = max(small, d / scale)
    return big, small


def extra_mixed256(torch, mp, W, steps=2):
    """The 256^3 cell, its first load steps solved in the mixed form and in
    FP64, each converged at tolerance 1e-6 on its own schedule: iterations,
    throughput, the error of every mixed result against FP64, and the x pass
    of both against the HBM roofline (this grid's spectra do not fit in the
    Infinity Cache)."""
    wl = W.random_spheres_256(n_steps=steps)
    nvox = wl.phase_map.size
    res = {}
    for prec in ("mixed", "fp64"):
        plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision=prec)
        plan.profile(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = plan.solve(wl.times, wl.E, wl.G)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, n = plan.profile_read()["x_pass"]
        x_ms = ms / n
        w = 4 if prec == "mixed" else 8
        x_bytes = algorithmic_x_bytes(w) * nvox
        res[prec] = dict(iters=it, seconds=dt, fields=plan.fields(device=True), resp=plan.responses()[:, :40],
                         final_err=[float(plan.responses()[s][40]) for s in range(steps)],
                         reserved=[float(plan.error_parts(s + 1)[4]) for s in range(steps)],
                         x=dict(avg_ms=round(x_ms, 4), achieved_GBps=round(x_bytes / x_ms / 1e6, 1),
                                frac=round(x_bytes / x_ms / 1e6 / HBM_PEAK_GBS, 4)))
        plan.close()
        print(f"# 256^3 {prec}: iterations {it}, {dt:.2f} s, x pass {x_ms:.3f} ms", file=sys.stderr, flush=True)
    m, d = res["mixed"], res["fp64"]
    ferr = field_errors(torch, m["fields"], d["fields"])
    big, small = curve_errors(m["resp"], d["resp"], d["fields"])
    del m["fields"], d["fields"]
    torch.cuda.empty_cache()
    out = {"workload": WORKLOADS["spheres256_mixed"]["desc"] + f", load steps 1-{steps}", "tol": wl.tol}
    for k, r in res.items():
        out[k] = {"iterations": r["iters"], "seconds": round(r["seconds"], 3),
                  "voxel_iterations_per_s": sum(r["iters"]) * nvox / r["seconds"],
                  "final_error_measure": r["final_err"], "floor_stop": r["reserved"],
                  "x_pass_roofline": r["x"]}
    out["mixed_vs_fp64"] = {"field_rel": {k: float("%.3g" % v) for k, v in ferr.items()},
                            "curve_rel_per_component": float("%.3g" % big),
                            "small_averages_rel_field_scale": float("%.3g" % small),
                            "solve_speedup": round(res["fp64"]["seconds"] / res["mixed"]["seconds"], 3)}
    return out


def extra_batch8(torch, mp, W, n_rves=8, n_steps=5):
    """The first RVEs of the many-RVE workload (edges 32-128, contrast 2-20,
    mixed, tolerance 1e-6), on shorter load paths: one resident batch against
    the same RVEs solved one after another with FP64 plans."""
    rves = W.batch_rves(seed=3, count=64, n_steps=n_steps)[:n_rves]
    shapes = sorted({w.phase_map.shape[::-1] for w in rves})
    probe = mp.Batch(shapes, arena_bytes=64 << 20, precision="mixed", max_rves=4, autotune=False)
    need = sum(probe.footprint(w.phase_map, w.phases, len(w.E), tol=w.tol) for w in rves)
    probe.close()
    B = mp.Batch(shapes, arena_bytes=need + (1 << 30), precision="mixed", max_rves=16, iters_per_launch=8,
                 autotune=True)
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in rves]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches = B.drain()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = [B.query(i) for i in ids]
    B.close()
    t1 = time.perf_counter()
    seq_its = []
    for w in rves:
        plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, precision="fp64")
        seq_its.append(sum(plan.solve(w.times, w.E, w.G, raise_on_error=False)[1]))
        plan.close()
    torch.cuda.synchronize()
    d1 = time.perf_counter() - t1
    print(f"# batch of {n_rves}: {dt:.2f} s batched mixed, {d1:.2f} s sequential FP64", file=sys.stderr, flush=True)
    return {"rves": n_rves, "load_steps": n_steps, "edges": [int(w.phase_map.shape[0]) for w in rves],
            "batched_mixed": {"seconds": round(dt, 3), "rve_solves_per_s": n_rves / dt, "graph_launches": launches,
                              "iterations": [int(x[3]) for x in q], "statuses": [int(x[1]) for x in q]},
            "sequential_fp64": {"seconds": round(d1, 3), "rve_solves_per_s": n_rves / d1,
                                "iterations": seq_its},
            "speedup": round(d1 / dt, 3)}


def extra_ratchet(torch, mp, W, steps=1000):
    """The Sec. 3.2 ratcheting path (4^3 Tab. 2 laminate, ten cycles of 100
    steps of 0.01 s) on one FP64 plan: a small cell, whose steps run the
    one-block loop.  A first plan over 20 steps warms the kernels up."""
    w = W.ratchet_laminate(cycles=10)
    warm = mp.Plan(w.phase_map, w.phases, h=w.h, tol=w.tol)
    warm.solve(w.times[:21], w.E[:20], w.G[:20])
    warm.close()
    plan = mp.Plan(w.phase_map, w.phases, h=w.h, tol=w.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = plan.solve(w.times[: steps + 1], w.E[:steps], w.G[:steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = plan.responses()[:, 37]
    plan.close()
    return {"steps": steps, "seconds": round(dt, 4), "iterations": int(sum(it)), "steps_per_s": round(steps / dt, 1),
            "iterations_per_s": round(sum(it) / dt, 1), "Q_end": float(q[-1])}


def run_sweep(torch, mp, W, n=10, precision="mixed"):
    """The Sec. 3.3 length-scale study as batched dataset generation: an n x n
    sweep of the elastic and plastic lengths over [0.1, 1] on the 16^3
    four-sphere cell (100 load steps each), every cell an RVE of one resident
    batch, drained to completion."""
    vals = np.linspace(0.1, 1.0, n)
    cells = [W.length_scale_rve(le, lp) for le in vals for lp in vals]
    shape = cells[0].phase_map.shape[::-1]
    B = mp.Batch([shape], arena_bytes=2 << 30, precision=precision, max_rves=len(cells))
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, h=w.h) for w in cells]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches = B.drain()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = [B.query(i) for i in ids]
    B.close()
    its = [int(x[3]) for x in q]
    nvox = int(cells[0].phase_map.size)
    return {"workload": f"length-scale sweep: {n} x {n} cells (l_e, l_p in [0.1, 1]), 16^3 four spheres, "
                        f"100 load steps each, {precision}, one resident batch",
            "rves": len(cells), "seconds": round(dt, 3), "rve_solves_per_s": round(len(cells) / dt, 2),
            "voxel_iterations_per_s": sum(its) * nvox / dt, "graph_launches": int(launches),
            "iterations_total": sum(its), "iterations_max": max(its), "iterations_median": float(np.median(its)),
            "statuses": sorted({int(x[1]) for x in q})}


def extra_serve(torch, mp, W, n=8):
    """A short Poisson trace of the serving workload (edges 32-128 only, 10-12
    load steps): the closed-loop saturation of continuous batching, then the
    trace at 0.8x that rate through continuous batching (mixed) and through
    sequential FP64 plans, with p50 / p99 latency including the replies."""
    base = W.serve_trace(seed=4, n_req=n, rate=1.0, sizes=(32, 64, 128), weights=(0.5, 0.3, 0.2), steps=(10, 12))
    wls = [w for _, w in base]
    shapes = sorted({w.phase_map.shape[::-1] for w in wls})

    def items(arr):
        return [(a, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol)) for a, w in zip(arr, wls)]

    B = mp.Batch(shapes, arena_bytes=8 << 30, precision="mixed", max_rves=64, iters_per_launch=8, autotune=True)
    _, td, _, _ = mp.serve_batched(B, mp.Requests(items(np.zeros(n)), "mixed"))
    rate = 0.8 * n / float(td.max())
    gaps = np.random.default_rng(4).exponential(1.0 / rate, size=n)
    arr = np.cumsum(gaps) - gaps[0]
    _, td2, st2, _ = mp.serve_batched(B, mp.Requests(items(arr), "mixed"))
    B.close()
    ws = torch.empty(2 << 30, dtype=torch.uint8, device="cuda:0")
    _, td3, st3, _ = mp.serve_sequential(mp.Requests(items(arr), "fp64"), ws)
    del ws
    torch.cuda.empty_cache()

    def lat(done):
        L = np.asarray(done) - arr
        return {"p50_s": round(float(np.percentile(L, 50)), 3), "p99_s": round(float(np.percentile(L, 99)), 3),
                "makespan_s": round(float(np.max(done)), 3)}

    print(f"# serving {n} requests at {rate:.3f}/s", file=sys.stderr, flush=True)
    return {"requests": n, "edges": [int(w.phase_map.shape[0]) for w in wls], "closed_loop_requests_per_s": n / float(td.max()),
            "arrival_rate_per_s": rate, "batched_mixed": dict(lat(td2), statuses=sorted({int(v) for v in st2})),
            "sequential_fp64": dict(lat(td3), statuses=sorted({int(v) for v in st3}))}


def run_batch(args, torch, mp, W):
    """Many-RVE batch: every RVE admitted at once, drained; against the same
    RVEs solved one after another with FP64 plans (first --seq-rves of them)."""
    rves = W.batch_rves(seed=3, count=args.rves)
    shapes = sorted({w.phase_map.shape[::-1] for w in rves})
    probe = mp.Batch(shapes, arena_bytes=64 << 20, precision="mixed", max_rves=4, autotune=False)
    need = sum(probe.footprint(w.phase_map, w.phases, len(w.E), tol=w.tol) for w in rves)
    probe.close()
    print(f"# {len(rves)} RVEs, {sum(w.phase_map.size for w in rves) / 1e6:.1f} M voxels, "
          f"arena {need / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    B = mp.Batch(shapes, arena_bytes=need + (2 << 30), precision="mixed", max_rves=max(64, len(rves)),
                 iters_per_launch=args.iters_per_launch, autotune=True)
    sched = {"x".join(map(str, sh)): B.schedule(c) for c, sh in enumerate(shapes)}
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol) for w in rves]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    active, launches = len(ids), 0
    while active:
        active = B.run()
        launches += 1
        if launches % 25 == 0:
            print(f"# launches {launches}, active {active}, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = [B.query(i) for i in ids]
    vox_it = sum(qq[3] * w.phase_map.size for qq, w in zip(q, rves))
    statuses = [qq[1] for qq in q]
    B.close()
    seq = None
    if args.seq_rves:
        sub = rves[: args.seq_rves]
        t1 = time.perf_counter()
        its = 0
        for w in sub:
            plan = mp.Plan(w.phase_map, w.phases, tol=w.tol, precision="fp64")
            it = plan.solve(w.times, w.E, w.G, raise_on_error=False)[1]
            its += sum(it) * w.phase_map.size
            plan.close()
            print(f"# sequential fp64 rve {w.name}: {sum(it)} iterations", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        d1 = time.perf_counter() - t1
        seq = {"rves": len(sub), "seconds": round(d1, 3), "rve_solves_per_s": len(sub) / d1,
               "voxel_iterations_per_s": its / d1}
    return {
        "metric": "voxel-iterations/s", "value": vox_it / dt, "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 bulk / f64 reductions",
        "data": "synthetic (seeded random-sphere RVEs)",
        "config": {"workload": WORKLOADS["batch64_mixed"]["desc"], "rves": len(rves),
                   "voxels": int(sum(w.phase_map.size for w in rves)),
                   "iters_per_launch": args.iters_per_launch, "graph_launches": launches,
                   "parallelism": "single GPU"},
        "rve_solves_per_s": len(rves) / dt,
        "statuses": {str(k): statuses.count(k) for k in sorted(set(statuses))},
        "schedules": sched,
        "sequential_fp64": seq,
    }


def run_serve(args, torch, mp, W):
    """Poisson trace: closed-loop saturation of the batched server, then the
    open-loop trace at 0.8x that rate through continuous batching (mixed) and
    through sequential FP64 plans."""
    n = args.requests
    base = W.serve_trace(seed=4, n_req=n, rate=1.0)
    wls = [w for _, w in base]
    shapes = sorted({w.phase_map.shape[::-1] for w in wls})
    arena = args.arena_gib << 30

    def items(arrivals):
        return [(a, w.phase_map, w.phases, w.times, w.E, w.G, dict(tol=w.tol)) for a, w in zip(arrivals, wls)]

    def lat(arr, done):
        L = np.asarray(done) - np.asarray(arr)
        return {"p50_s": float(np.percentile(L, 50)), "p99_s": float(np.percentile(L, 99)),
                "mean_s": float(L.mean())}

    vox = np.array([w.phase_map.size for w in wls])
    closed = batched = sequential = None
    if args.servers == "none" and args.serve_rate > 0:
        raise SystemExit("--servers none runs the closed loop only; it takes no --serve-rate")
    if args.serve_rate > 0:
        # the open-loop rate of an earlier closed-loop run: the same trace again
        rate = args.serve_rate
    else:
        B = mp.Batch(shapes, arena_bytes=arena, precision="mixed", max_rves=256,
                     iters_per_launch=args.iters_per_launch, autotune=True)
        print(f"# closed loop: {n} requests at t = 0", file=sys.stderr, flush=True)
        ta, td, st, it = mp.serve_batched(B, mp.Requests(items(np.zeros(n)), "mixed"), progress_s=20.0)
        B.close()
        del B
        torch.cuda.empty_cache()
        makespan = float(td.max())
        sat = n / makespan
        rate = 0.8 * sat
        closed = {"requests_per_s": sat, "makespan_s": makespan,
                  "voxel_iterations_per_s": float((it * vox).sum()) / makespan}
    gaps = np.random.default_rng(4).exponential(1.0 / rate, size=n)
    arr = np.cumsum(gaps) - gaps[0]
    if args.servers in ("both", "batched"):
        print(f"# open loop at {rate:.4f} req/s, continuous batching", file=sys.stderr, flush=True)
        B = mp.Batch(shapes, arena_bytes=arena, precision="mixed", max_rves=256,
                     iters_per_launch=args.iters_per_launch, autotune=True)
        ta2, td2, st2, it2 = mp.serve_batched(B, mp.Requests(items(arr), "mixed"), progress_s=20.0)
        B.close()
        del B
        torch.cuda.empty_cache()
        batched = dict(lat(arr, td2), makespan_s=float(td2.max()), statuses=[int(v) for v in set(st2)],
                       voxel_iterations_per_s=float((it2 * vox).sum()) / float(td2.max()))
    if args.servers in ("both", "sequential"):
        print(f"# open loop at {rate:.4f} req/s, sequential fp64", file=sys.stderr, flush=True)
        ws = torch.empty(arena, dtype=torch.uint8, device="cuda:0")
        ts3, td3, st3, it3 = mp.serve_sequential(mp.Requests(items(arr), "fp64"), ws, progress_s=20.0)
        sequential = dict(lat(arr, td3), makespan_s=float(td3.max()), statuses=[int(v) for v in set(st3)],
                          voxel_iterations_per_s=float((it3 * vox).sum()) / float(td3.max()))
    head = batched or sequential or {"makespan_s": closed["makespan_s"]}
    return {
        "metric": "requests/s", "value": n / head["makespan_s"], "unit": "requests/s", "n_gpus": 1,
        "steps": n, "warmup": 0, "ms_per_step": head["makespan_s"] / n * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if sequential and not batched else "f32 bulk / f64 reductions",
        "data": "synthetic (seeded Poisson trace of random-sphere RVEs)",
        "config": {"workload": WORKLOADS["serve_mixed"]["desc"], "requests": n,
                   "arrival_rate_per_s": rate, "iters_per_launch": args.iters_per_launch,
                   "arena_gib": args.arena_gib, "servers": args.servers,
                   "parallelism": "single GPU"},
        "closed_loop": closed,
        "batched_mixed": batched,
        "sequential_fp64": sequential,
    }


def run_green_ab(torch, mp, W):
    """The Green operator stored per frequency (Sec. 2.4) against computed
    per frequency, on cubic RVEs of the many-RVE workload's kind (32^3 to
    256^3), FP64 and mixed, on a fixed schedule: the z pass (forward z
    transform, Green operator, inverse z transform) from HIP events between
    the loop kernels, and the whole loop iteration from the wall clock
    without events.  The stored table adds 21 words per frequency to the z
    pass's 72 (the spectrum read and written)."""
    rows = []
    for n, iters in ((32, 200), (64, 100), (128, 40), (256, 12)):
        wl = W.random_rve(seed=5, n=n, n_steps=3)
        for prec in ("fp64", "mixed"):
            w = 8 if prec == "fp64" else 4
            row = {"n": n, "precision": prec}
            for green in ("computed", "stored"):
                plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision=prec, green=green)
                plan.set_fixed_iterations(iters)
                plan.solve(wl.times[:2], wl.E[:1], wl.G[:1])        # warm-up step
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan.solve(wl.times[1:3], wl.E[1:2], wl.G[1:2])
                torch.cuda.synchronize()
                it_ms = (time.perf_counter() - t0) / iters * 1e3
                plan.profile(1)
                plan.solve(wl.times[2:4], wl.E[2:3], wl.G[2:3])
                ms, k = plan.profile_read()["z_green"]
                plan.close()
                z_ms = ms / k
                zb = (72 + (21 if green == "stored" else 0)) * w * (n // 2) * n * n
                row[green] = {"z_pass_ms": round(z_ms, 5), "z_pass_GBps": round(zb / z_ms / 1e6, 1),
                              "iteration_ms": round(it_ms, 5)}
            row["stored_over_computed"] = {"z_pass": round(row["stored"]["z_pass_ms"] / row["computed"]["z_pass_ms"], 3),
                                           "iteration": round(row["stored"]["iteration_ms"] /
                                                              row["computed"]["iteration_ms"], 3)}
            print(f"# green A/B n={n} {prec}: {row['stored_over_computed']}", file=sys.stderr, flush=True)
            rows.append(row)
    # resident batches of small RVEs (each its own reference medium, so each
    # its own table), 2 load steps of 40 fixed iterations
    brows = []
    for n, count in ((32, 64), (64, 16)):
        rves = [W.random_rve(seed=100 + i, n=n, n_steps=2) for i in range(count)]
        for prec in ("fp64", "mixed"):
            row = {"rves": count, "n": n, "precision": prec}
            for green in ("computed", "stored"):
                B = mp.Batch([(n, n, n)], arena_bytes=12 << 30, precision=prec, max_rves=count,
                             iters_per_launch=8, autotune=True)
                ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, green=green) for w in rves]
                for rid in ids:
                    B.set_fixed_iterations(rid, 40)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                launches = B.drain()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                B.close()
                row[green] = {"seconds": round(dt, 4), "graph_launches": launches,
                              "voxel_iterations_per_s": count * n ** 3 * 80 / dt}
            row["stored_over_computed"] = round(row["stored"]["seconds"] / row["computed"]["seconds"], 3)
            print(f"# green A/B batch {count} x {n}^3 {prec}: {row['stored_over_computed']}", file=sys.stderr,
                  flush=True)
            brows.append(row)
    return {"green_ab": rows, "green_ab_batches": brows,
            "data": "synthetic (seeded random-sphere RVEs, W.random_rve seeds 5 and 100..163)"}


def run_al_ab(torch, mp, W):
    """The augmented-Lagrangian scheme (geometric-mean penalty, over-relaxation
    1.7) against the basic scheme (phase-mean reference) on the 128^3 and
    256^3 sphere cells with their inclusions at contrast 20, FP64, each
    converged on its own schedule at the cell's tolerance: iterations per
    step, wall time, the x pass from HIP events, and the largest difference
    of the 40 response columns on the response's scale."""
    rows = []
    for label, make in (("spheres128_fp64 cell, inclusions at contrast 20, load steps 1-3",
                         lambda: W.random_spheres_128(n_steps=3)),
                        ("spheres256 cell, inclusions at contrast 20, FP64, load steps 1-2",
                         lambda: W.random_spheres_256(n_steps=2))):
        wl = make()
        wl.phases = [wl.phases[0], wl.phases[0].scaled_moduli(20.0)]
        row = {"cell": label, "tol": wl.tol}
        resp = {}
        for scheme, kw in (("basic", dict(scheme="basic", ref_mode="phase_mean")),
                           ("al", dict(scheme="al", ref_mode="geometric_mean", relax=1.7))):
            plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, **kw)
            plan.profile(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = plan.solve(wl.times, wl.E, wl.G)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ms, k = plan.profile_read()["x_pass"]
            resp[scheme] = plan.responses()[:, :40]
            plan.close()
            row[scheme] = {"iterations": it, "seconds": round(dt, 3), "ms_per_iteration": round(dt / sum(it) * 1e3, 4),
                           "x_pass_ms": round(ms / k, 4)}
            print(f"# AL A/B {label}: {scheme} {it}, {dt:.2f} s", file=sys.stderr, flush=True)
        scale = np.abs(resp["basic"]).max()
        row["al_over_basic"] = {"iterations": round(sum(row["al"]["iterations"]) / sum(row["basic"]["iterations"]), 3),
                                "seconds": round(row["al"]["seconds"] / row["basic"]["seconds"], 3),
                                "ms_per_iteration": round(row["al"]["ms_per_iteration"] / row["basic"]["ms_per_iteration"], 3)}
        row["response_difference"] = float("%.3g" % (np.abs(resp["al"] - resp["basic"]).max() / scale))
        rows.append(row)
    return {"al_ab": rows, "data": "synthetic (seeded random-sphere microstructure)"}


def run_al_batch(torch, mp, W, count=16, n_steps=5):
    """The first RVEs of the many-RVE workload (edges 32-128, contrast
    2-20, tolerance 1e-6) on a shortened load path, each converged on its own
    schedule in one resident batch: FP64 with the augmented-Lagrangian scheme
    (geometric-mean penalty, over-relaxation 1.7) against FP64 and mixed with
    the basic scheme (phase-mean reference)."""
    rves = W.batch_rves(seed=3, count=64, n_steps=n_steps)[:count]
    shapes = sorted({w.phase_map.shape[::-1] for w in rves})
    out = {"rves": count, "load_steps": n_steps, "edges": [int(w.phase_map.shape[0]) for w in rves]}
    for name, prec, kw in (("basic_mixed", "mixed", {}), ("basic_fp64", "fp64", {}),
                           ("al_fp64", "fp64", dict(scheme="al", ref_mode="geometric_mean", relax=1.7))):
        B = mp.Batch(shapes, arena_bytes=24 << 30, precision=prec, max_rves=count, iters_per_launch=8,
                     autotune=True)
        ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, **kw) for w in rves]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        launches = B.drain()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        q = [B.query(i) for i in ids]
        B.close()
        out[name] = {"seconds": round(dt, 3), "rve_solves_per_s": count / dt, "graph_launches": launches,
                     "iterations": [int(x[3]) for x in q], "statuses": sorted({int(x[1]) for x in q})}
        print(f"# AL batch: {name} {dt:.2f} s, iterations {sum(x[3] for x in q)}", file=sys.stderr, flush=True)
    return {"al_batch": out, "data": "synthetic (seeded random-sphere RVEs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed, batch and serving samples added to the default line")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--workload", default="spheres128_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="run every load step for exactly this many iterations (profiling runs)")
    ap.add_argument("--rves", type=int, default=64, help="batch64_mixed: RVEs in the batch")
    ap.add_argument("--seq-rves", type=int, default=0,
                    help="batch64_mixed: also solve the first N RVEs one by one with FP64 plans")
    ap.add_argument("--requests", type=int, default=24, help="serve_mixed: requests in the trace")
    ap.add_argument("--arena-gib", type=int, default=48, help="serve_mixed: device arena (GiB)")
    ap.add_argument("--servers", default="both", choices=("both", "batched", "sequential", "none"),
                    help="serve_mixed: which servers replay the open-loop trace (none: the closed loop only)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="serve_mixed: open-loop arrival rate (req/s) instead of 0.8x a closed-loop run")
    ap.add_argument("--iters-per-launch", type=int, default=8,
                    help="batch / serve: loop iterations per graph launch")
    ap.add_argument("--al-batch", action="store_true",
                    help="only time a batch of 16 RVEs: augmented Lagrangian FP64 against basic FP64 and mixed")
    ap.add_argument("--al-ab", action="store_true",
                    help="only time the augmented-Lagrangian against the basic scheme at contrast 20")
    ap.add_argument("--green-ab", action="store_true",
                    help="only time the stored against the computed Green operator (32^3-256^3)")
    ap.add_argument("--sweep", action="store_true",
                    help="only time the 10 x 10 length-scale sweep (16^3 cells, 100 steps each) as one mixed batch")
    ap.add_argument("--ratchet", action="store_true",
                    help="only time the Sec. 3.2 ratcheting path (1000 steps on the 4^3 laminate, FP64 plan)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "dispatches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_10774_amd import mp, workloads as W

    if args.green_ab:
        print(json.dumps(run_green_ab(torch, mp, W)), flush=True)
        return
    if args.al_ab:
        print(json.dumps(run_al_ab(torch, mp, W)), flush=True)
        return
    if args.al_batch:
        print(json.dumps(run_al_batch(torch, mp, W)), flush=True)
        return
    if args.ratchet:
        print(json.dumps(extra_ratchet(torch, mp, W)), flush=True)
        return
    if args.sweep:
        print(json.dumps(run_sweep(torch, mp, W)), flush=True)
        return
    if args.workload in ("batch64_mixed", "serve_mixed"):
        run = run_batch if args.workload == "batch64_mixed" else run_serve
        print(json.dumps(run(args, torch, mp, W)), flush=True)
        return

    W_, K = args.warmup, args.steps
    cfg = WORKLOADS[args.workload]
    if args.workload == "spheres128_fp64":
        wl = W.random_spheres_128(n_steps=W_ + K)
    elif args.workload == "aniso128_fp64":
        wl = W.anisotropic_spheres_128(n_steps=W_ + K)
    else:   # spheres256_mixed, spheres256_fp64
        wl = W.random_spheres_256(n_steps=W_ + K)
    nvox = wl.phase_map.size
    BYTES_PER_VOXEL = algorithmic_bytes_per_voxel(8 if cfg["precision"] == "fp64" else 4)
    BYTES_PER_VOXEL_ITER = sum(BYTES_PER_VOXEL.values())
    DESIGN_BYTES = bytes_per_voxel(8 if cfg["precision"] == "fp64" else 4)
    plan = mp.Plan(wl.phase_map, wl.phases, tol=wl.tol, precision=cfg["precision"], ref_mode=wl.ref_mode)
    if args.fixed_iters:
        plan.set_fixed_iterations(args.fixed_iters)
    print(f"# workload {wl.name}: {wl.info}, warmup {W_} step(s), timed {K}", file=sys.stderr,
          flush=True)
    # warm-up steps with events between every loop kernel (the per-kernel
    # breakdown); the timed steps with events around the x pass only, which
    # is the dominant kernel and the one the roofline line reports
    prof_w = {}
    if W_ > 0:
        plan.profile(not args.no_profile)
        it_w = plan.solve(wl.times[: W_ + 1], wl.E[:W_], wl.G[:W_])
        prof_w = plan.profile_read()
        print(f"# warmup iterations {it_w}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    plan.profile(0 if args.no_profile else 2)
    t0 = time.perf_counter()
    iters = plan.solve(wl.times[W_: W_ + K + 1], wl.E[W_: W_ + K], wl.G[W_: W_ + K])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    print(f"# timed iterations {iters}, {dt:.3f} s", file=sys.stderr, flush=True)
    value = sum(iters) * nvox / dt

    kernels = {}
    for k, (ms, n) in prof_w.items():
        if n:
            avg = ms / n
            b = BYTES_PER_VOXEL[k] * nvox
            kernels[k] = {"avg_ms": round(avg, 4), "launches": n, "share": None,
                          "GBps": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
    tot = sum(prof_w[k][0] for k in prof_w)
    for k in kernels:
        kernels[k]["share"] = round(prof_w[k][0] / tot, 4)
    roof = None
    dom = "x_pass"
    if prof[dom][1]:
        avg = prof[dom][0] / prof[dom][1] * 1e-3
        achieved = BYTES_PER_VOXEL[dom] * nvox / avg / 1e9
        mt = MEASURED_TRAFFIC.get(args.workload)
        traffic = None
        if mt and mt["kernel"] == dom and mt["src_sha1"] == kernel_src_sha1():
            traffic = mt["bytes"]
        moved = DESIGN_BYTES[dom] * nvox / avg / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_voxel": BYTES_PER_VOXEL[dom], "bytes_per_launch": BYTES_PER_VOXEL[dom] * nvox,
                "avg_ms": round(avg * 1e3, 4), "launches": prof[dom][1],
                "design_bytes": {"bytes_per_voxel": DESIGN_BYTES[dom], "achieved": round(moved, 1),
                                 "frac": round(moved / HBM_PEAK_GBS, 4)}}

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
        "dtype": cfg["dtype"],
        "data": "synthetic (seeded random-sphere microstructure)",
        "config": {"workload": cfg["desc"], "timed_load_steps": [W_ + 1, W_ + K],
                   "iterations": iters, "fixed_iters": args.fixed_iters or None,
                   "parallelism": "single GPU"},
        "iteration_hbm_frac": round(BYTES_PER_VOXEL_ITER * value / (HBM_PEAK_GBS * 1e9), 4),
        "iteration_hbm_frac_design_bytes": round(sum(DESIGN_BYTES.values()) * value / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roof,
        "kernels": kernels,
        "kernels_measured": "warm-up steps, HIP events between every loop kernel",
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(wl),
    }
    if args.workload == "spheres128_fp64" and not args.no_extras:
        # samples of the precision, batching and serving forms on the same
        # GPU, outside the timed region
        line["extras"] = {"mixed256": extra_mixed256(torch, mp, W), "batch8": extra_batch8(torch, mp, W),
                          "serve": extra_serve(torch, mp, W), "ratchet4": extra_ratchet(torch, mp, W)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

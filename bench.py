#!/usr/bin/env python3
"""Benchmark of the LTS3 hot path on one MI355X.

A step is one LTS3 coarse step (Algorithm 2.2: coarse stages, M fine SSPRK3
substeps with interface prediction and accumulation, interface correction) of
the variable-resolution planar workload: 200,000 Voronoi cells, M = 8, FP64.

Reported (one JSON line on stdout):
  value      effective cell-updates/s = N_cells * M * steps / t  (fine-step
             equivalents, the rate global SSPRK3 at the fine step would need)
  extras     global SSPRK3 at the fine step (same GPU, same library), LTS3 in
             FP32, L2 height errors of all three against an FP64 SSPRK3
             reference at a quarter of the fine step
  roofline   the dominant kernel's algorithmic bytes per launch over its mean
             duration (HIP events bracketing each launch, timing pass right
             after the timed region), against 8 TB/s
  cpu_baseline  the FP64 oracle on the host, one thread, on a bounded number
             of coarse steps of the same workload
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s, LTS3 vs global RK3 on 1 GPU at fixed L2 height error; HBM GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b, w):
    import numpy as np
    return float(np.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum()))


def timed(torch, stream, fn):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["vr", "igw", "ensemble"], default="vr")
    ap.add_argument("--members", type=int, default=64, help="ensemble members")
    ap.add_argument("--lloyd", type=int, default=10,
                    help="minimum Lloyd iterations per ensemble member")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--quick", action="store_true",
                    help="LTS3 FP64 timed region only (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(every box here has a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble":
        return bench_ensemble(args)
    import numpy as np
    import torch
    from paper_2106_07154_amd.build import LIB
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2106_07154_amd import lts
    from paper_2106_07154_amd.inputs import workloads

    t0 = time.time()
    w = workloads.vr_planar() if args.workload == "vr" else workloads.igw_hex()
    m = w.mesh
    log(f"workload {w.name}: {m.nCells} cells {m.nEdges} edges, M={w.M} "
        f"dt_coarse={w.dt_coarse:.4f}s ({time.time() - t0:.1f}s to build)")
    # a dedicated (default-priority) stream: the library enqueues on it and the
    # timing events are recorded on it
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    K, W, M, dt = args.steps, args.warmup, w.M, w.dt_coarse

    def make(prec):
        c = lts.LTSContext(0, prec, stream=sp)
        c.upload_mesh(m, w.fine_mask, w.n_if1, w.n_if2, w.gravity)
        c.init_state(w.h0, w.u0)
        return c

    ctx = make("fp64")
    cells, edges, fbar = ctx.region_counts()
    ctx.step(dt, M, W)
    ctx.init_state(w.h0, w.u0)
    ms = timed(torch, stream, lambda: ctx.step(dt, M, K))
    value = m.nCells * M * K / (ms / 1e3)
    log(f"LTS3 fp64: {ms / K:.3f} ms/coarse step, {value:.4e} cell-updates/s")
    d = ctx.diagnostics()
    h_lts, _ = ctx.get_state()

    # per-kernel timing pass (HIP events around every launch, same stream)
    ctx.init_state(w.h0, w.u0)
    ctx.set_timing(True)
    ctx.step(dt, M, K)
    stats = ctx.kernel_stats()
    ctx.set_timing(False)
    dom = max(stats, key=lambda k: stats[k]["ms"])
    st = stats[dom]
    avg_ms = st["ms"] / st["launches"]
    bytes_per_launch = st["bytes"] / st["launches"]
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": dom, "launches": st["launches"], "avg_us": round(avg_ms * 1e3, 2),
                "bytes_per_launch": round(bytes_per_launch)}
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "GB/s": round(v["bytes"] / max(v["ms"], 1e-12) / 1e6, 1)}
               for k, v in stats.items() if v["launches"]}
    log("kernels:", json.dumps(kernels))

    out = {"metric": METRIC, "value": round(value, 1), "unit": "cell-updates/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": round(ms / K, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": w.name, "cells": m.nCells, "edges": m.nEdges,
                      "vertices": m.nVertices, "M": M, "dt_coarse_s": round(dt, 6),
                      "interface_rings": [w.n_if1, w.n_if2],
                      "region_cells": {"F": int(cells[3]), "I1": int(cells[2]),
                                       "I2": int(cells[1]), "C": int(cells[0]),
                                       "Fbar": int(fbar[0])}},
           "roofline": roofline, "kernels": kernels}

    if not args.quick:
        # global SSPRK3 at the fine step over the same simulated time
        rk = make("fp64")
        rk.step_rk3(dt / M, W * M)
        rk.init_state(w.h0, w.u0)
        ms_rk = timed(torch, stream, lambda: rk.step_rk3(dt / M, K * M))
        v_rk = m.nCells * K * M / (ms_rk / 1e3)
        h_rk, _ = rk.get_state()
        log(f"SSPRK3 fp64 at dt/M: {ms_rk / K:.3f} ms per coarse-step interval, {v_rk:.4e}")
        # FP32 LTS3
        c32 = make("fp32")
        c32.step(dt, M, W)
        c32.init_state(w.h0, w.u0)
        ms32 = timed(torch, stream, lambda: c32.step(dt, M, K))
        v32 = m.nCells * K * M / (ms32 / 1e3)
        h32, _ = c32.get_state()
        log(f"LTS3 fp32: {ms32 / K:.3f} ms/coarse step, {v32:.4e}")
        # reference: FP64 SSPRK3 at dt/(4M)
        ref = make("fp64")
        ref.step_rk3(dt / (4 * M), K * M * 4)
        h_ref, _ = ref.get_state()
        H = float(w.h0.min())
        wA = m.areaCell
        err = {"reference": "FP64 SSPRK3 at dt_fine/4",
               "t_end_s": round(K * dt, 3),
               "lts3_fp64": rel_l2(h_lts - H, h_ref - H, wA),
               "rk3_fp64": rel_l2(h_rk - H, h_ref - H, wA),
               "lts3_fp32": rel_l2(h32 - H, h_ref - H, wA),
               "norm": "area-weighted L2 of h - H relative to the reference perturbation"}
        log("errors:", json.dumps(err))
        out["comparisons"] = {"rk3_fp64_value": round(v_rk, 1),
                              "lts3_over_rk3": round(value / v_rk, 3),
                              "lts3_fp32_value": round(v32, 1),
                              "fp32_over_rk3_fp64": round(v32 / v_rk, 3),
                              "ideal_work_ratio": round(
                                  3 * M * m.nCells / (3 * int(cells[0]) + (2 + 3 * M) * int(cells[1] + cells[2])
                                                      + 3 * M * int(cells[3]) + int(fbar[0])), 3),
                              "l2_height_error": err,
                              "mass_rel_drift": None}
        rk.close(), c32.close(), ref.close()
        ctx.init_state(w.h0, w.u0)
        d0 = ctx.diagnostics()
        out["comparisons"]["mass_rel_drift"] = abs(d.mass - d0.mass) / d0.mass

        # CPU baseline: the FP64 oracle, one thread, bounded sample
        from oracle import Oracle
        o = Oracle(m, w.gravity)
        R = o.regions(w.fine_mask, w.n_if1, w.n_if2)
        t1 = time.time()
        o.lts(w.h0, w.u0, dt, M, R, n=1)
        one = time.time() - t1
        n_cpu = max(1, int(args.cpu_seconds / max(one, 1e-3)))
        t1 = time.time()
        o.lts(w.h0, w.u0, dt, M, R, n=n_cpu)
        tc = time.time() - t1
        out["cpu_baseline"] = {"value": round(m.nCells * M * n_cpu / tc, 1),
                               "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n_cpu} LTS3 coarse steps (M={M}) of {w.name} in "
                                         f"{tc:.1f}s on {os.cpu_count()} host cores (1 used)"}
        log(f"cpu baseline: {out['cpu_baseline']}")
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """Batched ensemble: every member advances K coarse steps (FP32, its own dt
    and M) through shared launches; compared with FP64 global SSPRK3 run member
    by member over the same simulated time."""
    from paper_2106_07154_amd.inputs import workloads
    t0 = time.time()
    cache = os.environ.get("LTS_ENSEMBLE_CACHE")  # a file this script itself wrote
    if cache and os.path.exists(cache):
        import pickle
        with open(cache, "rb") as f:
            mem = pickle.load(f)
    else:
        mem = workloads.ensemble_members(args.members, iters=args.lloyd)  # before any GPU use
        if cache:
            import pickle
            with open(cache, "wb") as f:
                pickle.dump(mem, f)
    log(f"{len(mem)} members, {sum(w.mesh.nCells for w in mem)} cells, "
        f"generated in {time.time() - t0:.0f}s")
    import numpy as np
    import torch
    from paper_2106_07154_amd.build import LIB
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2106_07154_amd import lts
    stream = torch.cuda.Stream()
    K, W = args.steps, args.warmup
    ens = lts.Ensemble(0, "fp32", stream=stream)
    for w in mem:
        ens.add_member(w.mesh, w.fine_mask, w.dt_coarse, w.M, w.n_if1, w.n_if2, w.gravity)
    for j, w in enumerate(mem):
        ens.init_member(j, w.h0, w.u0)
    t1 = time.time()
    ens.build(autotune=True)
    info = ens.info()
    log(f"build + autotune {time.time() - t1:.1f}s: {json.dumps(info)}")
    ens.step(W)
    for j, w in enumerate(mem):
        ens.init_member(j, w.h0, w.u0)
    ms = timed(torch, stream, lambda: ens.step(K))
    updates = sum(w.mesh.nCells * w.M for w in mem) * K
    value = updates / (ms / 1e3)
    total_bytes = sum(info["step_bytes"].values()) * K
    gbs = total_bytes / (ms / 1e3) / 1e9
    log(f"ensemble fp32: {ms / K:.3f} ms/step, {value:.4e} cell-updates/s, {gbs:.0f} GB/s")
    ok = all(ens.diagnostics(j).n_nonfinite == 0 for j in range(len(mem)))
    # FP64 global SSPRK3 at each member's fine step, member by member
    rk_ms = 0.0
    sample = sorted(range(len(mem)), key=lambda j: mem[j].mesh.nCells)
    sample = [sample[0], sample[len(sample) // 2], sample[-1]]
    errs = {}
    for j, w in enumerate(mem):
        c = lts.LTSContext(0, "fp64", stream=stream)
        c.upload_mesh(w.mesh, w.fine_mask, w.n_if1, w.n_if2, w.gravity)
        c.init_state(w.h0, w.u0)
        c.step_rk3(w.dt_coarse / w.M, 2)
        c.init_state(w.h0, w.u0)
        rk_ms += timed(torch, stream, lambda: c.step_rk3(w.dt_coarse / w.M, K * w.M))
        if j in sample:
            h_rk, _ = c.get_state()
            c.init_state(w.h0, w.u0)
            c.step_rk3(w.dt_coarse / (4 * w.M), K * w.M * 4)
            h_ref, _ = c.get_state()
            h_e, _ = ens.get_member(j)
            H = float(w.h0.min())
            errs[f"member{j}_{w.mesh.nCells}cells_M{w.M}"] = {
                "lts3_fp32_ensemble": rel_l2(h_e - H, h_ref - H, w.mesh.areaCell),
                "rk3_fp64": rel_l2(h_rk - H, h_ref - H, w.mesh.areaCell)}
        c.close()
    log(f"FP64 SSPRK3 member by member: {rk_ms:.1f} ms; errors {json.dumps(errs)}")
    out = {"metric": "cell-updates/s (ensemble aggregate, FP32 LTS3) and time-to-solution vs FP64 "
                     "global SSPRK3",
           "value": round(value, 1), "unit": "cell-updates/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": round(ms / K, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"ensemble-{len(mem)}-planar-vr",
                      "cells": int(sum(w.mesh.nCells for w in mem)),
                      "member_cells": [int(w.mesh.nCells) for w in mem],
                      "member_M": [int(w.M) for w in mem],
                      "lloyd_iterations": [int(w.extra["lloyd_iterations"]) for w in mem]},
           "achieved_GBs_all_kernels": round(gbs, 1), "hbm_frac_all_kernels": round(gbs / HBM_PEAK_GBS, 4),
           "ensemble": info, "all_finite": ok,
           "time_to_solution": {"ensemble_lts3_fp32_ms": round(ms, 2),
                                "rk3_fp64_member_by_member_ms": round(rk_ms, 2),
                                "speedup": round(rk_ms / ms, 3),
                                "l2_height_error_sampled": errs,
                                "reference": "FP64 SSPRK3 at a quarter of each member's fine step"}}
    ens.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

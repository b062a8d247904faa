"""Benchmark of the hierarchical-grid hot path on one MI355X.

One step = the whole path over one batch: grid_build (GPU construction with
per-node density sampling and the mass criterion) followed by grid_trace of
every path of the batch with the FP32-with-FP64-recheck walk in records mode
(counting walk, prefix sum, record-filling walk).  Inputs (ray origins and
directions) are resident in HBM before the timed region.

Default workload: the k-d tree of about 1e6 leaves on the exponential disk
(mass threshold 1e-6, max level 24) with 1e7 paths emitted by a stellar disk
and isotropic directions.  Besides the step throughput the JSON line carries
the FP64 tracer's throughput on the same paths, the leaf-for-leaf comparison
FP32-recheck vs FP64, an oracle spot check, the roofline of the dominant
kernel and the CPU oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "crossings/sec & rays/sec, FP32+FP64-recheck vs plain FP64, tau rel err <=1e-5"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes (what the method itself moves), per crossing and per path.
#   FP32-recheck, records: 4 B rope + 4 B rho32 + 16 B leaf geometry read,
#   4 B leaf id + 4 B ds32 written = 32 B per crossing.
#   The record-filling walk also reads the path (48 B) and its offset (8 B).
#   The counting (tau-only) walk reads 24 B per crossing, the path (48 B), and
#   writes tau + count (12 B).
# HBM traffic of the dominant kernel from rocprofv3 --pmc runs (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch), scaled by what the same counters read for a
# 1 GiB device copy (FETCH_SIZE reads 0.5 GiB for it, WRITE_SIZE 1.0 GiB).
# Valid only for the walk source it was measured on (sha256 of trace.hip).
TRAFFIC = {"trace_sha256": "b4f12bc0c7bd9e93626cc32a1a383fe05fb3af5f38fc8354b4810373c542185b",
           "fetch_kib": 32660382.3, "write_kib": 10795357.5,
           "fetch_scale": 2.0, "write_scale": 1.0}

B_X_FILL32 = 32
B_RAY_FILL = 48 + 8
B_X_COUNT32 = 24
B_RAY_COUNT = 48 + 12
B_X_FILL64 = 40
B_X_COUNT64 = 28


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", type=int, default=2, choices=[1, 2, 3])
    p.add_argument("--tree", choices=["kd", "octree"], default=None)
    p.add_argument("--rays", type=int, default=None, help="override the path count")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="target CPU time of the oracle baseline sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--calib-copy", type=int, default=0,
                   help="also run a device copy of this many MiB (counter calibration)")
    return p.parse_args()


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; runs on more than one GPU are not "
              "part of it (rays shard with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1311_0705_amd as hg
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tree = None if a.tree is None else (W.KDTREE if a.tree == "kd" else W.OCTREE)
    w = W.workload(a.workload, tree_type=tree, n_rays=a.rays)
    print(f"[bench] workload {w.name}: {w.n_rays} paths ({w.ray_kind} origins)", file=sys.stderr,
          flush=True)
    o_np, k_np = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
    o = torch.from_numpy(o_np).to(dev)
    k = torch.from_numpy(k_np).to(dev)
    n = o.shape[0]
    stream = torch.cuda.current_stream()

    if a.calib_copy:
        src = torch.empty(a.calib_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- warm-up (also sizes the record buffers) ----
    g = hg.build(w.density, w.criteria, w.tree_type, device=dev)
    n_leaves, n_nodes = g.n_leaves, g.n_nodes
    res = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, timing=True,
                  count_rechecks=True)
    needed = res["needed"]
    rechecks = res["rechecks"]
    g.free()
    del g
    for _ in range(max(0, a.warmup - 1)):
        g = hg.build(w.density, w.criteria, w.tree_type, device=dev)
        g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=res, capacity=needed)
        g.free()
    print(f"[bench] grid: {n_leaves} leaves, {n_nodes} nodes; {needed} crossings", file=sys.stderr,
          flush=True)

    # ---- timed steps: build + FP32-recheck records trace ----
    torch.cuda.synchronize()
    fill_ms, count_ms, build_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        tb0 = time.perf_counter()
        g = hg.build(w.density, w.criteria, w.tree_type, device=dev)
        build_ms.append((time.perf_counter() - tb0) * 1e3)
        r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=res, capacity=needed,
                    timing=True)
        count_ms.append(r["kernel_ms"][0])
        fill_ms.append(r["kernel_ms"][2])
        if _ < a.steps - 1:
            g.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / a.steps
    crossings = int(res["needed"])
    value = crossings / step_s
    print(f"[bench] step {step_s*1e3:.2f} ms (build ~{np.mean(build_ms):.2f} ms host-timed)",
          file=sys.stderr, flush=True)

    # ---- trace-only throughput, FP32-recheck vs FP64 (same grid, same paths) ----
    def time_trace(prec, reps=3):
        ms_tot, ms_c, ms_f = [], [], []
        out = {}
        for i in range(reps + 1):
            rr = g.trace(o, k, precision=prec, mode=hg.RECORDS, out=out, capacity=needed,
                         timing=True)
            if i:
                ms_tot.append(rr["kernel_ms"][3])
                ms_c.append(rr["kernel_ms"][0])
                ms_f.append(rr["kernel_ms"][2])
        return out, float(np.median(ms_tot)), float(np.median(ms_c)), float(np.median(ms_f))

    r32, ms32, c32, f32 = time_trace(hg.FP32_RECHECK)
    r64, ms64, c64, f64 = time_trace(hg.FP64)
    tau_only = {}
    for prec in (hg.FP32_RECHECK, hg.FP64):
        ts = []
        tout = {}
        for i in range(4):
            rr = g.trace(o, k, precision=prec, mode=hg.TAU_ONLY, out=tout, timing=True)
            if i:
                ts.append(rr["kernel_ms"][0])
        tau_only[prec] = float(np.median(ts))

    extra = {}
    if not a.no_compare:
        same_counts = bool(torch.equal(r32["count"], r64["count"]))
        leaf_exact = same_counts and bool(torch.equal(r32["leaf"][:crossings],
                                                      r64["leaf"][:crossings]))
        ds_exact = bool(torch.equal(r32["ds"][:crossings], r64["ds"][:crossings].float()))
        t64 = r64["tau"]
        rel = ((r32["tau"] - t64).abs() / t64.abs().clamp_min(1e-300))
        extra.update(leaf_exact_vs_fp64=leaf_exact, ds32_equals_rounded_fp64=ds_exact,
                     tau_max_rel_err_vs_fp64=float(rel.max().item()))
        # oracle spot check on a sample of paths through the same grid
        import oracle as O
        e = g.export()
        og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(),
                                     e["rho"].cpu().numpy())
        rng = np.random.default_rng(1)
        idx = np.sort(rng.choice(n, size=min(n, 4000), replace=False))
        ref = og.trace(o_np[idx], k_np[idx])
        off64 = r64["offsets"].cpu().numpy()
        ok = np.array_equal(r64["count"].cpu().numpy()[idx], ref["count"])
        ok = ok and np.array_equal(r64["tau"].cpu().numpy()[idx], ref["tau"])
        if ok:
            pos = np.concatenate([np.arange(off64[i], off64[i + 1]) for i in idx])
            pos_t = torch.from_numpy(pos).to(dev)
            gl = r64["leaf"].index_select(0, pos_t).cpu().numpy()
            gd = r64["ds"].index_select(0, pos_t).cpu().numpy()
            ok = np.array_equal(gl, ref["leaf"]) and np.array_equal(gd, ref["ds"])
        extra.update(oracle_sample_paths=int(idx.size), oracle_sample_bitwise_fp64=bool(ok))
        del e, og
    g.free()

    # ---- roofline of the dominant kernel (record-filling FP32-recheck walk) ----
    fill_avg = float(np.mean(fill_ms))
    count_avg = float(np.mean(count_ms))
    alg_fill = crossings * B_X_FILL32 + n * B_RAY_FILL
    achieved = alg_fill / (fill_avg * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(a.workload),
                "kernel": "k_walk_persistent<kd,fp32_recheck,fill>" if w.tree_type == W.KDTREE
                else "k_walk_persistent<octree,fp32_recheck,fill>",
                "kernel_ms": round(fill_avg, 3),
                "alg_bytes_per_launch": int(alg_fill)}

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "crossings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "tree": "kd" if w.tree_type == W.KDTREE else "octree",
                   "leaves": int(n_leaves), "nodes": int(n_nodes), "paths": int(n),
                   "precision": "fp32_recheck", "mode": "records",
                   "step": "grid_build + grid_trace"},
        "rays_per_s": round(n / step_s, 1),
        "crossings_per_path": round(crossings / n, 3),
        "trace_fp32r": {"crossings_per_s": round(crossings / (ms32 * 1e-3), 1),
                        "rays_per_s": round(n / (ms32 * 1e-3), 1), "ms": round(ms32, 3),
                        "count_ms": round(c32, 3), "fill_ms": round(f32, 3),
                        "tau_only_ms": round(tau_only[hg.FP32_RECHECK], 3)},
        "trace_fp64": {"crossings_per_s": round(crossings / (ms64 * 1e-3), 1),
                       "rays_per_s": round(n / (ms64 * 1e-3), 1), "ms": round(ms64, 3),
                       "count_ms": round(c64, 3), "fill_ms": round(f64, 3),
                       "tau_only_ms": round(tau_only[hg.FP64], 3)},
        "fp32r_over_fp64": round(ms64 / ms32, 3),
        "fp32r_over_fp64_tau_only": round(tau_only[hg.FP64] / tau_only[hg.FP32_RECHECK], 3),
        "recheck_rate": round(rechecks / max(crossings, 1), 6),
        "build_ms": round(float(np.mean(build_ms)), 3),
        "count_walk_ms": round(count_avg, 3),
        "roofline": roofline,
    }
    line.update(extra)

    # ---- CPU baseline: the oracle on the host cores ----
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, o_np, k_np, crossings, a.cpu_seconds)
    print(json.dumps(line), flush=True)


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel, if the counters were taken
    on the current walk source; else None."""
    import hashlib
    if workload != 2 or TRAFFIC["trace_sha256"] is None:
        return None
    src = os.path.join(ROOT, "paper_1311_0705_amd", "csrc", "trace.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["trace_sha256"]:
            return None
    return int(TRAFFIC["fetch_kib"] * 1024 * TRAFFIC["fetch_scale"]
               + TRAFFIC["write_kib"] * 1024 * TRAFFIC["write_scale"])


def cpu_baseline(w, o_np, k_np, crossings_total, budget_s):
    import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores), 64))
    t0 = time.perf_counter()
    og = O.Grid.build(w.density, w.criteria, w.tree_type)
    t_build = time.perf_counter() - t0
    n = o_np.shape[0]
    m = min(n, 20000)
    t0 = time.perf_counter()
    r = og.trace(o_np[:m], k_np[:m], records=True, nthreads=cores)
    t_probe = time.perf_counter() - t0
    left = max(0.0, budget_s - t_build - t_probe)
    m2 = int(min(n, max(m, m * left / max(t_probe, 1e-6))))
    if m2 > m:
        t0 = time.perf_counter()
        r = og.trace(o_np[:m2], k_np[:m2], records=True, nthreads=cores)
        t_probe = time.perf_counter() - t0
        m = m2
    x_sample = int(r["count"].sum())
    trace_rate = x_sample / t_probe
    # whole step extrapolated: one build plus the trace of all n paths
    t_step = t_build + t_probe * (n / m)
    return {"value": round(crossings_total / t_step, 1), "unit": "crossings/s", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle build of the full grid ({t_build:.2f} s, one thread) + FP64 "
                      f"records trace of the first {m} of {n} paths on {cores} threads "
                      f"({t_probe:.2f} s, {x_sample} crossings); step time extrapolated "
                      f"to all paths",
            "trace_crossings_per_s": round(trace_rate, 1),
            "build_s": round(t_build, 3),
            "oracle_leaves": int(og.n_leaves)}


if __name__ == "__main__":
    main()

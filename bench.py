"""Benchmark of the hierarchical-grid hot path on one MI355X.

One step = the whole path over one batch of synthetic input: grid_build (GPU
construction with per-node density sampling and the stopping criteria)
followed by grid_trace of every path of the batch with the
FP32-with-FP64-recheck walk.  Inputs (ray origins and directions) are
resident in HBM before the timed region.

Workloads (--workload):
  3 (default)  torus plus 500 clumps, k-d tree of about 4e6 leaves (--tree
               octree for the octree), 1e8 uniform paths: tau-only walk over
               all of them, records mode on the first batch of 1e7.  The JSON
               line also carries the FP64 tracer's throughput on the same
               paths, the comparison FP32-recheck vs FP64, the FP64 walk
               against the oracle on the first 1e6 paths (bitwise), the
               roofline of the dominant kernel and the CPU oracle's rate on the
               host cores (its construction timed on a sample of the grid's
               nodes, its walk on a sample of the paths).
  2            k-d tree of about 1e6 leaves on the exponential disk (mass
               threshold 1e-6, max level 24), 1e7 stellar-disk paths,
               records mode.
  1            octree of about 5e3 leaves on the same disk, 1e4 paths (FP64
               parity case; timed like 2).
  4            64 clump grids of uneven size (octree and k-d), 10^U[3,6]
               paths each: the batch built and traced by one replay of a
               captured graph, against the same 64 grids built and traced one
               by one.
  5            k-d tree of about 2e7 leaves on 97336 clustered clumps: the
               build timed end to end, then batches of 1e8 stellar-disk paths
               in tau-only mode.
The launch shape of the walk is autotuned (grid_tune, memoised per device and
grid class in the tuning cache file; batch_tune for workload 4) before the
timed region unless --no-tune is given.
"""
from __future__ import annotations

import argparse
import hashlib
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
#   writes tau + count (12 B).  FP64: 28 B (tau-only) / 40 B (records).
B_X_FILL32 = 32
B_RAY_FILL = 48 + 8
B_X_COUNT32 = 24
B_RAY_COUNT = 48 + 12
B_X_FILL64 = 40
B_X_COUNT64 = 28
# The one-pass records walk reads the path (48 B) and writes tau + count (12 B).
B_RAY_SLAB = 48 + 12

# Paths the launch-shape autotuner times each candidate on (a sample large
# enough that the walk's tail does not dominate the timing); the tau-only
# walks over 1e8 paths take a larger one, on which the candidates' order
# matches the full run's more often.
TUNE_PATHS = 10_000_000
TUNE_PATHS_TAU = 30_000_000

# HBM traffic of the dominant kernel from rocprofv3 --pmc runs (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch), scaled by what the same counters read for a
# 1 GiB device copy (FETCH_SIZE reads 0.5 GiB for it, WRITE_SIZE 1.0 GiB).
# Valid only for the walk source it was measured on (sha256 of trace.hip) and
# the workload it was measured on.
TRAFFIC = {
    "w2_slab": {"trace_sha256": "c18f1b6b3d9b6ab484e9bd7258dd9233c3d93c3f6a2c4c7f222613edf8ed5a77",
                "fetch_kib": 28233007.0, "write_kib": 5905506.9, "fetch_scale": 2.0, "write_scale": 1.0},
    "w3kd_tau": {"trace_sha256": "c18f1b6b3d9b6ab484e9bd7258dd9233c3d93c3f6a2c4c7f222613edf8ed5a77",
                 "fetch_kib": 81700626.0, "write_kib": 6899754.9, "fetch_scale": 2.0, "write_scale": 1.0},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", type=int, default=3, choices=[1, 2, 3, 4, 5])
    p.add_argument("--tree", choices=["kd", "octree"], default=None)
    p.add_argument("--rays", type=int, default=None, help="override the path count")
    p.add_argument("--batches", type=int, default=10, help="workload 5: batches of 1e8 paths")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="target wall time of the oracle baseline samples")
    p.add_argument("--parity-paths", type=int, default=1_000_000,
                   help="workloads 3 and 5: paths compared with the oracle bit for bit")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--no-tune", action="store_true")
    p.add_argument("--max-nodes", type=int, default=None,
                   help="node capacity passed to grid_build (0: size levels on the host); "
                        "default 2^22 for workloads 1-2, 2^24 for workload 3")
    p.add_argument("--calib-copy", type=int, default=0,
                   help="also run a device copy of this many MiB (counter calibration)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def trace_sha():
    src = os.path.join(ROOT, "paper_1311_0705_amd", "csrc", "trace.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of the dominant kernel, if its counters were taken
    on the current walk source for this workload; else None."""
    t = TRAFFIC.get(key)
    if not t or t["trace_sha256"] != trace_sha():
        return None
    return int(t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"])


def roofline(kernel, ms, alg_bytes, traffic_key):
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(traffic_key),
            "kernel": kernel, "kernel_ms": round(ms, 3), "alg_bytes_per_launch": int(alg_bytes)}


def base_line(a, value, step_s, unit, dtype, config):
    return {"metric": METRIC, "value": round(value, 1), "unit": unit, "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(step_s * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def tree_name(t):
    import workloads as W
    return "kd" if t == W.KDTREE else "octree"


def persistent_kernel(tree, prec, mode, block, wide=False):
    mode = {True: "fill", False: "count"}.get(mode, mode)
    return (f"k_walk_persistent<{'kd' if tree == 1 else 'octree'},"
            f"{'fp32_recheck' if prec == 1 else 'fp64'},{mode},{'u64' if wide else 'u32'},{block}>")


def oracle_sample_check(g, w, o_np, k_np, r64, dev, m=4000):
    """FP64 GPU walk vs the oracle on a sample of paths through the same grid."""
    import torch

    import oracle as O
    n = o_np.shape[0]
    e = g.export()
    og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(n, size=min(n, m), replace=False))
    ref = og.trace(o_np[idx], k_np[idx])
    ok = np.array_equal(r64["count"].cpu().numpy()[idx], ref["count"])
    ok = ok and np.array_equal(r64["tau"].cpu().numpy()[idx], ref["tau"])
    if ok and "offsets" in r64:
        off = r64["offsets"].cpu().numpy()
        pos = torch.from_numpy(np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])).to(dev)
        ok = (np.array_equal(r64["leaf"].index_select(0, pos).cpu().numpy(), ref["leaf"])
              and np.array_equal(r64["ds"].index_select(0, pos).cpu().numpy(), ref["ds"]))
    return {"oracle_sample_paths": int(idx.size), "oracle_sample_bitwise_fp64": bool(ok)}


def oracle_first_paths(g, w, o, k, o_np, k_np, m, cores):
    """The first m paths through the grid, GPU FP64 and FP32-recheck records
    walks against the oracle's FP64 walk of the same imported grid: leaf ids,
    counts, ds and tau bitwise for FP64; leaf for leaf and tau within 1e-5 for
    FP32-recheck.  Also returns the oracle's timing of that walk."""
    import paper_1311_0705_amd as hg
    import oracle as O
    m = min(m, o_np.shape[0])
    e = g.export()
    og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    del e
    t0 = time.perf_counter()
    ref = og.trace(o_np[:m], k_np[:m], records=True, nthreads=cores)
    t_or = time.perf_counter() - t0
    r64 = g.trace(o[:m], k[:m], precision=hg.FP64, mode=hg.RECORDS)
    x = r64["needed"]
    ok64 = (x == ref["leaf"].size
            and np.array_equal(r64["count"].cpu().numpy(), ref["count"])
            and np.array_equal(r64["tau"].cpu().numpy(), ref["tau"])
            and np.array_equal(r64["leaf"][:x].cpu().numpy(), ref["leaf"])
            and np.array_equal(r64["ds"][:x].cpu().numpy(), ref["ds"]))
    del r64
    r32 = g.trace(o[:m], k[:m], precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacity=x)
    leaf32 = (r32["needed"] == ref["leaf"].size
              and np.array_equal(r32["count"].cpu().numpy(), ref["count"])
              and np.array_equal(r32["leaf"][:x].cpu().numpy(), ref["leaf"]))
    t32 = r32["tau"].cpu().numpy()
    rel = np.abs(t32 - ref["tau"]) / np.maximum(np.abs(ref["tau"]), 1e-300)
    del r32
    out = {"oracle_paths": int(m), "oracle_crossings": int(ref["leaf"].size),
           "fp64_bitwise_vs_oracle": bool(ok64), "fp32r_leaf_exact_vs_oracle": bool(leaf32),
           "fp32r_tau_max_rel_err_vs_oracle": float(rel.max(initial=0.0))}
    return out, og, t_or, int(ref["leaf"].size)


def oracle_build_estimate(g, w, budget_s, seed=7):
    """The oracle's construction time for this grid, extrapolated: its
    per-node work (Eq. 1 sampling plus the criteria, one thread, as in its
    construction loop) timed on a uniform random sample of the grid's nodes,
    times the node count.  The sampled statistics are also compared with the
    GPU build's, node for node (equal up to the last bits of exp() between the
    host's libm and the GPU's: the largest relative difference is reported)."""
    import oracle as O
    e = g.export()
    n = int(g.n_nodes)
    rng = np.random.default_rng(seed)
    lv_all = e["level"].cpu().numpy()
    co_all = e["coord"].cpu().numpy().reshape(-1, 3)
    S_all = e["S"].cpu().numpy()
    del e
    m, t, done, worst = 256, 0.0, 0, 0.0
    while True:
        idx = rng.integers(0, n, size=m)
        t0 = time.perf_counter()
        r = O.sample_nodes(w.density, w.criteria, w.tree_type, lv_all[idx], co_all[idx])
        t += time.perf_counter() - t0
        done += m
        d = np.abs(r["S"] - S_all[idx]) / np.maximum(np.abs(r["S"]), 1e-300)
        worst = max(worst, float(d.max(initial=0.0)))
        if t >= budget_s or done >= n:
            break
        m = int(min(n, max(m, m * (budget_s - t) / max(t, 1e-6))))
    return {"build_s_est": t / done * n, "nodes_timed": int(done), "nodes_timed_s": round(t, 3),
            "nodes": n, "sampled_S_max_rel_diff": worst}


def compare_fp32r_fp64(r32, r64, records):
    import torch
    out = {}
    same_counts = bool(torch.equal(r32["count"], r64["count"]))
    if records:
        x = int(r64["needed"])
        out["leaf_exact_vs_fp64"] = same_counts and bool(torch.equal(r32["leaf"][:x], r64["leaf"][:x]))
        out["ds32_equals_rounded_fp64"] = bool(torch.equal(r32["ds"][:x], r64["ds"][:x].float()))
    else:
        out["counts_equal_fp64"] = same_counts
    t64 = r64["tau"]
    rel = (r32["tau"] - t64).abs() / t64.abs().clamp_min(1e-300)
    out["tau_max_rel_err_vs_fp64"] = float(rel.max().item())
    return out


def grid_quality(g, w, dev, n_pts=1_000_000, n_seg=100_000, seed=0x5EED):
    """The grid-quality measures of Sect. 3.2 on this grid: the standard
    deviations of rho_t - rho_g over uniform points and of tau_t - tau_g over
    segments with uniform start and end points (16-node Gauss-Legendre per
    cell piece for tau_t)."""
    import torch

    import paper_1311_0705_amd as hg
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, size=(n_pts, 3))
    a = rng.uniform(-1, 1, size=(n_seg, 3))
    b = rng.uniform(-1, 1, size=(n_seg, 3))
    L = np.linalg.norm(b - a, axis=1)
    k = (b - a) / L[:, None]
    drho = g.density_diff(w.density, pts)
    r = g.trace(a, k, precision=hg.FP64, mode=hg.RECORDS)
    tg = g.segment_tau(r, L)
    tt = g.true_tau(w.density, a, k, r, L)
    return {"delta_rho": float(drho.std().item()), "delta_tau": float((tt - tg).std().item()),
            "mean_tau_t": float(tt.mean().item()), "points": n_pts, "segments": n_seg}


def cpu_cores():
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(int(cores), 64))


def cpu_trace_sample(og, o_np, k_np, budget_s, records=True):
    """Oracle FP64 trace of the first paths, sized to about budget_s."""
    cores = cpu_cores()
    n = o_np.shape[0]
    m = min(n, 20000)
    t0 = time.perf_counter()
    r = og.trace(o_np[:m], k_np[:m], records=records, nthreads=cores)
    t = time.perf_counter() - t0
    m2 = int(min(n, max(m, m * max(0.0, budget_s - t) / max(t, 1e-6))))
    if m2 > m:
        t0 = time.perf_counter()
        r = og.trace(o_np[:m2], k_np[:m2], records=records, nthreads=cores)
        t = time.perf_counter() - t0
        m = m2
    return m, t, int(r["count"].sum()), cores


# ---------------------------------------------------------------------------
# workloads 1 and 2: build + records trace of one grid
# ---------------------------------------------------------------------------

def run_single(a, w):
    import torch

    import paper_1311_0705_amd as hg
    import workloads as W
    dev = torch.device("cuda:0")
    o_np, k_np = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
    o = torch.from_numpy(o_np).to(dev)
    k = torch.from_numpy(k_np).to(dev)
    n = o.shape[0]

    # ---- warm-up: sizes the record buffers and tunes the walk's launch shape ----
    mx = (1 << 22) if a.max_nodes is None else a.max_nodes
    g = hg.build(w.density, w.criteria, w.tree_type, device=dev, max_nodes=mx)
    n_leaves, n_nodes = g.n_leaves, g.n_nodes
    res = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, count_rechecks=True)
    needed, rechecks, descents = res["needed"], res["rechecks"], res["descents"]
    tuned = {}
    if not a.no_tune:
        m = min(n, TUNE_PATHS)
        for prec in (hg.FP32_RECHECK, hg.FP64):
            tuned[prec] = hg.tune_cached(g, o[:m], k[:m], precision=prec, mode=hg.RECORDS)
        log(f"tuned launch shapes: {tuned}")
    t32 = tuned.get(hg.FP32_RECHECK)
    g.free()
    for _ in range(max(0, a.warmup - 1)):
        g = hg.build(w.density, w.criteria, w.tree_type, device=dev, max_nodes=mx)
        g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=res, capacity=needed, tuned=t32)
        g.free()
    log(f"grid: {n_leaves} leaves, {n_nodes} nodes; {needed} crossings")

    # ---- timed steps: build + FP32-recheck records trace ----
    torch.cuda.synchronize()
    fill_ms, count_ms, build_ms = [], [], []
    t0 = time.perf_counter()
    for i in range(a.steps):
        tb0 = time.perf_counter()
        g = hg.build(w.density, w.criteria, w.tree_type, device=dev, max_nodes=mx)
        build_ms.append((time.perf_counter() - tb0) * 1e3)
        r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=res, capacity=needed,
                    timing=True, tuned=t32)
        count_ms.append(r["kernel_ms"][0])
        fill_ms.append(r["kernel_ms"][2])
        if i < a.steps - 1:
            g.free()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / a.steps
    crossings = int(res["needed"])
    log(f"step {step_s * 1e3:.2f} ms (build ~{np.mean(build_ms):.2f} ms host-timed)")

    # ---- trace-only throughput, FP32-recheck vs FP64 (same grid, same paths) ----
    def time_trace(prec, mode, t, reps=3):
        out, ms = {}, []
        for i in range(reps + 1):
            rr = g.trace(o, k, precision=prec, mode=mode, out=out, capacity=needed, timing=True,
                         tuned=t)
            if i:
                ms.append(rr["kernel_ms"])
        ms = np.median(np.array(ms), axis=0)
        return out, [float(x) for x in ms]

    r32, ms32 = time_trace(hg.FP32_RECHECK, hg.RECORDS, t32)
    r64, ms64 = time_trace(hg.FP64, hg.RECORDS, tuned.get(hg.FP64))
    _, tau32 = time_trace(hg.FP32_RECHECK, hg.TAU_ONLY, t32)
    _, tau64 = time_trace(hg.FP64, hg.TAU_ONLY, tuned.get(hg.FP64))
    default_ms = None
    if tuned:
        _, dms = time_trace(hg.FP32_RECHECK, hg.RECORDS, None)
        default_ms = dms[3]
    two = {}
    ms2 = []
    for i in range(4):
        rr = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=two, capacity=needed,
                     timing=True, passes=2)
        if i:
            ms2.append(rr["kernel_ms"][3])
    two_ms = float(np.median(ms2))
    del two
    extra = {}
    if not a.no_compare:
        extra.update(compare_fp32r_fp64(r32, r64, True))
        extra.update(oracle_sample_check(g, w, o_np, k_np, r64, dev))
        extra["grid_quality"] = grid_quality(g, w, dev)
    g.free()

    block = t32["block"] if t32 else 256
    count_avg = float(np.mean(count_ms))
    line = base_line(a, crossings / step_s, step_s, "crossings/s", "f32+f64",
                     {"workload": w.name, "tree": tree_name(w.tree_type), "leaves": int(n_leaves),
                      "nodes": int(n_nodes), "paths": int(n), "precision": "fp32_recheck",
                      "mode": "records", "step": "grid_build + grid_trace", "max_nodes": mx})

    def trace_entry(ms, tau_ms):
        # records mode in one walk: [0] the walk into per-path rows, [1] prefix
        # sum + overflow list, [2] copy into the CSR slices (+ overflow walk)
        return {"crossings_per_s": round(crossings / (ms[3] * 1e-3), 1),
                "rays_per_s": round(n / (ms[3] * 1e-3), 1), "ms": round(ms[3], 3),
                "walk_ms": round(ms[0], 3), "scan_ms": round(ms[1], 3), "copy_ms": round(ms[2], 3),
                "tau_only_ms": round(tau_ms[0], 3),
                "tau_only_crossings_per_s": round(crossings / (tau_ms[0] * 1e-3), 1)}

    line.update({
        "rays_per_s": round(n / step_s, 1),
        "crossings_per_path": round(crossings / n, 3),
        "trace_fp32r": trace_entry(ms32, tau32),
        "trace_fp64": trace_entry(ms64, tau64),
        "fp32r_over_fp64": round(ms64[3] / ms32[3], 3),
        "fp32r_over_fp64_tau_only": round(tau64[0] / tau32[0], 3),
        "recheck_rate": round(rechecks / max(crossings, 1), 6),
        "descent_levels_per_crossing": round(descents / max(crossings, 1), 4),
        "build_ms": round(float(np.mean(build_ms)), 3),
        "tuned": {str(kk): v for kk, v in tuned.items()} or None,
        "untuned_fp32r_trace_ms": None if default_ms is None else round(default_ms, 3),
        "two_pass_fp32r_trace_ms": round(two_ms, 3),
        "roofline": roofline(persistent_kernel(w.tree_type, 1, "slab", block), count_avg,
                             crossings * B_X_FILL32 + n * B_RAY_SLAB, f"w{a.workload}_slab"),
    })
    line.update(extra)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline_single(w, o_np, k_np, crossings, a.cpu_seconds)
    return line


def cpu_baseline_single(w, o_np, k_np, crossings_total, budget_s):
    import oracle as O
    t0 = time.perf_counter()
    og = O.Grid.build(w.density, w.criteria, w.tree_type)
    t_build = time.perf_counter() - t0
    n = o_np.shape[0]
    m, t, xs, cores = cpu_trace_sample(og, o_np, k_np, budget_s - t_build)
    t_step = t_build + t * (n / m)
    return {"value": round(crossings_total / t_step, 1), "unit": "crossings/s", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle build of the full grid ({t_build:.2f} s, one thread) + FP64 "
                      f"records trace of the first {m} of {n} paths on {cores} threads "
                      f"({t:.2f} s, {xs} crossings); step time extrapolated to all paths",
            "trace_crossings_per_s": round(xs / t, 1), "build_s": round(t_build, 3),
            "oracle_leaves": int(og.n_leaves)}


# ---------------------------------------------------------------------------
# workload 3: build + tau-only trace of 1e8 paths (records on the first 1e7)
# ---------------------------------------------------------------------------

def run_c3(a, w):
    import torch

    import paper_1311_0705_amd as hg
    import workloads as W
    dev = torch.device("cuda:0")
    log(f"generating {w.n_rays} paths")
    o_np, k_np = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
    o = torch.from_numpy(o_np).to(dev)
    k = torch.from_numpy(k_np).to(dev)
    n = o.shape[0]
    nb = min(n, 10_000_000)
    mx = (1 << 24) if a.max_nodes is None else a.max_nodes
    g = hg.build(w.density, w.criteria, w.tree_type, device=dev, max_nodes=mx)
    n_leaves, n_nodes = g.n_leaves, g.n_nodes
    tuned = {}
    if not a.no_tune:
        for mode, m in ((hg.TAU_ONLY, TUNE_PATHS_TAU), (hg.RECORDS, TUNE_PATHS)):
            tuned[mode] = hg.tune_cached(g, o[:m], k[:m], precision=hg.FP32_RECHECK, mode=mode)
        tuned["fp64_tau"] = hg.tune_cached(g, o[:TUNE_PATHS_TAU], k[:TUNE_PATHS_TAU], precision=hg.FP64,
                                           mode=hg.TAU_ONLY)
        log(f"tuned launch shapes: {tuned}")
    tt = tuned.get(hg.TAU_ONLY)
    res = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY, tuned=tt, count_rechecks=True)
    crossings = int(res["count"].sum().item())
    rechecks, descents = res["rechecks"], res["descents"]
    g.free()
    log(f"grid: {n_leaves} leaves; {crossings} crossings over {n} paths")
    torch.cuda.synchronize()
    build_ms, tau_ms = [], []
    t0 = time.perf_counter()
    for i in range(a.steps):
        tb = time.perf_counter()
        g = hg.build(w.density, w.criteria, w.tree_type, device=dev, max_nodes=mx)
        build_ms.append((time.perf_counter() - tb) * 1e3)
        r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY, out=res, timing=True, tuned=tt)
        tau_ms.append(r["kernel_ms"][0])
        if i < a.steps - 1:
            g.free()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / a.steps
    log(f"step {step_s * 1e3:.1f} ms")
    # FP64 tau-only over all paths; records mode on the first batch, both precisions
    t64 = g.trace(o, k, precision=hg.FP64, mode=hg.TAU_ONLY, timing=True, tuned=tuned.get("fp64_tau"))
    t64 = g.trace(o, k, precision=hg.FP64, mode=hg.TAU_ONLY, out=t64, timing=True,
                  tuned=tuned.get("fp64_tau"))
    ob, kb = o[:nb], k[:nb]
    tr = tuned.get(hg.RECORDS)
    rec32 = g.trace(ob, kb, precision=hg.FP32_RECHECK, mode=hg.RECORDS, tuned=tr)
    rec32 = g.trace(ob, kb, precision=hg.FP32_RECHECK, mode=hg.RECORDS, out=rec32, timing=True,
                    capacity=rec32["needed"], tuned=tr)
    rec64 = g.trace(ob, kb, precision=hg.FP64, mode=hg.RECORDS, capacity=rec32["needed"], tuned=tr)
    rec64 = g.trace(ob, kb, precision=hg.FP64, mode=hg.RECORDS, out=rec64, timing=True,
                    capacity=rec32["needed"], tuned=tr)
    xb = rec32["needed"]
    extra = {}
    if not a.no_compare:
        extra.update(compare_fp32r_fp64(res, t64, False))
        extra["records_first_batch"] = compare_fp32r_fp64(rec32, rec64, True)
        extra.update(oracle_sample_check(g, w, o_np[:nb], k_np[:nb], rec64, dev, m=2000))
    cores = cpu_cores()
    first = None
    if not (a.no_compare and a.no_cpu):
        log(f"oracle: first {a.parity_paths} paths")
        first = oracle_first_paths(g, w, o, k, o_np, k_np, a.parity_paths, cores)
        extra["oracle_first_paths"] = first[0]
        log(f"oracle: {first[0]}")
    if not a.no_compare:
        extra["grid_quality"] = grid_quality(g, w, dev)
    tau_avg = float(np.mean(tau_ms))
    block = tt["block"] if tt else 256
    line = base_line(a, crossings / step_s, step_s, "crossings/s", "f32+f64",
                     {"workload": w.name, "tree": tree_name(w.tree_type), "leaves": int(n_leaves),
                      "nodes": int(n_nodes), "paths": int(n), "precision": "fp32_recheck",
                      "mode": "tau_only", "step": "grid_build + grid_trace (tau-only)",
                      "max_nodes": mx})
    line.update({
        "rays_per_s": round(n / step_s, 1),
        "crossings_per_path": round(crossings / n, 3),
        "build_ms": round(float(np.mean(build_ms)), 3),
        "trace_fp32r_tau_only": {"ms": round(tau_avg, 3),
                                 "crossings_per_s": round(crossings / (tau_avg * 1e-3), 1),
                                 "rays_per_s": round(n / (tau_avg * 1e-3), 1)},
        "trace_fp64_tau_only": {"ms": round(t64["kernel_ms"][0], 3),
                                "crossings_per_s": round(crossings / (t64["kernel_ms"][0] * 1e-3), 1)},
        "fp32r_over_fp64_tau_only": round(t64["kernel_ms"][0] / tau_avg, 3),
        "records_batch": {"paths": int(nb), "crossings": int(xb),
                          "fp32r_ms": round(rec32["kernel_ms"][3], 3),
                          "fp32r_crossings_per_s": round(xb / (rec32["kernel_ms"][3] * 1e-3), 1),
                          "fp32r_walk_ms": round(rec32["kernel_ms"][0], 3),
                          "fp32r_copy_ms": round(rec32["kernel_ms"][2], 3),
                          "fp64_ms": round(rec64["kernel_ms"][3], 3),
                          "fp64_crossings_per_s": round(xb / (rec64["kernel_ms"][3] * 1e-3), 1),
                          "walk_roofline": roofline(
                              persistent_kernel(w.tree_type, 1, "slab", tr["block"] if tr else 256),
                              rec32["kernel_ms"][0], xb * B_X_FILL32 + nb * B_RAY_SLAB,
                              f"w3{tree_name(w.tree_type)}_slab")},
        "recheck_rate": round(rechecks / max(crossings, 1), 6),
        "descent_levels_per_crossing": round(descents / max(crossings, 1), 4),
        "tuned": {str(kk): v for kk, v in tuned.items()} or None,
        "roofline": roofline(persistent_kernel(w.tree_type, 1, False, block), tau_avg,
                             crossings * B_X_COUNT32 + n * B_RAY_COUNT,
                             f"w3{tree_name(w.tree_type)}_tau"),
    })
    line.update(extra)
    if not a.no_cpu:
        og = first[1]
        be = oracle_build_estimate(g, w, 0.25 * a.cpu_seconds)
        log(f"oracle build estimate: {be}")
        m, t, xs, cores = cpu_trace_sample(og, o_np, k_np, 0.75 * a.cpu_seconds, records=False)
        t_trace = t * (n / m)
        t_step = be["build_s_est"] + t_trace
        line["cpu_baseline"] = {
            "value": round(crossings / t_step, 1), "unit": "crossings/s", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle construction timed on {be['nodes_timed']} of the grid's {be['nodes']} "
                      f"nodes drawn uniformly ({be['nodes_timed_s']:.2f} s, one thread, the "
                      f"construction loop's per-node sampling and criteria), extrapolated to all "
                      f"nodes: {be['build_s_est']:.1f} s; FP64 tau-only walk of the first {m} of {n} "
                      f"paths ({xs} crossings, {t:.2f} s on {cores} threads) through the GPU-built "
                      f"grid imported into the oracle, extrapolated to all paths: {t_trace:.1f} s; "
                      f"value = crossings of the step / (construction + walk)",
            "trace_crossings_per_s": round(xs / t, 1),
            "build_s_est": round(be["build_s_est"], 2),
            "build_sampled_S_max_rel_diff_vs_gpu": be["sampled_S_max_rel_diff"],
            "records_walk_first_paths_s": round(first[2], 3),
            "records_walk_first_paths_crossings_per_s": round(first[3] / first[2], 1)}
    g.free()
    return line


# ---------------------------------------------------------------------------
# workload 4: 64 grids, one captured build-then-trace graph vs one by one
# ---------------------------------------------------------------------------

def run_c4(a):
    import torch

    import paper_1311_0705_amd as hg
    import workloads as W
    dev = torch.device("cuda:0")
    ws = [W.workload(4, i) for i in range(64)]
    rays = [W.rays(x.ray_kind, x.n_rays, x.ray_seed) for x in ws]
    os_ = [torch.from_numpy(p).to(dev) for p, _ in rays]
    ks_ = [torch.from_numpy(q).to(dev) for _, q in rays]
    n = sum(x.n_rays for x in ws)

    def one_by_one(outs=None):
        gs, rs = [], []
        for i, x in enumerate(ws):
            g = hg.build(x.density, x.criteria, x.tree_type, device=dev)
            rs.append(g.trace(os_[i], ks_[i], precision=hg.FP32_RECHECK, mode=hg.RECORDS,
                              out=None if outs is None else outs[i],
                              capacity=None if outs is None else outs[i]["leaf"].numel()))
            gs.append(g)
        return gs, rs

    gs, ref = one_by_one()
    caps_nodes = [g.n_nodes + 64 for g in gs]
    needed = [r["needed"] for r in ref]
    crossings = sum(needed)
    leaves = sum(g.n_leaves for g in gs)
    for g in gs:
        g.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        gs, _ = one_by_one(ref)
        for g in gs:
            g.free()
    torch.cuda.synchronize()
    obo_s = (time.perf_counter() - t0) / a.steps
    log(f"one by one: {obo_s * 1e3:.1f} ms per pass; {leaves} leaves, {crossings} crossings")

    b = hg.Batch([x.density for x in ws], [x.criteria for x in ws], [x.tree_type for x in ws],
                 caps_nodes, device=dev)
    res = b.bind(os_, ks_, precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacities=needed)
    b.run(hg.STAGE_ALL)
    b.result()
    tuned = None
    if not a.no_tune:
        tuned = b.tune()
        res = b.results
        log(f"tuned batch walk: {tuned}")
    tk = dict(chunk=tuned["chunk"], refill_min=tuned["refill_min"], block=tuned["block"]) if tuned \
        else {}
    side = torch.cuda.Stream(dev)
    # eager batch (no graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.run(hg.STAGE_ALL, stream=side)
    b.result(side)
    eager_s = (time.perf_counter() - t0) / a.steps
    b.capture(hg.STAGE_ALL, stream=side)
    for _ in range(a.warmup):
        b.replay(side)
    b.result(side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.replay(side)
    b.result(side)
    step_s = (time.perf_counter() - t0) / a.steps
    log(f"graph replay {step_s * 1e3:.2f} ms, eager batch {eager_s * 1e3:.2f} ms")
    same = all(res[i]["needed"] == ref[i]["needed"]
               and torch.equal(res[i]["tau"], ref[i]["tau"])
               and torch.equal(res[i]["leaf"][:needed[i]], ref[i]["leaf"][:needed[i]])
               and torch.equal(res[i]["ds"][:needed[i]], ref[i]["ds"][:needed[i]])
               for i in range(64))
    # the bound trace stage on its own (one walk into per-path rows, the row
    # copy and the resume walk), timed with HIP events on its stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.run(hg.STAGE_TRACE, stream=side)
    e0.record(side)
    for _ in range(a.steps):
        b.run(hg.STAGE_TRACE, stream=side)
    e1.record(side)
    b.result(side)
    e1.synchronize()
    trace_stage_ms = e0.elapsed_time(e1) / a.steps
    same = same and all(torch.equal(res[i]["leaf"][:needed[i]], ref[i]["leaf"][:needed[i]])
                        for i in range(64))
    log(f"batch trace stage {trace_stage_ms:.3f} ms")
    # the batched walks on their own, timed with HIP events (eager, same grids)
    log("batched walk timing")
    grids = [b.grid(i) for i in range(64)]
    grids_fc = {}
    if not a.no_cpu:
        for i in range(0, 64, 8):
            e = grids[i].export()
            grids_fc[i] = (e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
            del e
    tb = hg.trace_batched(grids, os_, ks_, precision=hg.FP32_RECHECK, mode=hg.RECORDS,
                          capacities=needed, timing=True, **tk)
    tb = hg.trace_batched(grids, os_, ks_, precision=hg.FP32_RECHECK, mode=hg.RECORDS,
                          capacities=needed, timing=True, outs=tb, **tk)
    kms = tb[0]["kernel_ms"]
    for g in grids:
        g.free()
    b.free()
    line = base_line(a, crossings / step_s, step_s, "crossings/s", "f32+f64",
                     {"workload": "clumps-batch-64", "grids": 64, "leaves": int(leaves),
                      "paths": int(n), "precision": "fp32_recheck", "mode": "records",
                      "step": "captured graph: batched grid build + batched trace"})
    line.update({
        "rays_per_s": round(n / step_s, 1),
        "one_by_one_ms": round(obo_s * 1e3, 3),
        "eager_batch_ms": round(eager_s * 1e3, 3),
        "graph_over_one_by_one": round(obo_s / step_s, 3),
        "batch_equals_one_by_one": bool(same),
        "batch_trace_stage_ms": round(trace_stage_ms, 3),
        "trace_batched_two_walks_ms": {"count": round(kms[0], 3), "scan": round(kms[1], 3),
                                       "fill": round(kms[2], 3)},
        "tuned": tuned,
        "roofline": roofline("batch trace stage (one-pass batched walk, row copy, resume walk)",
                             trace_stage_ms, crossings * B_X_FILL32 + n * B_RAY_SLAB, "w4_stage"),
    })
    if not a.no_cpu:
        import oracle as O
        t_t, xs, m_tot = 0.0, 0, 0
        cores = cpu_cores()
        log("oracle trace sample")
        for i in range(0, 64, 8):
            e = grids_fc[i]
            og = O.Grid.from_first_child(ws[i].tree_type, e[0], e[1])
            m = min(20_000, ws[i].n_rays)
            t0 = time.perf_counter()
            r = og.trace(rays[i][0][:m], rays[i][1][:m], nthreads=cores)
            t_t += time.perf_counter() - t0
            xs += int(r["count"].sum())
            m_tot += m
        line["cpu_baseline"] = {
            "value": round(xs / t_t, 1), "unit": "crossings/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 records trace of the first (up to) 2e4 paths of grids 0, 8, ..., 56 "
                      f"({m_tot} paths, {xs} crossings, {t_t:.2f} s on {cores} threads) through "
                      f"the GPU-built grids imported into the oracle; the oracle builds (a plain "
                      f"loop over up to 2000 clumps per sample) are not timed"}
    return line


# ---------------------------------------------------------------------------
# workload 5: large clumpy k-d tree, build timed, batches of 1e8 tau-only
# ---------------------------------------------------------------------------

def run_c5(a, w):
    import torch

    import paper_1311_0705_amd as hg
    import workloads as W
    dev = torch.device("cuda:0")
    per = 100_000_000 if a.rays is None else a.rays
    log(f"generating {per} paths")
    o_np, k_np = W.rays(w.ray_kind, per, w.ray_seed)
    o = torch.from_numpy(o_np).to(dev)
    k0 = torch.from_numpy(k_np).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = hg.build(w.density, w.criteria, w.tree_type, device=dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"build {build_s:.2f} s: {g.n_leaves} leaves")
    tt = None
    if not a.no_tune:
        tt = hg.tune_cached(g, o[:TUNE_PATHS_TAU], k0[:TUNE_PATHS_TAU], precision=hg.FP32_RECHECK,
                            mode=hg.TAU_ONLY)
        log(f"tuned {tt}")
    res = g.trace(o, k0, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY, tuned=tt)
    batch_ms, xs = [], []
    k = torch.empty_like(k0)
    for bi in range(a.batches):
        # batch bi: the paths of batch 0 with directions turned about z by 2 pi bi / batches
        ang = 2.0 * math.pi * bi / a.batches
        c, s = math.cos(ang), math.sin(ang)
        k[:, 0] = c * k0[:, 0] - s * k0[:, 1]
        k[:, 1] = s * k0[:, 0] + c * k0[:, 1]
        k[:, 2] = k0[:, 2]
        k.div_(k.norm(dim=1, keepdim=True))
        r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY, out=res, timing=True, tuned=tt)
        batch_ms.append(r["kernel_ms"][0])
        xs.append(int(r["count"].sum().item()))
        log(f"batch {bi}: {batch_ms[-1]:.1f} ms, {xs[-1]} crossings")
    tot_ms = float(np.sum(batch_ms))
    crossings = int(np.sum(xs))
    n = per * a.batches
    extra = {}
    if not a.no_compare:
        r64 = g.trace(o[:1_000_000], k0[:1_000_000], precision=hg.FP64, mode=hg.RECORDS)
        r32 = g.trace(o[:1_000_000], k0[:1_000_000], precision=hg.FP32_RECHECK, mode=hg.RECORDS,
                      capacity=r64["needed"])
        extra["first_1e6_paths"] = compare_fp32r_fp64(r32, r64, True)
        extra.update(oracle_sample_check(g, w, o_np[:1_000_000], k_np[:1_000_000], r64, dev, m=2000))
    step_s = build_s + tot_ms * 1e-3
    line = base_line(a, crossings / step_s, step_s, "crossings/s", "f32+f64",
                     {"workload": w.name, "tree": "kd", "leaves": int(g.n_leaves),
                      "nodes": int(g.n_nodes), "paths": int(n), "batches": a.batches,
                      "precision": "fp32_recheck", "mode": "tau_only",
                      "step": "grid_build + grid_trace of every batch"})
    line.update({
        "build_s": round(build_s, 3),
        "trace_ms_total": round(tot_ms, 3),
        "trace_ms_per_batch": [round(x, 3) for x in batch_ms],
        "trace_crossings_per_s": round(crossings / (tot_ms * 1e-3), 1),
        "trace_rays_per_s": round(n / (tot_ms * 1e-3), 1),
        "tuned": tt,
        "roofline": roofline(persistent_kernel(1, 1, False, tt["block"] if tt else 256,
                                               wide=g.n_leaves > (1 << 25)),
                             float(np.mean(batch_ms)),
                             crossings / a.batches * B_X_COUNT32 + per * B_RAY_COUNT, "w5_tau"),
    })
    line.update(extra)
    if not a.no_cpu:
        import oracle as O
        e = g.export()
        og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
        del e
        m, t, xs1, cores = cpu_trace_sample(og, o_np, k_np, a.cpu_seconds, records=False)
        line["cpu_baseline"] = {
            "value": round(xs1 / t, 1), "unit": "crossings/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 tau trace of the first {m} paths of batch 0 ({xs1} crossings, {t:.2f} s "
                      f"on {cores} threads) through the GPU-built grid imported into the oracle; "
                      f"the oracle build is not timed"}
    g.free()
    return line


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not implemented (paths would "
              "shard across GPUs with no exchange during the walk)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.calib_copy:
        src = torch.empty(a.calib_copy << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tree = None if a.tree is None else (W.KDTREE if a.tree == "kd" else W.OCTREE)
    if a.workload == 4:
        line = run_c4(a)
    else:
        w = W.workload(a.workload, tree_type=tree, n_rays=a.rays if a.workload != 5 else None)
        log(f"workload {w.name}")
        if a.workload in (1, 2):
            line = run_single(a, w)
        elif a.workload == 3:
            line = run_c3(a, w)
        else:
            line = run_c5(a, w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

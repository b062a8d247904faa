"""The FP32 exit decision with its FP64 recheck, on the rays that stress it.

Rays aimed at an edge of a leaf have two exit distances that are equal or
nearly so; turning the direction slightly away from the edge makes their gap
any chosen fraction of the leaf's smallest side, here from far below to far
above the 1e-5 threshold of the recheck.  Directions with a component that is
nonzero but below 1e-30 take the FP64 decision throughout.  On all of them the
FP32-recheck walk must give the oracle's leaf sequence exactly, ds equal to the
oracle's ds rounded to FP32 and tau within 1e-5; the FP64 walk must be bitwise
equal to the oracle.  A last test runs grid_trace from two host threads at once
on one grid (each its own stream and outputs) against a serial call.
"""
import math
import threading

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", params=[O.KDTREE, O.OCTREE], ids=["kd", "octree"])
def grid(request):
    w = W.workload(1)
    cr = w.criteria
    cr.max_level = 14 if request.param == O.KDTREE else 5
    cr.delta_max = 3e-4
    og = O.Grid.build(w.density, cr, request.param)
    g = hg.import_grid(og.tree, og.nodes()["first_child"], og.leaves()["rho"], device=DEV)
    yield og, g
    g.free()


def near_edge_rays(og, n_leaves, seed):
    """Rays from inside random leaves toward an edge of the leaf, turned so
    that the gap between the two smallest exit distances is a chosen multiple
    of the leaf's smallest side."""
    rng = np.random.default_rng(seed)
    lo, hi = og.leaf_boxes()
    gaps = np.array([0.0, 1e-8, 1e-6, 5e-6, 9e-6, 9.9e-6, 1.01e-5, 1.1e-5, 2e-5, 1e-4, 1e-3])
    o, k = [], []
    for leaf in rng.choice(og.n_leaves, size=n_leaves, replace=False):
        l, h = lo[leaf], hi[leaf]
        w = h - l
        hmin = w.min()
        a, b = rng.choice(3, size=2, replace=False)
        c = 3 - a - b
        p = l + w * rng.uniform(0.2, 0.8, size=3)
        e = np.empty(3)
        e[a] = h[a] if rng.random() < 0.5 else l[a]
        e[b] = h[b] if rng.random() < 0.5 else l[b]
        e[c] = l[c] + w[c] * rng.uniform(0.1, 0.9)
        v = e - p
        t = np.linalg.norm(v)
        k0 = v / t
        for g in gaps:
            for sgn in (1.0, -1.0):
                # t_b = |e_b - p_b| / |k_b| moves by about eps t when k_b is scaled by 1 + eps
                kk = k0.copy()
                kk[b] *= 1.0 + sgn * g * hmin / t
                kk /= np.linalg.norm(kk)
                o.append(p)
                k.append(kk)
    return np.array(o), np.array(k)


def tiny_component_rays(seed, n=64):
    rng = np.random.default_rng(seed)
    o, k = [], []
    for i in range(n):
        d = i % 3
        e = np.zeros(3)
        e[d] = 1.0 if i % 2 == 0 else -1.0
        tiny = [1e-35, -1e-35, 5e-31, -7e-40][i % 4]
        e[(d + 1) % 3] = tiny
        o.append(rng.uniform(-0.9, 0.9, size=3))
        k.append(e)
    return np.array(o), np.array(k)


def _check(og, g, o, k):
    ref = og.trace(o, k)
    r64 = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS)
    r32 = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, count_rechecks=True)
    n = ref["leaf"].size
    assert r64["needed"] == n and r32["needed"] == n
    assert np.array_equal(r64["count"].cpu().numpy(), ref["count"])
    assert np.array_equal(r64["leaf"][:n].cpu().numpy(), ref["leaf"])
    assert np.array_equal(r64["ds"][:n].cpu().numpy(), ref["ds"])
    assert np.array_equal(r64["tau"].cpu().numpy(), ref["tau"])
    assert np.array_equal(r32["count"].cpu().numpy(), ref["count"])
    assert np.array_equal(r32["leaf"][:n].cpu().numpy(), ref["leaf"])
    assert np.array_equal(r32["ds"][:n].cpu().numpy(), ref["ds"].astype(np.float32))
    t = r32["tau"].cpu().numpy()
    rel = np.abs(t - ref["tau"]) / np.maximum(np.abs(ref["tau"]), 1e-300)
    assert float(rel.max(initial=0.0)) <= 1e-5
    return r32["rechecks"], n


def test_near_edge_rays(grid):
    og, g = grid
    o, k = near_edge_rays(og, 300, 11)
    rechecks, n = _check(og, g, o, k)
    # the rays with a gap below the threshold take the FP64 decision
    assert rechecks >= 300
    print(f"{o.shape[0]} rays, {n} crossings, {rechecks} rechecks")


def test_tiny_direction_components(grid):
    og, g = grid
    o, k = tiny_component_rays(12)
    rechecks, n = _check(og, g, o, k)
    assert rechecks >= n   # every exit decision of these paths is taken in FP64


def test_concurrent_host_threads(grid):
    og, g = grid
    o, k = W.rays("uniform", 200_000, 99)
    o = torch.from_numpy(o).to(DEV)
    k = torch.from_numpy(k).to(DEV)
    ref = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    results, errors = [None, None], []

    def run(i):
        try:
            s = torch.cuda.Stream(DEV)
            with torch.cuda.stream(s):
                r = g.trace(o, k, precision=hg.FP32_RECHECK if i == 0 else hg.FP64, mode=hg.RECORDS,
                            stream=s)
            s.synchronize()
            results[i] = r
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    r32, r64 = results
    n = ref["needed"]
    assert r32["needed"] == n and r64["needed"] == n
    assert torch.equal(r32["leaf"][:n], ref["leaf"][:n]) and torch.equal(r32["ds"][:n], ref["ds"][:n])
    assert torch.equal(r32["tau"], ref["tau"])
    assert torch.equal(r64["leaf"][:n], ref["leaf"][:n])
    assert torch.equal(r64["ds"][:n].float(), ref["ds"][:n])

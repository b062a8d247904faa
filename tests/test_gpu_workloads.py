"""Parity on the clumpy workloads at full size: the torus plus 500 truncated
Gaussian clumps with the combined mass, optical-depth and dispersion
criteria (about 4e6 k-d leaves, 7.6e6 octree leaves), traced with 1e7 of its
uniformly emitted paths.

The oracle cannot rebuild these trees in test time, so it checks them piece by
piece: sampled nodes are re-sampled one by one (statistics within 1e-13,
identical split decisions), and a sample of paths is traced by the oracle on
the exported grid (bitwise FP64 parity).  FP32-with-recheck equals FP64 leaf
for leaf on every path; the lengths along every path sum to its chord.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"
N_PATHS = 10_000_000


@pytest.fixture(scope="module", params=[W.KDTREE, W.OCTREE], ids=["kd", "octree"])
def clumpy(request):
    w = W.workload(3, tree_type=request.param)
    print(f"[gpu] {w.name}: building", flush=True)
    g = hg.build(w.density, w.criteria, w.tree_type, device=DEV)
    o_np, k_np = W.rays(w.ray_kind, N_PATHS, w.ray_seed)
    o = torch.from_numpy(o_np).to(DEV)
    k = torch.from_numpy(k_np).to(DEV)
    print(f"[gpu] {w.name}: {g.n_leaves} leaves, tracing", flush=True)
    r64 = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS)
    r32 = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacity=r64["needed"])
    yield w, g, o_np, k_np, o, k, r64, r32
    g.free()


def test_leaf_count_order(clumpy):
    w, g, *_ = clumpy
    assert 2e6 < g.n_leaves < 2e7


def test_fp32_recheck_equals_fp64(clumpy):
    w, g, o_np, k_np, o, k, r64, r32 = clumpy
    n = r64["needed"]
    assert n == r32["needed"]
    assert torch.equal(r64["count"], r32["count"])
    assert torch.equal(r64["leaf"][:n], r32["leaf"][:n])
    assert torch.equal(r64["ds"][:n].float(), r32["ds"][:n])
    rel = (r32["tau"] - r64["tau"]).abs() / r64["tau"].abs().clamp_min(1e-300)
    assert float(rel.max()) <= 1e-5, float(rel.max())


def test_lengths_sum_to_chord(clumpy):
    w, g, o_np, k_np, o, k, r64, r32 = clumpy
    n = r64["needed"]
    ray = torch.repeat_interleave(torch.arange(o.shape[0], device=DEV), r64["count"].long())
    s = torch.zeros(o.shape[0], dtype=torch.float64, device=DEV)
    s.index_add_(0, ray, r64["ds"][:n])
    inv = 1.0 / k
    t1 = (-1.0 - o) * inv
    t2 = (1.0 - o) * inv
    tn = torch.minimum(t1, t2).nan_to_num(nan=-np.inf).amax(dim=1).clamp_min(0.0)
    tf = torch.maximum(t1, t2).nan_to_num(nan=np.inf).amin(dim=1)
    assert float((s - (tf - tn).clamp_min(0.0)).abs().max()) <= 1e-12


def test_oracle_sample(clumpy):
    w, g, o_np, k_np, o, k, r64, r32 = clumpy
    e = g.export()
    og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    idx = np.sort(np.random.default_rng(3).choice(o_np.shape[0], size=2000, replace=False))
    ref = og.trace(o_np[idx], k_np[idx])
    assert np.array_equal(r64["count"].cpu().numpy()[idx], ref["count"])
    assert np.array_equal(r64["tau"].cpu().numpy()[idx], ref["tau"])
    off = r64["offsets"].cpu().numpy()
    pos = torch.from_numpy(np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])).to(DEV)
    assert np.array_equal(r64["leaf"].index_select(0, pos).cpu().numpy(), ref["leaf"])
    assert np.array_equal(r64["ds"].index_select(0, pos).cpu().numpy(), ref["ds"])
    pts = np.random.default_rng(4).uniform(-1, 1, size=(20000, 3))
    assert np.array_equal(g.locate(pts).cpu().numpy(), og.locate(pts))


def test_build_sampled_nodes(clumpy):
    w, g, *_ = clumpy
    e = g.export()
    fc = e["first_child"].cpu().numpy()
    lv = e["level"].cpu().numpy()
    co = e["coord"].cpu().numpy().astype(np.uint32)
    S = e["S"].cpu().numpy()
    mn = e["rho_min"].cpu().numpy()
    mx = e["rho_max"].cpu().numpy()
    rng = np.random.default_rng(5)
    # every level is represented, plus random nodes (weighted toward the deep ones)
    idx = [int(np.nonzero(lv == l)[0][0]) for l in np.unique(lv)]
    idx += list(rng.choice(fc.size, size=600, replace=False))
    for i in idx:
        s = O.sample_node(w.density, w.criteria, w.tree_type, int(lv[i]), co[i])
        assert abs(s["S"] - S[i]) <= 1e-13 * abs(s["S"]), i
        assert abs(s["rmin"] - mn[i]) <= 1e-13 * abs(s["rmin"]), i
        assert abs(s["rmax"] - mx[i]) <= 1e-13 * abs(s["rmax"]), i
        if s["split"] != (fc[i] >= 0):
            near = min(abs(s["delta"] / w.criteria.delta_max - 1.0),
                       abs(s["tau"] / w.criteria.tau_max - 1.0),
                       abs(s["q"] / w.criteria.q_max - 1.0))
            assert near < 1e-12, i

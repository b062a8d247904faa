"""Parity at the benchmark's full size: the k-d tree of about 1e6 leaves on the
exponential disk and its 1e7 paths, in the launch configuration bench.py
times (persistent walk, records mode).

* FP32-with-recheck vs FP64 on every path: identical counts and leaf
  sequences, ds32 equal to ds64 rounded, tau within 1e-5 relative.
* Sum of ds along every path equals its chord through the domain (1e-12).
* A sample of paths is traced by the oracle on the same (exported) grid and
  matches the FP64 walk bitwise.
* A sample of nodes is re-sampled by the oracle one by one: sampled
  statistics within 1e-13 relative and split decisions identical.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def setup():
    w = W.workload(2)
    print(f"[gpu] full size {w.name}: building", flush=True)
    g = hg.build(w.density, w.criteria, w.tree_type, device=DEV)
    o_np, k_np = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
    o = torch.from_numpy(o_np).to(DEV)
    k = torch.from_numpy(k_np).to(DEV)
    print(f"[gpu] full size: {g.n_leaves} leaves, tracing {o.shape[0]} paths", flush=True)
    r64 = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS)
    r32 = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacity=r64["needed"])
    return w, g, o_np, k_np, o, k, r64, r32


def test_fp32_recheck_equals_fp64_on_every_path(setup):
    w, g, o_np, k_np, o, k, r64, r32 = setup
    n = r64["needed"]
    assert n == r32["needed"] and n > 1e8
    assert torch.equal(r64["count"], r32["count"])
    assert torch.equal(r64["offsets"], r32["offsets"])
    assert torch.equal(r64["leaf"][:n], r32["leaf"][:n])
    assert torch.equal(r64["ds"][:n].float(), r32["ds"][:n])
    t64 = r64["tau"]
    rel = (r32["tau"] - t64).abs() / t64.abs().clamp_min(1e-300)
    assert float(rel.max()) <= 1e-5, float(rel.max())
    # tau-only mode gives the same tau and counts
    t = g.trace(o, k, precision=hg.FP64, mode=hg.TAU_ONLY)
    assert torch.equal(t["tau"], t64) and torch.equal(t["count"], r64["count"])
    t = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY)
    assert torch.equal(t["tau"], r32["tau"]) and torch.equal(t["count"], r32["count"])


def test_path_lengths_sum_to_chord(setup):
    w, g, o_np, k_np, o, k, r64, r32 = setup
    n = r64["needed"]
    cnt = r64["count"].long()
    ray = torch.repeat_interleave(torch.arange(o.shape[0], device=DEV), cnt)
    s = torch.zeros(o.shape[0], dtype=torch.float64, device=DEV)
    s.index_add_(0, ray, r64["ds"][:n])
    del ray
    lo, hi = -1.0, 1.0
    kk = k.clone()
    inv = 1.0 / kk
    t1 = (lo - o) * inv
    t2 = (hi - o) * inv
    tn = torch.minimum(t1, t2).nan_to_num(nan=-np.inf).amax(dim=1).clamp_min(0.0)
    tf = torch.maximum(t1, t2).nan_to_num(nan=np.inf).amin(dim=1)
    L = (tf - tn).clamp_min(0.0)
    err = (s - L).abs()
    assert float(err.max()) <= 1e-12, float(err.max())


def test_oracle_sample_bitwise(setup):
    w, g, o_np, k_np, o, k, r64, r32 = setup
    e = g.export()
    og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(o_np.shape[0], size=3000, replace=False))
    idx = np.concatenate([np.arange(200), idx[idx >= 200]])
    ref = og.trace(o_np[idx], k_np[idx])
    assert np.array_equal(r64["count"].cpu().numpy()[idx], ref["count"])
    assert np.array_equal(r64["tau"].cpu().numpy()[idx], ref["tau"])
    off = r64["offsets"].cpu().numpy()
    pos = torch.from_numpy(np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])).to(DEV)
    assert np.array_equal(r64["leaf"].index_select(0, pos).cpu().numpy(), ref["leaf"])
    assert np.array_equal(r64["ds"].index_select(0, pos).cpu().numpy(), ref["ds"])
    pts = np.random.default_rng(8).uniform(-1, 1, size=(20000, 3))
    assert np.array_equal(g.locate(pts).cpu().numpy(), og.locate(pts))


def test_build_sampled_nodes(setup):
    w, g, o_np, k_np, o, k, r64, r32 = setup
    e = g.export()
    fc = e["first_child"].cpu().numpy()
    lv = e["level"].cpu().numpy()
    co = e["coord"].cpu().numpy().astype(np.uint32)
    S = e["S"].cpu().numpy()
    mn = e["rho_min"].cpu().numpy()
    mx = e["rho_max"].cpu().numpy()
    rng = np.random.default_rng(9)
    idx = np.concatenate([np.arange(64), rng.choice(fc.size, size=1500, replace=False)])
    for i in idx:
        s = O.sample_node(w.density, w.criteria, w.tree_type, int(lv[i]), co[i])
        assert abs(s["S"] - S[i]) <= 1e-13 * abs(s["S"]), i
        assert abs(s["rmin"] - mn[i]) <= 1e-13 * abs(s["rmin"]), i
        assert abs(s["rmax"] - mx[i]) <= 1e-13 * abs(s["rmax"]), i
        if s["split"] != (fc[i] >= 0):
            # allowed only within rounding of the mass threshold
            assert abs(s["delta"] / w.criteria.delta_max - 1.0) < 1e-12, i
    # leaf density is S / N
    rho = e["rho"].cpu().numpy()
    no = e["node_of"].cpu().numpy()
    assert np.array_equal(rho, S[no] / w.criteria.n_samples)

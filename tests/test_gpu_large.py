"""Parity on the largest workload: the k-d tree on 97336 clustered clumps
(mass threshold 1e-8, max level 40, min level 9), which needs the wide
reference layout, traced with stellar-disk paths in tau-only mode as the
batches of 1e8 are.

The oracle cannot rebuild this tree in test time, so it checks it piece by
piece: sampled nodes are re-sampled one by one (statistics within 1e-13,
identical split decisions), and a sample of paths is traced by the oracle on
the exported grid (bitwise FP64 parity).  FP32-with-recheck equals FP64 path
for path on the first 1e6 paths; tau-only mode gives the records mode's tau
and counts.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"
N_PATHS = 1_000_000


@pytest.fixture(scope="module")
def large():
    w = W.workload(5)
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


def test_size_and_layout(large):
    w, g, *_ = large
    assert g.n_leaves > (1 << 25)   # beyond the compact layout: wide references
    assert g.max_level <= w.criteria.max_level


def test_fp32_recheck_equals_fp64_and_tau_only(large):
    w, g, o_np, k_np, o, k, r64, r32 = large
    n = r64["needed"]
    assert n == r32["needed"] and torch.equal(r64["count"], r32["count"])
    assert torch.equal(r64["leaf"][:n], r32["leaf"][:n])
    assert torch.equal(r64["ds"][:n].float(), r32["ds"][:n])
    rel = (r32["tau"] - r64["tau"]).abs() / r64["tau"].abs().clamp_min(1e-300)
    assert float(rel.max()) <= 1e-5, float(rel.max())
    t = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY)
    assert torch.equal(t["tau"], r32["tau"]) and torch.equal(t["count"], r32["count"])


def test_oracle_sample(large):
    w, g, o_np, k_np, o, k, r64, r32 = large
    e = g.export()
    og = O.Grid.from_first_child(w.tree_type, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    del e
    idx = np.sort(np.random.default_rng(11).choice(o_np.shape[0], size=1500, replace=False))
    ref = og.trace(o_np[idx], k_np[idx])
    assert np.array_equal(r64["count"].cpu().numpy()[idx], ref["count"])
    assert np.array_equal(r64["tau"].cpu().numpy()[idx], ref["tau"])
    off = r64["offsets"].cpu().numpy()
    pos = torch.from_numpy(np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])).to(DEV)
    assert np.array_equal(r64["leaf"].index_select(0, pos).cpu().numpy(), ref["leaf"])
    assert np.array_equal(r64["ds"].index_select(0, pos).cpu().numpy(), ref["ds"])
    pts = np.random.default_rng(12).uniform(-1, 1, size=(20000, 3))
    assert np.array_equal(g.locate(pts).cpu().numpy(), og.locate(pts))


def test_build_sampled_nodes(large):
    w, g, *_ = large
    e = g.export()
    fc = e["first_child"].cpu().numpy()
    lv = e["level"].cpu().numpy()
    co = e["coord"].cpu().numpy().astype(np.uint32)
    S = e["S"].cpu().numpy()
    mn = e["rho_min"].cpu().numpy()
    mx = e["rho_max"].cpu().numpy()
    del e
    rng = np.random.default_rng(13)
    # one node of every level, then random ones (each costs the oracle a plain
    # loop over all clumps per sample)
    idx = [int(np.nonzero(lv == l)[0][0]) for l in np.unique(lv)]
    idx += list(rng.choice(fc.size, size=60, replace=False))
    for i in idx:
        s = O.sample_node(w.density, w.criteria, w.tree_type, int(lv[i]), co[i])
        assert abs(s["S"] - S[i]) <= 1e-13 * abs(s["S"]), i
        assert abs(s["rmin"] - mn[i]) <= 1e-13 * abs(s["rmin"]), i
        assert abs(s["rmax"] - mx[i]) <= 1e-13 * abs(s["rmax"]), i
        if s["split"] != (fc[i] >= 0):
            assert abs(s["delta"] / w.criteria.delta_max - 1.0) < 1e-12, i

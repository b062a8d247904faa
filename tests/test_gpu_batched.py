"""Batched tracing: many grids of uneven size (octree and k-d mixed) and path
batches of uneven length in one persistent launch per walk pass must give
exactly what separate per-grid calls give, and match the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def batch():
    grids, os_, ks_, ws = [], [], [], []
    for g in range(64):
        w = W.workload(4, g)
        grids.append(hg.build(w.density, w.criteria, w.tree_type, device=DEV))
        o, k = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
        os_.append(torch.from_numpy(o).to(DEV))
        ks_.append(torch.from_numpy(k).to(DEV))
        ws.append(w)
    print(f"[gpu] batch: {sum(g.n_leaves for g in grids)} leaves, "
          f"{sum(o.shape[0] for o in os_)} paths", flush=True)
    return grids, os_, ks_, ws


@pytest.mark.parametrize("block", [128, 256, 512])
@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
def test_batched_equals_one_by_one(batch, prec, block):
    # every block size (records staged in LDS in groups of 16, or 8 for
    # 512-thread blocks)
    grids, os_, ks_, ws = batch
    rb = hg.trace_batched(grids, os_, ks_, precision=prec, mode=hg.RECORDS, chunk=333, block=block)
    tb = hg.trace_batched(grids, os_, ks_, precision=prec, mode=hg.TAU_ONLY, block=block)
    for i, g in enumerate(grids):
        r1 = g.trace(os_[i], ks_[i], precision=prec, mode=hg.RECORDS)
        n = r1["needed"]
        assert rb[i]["needed"] == n
        for key in ("tau", "count", "offsets"):
            assert torch.equal(rb[i][key], r1[key]), (i, key)
        assert torch.equal(rb[i]["leaf"][:n], r1["leaf"][:n]), i
        assert torch.equal(rb[i]["ds"][:n], r1["ds"][:n]), i
        assert torch.equal(tb[i]["tau"], r1["tau"]) and torch.equal(tb[i]["count"], r1["count"])


def test_batched_oracle_sample(batch):
    grids, os_, ks_, ws = batch
    rb = hg.trace_batched(grids, os_, ks_, precision=hg.FP64, mode=hg.RECORDS)
    for i in (0, 1, 2, 3, 10, 63):
        e = grids[i].export()
        og = O.Grid.from_first_child(ws[i].tree_type, e["first_child"].cpu().numpy(),
                                     e["rho"].cpu().numpy())
        m = min(300, os_[i].shape[0])
        ref = og.trace(os_[i][:m].cpu().numpy(), ks_[i][:m].cpu().numpy())
        tot = int(ref["offsets"][-1])
        assert np.array_equal(rb[i]["count"][:m].cpu().numpy(), ref["count"])
        assert np.array_equal(rb[i]["tau"][:m].cpu().numpy(), ref["tau"])
        assert np.array_equal(rb[i]["leaf"][:tot].cpu().numpy(), ref["leaf"])
        assert np.array_equal(rb[i]["ds"][:tot].cpu().numpy(), ref["ds"])


def test_batched_edge_cases(batch):
    grids, os_, ks_, ws = batch
    # empty batches among non-empty ones, a single-path batch
    sel = [grids[0], grids[1], grids[2]]
    o = [os_[0][:0], os_[1][:1], os_[2]]
    k = [ks_[0][:0], ks_[1][:1], ks_[2]]
    rb = hg.trace_batched(sel, o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    assert rb[0]["needed"] == 0 and rb[0]["offsets"].cpu().tolist() == [0]
    r1 = grids[1].trace(o[1], k[1], precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    assert torch.equal(rb[1]["tau"], r1["tau"])
    # a bad direction in one grid's batch is reported for the batch
    kb = ks_[2].clone()
    kb[5] = torch.tensor([2.0, 0.0, 0.0], dtype=torch.float64)
    with pytest.raises(hg.HGError) as ei:
        hg.trace_batched(sel, o, [k[0], k[1], kb], precision=hg.FP64, mode=hg.TAU_ONLY)
    assert ei.value.code == hg.HG_E_DIR

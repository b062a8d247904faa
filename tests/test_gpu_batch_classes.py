"""Batches whose grids fall in several level-table classes (tree type, finest
per-axis depth, domain side): the batched walk takes the classes one at a
time in each block, with one level table, so every class must be walked
and every grid's build and trace must still equal grid_build and grid_trace
bit for bit, for the bound one-walk trace, its graph replay and the two-walk
grid_trace_batched."""
import dataclasses

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"

# (tree, max level, domain side or None for the [-1, 1] cube, paths)
SPECS = [(W.OCTREE, 5, None, 3000), (W.KDTREE, 14, None, 20000), (W.OCTREE, 7, None, 1),
         (W.KDTREE, 20, None, 9000), (W.KDTREE, 14, 4.0, 5000), (W.OCTREE, 6, 4.0, 777),
         (W.KDTREE, 17, None, 12000), (W.OCTREE, 5, None, 64)]


@pytest.fixture(scope="module")
def mixed():
    dens, crit, trees, os_, ks_ = [], [], [], [], []
    for i, (tree, ml, side, n) in enumerate(SPECS):
        w = W.workload(4, i)
        d = w.density if side is None else dataclasses.replace(w.density, lo=(-2.0, -2.0, -2.0), side=side)
        cr = dataclasses.replace(w.criteria, max_level=ml, min_level=min(w.criteria.min_level, ml))
        o, k = W.rays("uniform", n, 7000 + i)
        dens.append(d)
        crit.append(cr)
        trees.append(tree)
        os_.append(torch.from_numpy(o).to(DEV))
        ks_.append(torch.from_numpy(k).to(DEV))
    singles = [hg.build(d, c, t, device=DEV) for d, c, t in zip(dens, crit, trees)]
    print(f"[gpu] batch classes: {len(SPECS)} grids, {sum(g.n_leaves for g in singles)} leaves", flush=True)
    yield dens, crit, trees, os_, ks_, singles
    for g in singles:
        g.free()


def _same(res, ref):
    for i, r in enumerate(ref):
        n = r["needed"]
        assert res[i]["needed"] == n, i
        for key in ("tau", "count", "offsets"):
            assert torch.equal(res[i][key], r[key]), (i, key)
        assert torch.equal(res[i]["leaf"][:n], r["leaf"][:n]), i
        assert torch.equal(res[i]["ds"][:n], r["ds"][:n]), i


@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
def test_classes_batch_equals_single(mixed, prec):
    dens, crit, trees, os_, ks_, singles = mixed
    ref = [g.trace(os_[i], ks_[i], precision=prec, mode=hg.RECORDS) for i, g in enumerate(singles)]
    caps = [2 * g.n_nodes + 64 for g in singles]
    b = hg.Batch(dens, crit, trees, caps, device=DEV)
    # short rows, so that some paths are resumed past their row
    res = b.bind(os_, ks_, precision=prec, mode=hg.RECORDS, capacities=[r["needed"] for r in ref],
                 chunk=500, slab=8)
    b.run(hg.STAGE_ALL)
    nn, nl = b.result()
    for i, g in enumerate(singles):
        assert nn[i] == g.n_nodes and nl[i] == g.n_leaves, i
        gb = b.grid(i)
        ea, eb = gb.export(), g.export()
        assert torch.equal(ea["first_child"], eb["first_child"]), i
        assert torch.equal(ea["rho"], eb["rho"]), i
        del ea
        gb.free()
    _same(res, ref)
    b.capture(hg.STAGE_TRACE)
    for rep in range(2):
        for r in res:
            r["tau"].zero_()
            r["leaf"].fill_(-7)
        torch.cuda.synchronize()
        b.replay(b._capture_stream)
        b.result(b._capture_stream)
        _same(res, ref)
    b.free()
    tb = hg.trace_batched(singles, os_, ks_, precision=prec, mode=hg.RECORDS, chunk=256)
    _same(tb, ref)

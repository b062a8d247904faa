"""Batches built and traced without host synchronisation (batch_* calls):
the level-synchronous construction of all grids at once must give every
grid's arrays exactly as grid_build does, the bound trace exactly what
grid_trace gives, and a captured graph must reproduce the eager pass on every
replay.  Capacity overruns (nodes, records) are reported per batch while the
other grids stay correct."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"
ARRAYS = ("first_child", "level", "coord", "S", "rho_min", "rho_max", "rho", "leaf_of",
          "node_of", "rope")


@pytest.fixture(scope="module")
def clumps():
    ws = [W.workload(4, g) for g in range(64)]
    singles = [hg.build(w.density, w.criteria, w.tree_type, device=DEV) for w in ws]
    rays = [W.rays(w.ray_kind, w.n_rays, w.ray_seed) for w in ws]
    os_ = [torch.from_numpy(o).to(DEV) for o, _ in rays]
    ks_ = [torch.from_numpy(k).to(DEV) for _, k in rays]
    print(f"[gpu] forest: {sum(g.n_leaves for g in singles)} leaves in 64 grids", flush=True)
    yield ws, singles, os_, ks_
    for g in singles:
        g.free()


def _batch(ws, caps):
    return hg.Batch([w.density for w in ws], [w.criteria for w in ws],
                    [w.tree_type for w in ws], caps, device=DEV)


def _same_arrays(a, b):
    ea, eb = a.export(), b.export()
    assert ea["n_nodes"] == eb["n_nodes"] and ea["n_leaves"] == eb["n_leaves"]
    for key in ARRAYS:
        assert torch.equal(ea[key], eb[key]), key


def test_batch_build_equals_grid_build(clumps):
    ws, singles, os_, ks_ = clumps
    caps = [2 * g.n_nodes + 64 for g in singles]
    b = _batch(ws, caps)
    b.run(hg.STAGE_BUILD)
    nn, nl = b.result()
    assert nn == [g.n_nodes for g in singles]
    assert nl == [g.n_leaves for g in singles]
    for i in range(64):
        g = b.grid(i)
        assert g.max_level == singles[i].max_level
        _same_arrays(g, singles[i])
        g.free()
    b.free()


# records: one walk into rows of the library's size, one walk into rows of 4
# (nearly every path resumes past its row), and a counting plus a filling walk
WALKS = {"one-pass": dict(), "rows4": dict(slab=4), "two-pass": dict(passes=2)}


@pytest.mark.parametrize("walk", list(WALKS))
@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
def test_batch_trace_and_graph_replays(clumps, prec, walk):
    ws, singles, os_, ks_ = clumps
    ref = [g.trace(os_[i], ks_[i], precision=prec, mode=hg.RECORDS)
           for i, g in enumerate(singles)]
    caps = [2 * g.n_nodes + 64 for g in singles]
    b = _batch(ws, caps)
    res = b.bind(os_, ks_, precision=prec, mode=hg.RECORDS,
                 capacities=[r["needed"] for r in ref], chunk=700, count_rechecks=True, **WALKS[walk])

    def check():
        for i, r in enumerate(ref):
            n = r["needed"]
            assert res[i]["needed"] == n, i
            for key in ("tau", "count", "offsets"):
                assert torch.equal(res[i][key], r[key]), (i, key)
            assert torch.equal(res[i]["leaf"][:n], r["leaf"][:n]), i
            assert torch.equal(res[i]["ds"][:n], r["ds"][:n]), i

    b.run(hg.STAGE_ALL)
    b.result()
    check()
    b.capture(hg.STAGE_ALL)
    for rep in range(3):
        for r in res:
            r["tau"].zero_()
            r["count"].zero_()
            r["offsets"].fill_(-1)
            r["leaf"].fill_(-7)
        torch.cuda.synchronize()
        b.replay(b._capture_stream)
        b.result(b._capture_stream)
        check()
        # eager work of the program between replays
        singles[rep].trace(os_[rep], ks_[rep], precision=prec, mode=hg.TAU_ONLY)
        torch.cuda.synchronize()
    b.free()


def test_batch_oracle_sample(clumps):
    ws, singles, os_, ks_ = clumps
    sel = [0, 1, 7, 40]
    b = _batch([ws[i] for i in sel], [2 * singles[i].n_nodes + 64 for i in sel])
    res = b.bind([os_[i][:400] for i in sel], [ks_[i][:400] for i in sel], precision=hg.FP64,
                 mode=hg.RECORDS)
    b.run(hg.STAGE_ALL)
    b.result()
    for j, i in enumerate(sel):
        g = b.grid(j)
        e = g.export()
        og = O.Grid.from_first_child(ws[i].tree_type, e["first_child"].cpu().numpy(),
                                     e["rho"].cpu().numpy())
        ref = og.trace(os_[i][:400].cpu().numpy(), ks_[i][:400].cpu().numpy())
        tot = int(ref["offsets"][-1])
        assert np.array_equal(res[j]["count"].cpu().numpy(), ref["count"])
        assert np.array_equal(res[j]["tau"].cpu().numpy(), ref["tau"])
        assert np.array_equal(res[j]["leaf"][:tot].cpu().numpy(), ref["leaf"])
        assert np.array_equal(res[j]["ds"][:tot].cpu().numpy(), ref["ds"])
        g.free()
    b.free()


def test_node_capacity_overrun_is_reported(clumps):
    ws, singles, os_, ks_ = clumps
    sel = [2, 3]
    caps = [singles[2].n_nodes - 1, singles[3].n_nodes]
    b = _batch([ws[i] for i in sel], caps)
    b.run(hg.STAGE_BUILD)
    with pytest.raises(hg.HGError) as ei:
        b.result()
    assert ei.value.code == hg.HG_E_LIMIT
    with pytest.raises(hg.HGError):
        b.grid(0)
    g = b.grid(1)
    _same_arrays(g, singles[3])
    g.free()
    b.free()


@pytest.mark.parametrize("walk", list(WALKS))
def test_record_capacity_overrun_and_empty_batch(clumps, walk):
    ws, singles, os_, ks_ = clumps
    sel = [4, 5, 6]
    ref = [singles[i].trace(os_[i], ks_[i], precision=hg.FP32_RECHECK, mode=hg.RECORDS)
           for i in sel]
    b = _batch([ws[i] for i in sel], [2 * singles[i].n_nodes + 64 for i in sel])
    o = [os_[4], os_[5][:0], os_[6]]
    k = [ks_[4], ks_[5][:0], ks_[6]]
    caps = [ref[0]["needed"], 0, ref[2]["needed"] - 1]
    res = b.bind(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacities=caps, **WALKS[walk])
    b.run(hg.STAGE_ALL)
    with pytest.raises(hg.HGError) as ei:
        b.result()
    assert ei.value.code == hg.HG_E_CAPACITY
    assert res[1]["needed"] == 0 and res[1]["offsets"].cpu().tolist() == [0]
    assert res[2]["needed"] == ref[2]["needed"]
    assert torch.equal(res[2]["tau"], ref[2]["tau"])
    n = ref[0]["needed"]
    assert torch.equal(res[0]["leaf"][:n], ref[0]["leaf"][:n])
    assert torch.equal(res[0]["ds"][:n], ref[0]["ds"][:n])
    b.free()


@pytest.mark.parametrize("tree", [W.OCTREE, W.KDTREE], ids=["octree", "kd"])
def test_grid_build_with_capacity_equals_level_synchronised(tree):
    # grid_build with a node capacity runs the batch construction for one grid
    w = W.workload(3, tree_type=tree)
    cr = w.criteria
    cr.max_level = 9 if tree == W.OCTREE else 24
    a = hg.build(w.density, cr, tree, device=DEV)
    b = hg.build(w.density, cr, tree, device=DEV, max_nodes=a.n_nodes + 10)
    _same_arrays(a, b)
    o, k = W.rays("uniform", 20000, 5)
    ra = a.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    rb = b.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    assert torch.equal(ra["tau"], rb["tau"]) and torch.equal(ra["leaf"][:ra["needed"]], rb["leaf"][:rb["needed"]])
    with pytest.raises(hg.HGError) as ei:
        hg.build(w.density, cr, tree, device=DEV, max_nodes=a.n_nodes - 1)
    assert ei.value.code == hg.HG_E_LIMIT
    a.free()
    b.free()

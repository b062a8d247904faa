"""The walk's launch shape changes its speed, never its results: every
candidate shape the autotuners try traces bit for bit like the defaults, and
the tuned shapes (single grid and batch) are valid and give the same
results."""
import itertools
import json

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def disk():
    w = W.workload(2)
    w.criteria.delta_max = 1e-5   # about 1e5 leaves: a quick but multi-level tree
    g = hg.build(w.density, w.criteria, w.tree_type, device=DEV)
    o, k = W.rays(w.ray_kind, 200_000, w.ray_seed)
    yield w, g, torch.from_numpy(o).to(DEV), torch.from_numpy(k).to(DEV)
    g.free()


def _same(a, b, records=True):
    assert torch.equal(a["tau"], b["tau"]) and torch.equal(a["count"], b["count"])
    if records:
        n = a["needed"]
        assert n == b["needed"] and torch.equal(a["offsets"], b["offsets"])
        assert torch.equal(a["leaf"][:n], b["leaf"][:n]) and torch.equal(a["ds"][:n], b["ds"][:n])


@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
def test_every_launch_shape_gives_the_same_result(disk, prec):
    w, g, o, k = disk
    o, k = o[:20000], k[:20000]
    ref = g.trace(o, k, precision=prec, mode=hg.RECORDS, persistent=0)
    for block, lds, chunk, refill in itertools.product((128, 256, 512), (-1, 4096, 65536),
                                                       (32, 1024), (4, 32)):
        r = g.trace(o, k, precision=prec, mode=hg.RECORDS, block=block, lds_bytes=lds,
                    chunk=chunk, refill_min=refill, capacity=ref["needed"])
        _same(ref, r)


def test_grid_tune_and_cache(disk, tmp_path):
    w, g, o, k = disk
    for mode in (hg.TAU_ONLY, hg.RECORDS):
        t = g.tune(o, k, precision=hg.FP32_RECHECK, mode=mode)
        assert t["block"] in (128, 256, 512) and t["chunk"] > 0 and 1 <= t["refill_min"] <= 64
        assert t["lds_bytes"] <= 65536 and t["ms"] > 0
        ref = g.trace(o, k, precision=hg.FP32_RECHECK, mode=mode)
        r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=mode, tuned=t)
        _same(ref, r, records=mode == hg.RECORDS)
    path = str(tmp_path / "tune.json")
    t1 = hg.tune_cached(g, o, k, path=path)
    t2 = hg.tune_cached(g, o, k, path=path)
    assert t1 == t2 and len(json.load(open(path))) == 1


def test_batch_tune(disk):
    ws = [W.workload(4, i) for i in range(8)]
    singles = [hg.build(x.density, x.criteria, x.tree_type, device=DEV) for x in ws]
    rays = [W.rays(x.ray_kind, x.n_rays, x.ray_seed) for x in ws]
    os_ = [torch.from_numpy(a).to(DEV) for a, _ in rays]
    ks_ = [torch.from_numpy(b).to(DEV) for _, b in rays]
    ref = [s.trace(os_[i], ks_[i], precision=hg.FP32_RECHECK, mode=hg.RECORDS)
           for i, s in enumerate(singles)]
    b = hg.Batch([x.density for x in ws], [x.criteria for x in ws], [x.tree_type for x in ws],
                 [2 * s.n_nodes + 64 for s in singles], device=DEV)
    res = b.bind(os_, ks_, precision=hg.FP32_RECHECK, mode=hg.RECORDS,
                 capacities=[r["needed"] for r in ref])
    b.run(hg.STAGE_BUILD)
    b.result()
    t = b.tune()
    assert t["ms"] > 0 and t["block"] in (128, 256, 512) and t["chunk"] > 0
    res = b.results
    b.capture(hg.STAGE_ALL)
    b.replay(b._capture_stream)
    b.result(b._capture_stream)
    for i in range(8):
        _same(ref[i], res[i])
    b.free()
    for s in singles:
        s.free()

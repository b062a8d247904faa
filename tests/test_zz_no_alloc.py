"""grid_trace_noalloc (the entry point for callers that cannot allocate) gives
exactly what grid_trace gives, called through the C ABI twice in a row on one
device, the second time with fewer paths (the fixed work space keeps the
first call's contents), in both trace modes and both precisions."""
import ctypes as C

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def disk():
    w = W.workload(2)
    w.criteria.delta_max = 1e-5
    g = hg.build(w.density, w.criteria, w.tree_type, device=DEV)
    o, k = W.rays(w.ray_kind, 400_000, w.ray_seed)
    o = torch.from_numpy(o).to(DEV)
    k = torch.from_numpy(k).to(DEV)
    # a path that misses and one that starts outside the domain
    o[:2] = torch.tensor([[3.0, 0, 0], [-1.5, 0.1, 0.2]], dtype=torch.float64)
    k[:2] = torch.tensor([[1.0, 0, 0], [1.0, 0, 0]], dtype=torch.float64)
    yield g, o, k
    g.free()


def _same(a, b, records):
    for key in ("tau", "count") + (("offsets",) if records else ()):
        assert torch.equal(a[key], b[key]), key
    if records:
        n = a["needed"]
        assert n == b["needed"]
        assert torch.equal(a["leaf"][:n], b["leaf"][:n])
        assert torch.equal(a["ds"][:n], b["ds"][:n])


@pytest.mark.parametrize("mode", [hg.TAU_ONLY, hg.RECORDS], ids=["tau", "records"])
@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
def test_noalloc_equals_grid_trace(disk, mode, prec):
    g, o, k = disk
    records = mode == hg.RECORDS
    for n in (o.shape[0], 123_457):   # the second call smaller than the first
        print(f"noalloc: mode {mode} precision {prec} n {n}", flush=True)
        ref = g.trace(o[:n], k[:n], precision=prec, mode=mode)
        cap = ref["needed"] if records else None
        got = g.trace(o[:n], k[:n], precision=prec, mode=mode, capacity=cap, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got, records)


def test_noalloc_capacity_and_limit(disk):
    g, o, k = disk
    ref = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    need = ref["needed"]
    with pytest.raises(hg.HGError) as ei:
        g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, capacity=need - 1, noalloc=True)
    assert ei.value.code == hg.HG_E_CAPACITY
    # more paths than the fixed work space allows: rejected before any work is enqueued
    opts = hg.TraceOpts()
    opts.precision = hg.FP32_RECHECK
    opts.mode = hg.TAU_ONLY
    opts.kappa = 1.0
    to = hg.TraceOut()
    tau = torch.empty(1, dtype=torch.float64, device=DEV)
    cnt = torch.empty(1, dtype=torch.int32, device=DEV)
    to.tau = tau.data_ptr()
    to.count = cnt.data_ptr()
    n_max = (hg.NOALLOC_SCRATCH_BYTES // 8 - 1) * 2048
    rc = hg.lib().grid_trace_noalloc(g._h, C.c_void_p(o.data_ptr()), C.c_void_p(k.data_ptr()), n_max + 1,
                                     C.byref(opts), C.byref(to), None)
    assert rc == hg.HG_E_LIMIT

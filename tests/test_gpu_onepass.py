"""Records mode in one walk (per-path rows, copy into the CSR slices, a
filling walk over the paths whose records overflow their row) gives exactly
the two-walk result, for any row size."""
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
    o, k = W.rays(w.ray_kind, 300_000, w.ray_seed)
    o = torch.from_numpy(o).to(DEV)
    k = torch.from_numpy(k).to(DEV)
    # a few paths that miss, start outside, or run along axes
    o[:4] = torch.tensor([[3.0, 0, 0], [-1.5, 0.1, 0.2], [0.0, 0.0, 0.0], [0.5, -0.25, 0.125]],
                         dtype=torch.float64)
    k[:4] = torch.tensor([[1.0, 0, 0], [1.0, 0, 0], [0, 0, 1.0], [0, -1.0, 0]], dtype=torch.float64)
    yield g, o, k
    g.free()


def _same(a, b):
    n = a["needed"]
    assert n == b["needed"]
    for key in ("tau", "count", "offsets"):
        assert torch.equal(a[key], b[key]), key
    assert torch.equal(a["leaf"][:n], b["leaf"][:n]) and torch.equal(a["ds"][:n], b["ds"][:n])


@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
@pytest.mark.parametrize("slab", [4, 16, 128, 1024])
def test_one_pass_equals_two_pass(disk, prec, slab):
    g, o, k = disk
    two = g.trace(o, k, precision=prec, mode=hg.RECORDS, passes=2)
    one = g.trace(o, k, precision=prec, mode=hg.RECORDS, passes=1, slab=slab,
                  capacity=two["needed"], count_rechecks=True)
    _same(two, one)
    assert int(two["count"].max()) > 16   # the small rows do overflow


def test_one_pass_capacity_error(disk):
    g, o, k = disk
    r = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.TAU_ONLY)
    need = int(r["count"].sum())
    with pytest.raises(hg.HGError) as ei:
        g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=1, capacity=need - 1)
    assert ei.value.code == hg.HG_E_CAPACITY
    # the binding retries with the size it reports
    r1 = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=1)
    assert r1["needed"] == need and torch.equal(r1["tau"], r["tau"])


def test_scratch_grows_and_is_released(disk):
    # the one-walk scratch is kept per device: a smaller call after a larger
    # one reuses it, a larger row size grows it, and after its release the
    # next call allocates it again; every result equals the two-walk result
    g, o, k = disk
    two = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=2)
    m = o.shape[0] // 3
    small = g.trace(o[:m], k[:m], precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=2)
    for slab, oo, kk, want in ((64, o, k, two), (64, o[:m], k[:m], small), (512, o, k, two)):
        _same(want, g.trace(oo, kk, precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=1, slab=slab))
    hg.release_scratch(DEV)
    hg.release_scratch(DEV)   # nothing held: a no-op
    _same(two, g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, passes=1))


@pytest.mark.parametrize("prec", [hg.FP32_RECHECK, hg.FP64], ids=["fp32r", "fp64"])
@pytest.mark.parametrize("persistent", [0, 1, 2])
def test_one_pass_walk_kinds(disk, prec, persistent):
    # one thread per path or persistent, for the row walk (bit 0) and the
    # resuming fill walk (bit 1): rows of separate leaf / ds areas or of
    # (leaf, ds) pairs, records staged in registers or in LDS
    g, o, k = disk
    two = g.trace(o, k, precision=prec, mode=hg.RECORDS, passes=2)
    one = g.trace(o, k, precision=prec, mode=hg.RECORDS, passes=1, slab=64, persistent=persistent,
                  capacity=two["needed"])
    _same(two, one)


def test_grid_blocks_are_reused():
    # a freed grid's array block serves the next build of the same size; the
    # grids built in reused blocks are the same grid bit for bit
    w = W.workload(1)
    ref = None
    for it in range(3):
        g = hg.build(w.density, w.criteria, w.tree_type, device=DEV, max_nodes=1 << 16)
        e = g.export()
        cur = (e["first_child"].cpu(), e["rho"].cpu())
        if ref is None:
            ref = cur
        else:
            assert torch.equal(ref[0], cur[0]) and torch.equal(ref[1], cur[1])
        g.free()
    hg.release_scratch(DEV)

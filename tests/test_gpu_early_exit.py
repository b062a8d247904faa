"""The early-exit walks against the oracle's consumers, bit for bit: the
segment optical depth of Sect. 3.2 (grid_trace_segment) and the Monte Carlo
interaction point (grid_trace_interact), both computed by the oracle from its
own full trace.  In both exit-decision precisions: the leaf sequence and the
FP64 ds are the same, and these walks sum tau in FP64 from the FP64 leaf
densities."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import oracle.quality as Q
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"
PRECS = [hg.FP64, hg.FP32_RECHECK]
PIDS = ["fp64", "fp32r"]


def _case(name):
    if name == "disk-octree":
        w = W.workload(1)
        return w.density, w.criteria, w.tree_type
    w = W.workload(3)
    cr = w.criteria
    cr.max_level = 18
    return w.density, cr, W.KDTREE


@pytest.fixture(scope="module", params=["disk-octree", "torus-clumps-kd18"])
def grid(request):
    d, cr, tree = _case(request.param)
    g = hg.build(d, cr, tree, device=DEV)
    e = g.export()
    og = O.Grid.from_first_child(tree, e["first_child"].cpu().numpy(), e["rho"].cpu().numpy())
    yield g, og
    g.free()


def _inside_paths(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, size=(n, 3))
    k = rng.normal(size=(n, 3))
    k /= np.linalg.norm(k, axis=1)[:, None]
    return a, k


def _segment_counts(ref, s_max):
    """Leaves with ds > 0 that the first s_max of each path enters."""
    ds = np.asarray(ref["ds"], dtype=np.float64)
    off = np.asarray(ref["offsets"])
    out = np.zeros(off.size - 1, dtype=np.int32)
    for i in range(off.size - 1):
        s = 0.0
        for d in ds[off[i]:off[i + 1]]:
            if not s < s_max[i]:
                break
            out[i] += 1
            s += d
    return out


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
def test_segment(grid, prec):
    g, og = grid
    a, k = _inside_paths(4000, 21)
    rng = np.random.default_rng(22)
    s_max = rng.uniform(0.0, 4.0, size=a.shape[0])   # some beyond the path's end
    s_max[:6] = [0.0, -1.0, 1e-300, math.inf, 5e-3, 3.5]
    tau, cnt = g.trace_segment(a, k, s_max, precision=prec)
    ref = og.trace(a, k)
    rho = og.leaves()["rho"]
    assert np.array_equal(tau.cpu().numpy(), Q.segment_tau(ref, rho, s_max))
    assert np.array_equal(cnt.cpu().numpy(), _segment_counts(ref, s_max))
    # an unbounded segment is the whole path: the FP64 tau-only walk's tau
    full = g.trace(a[:6], k[:6], precision=hg.FP64, mode=hg.TAU_ONLY)
    assert tau[3].item() == full["tau"][3].item()
    assert cnt[3].item() == full["count"][3].item()
    assert tau[0].item() == 0.0 and tau[1].item() == 0.0 and cnt[0].item() == 0


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
def test_interaction(grid, prec):
    g, og = grid
    a, k = _inside_paths(4000, 31)
    ref = og.trace(a, k)
    # tau* = -ln(1 - u) on the scale of the paths' own optical depths
    u = np.random.default_rng(32).uniform(size=a.shape[0])
    tau_star = -np.log1p(-u) * float(np.median(ref["tau"]))
    tau_star[:4] = [0.0, 1e300, 1e-12, math.inf]
    leaf, s = g.trace_interact(a, k, tau_star, precision=prec)
    want_leaf, want_s = Q.interaction(ref, og.leaves()["rho"], tau_star)
    assert np.array_equal(leaf.cpu().numpy(), want_leaf)
    assert np.array_equal(s.cpu().numpy(), want_s)
    assert leaf[1].item() == -1 and leaf[3].item() == -1
    # some paths interact and some do not
    hit = want_leaf >= 0
    assert 0.05 < hit.mean() < 0.95
    # the post-pass over a full records trace agrees
    r = g.trace(a, k, precision=hg.FP64, mode=hg.RECORDS)
    pl, ps = g.interact(r, tau_star)
    assert torch.equal(pl, leaf) and torch.equal(ps, s)


def test_paths_outside_and_nan(grid):
    g, og = grid
    # a miss (outside, pointing away), an entry from outside, a NaN s_max
    a = np.array([[3.0, 0.0, 0.0], [-3.0, 0.1, 0.2], [0.1, 0.2, 0.3]])
    k = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    tau, cnt = g.trace_segment(a, k, [1.0, math.inf, math.nan])
    full = g.trace(a, k, precision=hg.FP64, mode=hg.TAU_ONLY)
    assert tau[0].item() == 0.0 and cnt[0].item() == 0
    assert tau[1].item() == full["tau"][1].item() and cnt[1].item() == full["count"][1].item()
    assert tau[2].item() == 0.0 and cnt[2].item() == 0
    # s counts from the origin: a segment ending before the domain entry is empty
    tau2, cnt2 = g.trace_segment(a[1:2], k[1:2], [1.5])
    assert tau2[0].item() == 0.0 and cnt2[0].item() == 0
    leaf, s = g.trace_interact(a, k, [1.0, 1e300, 1e300])
    assert leaf[0].item() == -1 and s[0].item() == 0.0
    assert leaf[1].item() == -1 and s[1].item() == 4.0   # enters at s = 2, leaves at s = 4
    # a direction that is not a unit vector is an error
    with pytest.raises(RuntimeError):
        g.trace_interact(a[:1], np.array([[2.0, 0.0, 0.0]]), [1.0])

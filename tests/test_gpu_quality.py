"""The walk's consumers on the GPU against the oracle: density differences
and grid optical depths bit for bit, interaction points bit for bit, the
Gauss-Legendre true optical depth within rounding (its sums run in a
different order)."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.quality as Q
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


def _segments(n, seed):
    # start and end points uniform in the domain (Sect. 3.2)
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, size=(n, 3))
    b = rng.uniform(-1, 1, size=(n, 3))
    L = np.linalg.norm(b - a, axis=1)
    return a, (b - a) / L[:, None], L


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
    yield d, g, og
    g.free()


def test_density_diff(grid):
    d, g, og = grid
    pts = np.random.default_rng(1).uniform(-1, 1, size=(20000, 3))
    pts[:3] = [[1.0, 1.0, 1.0], [-1.0, 0.0, 0.5], [1.5, 0.0, 0.0]]   # faces, outside
    got = g.density_diff(d, pts).cpu().numpy()
    want = Q.density_diff(og, d, pts)
    assert np.array_equal(np.isnan(got), np.isnan(want)) and np.isnan(got[2])
    ok = ~np.isnan(want)
    # rho_g is bitwise the oracle's; rho_t differs by the last-bit rounding of
    # the device exp against the host exp (as in the build's sampled sums)
    rho_g = og.leaves()["rho"][og.locate(pts[ok])]
    rho_t = want[ok] + rho_g
    assert np.all(np.abs(got[ok] - want[ok]) <= 1e-14 * (np.abs(rho_t) + np.abs(rho_g)) + 1e-300)
    assert np.mean(got[ok] == want[ok]) > 0.5


@pytest.mark.parametrize("prec", [hg.FP64, hg.FP32_RECHECK], ids=["fp64", "fp32r"])
def test_segment_and_true_tau(grid, prec):
    d, g, og = grid
    a, k, L = _segments(3000, 2)
    r = g.trace(a, k, precision=prec, mode=hg.RECORDS)
    tg = g.segment_tau(r, L).cpu().numpy()
    tt = g.true_tau(d, a, k, r, L).cpu().numpy()
    ref = og.trace(a, k)
    if prec == hg.FP32_RECHECK:
        # the FP32-recheck walk records ds32 = ds64 rounded to FP32
        ref = dict(ref, ds=ref["ds"].astype(np.float32).astype(np.float64))
    assert np.array_equal(tg, Q.segment_tau(ref, og.leaves()["rho"], L))
    want_tt = Q.true_tau(d, a, k, ref, L)
    assert np.allclose(tt, want_tt, rtol=1e-12, atol=1e-15)
    # the measure itself: a finite spread of tau_t - tau_g
    dtau = tt - tg
    assert np.isfinite(dtau).all() and dtau.std() > 0


def test_interaction(grid):
    d, g, og = grid
    o, k = W.rays("uniform", 5000, 3)
    r = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS)
    u = np.random.default_rng(4).uniform(0, 1, 5000)
    tau_star = -np.log1p(-u) * 0.2
    leaf, s = g.interact(r, tau_star)
    ref = og.trace(o, k)
    wl, ws = Q.interaction(ref, og.leaves()["rho"], tau_star)
    assert np.array_equal(leaf.cpu().numpy(), wl)
    assert np.array_equal(s.cpu().numpy(), ws)
    assert (wl >= 0).any() and (wl < 0).any()

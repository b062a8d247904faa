"""Degenerate grids: a single cell (the root never split) and a single
level.  Every path inside the domain crosses the one cell, with its chord
as ds and tau = kappa rho chord, in every precision and records mode."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


def _chord(o, k):
    with np.errstate(divide="ignore"):
        t = np.where(k > 0, (1 - o) / k, np.where(k < 0, (-1 - o) / k, np.inf))
    return t.min(axis=1)


@pytest.mark.parametrize("tree", [W.OCTREE, W.KDTREE], ids=["octree", "kd"])
def test_single_cell(tree):
    rho, kappa = 1.75, 0.5
    d = W.uniform(rho)
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=2.0, max_level=0, seed=1)
    g = hg.build(d, cr, tree, device=DEV)
    assert g.n_leaves == 1 and g.n_nodes == 1
    rng = np.random.default_rng(2)
    o = rng.uniform(-0.9, 0.9, size=(5000, 3))
    k = rng.normal(size=(5000, 3))
    k /= np.linalg.norm(k, axis=1)[:, None]
    L = _chord(o, k)
    for prec in (hg.FP64, hg.FP32_RECHECK):
        for passes in (1, 2):
            r = g.trace(o, k, precision=prec, mode=hg.RECORDS, kappa=kappa, passes=passes)
            assert r["needed"] == 5000
            assert np.all(r["count"].cpu().numpy() == 1)
            assert np.all(r["leaf"][:5000].cpu().numpy() == 0)
            ds = r["ds"][:5000].cpu().numpy().astype(np.float64)
            tol = 1e-12 if prec == hg.FP64 else 1e-6
            assert np.allclose(ds, L, rtol=tol, atol=0)
            assert np.allclose(r["tau"].cpu().numpy(), kappa * rho * L, rtol=max(tol, 1e-7), atol=0)
    # locate: every point inside is in leaf 0, outside -1
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [-1.0, 0.5, 0.25], [1.5, 0.0, 0.0]])
    assert g.locate(pts).cpu().numpy().tolist() == [0, 0, 0, -1]
    g.free()

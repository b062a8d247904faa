"""The optical-depth recipe of Sect. 4.1 on the GPU against the oracle's:
per-leaf optical depths, the order statistic found by radix select, and the
second grid."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import oracle.recipe as RC
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("tree,ml", [(W.OCTREE, 10), (W.KDTREE, 30)], ids=["octree", "kd"])
def test_recipe_matches_oracle(tree, ml):
    d = W.exp_disk()
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-4, max_level=ml, kappa=2.0, seed=3)
    # first pass: leaf optical depths and their order statistic
    g1 = hg.build(d, cr, tree, device=DEV)
    o1 = O.Grid.build(d, cr, tree)
    assert g1.n_leaves == o1.n_leaves
    got = g1.leaf_tau(cr.kappa, cr.n_samples).cpu().numpy()
    want = RC.leaf_tau(o1, cr.kappa, cr.n_samples)
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    for f in (0.0, 0.5, 0.9, 1.0):
        k = min(got.size - 1, int(math.floor(f * got.size)))
        assert g1.tau_percentile(cr.kappa, cr.n_samples, f) == np.sort(got)[k]
    g1.free()
    # the whole recipe
    g2, tm = hg.Grid.build_tau_recipe(d, cr, tree, fraction=0.9, device=DEV)
    o2, otm = RC.build_with_recipe(d, cr, tree)
    assert abs(tm - otm) <= 1e-13 * otm
    assert g2.n_leaves == o2.n_leaves > o1.n_leaves
    e = g2.export()
    assert np.array_equal(e["first_child"].cpu().numpy(), o2.nodes()["first_child"])
    g2.free()


def test_percentile_edge_cases():
    # ties everywhere (uniform medium) and a single-leaf grid
    d = W.Density(box=(-1, -1, -1, 1, 1, 1, 3.0))
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-3, max_level=12, seed=5)
    g = hg.build(d, cr, W.KDTREE, device=DEV)
    t = g.leaf_tau(1.0).cpu().numpy()
    assert np.all(t == t[0]) and g.tau_percentile(1.0, 64, 0.9) == t[0]
    g.free()
    cr.max_level = 0
    g = hg.build(d, cr, W.OCTREE, device=DEV)
    assert g.n_leaves == 1 and g.tau_percentile(1.0, 64, 0.9) == g.leaf_tau(1.0).item()
    g.free()

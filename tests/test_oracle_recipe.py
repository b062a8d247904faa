"""Pins of the optical-depth recipe of Sect. 4.1 (oracle/recipe.py)."""
import math

import numpy as np

import oracle as O
import oracle.recipe as RC
import workloads as W


def _box_tau(g, kappa):
    # Eq. (2) from the leaf boxes and the leaf densities (M = rho V)
    lo, hi = g.leaf_boxes()
    rho = g.leaves()["rho"]
    a, b, c = (hi - lo).T
    V = a * b * c
    return kappa * (rho * V) * np.sqrt(a * a + b * b + c * c) / (a * b * c)


def _disk_criteria():
    d = W.exp_disk()
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-4, max_level=18, kappa=2.0, seed=3)
    return d, cr


def test_leaf_tau_matches_leaf_boxes():
    d, cr = _disk_criteria()
    for tree in (W.OCTREE, W.KDTREE):
        cr.max_level = 8 if tree == W.OCTREE else 18
        g = O.Grid.build(d, cr, tree)
        assert np.array_equal(RC.leaf_tau(g, cr.kappa, cr.n_samples), _box_tau(g, cr.kappa))


def test_percentile_position():
    d, cr = _disk_criteria()
    g = O.Grid.build(d, cr, W.KDTREE)
    t = RC.leaf_tau(g, cr.kappa, cr.n_samples)
    tm = RC.tau_percentile(g, cr.kappa, cr.n_samples, 0.9)
    k = int(math.floor(0.9 * t.size))
    assert np.sum(t < tm) <= k < np.sum(t <= tm)
    assert RC.tau_percentile(g, cr.kappa, cr.n_samples, 0.0) == t.min()
    assert RC.tau_percentile(g, cr.kappa, cr.n_samples, 1.0) == t.max()


def test_uniform_medium_recipe_changes_nothing():
    d = W.Density(box=(-1, -1, -1, 1, 1, 1, 3.0))
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-3, max_level=12, seed=5)
    g1 = O.Grid.build(d, cr, W.KDTREE)
    g2, tm = RC.build_with_recipe(d, cr, W.KDTREE)
    t = RC.leaf_tau(g1, cr.kappa, cr.n_samples)
    assert np.all(t == t[0]) and tm == t[0]
    assert np.array_equal(g1.nodes()["first_child"], g2.nodes()["first_child"])


def test_recipe_grid_respects_tau_max():
    d, cr = _disk_criteria()
    for tree, ml in ((W.OCTREE, 10), (W.KDTREE, 30)):
        cr.max_level = ml
        g1 = O.Grid.build(d, cr, tree)
        g2, tm = RC.build_with_recipe(d, cr, tree)
        assert g2.n_leaves > g1.n_leaves
        t2 = _box_tau(g2, cr.kappa)
        lv = g2.nodes()["level"][g2.leaves()["node_of"]]
        assert np.all((t2 <= tm) | (lv == ml))

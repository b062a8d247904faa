"""Pins for the k-d split variants of Sect. 2.2 in the oracle.

* Orientation by the strongest density gradient (tree type KDGRAD): a medium
  that varies along z only splits every node across z unless the node is
  centred on the plane of symmetry (where no axis has a gradient); a uniform
  medium has no gradient anywhere, and the tie rule (fewest halvings, then
  lowest axis) reproduces the cyclic tree node for node.
* Equal-mass location: for a piecewise-constant medium the plane that halves
  the cell's mass has a closed form.
* The cyclic midpoint tree and the gradient tree compared on the disk (the
  comparison behind the paper's choice of the cyclic rule): both honour the
  same criteria, and their cell counts are reported.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _crit(**kw):
    base = dict(total_mass=8.0, delta_max=1.0, tau_max=math.inf, q_max=1.0, kappa=1.0,
                min_level=0, max_level=12, n_samples=64, seed=2024)
    base.update(kw)
    return W.Criteria(**base)


def _centres(nd, lo=-1.0, side=2.0):
    w = side * np.exp2(-nd["depth"].astype(np.float64))
    return lo + (nd["coord"].astype(np.float64) + 0.5) * w, w


def test_uniform_medium_gives_the_cyclic_tree():
    d = W.uniform(1.0)
    cr = _crit(delta_max=2e-3)
    cyc = O.Grid.build(d, cr, O.KDTREE)
    grd = O.Grid.build(d, cr, O.KDGRAD)
    a, b = cyc.nodes(), grd.nodes()
    assert np.array_equal(a["first_child"], b["first_child"])
    internal = a["first_child"] >= 0
    assert np.array_equal(b["axis"][internal], a["level"][internal] % 3)
    assert np.array_equal(a["depth"], b["depth"]) and np.array_equal(a["coord"], b["coord"])
    assert np.all(b["axis"][~internal] == -1)


def test_medium_varying_along_z_splits_across_z():
    # exp(-R/hR - |z|/hz) with hR = 1e300: R/hR never changes the exponent, so
    # the density depends on z alone and only z can have a gradient
    d = W.Density(disk=(1.0, 1e300, 0.1))
    mass = 4.0 * 2.0 * 0.1 * (1.0 - math.exp(-10.0))   # the z column times the 2 x 2 face
    cr = _crit(total_mass=mass, delta_max=1e-3, max_level=14)
    g = O.Grid.build(d, cr, O.KDGRAD)
    nd = g.nodes()
    internal = nd["first_child"] >= 0
    assert internal.sum() > 100
    c, _ = _centres(nd)
    on_plane = internal & (c[:, 2] == 0.0)
    off_plane = internal & (c[:, 2] != 0.0)
    assert off_plane.sum() > 0.9 * internal.sum()
    assert np.all(nd["axis"][off_plane] == 2)
    # on z = 0 no axis has a gradient: the axis with the fewest halvings
    dep = nd["depth"][on_plane].astype(int)
    fewest = np.argmin(dep, axis=1)    # lowest index among the minima
    assert np.array_equal(nd["axis"][on_plane], fewest)
    # children follow their parent's axis: depth grows on that axis only
    fc = nd["first_child"]
    for i in np.flatnonzero(internal)[:500]:
        ax = nd["axis"][i]
        for k in (0, 1):
            ddep = nd["depth"][fc[i] + k].astype(int) - nd["depth"][i].astype(int)
            assert ddep[ax] == 1 and ddep.sum() == 1
            assert nd["coord"][fc[i] + k][ax] == 2 * nd["coord"][i][ax] + k


def test_gradient_tree_is_a_partition_and_traces_like_brute_force():
    # leaf boxes tile the domain, and the top-down walk finds what brute force finds
    d = W.exp_disk()
    cr = _crit(total_mass=W.total_mass(d), delta_max=2e-4, max_level=14)
    g = O.Grid.build(d, cr, O.KDGRAD)
    lo, hi = g.leaf_boxes()
    assert math.isclose(float(np.prod(hi - lo, axis=1).sum()), 8.0, rel_tol=0, abs_tol=1e-12)
    nd = g.nodes()
    assert set(np.unique(nd["axis"][nd["first_child"] >= 0])) <= {0, 1, 2}
    rng = np.random.default_rng(4)
    o = rng.uniform(-1, 1, size=(40, 3))
    k = rng.normal(size=(40, 3))
    k /= np.linalg.norm(k, axis=1)[:, None]
    r = g.trace(o, k)
    for i in range(40):
        b = g.trace_brute(o[i], k[i])
        sl = slice(r["offsets"][i], r["offsets"][i + 1])
        assert np.array_equal(r["leaf"][sl], b["leaf"])
        assert np.allclose(r["ds"][sl], b["ds"], rtol=0, atol=1e-12)
    # a grid rebuilt from its first-child array and split axes is the same grid
    e = O.Grid.from_first_child(O.KDGRAD, nd["first_child"], g.leaves()["rho"], axis=nd["axis"])
    ne = e.nodes()
    assert np.array_equal(ne["depth"], nd["depth"]) and np.array_equal(ne["coord"], nd["coord"])
    pts = rng.uniform(-1, 1, size=(2000, 3))
    assert np.array_equal(e.locate(pts), g.locate(pts))


@pytest.mark.parametrize("edge,want", [(0.5, -0.25), (1.0, 0.0), (-0.5, -0.75)])
def test_equal_mass_plane_of_a_piecewise_constant_medium(edge, want):
    # density 3 on x <= edge, 0 beyond: the lower (edge + 1) / 2 of the filled
    # part holds half the mass, so the plane is at x = -1 + (edge + 1) / 2
    d = W.Density(box=(-1.0, -1.0, -1.0, edge, 1.0, 1.0, 3.0))
    x = O.equal_mass_plane(d, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), 0, m=64, iters=52)
    assert abs(x - want) <= 1e-12
    # across y the filled part spans the whole cell: the midpoint
    y = O.equal_mass_plane(d, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), 1, m=64, iters=52)
    assert abs(y) <= 1e-12


def test_cell_counts_cyclic_and_gradient_on_the_disk():
    d = W.exp_disk()
    cr = _crit(total_mass=W.total_mass(d), delta_max=1e-4, max_level=18)
    cyc = O.Grid.build(d, cr, O.KDTREE)
    grd = O.Grid.build(d, cr, O.KDGRAD)
    # every leaf of both trees meets the mass criterion or sits at the level cap
    for g in (cyc, grd):
        nd = g.nodes()
        leaf = nd["first_child"] < 0
        w = 2.0 * np.exp2(-nd["depth"][leaf].astype(np.float64))
        M = nd["S"][leaf] * np.prod(w, axis=1) / cr.n_samples
        assert np.all((M / cr.total_mass <= cr.delta_max) | (nd["level"][leaf] >= cr.max_level))
    print(f"disk, delta_max 1e-4, max level 18: cyclic {cyc.n_leaves} leaves, "
          f"gradient axis {grd.n_leaves} leaves")
    assert cyc.n_leaves > 1000 and grd.n_leaves > 1000

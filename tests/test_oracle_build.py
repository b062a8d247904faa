"""Pins for the oracle's grid construction (Sect. 2.2 and Eq. 1-3 of Sect. 4).

Each test fixes a result by something other than the oracle's own formulas:
a published test vector, a closed form for a special density, an exact leaf
count, or an independent quadrature of the density model.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _crit(**kw):
    base = dict(total_mass=8.0, delta_max=1.0, tau_max=math.inf, q_max=1.0, kappa=1.0,
                min_level=0, max_level=16, n_samples=64, seed=12345)
    base.update(kw)
    return W.Criteria(**base)


def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        want = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    got = [int(v) for v in O.splitmix64_stream(1234567, 5)]
    assert got == want


def test_eq1_constant_density_mass_is_volume():
    # rho == 1: every sample is 1, S = N exactly, M = S V / N = V exactly.
    d = W.uniform(1.0)
    for tree, dmax, lv, nl in ((O.OCTREE, 0.2, 1, 8), (O.KDTREE, 0.2, 3, 8)):
        g = O.Grid.build(d, _crit(delta_max=dmax), tree)
        nd = g.nodes()
        assert np.all(nd["S"] == 64.0)
        assert np.all(nd["rmin"] == 1.0) and np.all(nd["rmax"] == 1.0)
        lf = g.leaves()
        assert np.all(lf["rho"] == 1.0)
        assert g.n_leaves == nl
        lo, hi = g.leaf_boxes()
        vol = np.prod(hi - lo, axis=1)
        assert vol.sum() == 8.0                     # leaf masses sum to M_tot exactly
        assert np.all(nd["level"][nd["first_child"] < 0] == lv)


@pytest.mark.parametrize("tree,level,n", [(O.OCTREE, 5, 32768), (O.KDTREE, 14, 16384)])
def test_mass_only_uniform_is_regular(tree, level, n):
    # delta at level l is 8^-l (octree) or 2^-l (k-d); split while delta > 1e-4.
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=1e-4), tree)
    nd = g.nodes()
    leaf_lv = nd["level"][nd["first_child"] < 0]
    assert g.n_leaves == n
    assert np.all(leaf_lv == level)
    assert g.n_nodes == (2 * n - 1 if tree == O.KDTREE else (8 * n - 1) // 7)


def test_max_level_caps_subdivision():
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=1e-6, max_level=4), O.OCTREE)
    assert g.n_leaves == 4096


def test_min_level_forces_subdivision():
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=10.0, min_level=2), O.OCTREE)
    assert g.n_leaves == 64


def _kd_sides(level):
    return [2.0 * 2.0 ** -((level + 2 - d) // 3) for d in range(3)]


@pytest.mark.parametrize("kappa,rho,tau_max", [(1.0, 1.0, 0.5), (2.0, 1.0, 0.5), (1.0, 3.0, 0.8)])
def test_eq2_tau_only_uniform(kappa, rho, tau_max):
    # Uniform rho: a cuboid of sides a,b,c holds M = rho abc, so Eq. (2) gives
    # tau = kappa rho sqrt(a^2+b^2+c^2), the optical depth along its diagonal.
    d = W.uniform(rho)
    cr = _crit(total_mass=8.0 * rho, delta_max=10.0, tau_max=tau_max, kappa=kappa)
    # octree: cubes of side h = 2^(1-l)
    lv = 0
    while kappa * rho * math.sqrt(3.0) * 2.0 ** (1 - lv) > tau_max:
        lv += 1
    g = O.Grid.build(d, cr, O.OCTREE)
    assert g.n_leaves == 8 ** lv
    # k-d: sides follow the x,y,z cycle
    lv = 0
    while kappa * rho * math.sqrt(sum(s * s for s in _kd_sides(lv))) > tau_max:
        lv += 1
    g = O.Grid.build(d, cr, O.KDTREE)
    assert g.n_leaves == 2 ** lv
    nd = g.nodes()
    assert np.all(nd["level"][nd["first_child"] < 0] == lv)


def test_eq3_special_cases():
    # constant density: q = 0, never split even with q_max = 0
    g = O.Grid.build(W.uniform(2.5), _crit(total_mass=20.0, delta_max=10.0, q_max=0.0),
                     O.OCTREE)
    assert g.n_leaves == 1
    # zero density everywhere: rho_max = 0 gives q = 0
    d0 = W.Density(box=(-1, -1, -1, 1, 1, 1, 0.0))
    g = O.Grid.build(d0, _crit(total_mass=1.0, delta_max=10.0, q_max=0.0), O.KDTREE)
    assert g.n_leaves == 1
    # node with a zero sample and rho_max > 0 has q = 1 exactly
    d = W.Density(box=(-0.5, -0.5, -0.5, 0.5, 0.5, 0.5, 1.0))
    s = O.sample_node(d, _crit(total_mass=1.0, delta_max=10.0), O.OCTREE, 0, [0, 0, 0])
    assert s["rmin"] == 0.0 and s["rmax"] == 1.0 and s["q"] == 1.0
    assert s["split"] is False                      # q_max = 1 switches the criterion off


def _straddle_leaves(tree, box_lo, box_hi, max_level):
    """Leaves of the tree that splits exactly the cells cut by the box surface:
    a geometric enumeration, no sampling."""
    out = 0
    stack = [(0, np.array([-1.0] * 3), np.array([1.0] * 3))]
    while stack:
        lv, lo, hi = stack.pop()
        inter = np.minimum(hi, box_hi) - np.maximum(lo, box_lo)
        overlap = np.all(inter > 0)
        inside = np.all(lo >= box_lo) and np.all(hi <= box_hi)
        if overlap and not inside and lv < max_level:
            if tree == O.OCTREE:
                mid = 0.5 * (lo + hi)
                for k in range(8):
                    b = np.array([(k >> d) & 1 for d in range(3)])
                    stack.append((lv + 1, np.where(b, mid, lo), np.where(b, hi, mid)))
            else:
                a = lv % 3
                mid = 0.5 * (lo[a] + hi[a])
                h1 = hi.copy(); h1[a] = mid
                l2 = lo.copy(); l2[a] = mid
                stack += [(lv + 1, lo, h1), (lv + 1, l2, hi)]
        else:
            out += 1
    return out


@pytest.mark.parametrize("tree", [O.OCTREE, O.KDTREE])
@pytest.mark.parametrize("box", [(-0.5, 0.5), (-0.25, 0.75)])
def test_eq3_refines_sharp_edges(tree, box):
    # A box of constant density: cells cut by its surface have samples on both
    # sides (q = 1 > q_max) and split; cells inside (q = 0) or outside
    # (rho_max = 0, q = 0) stop.  With box faces on dyadic planes the tree is
    # exactly the set of cells cut by the surface.
    lo, hi = box
    d = W.Density(box=(lo, lo, lo, hi, hi, hi, 1.0))
    ml = 12 if tree == O.KDTREE else 4
    g = O.Grid.build(d, _crit(total_mass=1.0, delta_max=10.0, q_max=0.5, max_level=ml), tree)
    want = _straddle_leaves(tree, np.array([lo] * 3), np.array([hi] * 3), ml)
    assert g.n_leaves == want


def _leaf_mass_check(d, cr, tree, nsig=5.0):
    g = O.Grid.build(d, cr, tree)
    nd = g.nodes()
    lf = g.leaves()
    lo, hi = g.leaf_boxes()
    V = np.prod(hi - lo, axis=1)
    M = lf["rho"] * V
    rng = nd["rmax"][lf["node_of"]] - nd["rmin"][lf["node_of"]]
    # Popoviciu: the sample variance is at most (max-min)^2/4
    sig = math.sqrt(float(np.sum(V * V * rng * rng / 4.0 / cr.n_samples)))
    err = abs(float(M.sum()) - cr.total_mass)
    return err, sig, g


def test_leaf_masses_sum_to_total_disk():
    w = W.workload(1)
    err, sig, g = _leaf_mass_check(w.density, w.criteria, w.tree_type)
    assert err <= 5.0 * sig, (err, sig)
    assert err / w.criteria.total_mass < 0.02


def test_leaf_masses_sum_to_total_torus_clumps():
    rng = np.random.Generator(np.random.PCG64(7))
    c, s, a = W.clumps_uniform(rng, 40, 0.02, 0.06, 1.0)
    d = W.Density(torus=(0.5, 0.1, 1.0), clump_c=c, clump_sigma=s, clump_amp=a)
    # A regular 8^3 grid with 4096 samples per cell, so that every clump is hit
    # by many samples and the sample range bounds the sampling noise.
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=10.0, min_level=3, max_level=3,
                    n_samples=4096, seed=99)
    for tree in (O.OCTREE, O.KDTREE):
        if tree == O.KDTREE:
            cr.min_level = cr.max_level = 9
        err, sig, g = _leaf_mass_check(d, cr, tree)
        assert err <= 5.0 * sig, (err, sig)
        assert err / cr.total_mass < 0.01


def test_density_model_special_points():
    d = W.exp_disk()
    rho0, hR, hz = d.disk
    v = O.density(d, [[0, 0, 0], [hR, 0, 0], [0, 0, -hz], [0, 0.6, 0.0]])
    assert v[0] == rho0
    assert abs(v[1] / (rho0 / math.e) - 1) < 1e-15
    assert abs(v[2] / (rho0 / math.e) - 1) < 1e-15
    assert abs(v[3] / (rho0 * math.exp(-0.6 / hR)) - 1) < 1e-15
    t = W.Density(torus=(0.5, 0.1, 2.0))
    v = O.density(t, [[0.5, 0, 0], [0, -0.5, 0.1], [0.5, 0, 0.1001], [0, 0, 0], [0.61, 0, 0]])
    assert list(v) == [2.0, 2.0, 0.0, 0.0, 0.0]
    cl = W.Density(clump_c=np.array([[0.1, 0.2, 0.3]]), clump_sigma=np.array([0.05]),
                   clump_amp=np.array([4.0]), clump_trunc=3.0)
    v = O.density(cl, [[0.1, 0.2, 0.3], [0.1 + 0.05, 0.2, 0.3], [0.1, 0.2 + 0.151, 0.3]])
    assert v[0] == 4.0
    assert abs(v[1] / (4.0 * math.exp(-0.5)) - 1) < 1e-14
    assert v[2] == 0.0


def test_samples_stay_inside_node_and_are_uniform():
    # A thin slab density that is 1 only on the lower half of a cell on each
    # axis: the fraction of samples hitting it estimates 1/2 per axis.
    tot = 0.0
    for lvl, c in ((3, [1, 2, 5]), (4, [7, 0, 9]), (2, [3, 3, 3])):
        w = 2.0 * 2.0 ** -lvl
        lo = -1.0 + np.array(c) * w
        for ax in range(3):
            blo = list(lo - 1.0)
            bhi = list(lo + 4 * w)
            bhi[ax] = lo[ax] + 0.5 * w
            d = W.Density(box=tuple(blo + bhi + [1.0]))
            s = O.sample_node(d, _crit(total_mass=1.0, n_samples=4096), O.OCTREE, lvl, c)
            tot += s["S"] / 4096
        # a box that contains the node entirely but nothing outside it
        d = W.Density(box=tuple(list(lo) + list(lo + w) + [1.0]))
        s = O.sample_node(d, _crit(total_mass=1.0, n_samples=512), O.OCTREE, lvl, c)
        assert s["S"] == 512.0
    assert abs(tot / 9 - 0.5) < 0.02


def test_kd_half_the_cells_of_octree_sanity():
    # Sect. 3.3: at fixed delta_max the k-d tree needs about half the cells.
    d = W.exp_disk()
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-3, max_level=10, seed=3)
    go = O.Grid.build(d, cr, O.OCTREE)
    cr.max_level = 30
    gk = O.Grid.build(d, cr, O.KDTREE)
    r = gk.n_leaves / go.n_leaves
    assert 0.2 < r < 0.8, r


def test_node_list_is_breadth_first():
    w = W.workload(1)
    g = O.Grid.build(w.density, w.criteria, w.tree_type)
    nd = g.nodes()
    assert np.all(np.diff(nd["level"].astype(int)) >= 0)
    fc = nd["first_child"]
    internal = np.nonzero(fc >= 0)[0]
    assert np.all(fc[internal] == 1 + 8 * np.arange(internal.size))
    # leaf ids are ranks in list order
    lf = nd["leaf_of"]
    assert np.array_equal(lf[fc < 0], np.arange(g.n_leaves))


def test_import_roundtrip():
    w = W.workload(1)
    g = O.Grid.build(w.density, w.criteria, w.tree_type)
    nd = g.nodes()
    g2 = O.Grid.from_first_child(w.tree_type, nd["first_child"], g.leaves()["rho"])
    n2 = g2.nodes()
    assert np.array_equal(n2["level"], nd["level"])
    assert np.array_equal(n2["coord"], nd["coord"])
    with pytest.raises(RuntimeError):
        bad = nd["first_child"].copy()
        bad[0] = 2
        O.Grid.from_first_child(w.tree_type, bad)


def test_eq3_intermediate_dispersion():
    # Two media, rho = 1 everywhere plus 2 more in a sub-box: a node holding
    # samples of both has rho_min = 1, rho_max = 3, so q = (3-1)/3 = 2/3.
    d = W.Density(box=(-1, -1, -1, 1, 1, 1, 1.0))
    s = O.sample_node(d, _crit(total_mass=100.0, delta_max=10.0, q_max=0.6), O.OCTREE, 0,
                      [0, 0, 0])
    assert s["q"] == 0.0
    two = W.Density(box=(-1, -1, -1, 1, 1, 1, 1.0))
    # box component adds 1; the clump-free second medium is modelled by a
    # torus of density 2 (added after the box): samples are 1 or 3.
    two.torus = (0.5, 0.3, 2.0)
    s = O.sample_node(two, _crit(total_mass=100.0, delta_max=10.0, q_max=0.6), O.OCTREE, 0,
                      [0, 0, 0])
    assert s["rmin"] == 1.0 and s["rmax"] == 3.0
    assert s["q"] == (3.0 - 1.0) / 3.0
    assert s["split"] is True                                   # 2/3 > 0.6
    s = O.sample_node(two, _crit(total_mass=100.0, delta_max=10.0, q_max=0.7), O.OCTREE, 0,
                      [0, 0, 0])
    assert s["split"] is False                                  # 2/3 < 0.7


def test_mass_threshold_is_strict():
    # delta of a level-2 octree cell of a uniform medium is exactly 8^-2; the
    # paper splits only while delta > delta_max, so equality stops at level 2.
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=8.0 ** -2), O.OCTREE)
    assert g.n_leaves == 64
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=0.995 * 8.0 ** -2), O.OCTREE)
    assert g.n_leaves == 512
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=2.0 ** -9), O.KDTREE)
    assert g.n_leaves == 512

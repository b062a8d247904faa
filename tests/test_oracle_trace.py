"""Pins for the oracle's point location and path tracing (Sect. 2.3).

The walk's output is fixed by what geometry alone determines: the chord
length through the domain, the optical depth of a uniform medium, the number
of planes a line crosses in a regular grid, the leaves found by intersecting
the path with every leaf box, and the equivalence of an octree with the k-d
tree that has the same leaves (Sect. 2.1).
"""
import collections
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _crit(**kw):
    base = dict(total_mass=8.0, delta_max=1.0, tau_max=math.inf, q_max=1.0, kappa=1.0,
                min_level=0, max_level=10, n_samples=64, seed=777)
    base.update(kw)
    return W.Criteria(**base)


def chord(p0, k, lo=-1.0, hi=1.0):
    """Length of the part of the half-line p0 + t k (t >= 0) inside the cube."""
    t0, t1 = 0.0, math.inf
    for d in range(3):
        if k[d] == 0.0:
            if p0[d] < lo or p0[d] > hi:
                return 0.0
            continue
        a = (lo - p0[d]) / k[d]
        b = (hi - p0[d]) / k[d]
        t0 = max(t0, min(a, b))
        t1 = min(t1, max(a, b))
    return max(0.0, t1 - t0)


def small_trees():
    """A few trees of at most ~2e3 leaves, both types, smooth and sharp media."""
    out = []
    d = W.exp_disk()
    m = W.total_mass(d)
    out.append(("disk-oct", O.Grid.build(d, _crit(total_mass=m, delta_max=3e-3), O.OCTREE)))
    out.append(("disk-kd", O.Grid.build(d, _crit(total_mass=m, delta_max=2e-3, max_level=30),
                                         O.KDTREE)))
    t = W.Density(torus=(0.5, 0.1, 1.0))
    mt = W.total_mass(t)
    out.append(("torus-oct-q", O.Grid.build(t, _crit(total_mass=mt, delta_max=0.05, q_max=0.9,
                                                      max_level=4), O.OCTREE)))
    out.append(("torus-kd-q", O.Grid.build(t, _crit(total_mass=mt, delta_max=0.05, q_max=0.9,
                                                     max_level=11), O.KDTREE)))
    for name, g in out:
        assert 20 <= g.n_leaves <= 2500, (name, g.n_leaves)
    return out


TREES = small_trees()


def adversarial_rays():
    """Axis-parallel rays, rays lying in split planes, through edges and
    corners, origins on planes and on the domain faces, origins outside the
    domain, rays missing it."""
    o, k = [], []
    s3 = 1.0 / math.sqrt(3.0)
    s2 = 1.0 / math.sqrt(2.0)
    for d in range(3):
        for sgn in (1.0, -1.0):
            e = [0.0, 0.0, 0.0]
            e[d] = sgn
            for p in ([0.1, 0.2, 0.3], [0.0, 0.0, 0.0], [0.5, -0.25, 0.125], [0.0, 0.5, 0.0],
                      [-1.0, -1.0, -1.0], [1.0, 1.0, 1.0], [0.75, 0.0, -0.5]):
                o.append(p); k.append(e)
    for p in ([0.0, 0.0, 0.0], [-1.0, -1.0, -1.0], [0.5, 0.5, 0.5], [-0.5, 0.25, 0.0]):
        for kk in ([s3, s3, s3], [-s3, s3, -s3], [s2, s2, 0.0], [0.0, -s2, s2], [s2, 0.0, -s2]):
            o.append(p); k.append(kk)
    # outside origins, hitting and missing
    o += [[-2.0, 0.1, 0.2], [0.3, 3.0, -0.2], [-2.0, -2.0, -2.0], [-2.0, 2.0, 0.0],
          [1.0, 0.3, 0.3], [1.0, 0.3, 0.3], [2.0, 0.0, 0.0]]
    k += [[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [s3, s3, s3], [1.0, 0.0, 0.0],
          [-1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [-s2, s2, 0.0]]
    return np.array(o, float), np.array(k, float)


def random_rays(n, seed, outside=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = W.isotropic(rng, n)
    if outside:
        o = rng.uniform(-2.5, 2.5, size=(n, 3))
    else:
        o = rng.uniform(-1.0, 1.0, size=(n, 3))
    return o, k


@pytest.mark.parametrize("name,g", TREES)
def test_walk_equals_brute_force(name, g):
    o1, k1 = random_rays(150, 5, outside=False)
    o2, k2 = random_rays(150, 6, outside=True)
    o3, k3 = adversarial_rays()
    o = np.concatenate([o1, o2, o3])
    k = np.concatenate([k1, k2, k3])
    r = g.trace(o, k)
    for i in range(o.shape[0]):
        a, b = r["offsets"][i], r["offsets"][i + 1]
        lw, dw = r["leaf"][a:b], r["ds"][a:b]
        keep = dw >= 1e-12
        bf = g.trace_brute(o[i], k[i])
        assert np.array_equal(lw[keep], bf["leaf"]), (name, i, lw, bf["leaf"])
        assert np.allclose(dw[keep], bf["ds"], rtol=0, atol=1e-12), (name, i)
        assert abs(r["tau"][i] - bf["tau"]) <= 1e-12 * max(1.0, abs(bf["tau"]))


@pytest.mark.parametrize("name,g", TREES)
def test_path_lengths_sum_to_chord(name, g):
    o, k = random_rays(400, 11, outside=True)
    oa, ka = adversarial_rays()
    o = np.concatenate([o, oa])
    k = np.concatenate([k, ka])
    g.set_rho(np.ones(g.n_leaves))
    r = g.trace(o, k, kappa=1.0)
    L = np.array([chord(o[i], k[i]) for i in range(o.shape[0])])
    off = r["offsets"]
    s = np.array([math.fsum(r["ds"][off[i]:off[i + 1]]) for i in range(L.size)])
    assert np.allclose(s, L, rtol=0, atol=1e-12)
    # uniform medium: tau = kappa rho L
    g.set_rho(np.full(g.n_leaves, 2.5))
    r = g.trace(o, k, kappa=0.4, records=False)
    assert np.allclose(r["tau"], 0.4 * 2.5 * L, rtol=1e-12, atol=1e-13)


def test_uniform_tau_regular_grid_and_crossing_count():
    # Mass-only build of a uniform medium is the regular 32^3 grid (level 5).
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=1e-4), O.OCTREE)
    assert g.n_leaves == 32 ** 3
    o, k = random_rays(2000, 21)
    r = g.trace(o, k, records=False)
    planes = -1.0 + np.arange(1, 32) * (2.0 / 32)
    for i in range(o.shape[0]):
        L = chord(o[i], k[i])
        pe = o[i] + L * k[i]
        n = 1
        for d in range(3):
            a, b = sorted((o[i, d], pe[d]))
            n += int(np.sum((planes > a) & (planes < b)))
        assert r["count"][i] == n
        assert abs(r["tau"][i] - L) <= 1e-12 * max(L, 1e-300) + 1e-15


def _locate_brute(g, pts):
    lo, hi = g.leaf_boxes()
    out = np.full(pts.shape[0], -1, np.int32)
    for i, x in enumerate(pts):
        top = hi >= 1.0
        ins = np.all((lo <= x) & ((x < hi) | (top & (x == hi))), axis=1)
        idx = np.nonzero(ins)[0]
        if idx.size:
            assert idx.size == 1
            out[i] = idx[0]
    return out


@pytest.mark.parametrize("name,g", TREES)
def test_locate_equals_brute_force(name, g):
    rng = np.random.Generator(np.random.PCG64(3))
    pts = rng.uniform(-1.1, 1.1, size=(800, 3))
    grid = np.array([-1.0, -0.5, -0.25, 0.0, 0.125, 0.5, 0.75, 1.0])
    pts = np.concatenate([pts, rng.choice(grid, size=(400, 3)),
                          [[np.nan, 0, 0], [1.0 + 1e-16, 0, 0], [-1.0 - 1e-15, 0, 0]]])
    got = g.locate(pts)
    assert np.array_equal(got, _locate_brute(g, pts))


def octree_to_kd(fc_oct):
    """The k-d tree with the same leaves as an octree: each octree split becomes
    an x split, then y splits, then z splits (Sect. 2.1).  Returns the k-d
    first-child array in list order and, per k-d leaf, the octree leaf node."""
    nodes = [("o", 0)]
    fc = []
    i = 0
    while i < len(nodes):
        nd = nodes[i]
        kids = []
        if nd[0] == "o":
            if fc_oct[nd[1]] >= 0:
                kids = [("x", nd[1], 0), ("x", nd[1], 1)]
        elif nd[0] == "x":
            kids = [("y", nd[1], nd[2], 0), ("y", nd[1], nd[2], 1)]
        else:
            n, bx, by = nd[1], nd[2], nd[3]
            kids = [("o", fc_oct[n] + bx + 2 * by + 4 * bz) for bz in (0, 1)]
        if kids:
            fc.append(len(nodes))
            nodes.extend(kids)
        else:
            fc.append(-1)
        i += 1
    leaf_octnode = [nd[1] for nd, f in zip(nodes, fc) if f < 0]
    return np.array(fc, np.int32), np.array(leaf_octnode)


def test_octree_equals_kd_with_same_leaves():
    w = W.workload(1)
    go = O.Grid.build(w.density, w.criteria, O.OCTREE)
    nd = go.nodes()
    fc_kd, leaf_octnode = octree_to_kd(nd["first_child"])
    rho_o = go.leaves()["rho"]
    oct_leaf = nd["leaf_of"][leaf_octnode]
    gk = O.Grid.from_first_child(O.KDTREE, fc_kd, rho_o[oct_leaf])
    assert gk.n_leaves == go.n_leaves
    lo_o, hi_o = go.leaf_boxes()
    lo_k, hi_k = gk.leaf_boxes()
    assert np.array_equal(lo_k, lo_o[oct_leaf]) and np.array_equal(hi_k, hi_o[oct_leaf])
    o, k = W.rays("uniform", 3000, 99)
    oa, ka = adversarial_rays()
    o = np.concatenate([o, oa])
    k = np.concatenate([k, ka])
    ro = go.trace(o, k)
    rk = gk.trace(o, k)
    assert np.array_equal(ro["count"], rk["count"])
    assert np.array_equal(lo_o[ro["leaf"]], lo_k[rk["leaf"]])
    assert np.array_equal(hi_o[ro["leaf"]], hi_k[rk["leaf"]])
    assert np.array_equal(ro["ds"], rk["ds"])          # bitwise
    assert np.array_equal(ro["tau"], rk["tau"])


def test_neighbors_brute_regular_and_refined():
    g = O.Grid.build(W.uniform(1.0), _crit(delta_max=0.02), O.OCTREE)   # 4^3 regular
    assert g.n_leaves == 64
    lo, hi = g.leaf_boxes()
    for l in range(g.n_leaves):
        for f in range(6):
            a, up = divmod(f, 2)
            nb = g.neighbors_brute(l, f)
            on_boundary = (hi[l, a] == 1.0) if up else (lo[l, a] == -1.0)
            assert nb.size == (0 if on_boundary else 1)
            if nb.size:
                assert (lo[nb[0], a] == hi[l, a]) if up else (hi[nb[0], a] == lo[l, a])
    # one refined octant: the coarse neighbor across it sees 4 fine leaves
    d = W.Density(box=(0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0))
    g = O.Grid.build(d, _crit(total_mass=1.0, delta_max=0.1, max_level=2), O.OCTREE)
    lo, hi = g.leaf_boxes()
    coarse = [l for l in range(g.n_leaves) if hi[l, 0] - lo[l, 0] == 1.0
              and lo[l, 0] == -1.0 and lo[l, 1] == 0.0 and lo[l, 2] == 0.0]
    assert len(coarse) == 1
    assert g.neighbors_brute(coarse[0], 1).size == 4


def test_missing_and_empty():
    g = TREES[0][1]
    r = g.trace(np.zeros((0, 3)), np.zeros((0, 3)))
    assert r["count"].size == 0 and r["leaf"].size == 0
    r = g.trace([[-2.0, 2.0, 0.0], [3.0, 0.0, 0.0]], [[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    assert list(r["count"]) == [0, 0] and list(r["tau"]) == [0.0, 0.0]
    # origin on the upper domain face, moving out: nothing crossed
    r = g.trace([[1.0, 0.2, 0.3]], [[1.0, 0.0, 0.0]])
    assert r["count"][0] == 0

"""Pins of the oracle's walk consumers (Sect. 3.2 quality measures, the
interaction point) against closed forms and brute force."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.quality as Q
import workloads as W


def _uniform(c=2.5):
    return W.Density(box=(-1, -1, -1, 1, 1, 1, c))


def _grid(d, tree=W.KDTREE, delta=1e-2, max_level=9):
    cr = W.Criteria(total_mass=W.total_mass(d), delta_max=delta, max_level=max_level, seed=7)
    return O.Grid.build(d, cr, tree)


def _inside_rays(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(-0.95, 0.95, size=(n, 3))
    mu = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - mu * mu)
    k = np.stack([s * np.cos(ph), s * np.sin(ph), mu], axis=1)
    return o, k


def _chord_from_inside(o, k):
    with np.errstate(divide="ignore"):
        t = np.where(k > 0, (1 - o) / k, np.where(k < 0, (-1 - o) / k, np.inf))
    return t.min(axis=1)


def test_density_diff_uniform_is_zero():
    d = _uniform()
    g = _grid(d)
    pts = np.random.default_rng(1).uniform(-1, 1, size=(5000, 3))
    assert np.all(Q.density_diff(g, d, pts) == 0.0)


def test_density_diff_matches_brute_force_boxes():
    # a box not aligned with the cells: cells cut by its faces carry the
    # sampled mean, so the difference is nonzero exactly there
    d = W.Density(box=(-0.3, -0.2, -0.45, 0.37, 0.51, 0.23, 4.0))
    g = _grid(d, tree=W.OCTREE, delta=1e-3, max_level=5)
    pts = np.random.default_rng(2).uniform(-1, 1, size=(4000, 3))
    diff = Q.density_diff(g, d, pts)
    lo, hi = g.leaf_boxes()
    rho = g.leaves()["rho"]
    b = np.array(d.box[:6]).reshape(2, 3)
    for i in range(0, pts.shape[0], 37):
        p = pts[i]
        inl = np.nonzero(np.all((lo <= p) & (p < hi), axis=1))[0]
        assert inl.size == 1
        rt = 4.0 if np.all((b[0] <= p) & (p <= b[1])) else 0.0
        assert diff[i] == rt - rho[inl[0]]
    assert np.any(diff != 0.0) and np.mean(diff == 0.0) > 0.5


@pytest.mark.parametrize("tree", [W.OCTREE, W.KDTREE], ids=["octree", "kd"])
def test_segment_tau_uniform_closed_form(tree):
    c, kappa = 2.5, 1.7
    d = _uniform(c)
    g = _grid(d, tree=tree)
    o, k = _inside_rays(300, 3)
    L = _chord_from_inside(o, k)
    s_max = np.random.default_rng(4).uniform(0, 3.5, size=300)
    rec = g.trace(o, k, kappa=kappa)
    tau = Q.segment_tau(rec, g.leaves()["rho"], s_max, kappa=kappa)
    want = kappa * c * np.minimum(s_max, L)
    assert np.allclose(tau, want, rtol=1e-12, atol=1e-12)


def test_true_tau_disk_axis_closed_form():
    d = W.exp_disk()
    rho0, hR, hz = d.disk
    g = _grid(d, tree=W.KDTREE, delta=1e-4, max_level=18)
    z0 = np.array([-0.5, -0.2, 0.05, -0.9])
    z1 = np.array([0.7, 0.3, 0.6, 0.1])
    o = np.stack([np.zeros(4), np.zeros(4), z0], axis=1)
    k = np.tile([0.0, 0.0, 1.0], (4, 1))
    rec = g.trace(o, k)
    s_max = z1 - z0

    def prim(z):  # integral of exp(-|z|/hz) from 0 to z
        return math.copysign(hz * (1 - math.exp(-abs(z) / hz)), z)

    want = np.array([rho0 * (prim(b) - prim(a)) for a, b in zip(z0, z1)])
    got = Q.true_tau(d, o, k, rec, s_max)
    assert np.allclose(got, want, rtol=1e-11, atol=0)
    # the grid's tau over the same stretch differs by the discretisation
    tg = Q.segment_tau(rec, g.leaves()["rho"], s_max)
    assert np.all(np.abs(tg - want) < 0.2 * want)


def test_true_tau_uniform_is_segment_tau():
    c = 0.75
    d = _uniform(c)
    g = _grid(d, delta=3e-2)
    o, k = _inside_rays(100, 5)
    s_max = np.random.default_rng(6).uniform(0, 2.0, size=100)
    rec = g.trace(o, k)
    assert np.allclose(Q.true_tau(d, o, k, rec, s_max), c * np.minimum(s_max, _chord_from_inside(o, k)),
                       rtol=1e-12)


def test_interaction_uniform_closed_form():
    c, kappa = 1.3, 0.9
    d = _uniform(c)
    g = _grid(d, tree=W.OCTREE, delta=1e-2)
    o, k = _inside_rays(400, 8)
    L = _chord_from_inside(o, k)
    u = np.random.default_rng(9).uniform(0, 1, 400)
    tau_star = -np.log(1 - u)
    rec = g.trace(o, k, kappa=kappa)
    leaf, s = Q.interaction(rec, g.leaves()["rho"], tau_star, kappa=kappa)
    want_s = tau_star / (kappa * c)
    hit = want_s < L
    assert np.all((leaf >= 0) == hit)
    assert np.allclose(s[hit], want_s[hit], rtol=1e-12)
    assert np.allclose(s[~hit], L[~hit], rtol=1e-12)
    # the leaf holds the interaction point (brute force over the leaf boxes)
    lo, hi = g.leaf_boxes()
    for i in np.nonzero(hit)[0][:60]:
        p = o[i] + s[i] * k[i]
        j = leaf[i]
        assert np.all(lo[j] - 1e-12 <= p) and np.all(p <= hi[j] + 1e-12)


def test_interaction_on_disk_reaches_tau_star():
    d = W.exp_disk()
    g = _grid(d, tree=W.KDTREE, delta=1e-4, max_level=18)
    o, k = W.rays("disk", 300, 11)
    rec = g.trace(o, k)
    tau_star = np.random.default_rng(12).uniform(0, 1.0, 300) * rec["tau"]
    leaf, s = Q.interaction(rec, g.leaves()["rho"], tau_star)
    # the cumulative optical depth up to s equals tau_star
    tg = Q.segment_tau(rec, g.leaves()["rho"], s)
    ok = leaf >= 0
    assert np.allclose(tg[ok], tau_star[ok], rtol=1e-10, atol=1e-14)

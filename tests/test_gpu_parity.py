"""GPU parity: the HIP library against the FP64 CPU oracle, through the C ABI.

Trace parity is checked on one shared grid (built by the oracle, imported by
the library): leaf sequences identical, FP64 ds and tau bitwise equal,
FP32-with-recheck ds equal to the oracle's ds rounded to FP32 and tau within
1e-5 relative.  Build parity compares a GPU-built grid with the oracle's:
same topology and sampled statistics within 1e-13 relative (the two sides'
exp() may differ in the last bit).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1311_0705_amd as hg  # noqa: E402  (fails loudly if the library is missing)

DEV = "cuda:0"


def _crit(**kw):
    base = dict(total_mass=8.0, delta_max=1.0, tau_max=math.inf, q_max=1.0, kappa=1.0,
                min_level=0, max_level=10, n_samples=64, seed=777)
    base.update(kw)
    return W.Criteria(**base)


def to_gpu(og: O.Grid) -> hg.Grid:
    return hg.import_grid(og.tree, og.nodes()["first_child"], og.leaves()["rho"], device=DEV)


def adversarial_rays():
    s3 = 1.0 / math.sqrt(3.0)
    s2 = 1.0 / math.sqrt(2.0)
    o, k = [], []
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
    o += [[-2.0, 0.1, 0.2], [0.3, 3.0, -0.2], [-2.0, -2.0, -2.0], [-2.0, 2.0, 0.0],
          [1.0, 0.3, 0.3], [1.0, 0.3, 0.3], [2.0, 0.0, 0.0]]
    k += [[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [s3, s3, s3], [1.0, 0.0, 0.0],
          [-1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [-s2, s2, 0.0]]
    return np.array(o, float), np.array(k, float)


def random_rays(n, seed, lo=-1.0, hi=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(n, 3)), W.isotropic(rng, n)


def check_trace(og, g, o, k, kappa=1.0):
    out = None
    for persistent in (0, 3):
        out = _check_trace(og, g, o, k, kappa, persistent)
    return out


def _check_trace(og, g, o, k, kappa, persistent):
    ref = og.trace(o, k, kappa=kappa)
    n = o.shape[0]
    r = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS, kappa=kappa, persistent=persistent)
    tot = r["needed"]
    assert tot == int(ref["offsets"][-1])
    assert np.array_equal(r["count"].cpu().numpy(), ref["count"])
    assert np.array_equal(r["offsets"].cpu().numpy(), ref["offsets"])
    assert np.array_equal(r["leaf"][:tot].cpu().numpy(), ref["leaf"])
    assert np.array_equal(r["ds"][:tot].cpu().numpy(), ref["ds"])            # bitwise
    assert np.array_equal(r["tau"].cpu().numpy(), ref["tau"])                # same order, same ops
    t = g.trace(o, k, precision=hg.FP64, mode=hg.TAU_ONLY, kappa=kappa, persistent=persistent)
    assert np.array_equal(t["tau"].cpu().numpy(), ref["tau"])
    assert np.array_equal(t["count"].cpu().numpy(), ref["count"])
    f = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS, kappa=kappa,
                count_rechecks=True, persistent=persistent)
    assert f["needed"] == tot
    assert np.array_equal(f["count"].cpu().numpy(), ref["count"])
    assert np.array_equal(f["leaf"][:tot].cpu().numpy(), ref["leaf"])
    assert np.array_equal(f["ds"][:tot].cpu().numpy(), ref["ds"].astype(np.float32))
    tau32 = f["tau"].cpu().numpy()
    rel = np.abs(tau32 - ref["tau"]) / np.maximum(np.abs(ref["tau"]), 1e-300)
    assert float(rel.max(initial=0.0)) <= 1e-5, float(rel.max())
    return ref, r, f, n


def small_trees():
    d = W.exp_disk()
    m = W.total_mass(d)
    t = W.Density(torus=(0.5, 0.1, 1.0))
    mt = W.total_mass(t)
    return [
        ("disk-oct", O.Grid.build(d, _crit(total_mass=m, delta_max=3e-3), O.OCTREE)),
        ("disk-kd", O.Grid.build(d, _crit(total_mass=m, delta_max=2e-3, max_level=30), O.KDTREE)),
        ("torus-oct-q", O.Grid.build(t, _crit(total_mass=mt, delta_max=0.05, q_max=0.9,
                                              max_level=4), O.OCTREE)),
        ("torus-kd-q", O.Grid.build(t, _crit(total_mass=mt, delta_max=0.05, q_max=0.9,
                                             max_level=11), O.KDTREE)),
        ("root-leaf", O.Grid.build(W.uniform(1.0), _crit(delta_max=10.0), O.KDTREE)),
    ]


@pytest.fixture(scope="module")
def trees():
    return small_trees()


def test_trace_parity_small_trees(trees):
    for name, og in trees:
        print(f"[gpu] trace parity {name} leaves={og.n_leaves}", flush=True)
        g = to_gpu(og)
        o1, k1 = random_rays(300, 5)
        o2, k2 = random_rays(300, 6, -2.5, 2.5)
        oa, ka = adversarial_rays()
        check_trace(og, g, np.concatenate([o1, o2, oa]), np.concatenate([k1, k2, ka]), kappa=0.7)


def test_trace_parity_workload1():
    w = W.workload(1)
    print(f"[gpu] trace parity {w.name}", flush=True)
    og = O.Grid.build(w.density, w.criteria, w.tree_type)
    g = to_gpu(og)
    o, k = W.rays(w.ray_kind, w.n_rays, w.ray_seed)
    ref, r, f, n = check_trace(og, g, o, k)
    assert n == 10_000


def test_locate_parity(trees):
    rng = np.random.Generator(np.random.PCG64(3))
    grid = np.array([-1.0, -0.5, -0.25, 0.0, 0.125, 0.5, 0.75, 1.0])
    pts = np.concatenate([rng.uniform(-1.1, 1.1, size=(5000, 3)), rng.choice(grid, size=(2000, 3)),
                          [[np.nan, 0, 0], [1.0, 1.0, 1.0], [-1.0, -1.0, -1.0]]])
    for name, og in trees:
        g = to_gpu(og)
        got = g.locate(pts).cpu().numpy()
        assert np.array_equal(got, og.locate(pts)), name
    empty = to_gpu(trees[0][1]).locate(np.zeros((0, 3)))
    assert empty.numel() == 0


def _leaf_sets_under(fc, node, nc):
    """Node ids of the leaves in node's subtree."""
    out, st = [], [node]
    while st:
        n = st.pop()
        if fc[n] < 0:
            out.append(n)
        else:
            st.extend(range(fc[n], fc[n] + nc))
    return out


def test_ropes_are_smallest_neighbor_covers(trees):
    # The rope of each leaf face points at the smallest node whose subtree
    # holds every leaf sharing positive area with that face (the neighbor list
    # of the face, Sect. 2.3), or -1 on the domain boundary.
    for name, og in trees:
        g = to_gpu(og)
        e = g.export()
        rope = e["rope"].cpu().numpy()
        nd = og.nodes()
        fc = nd["first_child"]
        nc = 8 if og.tree == O.OCTREE else 2
        lf = og.leaves()
        for l in range(min(og.n_leaves, 400)):
            node = lf["node_of"][l]
            for f in range(6):
                nb = set(lf["node_of"][og.neighbors_brute(l, f)].tolist())
                t = rope[node, f]
                if not nb:
                    assert t == -1, (name, l, f)
                    continue
                assert t >= 0, (name, l, f)
                assert nb <= set(_leaf_sets_under(fc, t, nc)), (name, l, f)
                if fc[t] >= 0:
                    kids = [c for c in range(fc[t], fc[t] + nc)
                            if nb & set(_leaf_sets_under(fc, c, nc))]
                    assert len(kids) >= 2, (name, l, f, t)


def _compare_build(og, g, rtol=1e-13):
    e = g.export()
    nd = og.nodes()
    fc_g = e["first_child"].cpu().numpy()
    if not np.array_equal(fc_g, nd["first_child"]):
        # Only a split decision taken within rounding of its threshold may differ.
        lv = e["level"].cpu().numpy()
        co = e["coord"].cpu().numpy().astype(np.uint32)
        n = min(fc_g.size, nd["first_child"].size)
        bad = np.nonzero((fc_g[:n] >= 0) != (nd["first_child"][:n] >= 0))[0]
        assert bad.size, "topologies differ in length only"
        i = int(bad[0])
        assert lv[i] == nd["level"][i] and np.array_equal(co[i], nd["coord"][i])
        pytest.fail(f"split decision differs at node {i} (level {lv[i]})")
    for key, okey in (("S", "S"), ("rho_min", "rmin"), ("rho_max", "rmax")):
        a = e[key].cpu().numpy()
        b = nd[okey]
        assert np.allclose(a, b, rtol=rtol, atol=0), key
    assert np.allclose(e["rho"].cpu().numpy(), og.leaves()["rho"], rtol=rtol, atol=0)
    assert np.array_equal(e["leaf_of"].cpu().numpy(), nd["leaf_of"])
    assert np.array_equal(e["level"].cpu().numpy(), nd["level"])
    assert np.array_equal(e["coord"].cpu().numpy().astype(np.uint32), nd["coord"])
    return e


@pytest.mark.parametrize("case", ["disk-octree", "disk-kd", "uniform-octree", "torus-clumps-oct",
                                  "torus-clumps-kd", "box-q-kd"])
def test_build_parity(case):
    rng = np.random.Generator(np.random.PCG64(11))
    if case == "disk-octree":
        w = W.workload(1)
        d, cr, tree = w.density, w.criteria, w.tree_type
    elif case == "disk-kd":
        d = W.exp_disk()
        cr = W.Criteria(total_mass=W.total_mass(d), delta_max=2e-5, max_level=30, seed=5)
        tree = O.KDTREE
    elif case == "uniform-octree":
        d = W.uniform(1.0)
        cr = _crit(delta_max=1e-4, max_level=8)
        tree = O.OCTREE
    elif case.startswith("torus-clumps"):
        c, s, a = W.clumps_uniform(rng, 60, 0.005, 0.03, 1.0)
        d = W.Density(torus=(0.5, 0.1, 1.0), clump_c=c, clump_sigma=s, clump_amp=a)
        tree = O.OCTREE if case.endswith("oct") else O.KDTREE
        cr = W.Criteria(total_mass=W.total_mass(d), delta_max=1e-4, tau_max=0.1, q_max=0.9,
                        min_level=2 if tree == O.OCTREE else 6,
                        max_level=6 if tree == O.OCTREE else 17, seed=21)
    else:
        d = W.Density(box=(-0.25, -0.25, -0.25, 0.75, 0.75, 0.75, 1.0))
        cr = _crit(total_mass=1.0, delta_max=10.0, q_max=0.5, max_level=14)
        tree = O.KDTREE
    print(f"[gpu] build parity {case}", flush=True)
    og = O.Grid.build(d, cr, tree)
    g = hg.Grid.build(d, cr, tree, device=DEV)
    assert g.n_leaves == og.n_leaves and g.n_nodes == og.n_nodes
    _compare_build(og, g)
    # tracing the GPU-built grid equals tracing the oracle-built one
    o, k = random_rays(500, 17)
    ref = og.trace(o, k)
    r = g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS)
    assert np.array_equal(r["leaf"][: r["needed"]].cpu().numpy(), ref["leaf"])
    np.testing.assert_allclose(r["tau"].cpu().numpy(), ref["tau"], rtol=1e-12, atol=0)


def test_errors_and_edge_cases(trees):
    og = trees[0][1]
    g = to_gpu(og)
    o, k = random_rays(100, 1)
    bad = k.copy()
    bad[7] = [1.0, 1.0, 0.0]
    with pytest.raises(hg.HGError) as ei:
        g.trace(o, bad, precision=hg.FP64, mode=hg.TAU_ONLY)
    assert ei.value.code == hg.HG_E_DIR
    nan = k.copy()
    nan[3, 0] = np.nan
    with pytest.raises(hg.HGError) as ei:
        g.trace(o, nan, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    assert ei.value.code == hg.HG_E_DIR
    # capacity too small: tau, count, offsets and needed still valid
    with pytest.raises(hg.HGError) as ei:
        g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS, capacity=3)
    assert ei.value.code == hg.HG_E_CAPACITY
    res = {}
    try:
        g.trace(o, k, precision=hg.FP64, mode=hg.RECORDS, capacity=3, out=res)
    except hg.HGError:
        pass
    ref = og.trace(o, k)
    assert np.array_equal(res["count"].cpu().numpy(), ref["count"])
    assert np.array_equal(res["tau"].cpu().numpy(), ref["tau"])
    assert np.array_equal(res["offsets"].cpu().numpy(), ref["offsets"])
    # empty batch
    r = g.trace(np.zeros((0, 3)), np.zeros((0, 3)), precision=hg.FP64, mode=hg.RECORDS)
    assert r["needed"] == 0 and r["offsets"].cpu().numpy().tolist() == [0]
    # all rays miss
    r = g.trace([[-3.0, 3.0, 0.0]] * 5, [[1.0, 0.0, 0.0]] * 5, precision=hg.FP32_RECHECK,
                mode=hg.RECORDS)
    assert r["needed"] == 0 and float(r["tau"].abs().sum()) == 0.0
    # invalid construction inputs
    d = W.exp_disk()
    with pytest.raises(hg.HGError) as ei:
        hg.Grid.build(W.Density(disk=d.disk, lo=(-1.0, -1.0, -1.0), side=3.0),
                      _crit(total_mass=1.0), O.OCTREE, device=DEV)
    assert ei.value.code == hg.HG_E_DOMAIN
    with pytest.raises(hg.HGError) as ei:
        hg.Grid.build(d, _crit(total_mass=1.0, max_level=20), O.OCTREE, device=DEV)
    assert ei.value.code == hg.HG_E_INVAL
    with pytest.raises(hg.HGError) as ei:
        hg.Grid.build(W.uniform(1.0), _crit(delta_max=1e-6, max_level=12), O.OCTREE,
                      device=DEV, max_nodes=10000)
    assert ei.value.code == hg.HG_E_LIMIT
    with pytest.raises(hg.HGError) as ei:
        hg.import_grid(O.KDTREE, np.array([2, -1, -1], np.int32), np.zeros(2), device=DEV)
    assert ei.value.code == hg.HG_E_FORMAT


def test_deterministic_repeat():
    w = W.workload(1)
    g = hg.Grid.build(w.density, w.criteria, w.tree_type, device=DEV)
    o, k = W.rays(w.ray_kind, 20_000, 3)
    a = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    b = g.trace(o, k, precision=hg.FP32_RECHECK, mode=hg.RECORDS)
    for key in ("tau", "count", "offsets"):
        assert torch.equal(a[key], b[key])
    n = a["needed"]
    assert torch.equal(a["leaf"][:n], b["leaf"][:n]) and torch.equal(a["ds"][:n], b["ds"][:n])
    g2 = hg.Grid.build(w.density, w.criteria, w.tree_type, device=DEV)
    e1, e2 = g.export(), g2.export()
    for key in ("first_child", "S", "rope", "rho"):
        assert torch.equal(e1[key], e2[key])


def test_wide_reference_layout(trees, monkeypatch):
    # Trees beyond 2^25 leaves or internal nodes use 64-bit references and
    # 64-byte records; HGRID_WIDE_REFS=1 forces that layout on small trees.
    monkeypatch.setenv("HGRID_WIDE_REFS", "1")
    for name, og in trees:
        print(f"[gpu] wide layout {name}", flush=True)
        g = to_gpu(og)
        o1, k1 = random_rays(300, 15)
        oa, ka = adversarial_rays()
        check_trace(og, g, np.concatenate([o1, oa]), np.concatenate([k1, ka]), kappa=1.3)
        pts = np.random.default_rng(2).uniform(-1.05, 1.05, size=(3000, 3))
        assert np.array_equal(g.locate(pts).cpu().numpy(), og.locate(pts))
    w = W.workload(1)
    gw = hg.Grid.build(w.density, w.criteria, w.tree_type, device=DEV)
    monkeypatch.delenv("HGRID_WIDE_REFS")
    gc = hg.Grid.build(w.density, w.criteria, w.tree_type, device=DEV)
    o, k = W.rays(w.ray_kind, 20_000, 8)
    for prec in (hg.FP64, hg.FP32_RECHECK):
        a = gw.trace(o, k, precision=prec, mode=hg.RECORDS)
        b = gc.trace(o, k, precision=prec, mode=hg.RECORDS)
        n = a["needed"]
        assert n == b["needed"]
        for key in ("tau", "count", "offsets"):
            assert torch.equal(a[key], b[key])
        assert torch.equal(a["leaf"][:n], b["leaf"][:n]) and torch.equal(a["ds"][:n], b["ds"][:n])

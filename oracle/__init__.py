"""Python handle on the plain FP64 CPU oracle (``hgrid_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

The C file follows the paper step by step (construction loop of Sect. 2.2,
Eq. 1-3 of Sect. 4, traversal of Sect. 2.3); this module only marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgrid_oracle.c")
_LIB = os.path.join(_HERE, "libhgrid_oracle.so")

OCTREE = 0
KDTREE = 1
KDGRAD = 2   # k-d tree split across the axis of strongest density gradient (Sect. 2.2)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-std=c11", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Density(C.Structure):
    _fields_ = [
        ("has_box", C.c_int), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("box_rho", C.c_double),
        ("has_disk", C.c_int), ("disk_rho0", C.c_double), ("disk_hR", C.c_double),
        ("disk_hz", C.c_double),
        ("has_torus", C.c_int), ("torus_R0", C.c_double), ("torus_a", C.c_double),
        ("torus_rho", C.c_double),
        ("n_clumps", C.c_int64), ("clump_c", C.c_void_p), ("clump_sigma", C.c_void_p),
        ("clump_amp", C.c_void_p), ("clump_trunc", C.c_double),
    ]


class _Criteria(C.Structure):
    _fields_ = [
        ("total_mass", C.c_double), ("delta_max", C.c_double), ("tau_max", C.c_double),
        ("q_max", C.c_double), ("kappa", C.c_double),
        ("min_level", C.c_int), ("max_level", C.c_int), ("n_samples", C.c_int),
        ("seed", C.c_uint64),
    ]


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        L = C.CDLL(build())
        P = C.c_void_p
        L.or_splitmix64.restype = C.c_uint64
        L.or_splitmix64.argtypes = [C.c_uint64]
        L.or_splitmix64_stream.argtypes = [C.c_uint64, C.c_int, P]
        L.or_density_eval.argtypes = [P, P, C.c_int64, P]
        L.or_build.restype = P
        L.or_build.argtypes = [P, P, C.c_int, P, C.c_double, C.c_int64]
        L.or_import.restype = P
        L.or_import.argtypes = [C.c_int, P, C.c_double, C.c_int64, P, P]
        L.or_import_axes.restype = P
        L.or_import_axes.argtypes = [C.c_int, P, C.c_double, C.c_int64, P, P, P]
        L.or_get_axes.argtypes = [P, P, P]
        L.or_equal_mass_plane.restype = C.c_double
        L.or_equal_mass_plane.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int]
        L.or_free.argtypes = [P]
        L.or_n_nodes.restype = C.c_int64
        L.or_n_nodes.argtypes = [P]
        L.or_n_leaves.restype = C.c_int64
        L.or_n_leaves.argtypes = [P]
        L.or_get_nodes.argtypes = [P] * 8
        L.or_get_leaves.argtypes = [P, P, P]
        L.or_set_rho.argtypes = [P, P]
        L.or_leaf_boxes.argtypes = [P, P, P]
        L.or_sample_node.argtypes = [P, P, C.c_int, P, C.c_double, C.c_int, P, P]
        L.or_sample_nodes.argtypes = [P, P, C.c_int, P, C.c_double, C.c_int64, P, P, P]
        L.or_locate.argtypes = [P, P, C.c_int64, P]
        L.or_trace.restype = C.c_int
        L.or_trace.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_int, P, P, P, P, P]
        L.or_trace_brute.restype = C.c_int64
        L.or_trace_brute.argtypes = [P, P, P, C.c_double, C.c_double, P, P, P, C.c_int64]
        L.or_neighbors_brute.restype = C.c_int64
        L.or_neighbors_brute.argtypes = [P, C.c_int64, C.c_int, P, C.c_int64]
        _lib_handle = L
    return _lib_handle


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _DensityHolder:
    """Keeps the ctypes struct and the arrays it points to alive together."""

    def __init__(self, d):
        s = _Density()
        self.keep = []
        if d.box is not None:
            s.has_box = 1
            for i in range(3):
                s.box_lo[i] = d.box[i]
                s.box_hi[i] = d.box[3 + i]
            s.box_rho = d.box[6]
        if d.disk is not None:
            s.has_disk = 1
            s.disk_rho0, s.disk_hR, s.disk_hz = d.disk
        if d.torus is not None:
            s.has_torus = 1
            s.torus_R0, s.torus_a, s.torus_rho = d.torus
        if d.n_clumps:
            c = _f64(d.clump_c).reshape(-1, 3)
            sg = _f64(d.clump_sigma)
            am = _f64(d.clump_amp)
            self.keep += [c, sg, am]
            s.n_clumps = c.shape[0]
            s.clump_c, s.clump_sigma, s.clump_amp = _ptr(c), _ptr(sg), _ptr(am)
        s.clump_trunc = d.clump_trunc
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _criteria(cr) -> _Criteria:
    c = _Criteria()
    c.total_mass = cr.total_mass
    c.delta_max = cr.delta_max
    c.tau_max = cr.tau_max
    c.q_max = cr.q_max
    c.kappa = cr.kappa
    c.min_level = cr.min_level
    c.max_level = cr.max_level
    c.n_samples = cr.n_samples
    c.seed = cr.seed & ((1 << 64) - 1)
    return c


def splitmix64(x: int) -> int:
    return int(lib().or_splitmix64(x & ((1 << 64) - 1)))


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().or_splitmix64_stream(seed & ((1 << 64) - 1), n, _ptr(out))
    return out


def density(d, pts) -> np.ndarray:
    pts = _f64(pts).reshape(-1, 3)
    out = np.empty(pts.shape[0])
    h = _DensityHolder(d)
    lib().or_density_eval(h.ref, _ptr(pts), pts.shape[0], _ptr(out))
    return out


def sample_node(d, cr, tree, level, coord) -> dict:
    """Sampled statistics and criteria of one node, computed on its own."""
    h = _DensityHolder(d)
    c = _criteria(cr)
    lo = _f64(d.lo)
    cc = np.ascontiguousarray(coord, dtype=np.uint32)
    out = np.empty(7)
    lib().or_sample_node(h.ref, C.byref(c), tree, _ptr(lo), d.side, int(level), _ptr(cc),
                         _ptr(out))
    return dict(S=out[0], rmin=out[1], rmax=out[2], delta=out[3], tau=out[4], q=out[5],
                split=bool(out[6]))


def sample_nodes(d, cr, tree, levels, coords) -> dict:
    """sample_node for many nodes in one C loop (one thread): arrays S, rmin,
    rmax, delta, tau, q, split."""
    h = _DensityHolder(d)
    c = _criteria(cr)
    lo = _f64(d.lo)
    lv = np.ascontiguousarray(levels, dtype=np.uint8)
    cc = np.ascontiguousarray(coords, dtype=np.uint32).reshape(-1, 3)
    n = lv.shape[0]
    out = np.empty((max(n, 1), 7))
    lib().or_sample_nodes(h.ref, C.byref(c), tree, _ptr(lo), d.side, n, _ptr(lv), _ptr(cc), _ptr(out))
    out = out[:n]
    return dict(S=out[:, 0], rmin=out[:, 1], rmax=out[:, 2], delta=out[:, 3], tau=out[:, 4],
                q=out[:, 5], split=out[:, 6] != 0)


class Grid:
    """An oracle-built (or imported) tree with its breadth-first node list."""

    def __init__(self, handle, tree, lo, side):
        if not handle:
            raise RuntimeError("oracle: build/import failed")
        self._h = handle
        self.tree = tree
        self.lo = tuple(lo)
        self.side = side
        L = lib()
        self.n_nodes = int(L.or_n_nodes(handle))
        self.n_leaves = int(L.or_n_leaves(handle))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_free(h)
            self._h = None

    # -- construction -------------------------------------------------------
    @classmethod
    def build(cls, d, cr, tree, max_nodes: int = 0):
        h = _DensityHolder(d)
        c = _criteria(cr)
        lo = _f64(d.lo)
        g = lib().or_build(h.ref, C.byref(c), tree, _ptr(lo), d.side, max_nodes)
        return cls(g, tree, d.lo, d.side)

    @classmethod
    def from_first_child(cls, tree, first_child, rho=None, lo=(-1.0, -1.0, -1.0), side=2.0, axis=None):
        """The tree of a first-child array (and, for KDGRAD, the per-node
        split axes)."""
        fc = np.ascontiguousarray(first_child, dtype=np.int32)
        r = None if rho is None else _f64(rho)
        lo_a = _f64(lo)
        ax = None if axis is None else np.ascontiguousarray(axis, dtype=np.int8)
        g = lib().or_import_axes(tree, _ptr(lo_a), side, fc.shape[0], _ptr(fc), _ptr(ax), _ptr(r))
        return cls(g, tree, lo, side)

    # -- arrays ---------------------------------------------------------------
    def nodes(self) -> dict:
        n = self.n_nodes
        fc = np.empty(n, np.int32)
        lv = np.empty(n, np.uint8)
        co = np.empty((n, 3), np.uint32)
        S = np.empty(n)
        mn = np.empty(n)
        mx = np.empty(n)
        lf = np.empty(n, np.int32)
        lib().or_get_nodes(self._h, _ptr(fc), _ptr(lv), _ptr(co), _ptr(S), _ptr(mn), _ptr(mx),
                           _ptr(lf))
        ax = np.empty(n, np.int8)
        dep = np.empty((n, 3), np.uint8)
        lib().or_get_axes(self._h, _ptr(ax), _ptr(dep))
        return dict(first_child=fc, level=lv, coord=co, S=S, rmin=mn, rmax=mx, leaf_of=lf, axis=ax,
                    depth=dep)

    def leaves(self) -> dict:
        n = self.n_leaves
        no = np.empty(n, np.int32)
        rho = np.empty(n)
        lib().or_get_leaves(self._h, _ptr(no), _ptr(rho))
        return dict(node_of=no, rho=rho)

    def set_rho(self, rho):
        r = _f64(rho)
        assert r.shape[0] == self.n_leaves
        lib().or_set_rho(self._h, _ptr(r))

    def leaf_boxes(self):
        lo = np.empty((self.n_leaves, 3))
        hi = np.empty((self.n_leaves, 3))
        lib().or_leaf_boxes(self._h, _ptr(lo), _ptr(hi))
        return lo, hi

    # -- queries --------------------------------------------------------------
    def locate(self, pts) -> np.ndarray:
        pts = _f64(pts).reshape(-1, 3)
        out = np.empty(pts.shape[0], np.int32)
        lib().or_locate(self._h, _ptr(pts), pts.shape[0], _ptr(out))
        return out

    def trace(self, origins, dirs, kappa=1.0, records=True, nthreads=None):
        """Returns dict(tau, count[, offsets, leaf, ds])."""
        o = _f64(origins).reshape(-1, 3)
        k = _f64(dirs).reshape(-1, 3)
        n = o.shape[0]
        nt = nthreads or os.cpu_count() or 1
        tau = np.empty(n)
        cnt = np.empty(n, np.int32)
        rc = lib().or_trace(self._h, _ptr(o), _ptr(k), n, kappa, nt, _ptr(tau), _ptr(cnt),
                            None, None, None)
        if rc != 0:
            raise RuntimeError("oracle walk exceeded its step guard")
        out = dict(tau=tau, count=cnt)
        if records:
            off = np.zeros(n + 1, np.int64)
            np.cumsum(cnt, out=off[1:])
            tot = int(off[-1])
            leaf = np.empty(max(tot, 1), np.int32)
            ds = np.empty(max(tot, 1))
            tau2 = np.empty(n)
            rc = lib().or_trace(self._h, _ptr(o), _ptr(k), n, kappa, nt, _ptr(tau2), None,
                                _ptr(off), _ptr(leaf), _ptr(ds))
            if rc != 0:
                raise RuntimeError("oracle walk exceeded its step guard")
            out.update(offsets=off, leaf=leaf[:tot], ds=ds[:tot])
        return out

    def trace_brute(self, origin, direction, kappa=1.0, eps=1e-12):
        o = _f64(origin)
        k = _f64(direction)
        cap = self.n_leaves + 1
        leaf = np.empty(cap, np.int32)
        ds = np.empty(cap)
        tau = C.c_double()
        nh = lib().or_trace_brute(self._h, _ptr(o), _ptr(k), kappa, eps, C.byref(tau),
                                  _ptr(leaf), _ptr(ds), cap)
        return dict(tau=tau.value, leaf=leaf[:nh].copy(), ds=ds[:nh].copy())

    def neighbors_brute(self, leaf, face) -> np.ndarray:
        cap = self.n_leaves
        out = np.empty(max(cap, 1), np.int32)
        nf = lib().or_neighbors_brute(self._h, int(leaf), int(face), _ptr(out), cap)
        return out[:nf].copy()


def equal_mass_plane(d, lo, hi, axis, m=64, iters=50) -> float:
    """The plane across `axis` that splits the cell [lo, hi] into two parts of
    equal mass (midpoint-rule masses on m^3 points, bisection)."""
    h = _DensityHolder(d)
    lo_a, hi_a = _f64(lo), _f64(hi)
    return float(lib().or_equal_mass_plane(h.ref, _ptr(lo_a), _ptr(hi_a), int(axis), int(m), int(iters)))

"""Python binding of libhgrid.so, the gfx950 hierarchical-grid library.

Thin ctypes marshalling over the C ABI in include/hgrid.h: every step of grid
construction, traversal and location runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and the stream.  If the library has
not been built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HGRID_LIB names another build of the same library (e.g. one compiled with
# different launch bounds, for comparing builds); the default is the in-tree one.
LIB_PATH = os.environ.get("HGRID_LIB") or os.path.join(_HERE, "libhgrid.so")

OCTREE = 0
KDTREE = 1
KDGRAD = 2   # k-d tree split across the axis of strongest density gradient
FP64 = 0
FP32_RECHECK = 1
TAU_ONLY = 0
RECORDS = 1
FLAG_TIMING = 1
FLAG_RECHECKS = 2
STAGE_BUILD = 1
STAGE_TRACE = 2
STAGE_ALL = 3

HG_OK = 0
HG_E_INVAL = -1
HG_E_DOMAIN = -2
HG_E_DIR = -3
HG_E_CAPACITY = -4
HG_E_OOM = -5
HG_E_LIMIT = -6
HG_E_HIP = -7
HG_E_STEP = -8
HG_E_FORMAT = -9
# fixed work space of grid_trace_noalloc (hgrid.h)
NOALLOC_SCRATCH_BYTES = 512 * 1024


class HGError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})")


class Density(C.Structure):
    _fields_ = [
        ("lo", C.c_double * 3), ("side", C.c_double),
        ("has_box", C.c_int32), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("box_rho", C.c_double),
        ("has_disk", C.c_int32), ("disk_rho0", C.c_double), ("disk_hR", C.c_double),
        ("disk_hz", C.c_double),
        ("has_torus", C.c_int32), ("torus_R0", C.c_double), ("torus_a", C.c_double),
        ("torus_rho", C.c_double),
        ("n_clumps", C.c_int64), ("clump_c", C.c_void_p), ("clump_sigma", C.c_void_p),
        ("clump_amp", C.c_void_p), ("clump_trunc", C.c_double),
    ]


class Criteria(C.Structure):
    _fields_ = [
        ("total_mass", C.c_double), ("delta_max", C.c_double), ("tau_max", C.c_double),
        ("q_max", C.c_double), ("kappa", C.c_double),
        ("min_level", C.c_int32), ("max_level", C.c_int32), ("n_samples", C.c_int32),
        ("reserved", C.c_int32), ("seed", C.c_uint64), ("max_nodes", C.c_int64),
    ]


class TraceOpts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("mode", C.c_int32), ("kappa", C.c_double),
        ("flags", C.c_int32), ("block", C.c_int32), ("persistent", C.c_int32),
        ("chunk", C.c_int32), ("refill_min", C.c_int32), ("lds_bytes", C.c_int32),
        ("passes", C.c_int32), ("slab", C.c_int32),
    ]


class TraceOut(C.Structure):
    _fields_ = [
        ("tau", C.c_void_p), ("count", C.c_void_p), ("offsets", C.c_void_p),
        ("leaf", C.c_void_p), ("ds", C.c_void_p), ("capacity", C.c_int64),
        ("needed", C.c_int64), ("rechecks", C.c_int64), ("kernel_ms", C.c_float * 4),
        ("descents", C.c_int64),
    ]


class GridArrays(C.Structure):
    _fields_ = [
        ("tree_type", C.c_int32), ("max_level", C.c_int32), ("lo", C.c_double * 3),
        ("side", C.c_double), ("n_nodes", C.c_int64), ("n_leaves", C.c_int64),
        ("first_child", C.c_void_p), ("rho", C.c_void_p), ("level", C.c_void_p),
        ("coord", C.c_void_p), ("S", C.c_void_p), ("rho_min", C.c_void_p),
        ("rho_max", C.c_void_p), ("leaf_of", C.c_void_p), ("node_of", C.c_void_p),
        ("rope", C.c_void_p), ("geom", C.c_void_p),
    ]


_lib = None
_hip_lib = None

# (name, restype, argtypes) of every exported entry point
_SIGS = [
    ("grid_build", C.c_int, [C.POINTER(Density), C.POINTER(Criteria), C.c_int, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    ("grid_trace", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                             C.POINTER(TraceOpts), C.POINTER(TraceOut), C.c_void_p]),
    ("grid_trace_batched", C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                     C.POINTER(TraceOpts), C.POINTER(TraceOut), C.c_void_p]),
    ("grid_trace_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.POINTER(TraceOpts), C.POINTER(TraceOut), C.c_void_p]),
    ("grid_locate", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    ("grid_import", C.c_int, [C.POINTER(GridArrays), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("grid_export", C.c_int, [C.c_void_p, C.POINTER(GridArrays)]),
    ("grid_free", None, [C.c_void_p]),
    ("grid_release_scratch", C.c_int, []),
    ("batch_create", C.c_int, [C.c_int, C.POINTER(Density), C.POINTER(Criteria),
                               C.POINTER(C.c_int), C.POINTER(C.c_void_p)]),
    ("batch_bind", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                             C.POINTER(C.c_int64), C.POINTER(TraceOpts), C.POINTER(TraceOut)]),
    ("batch_run", C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    ("batch_capture", C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    ("batch_replay", C.c_int, [C.c_void_p, C.c_void_p]),
    ("batch_result", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                               C.POINTER(C.c_int64), C.POINTER(TraceOut)]),
    ("batch_grid", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    ("batch_free", None, [C.c_void_p]),
    ("batch_tune", C.c_int, [C.c_void_p, C.POINTER(TraceOpts), C.POINTER(C.c_float), C.c_void_p]),
    ("grid_density_diff", C.c_int, [C.c_void_p, C.POINTER(Density), C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p]),
    ("grid_segment_tau", C.c_int, [C.c_void_p, C.POINTER(TraceOut), C.c_int, C.c_int64, C.c_void_p,
                                   C.c_double, C.c_void_p, C.c_void_p]),
    ("grid_true_tau", C.c_int, [C.c_void_p, C.POINTER(Density), C.c_void_p, C.c_void_p,
                                C.POINTER(TraceOut), C.c_int, C.c_int64, C.c_void_p, C.c_double,
                                C.c_int, C.c_void_p, C.c_void_p]),
    ("grid_interact", C.c_int, [C.c_void_p, C.POINTER(TraceOut), C.c_int, C.c_int64, C.c_void_p,
                                C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grid_trace_segment", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.POINTER(TraceOpts), C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grid_trace_interact", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.POINTER(TraceOpts), C.c_void_p, C.c_void_p, C.c_void_p]),
    ("grid_leaf_tau", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_void_p, C.c_void_p]),
    ("grid_tau_percentile", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_double,
                                      C.POINTER(C.c_double), C.c_void_p]),
    ("grid_build_tau_recipe", C.c_int, [C.POINTER(Density), C.POINTER(Criteria), C.c_int, C.c_double,
                                        C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_double)]),
    ("grid_tune", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(TraceOpts),
                            C.POINTER(C.c_float), C.c_void_p]),
    ("grid_strerror", C.c_char_p, [C.c_int]),
    ("grid_last_hip_error", C.c_int, []),
]


def lib():
    """Load libhgrid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                "g.build()'` (hipcc, gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().grid_strerror(code).decode()
    except Exception:  # pragma: no cover - library missing
        return "?"


def _check(rc: int, what: str):
    if rc != HG_OK:
        raise HGError(rc, what)


def _hip():
    global _hip_lib
    if _hip_lib is None:
        h = C.CDLL("libamdhip64.so")
        h.hipMemcpy.restype = C.c_int
        h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip_lib = h
    return _hip_lib


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64x3(a, device) -> torch.Tensor:
    t = torch.as_tensor(a, dtype=torch.float64)
    t = t.reshape(-1, 3).to(device).contiguous()
    return t


def _density_struct(d):
    """Marshal a density description (attributes lo, side, box, disk, torus,
    clump_c, clump_sigma, clump_amp, clump_trunc) into the C struct."""
    s = Density()
    keep = []
    for i in range(3):
        s.lo[i] = float(d.lo[i])
    s.side = float(d.side)
    if getattr(d, "box", None) is not None:
        s.has_box = 1
        for i in range(3):
            s.box_lo[i] = d.box[i]
            s.box_hi[i] = d.box[3 + i]
        s.box_rho = d.box[6]
    if getattr(d, "disk", None) is not None:
        s.has_disk = 1
        s.disk_rho0, s.disk_hR, s.disk_hz = d.disk
    if getattr(d, "torus", None) is not None:
        s.has_torus = 1
        s.torus_R0, s.torus_a, s.torus_rho = d.torus
    cc = getattr(d, "clump_c", None)
    if cc is not None and len(cc):
        c = np.ascontiguousarray(cc, dtype=np.float64).reshape(-1, 3)
        sg = np.ascontiguousarray(d.clump_sigma, dtype=np.float64)
        am = np.ascontiguousarray(d.clump_amp, dtype=np.float64)
        keep += [c, sg, am]
        s.n_clumps = c.shape[0]
        s.clump_c = c.ctypes.data
        s.clump_sigma = sg.ctypes.data
        s.clump_amp = am.ctypes.data
    s.clump_trunc = float(getattr(d, "clump_trunc", 3.0))
    return s, keep


def _criteria_struct(cr, max_nodes: int = 0):
    c = Criteria()
    c.total_mass = cr.total_mass
    c.delta_max = cr.delta_max
    c.tau_max = cr.tau_max
    c.q_max = cr.q_max
    c.kappa = cr.kappa
    c.min_level = cr.min_level
    c.max_level = cr.max_level
    c.n_samples = cr.n_samples
    c.seed = cr.seed & ((1 << 64) - 1)
    c.max_nodes = max_nodes
    return c


class Grid:
    """A grid owned by the library (device memory)."""

    def __init__(self, handle: C.c_void_p, device):
        self._h = handle
        self.device = device
        a = GridArrays()
        _check(lib().grid_export(self._h, C.byref(a)), "grid_export")
        self.tree_type = a.tree_type
        self.max_level = a.max_level
        self.n_nodes = a.n_nodes
        self.n_leaves = a.n_leaves
        self.lo = tuple(a.lo)
        self.side = a.side

    # -- construction ------------------------------------------------------
    @classmethod
    def build(cls, density, criteria, tree_type: int, stream=None, device="cuda",
              max_nodes: int = 0):
        s, keep = _density_struct(density)
        c = _criteria_struct(criteria, max_nodes)
        h = C.c_void_p()
        with torch.cuda.device(device):
            rc = lib().grid_build(C.byref(s), C.byref(c), tree_type, _stream(stream), C.byref(h))
        del keep
        _check(rc, "grid_build")
        return cls(h, device)

    @classmethod
    def build_tau_recipe(cls, density, criteria, tree_type: int, fraction: float = 0.9, stream=None,
                         device="cuda", max_nodes: int = 0):
        """The optical-depth recipe of Sect. 4.1 (grid_build_tau_recipe):
        returns (grid, tau_max)."""
        s, keep = _density_struct(density)
        c = _criteria_struct(criteria, max_nodes)
        h = C.c_void_p()
        tm = C.c_double()
        with torch.cuda.device(device):
            rc = lib().grid_build_tau_recipe(C.byref(s), C.byref(c), tree_type, fraction,
                                             _stream(stream), C.byref(h), C.byref(tm))
        del keep
        _check(rc, "grid_build_tau_recipe")
        return cls(h, device), float(tm.value)

    def leaf_tau(self, kappa: float, n_samples: int = 64, stream=None) -> torch.Tensor:
        """Eq. (2) per leaf from its sampled mass (grid_leaf_tau)."""
        out = torch.empty(self.n_leaves, dtype=torch.float64, device=self.device)
        _check(lib().grid_leaf_tau(self._h, kappa, n_samples, _ptr(out), _stream(stream)),
               "grid_leaf_tau")
        return out

    def tau_percentile(self, kappa: float, n_samples: int = 64, fraction: float = 0.9,
                       stream=None) -> float:
        tm = C.c_double()
        _check(lib().grid_tau_percentile(self._h, kappa, n_samples, fraction, C.byref(tm),
                                         _stream(stream)), "grid_tau_percentile")
        return float(tm.value)

    @classmethod
    def from_arrays(cls, tree_type: int, first_child, rho, lo=(-1.0, -1.0, -1.0), side=2.0,
                    stream=None, device="cuda", axis=None):
        """grid_import; axis (KDGRAD): the split axis of every node (-1 for leaves)."""
        fc = torch.as_tensor(first_child, dtype=torch.int32).to(device).contiguous()
        r = torch.as_tensor(rho, dtype=torch.float64).to(device).contiguous()
        gm = None
        if axis is not None:
            ax = torch.as_tensor(axis, dtype=torch.int64)
            gm = torch.where(ax < 0, torch.full_like(ax, 3), ax) << 24
            gm = gm.to(torch.int32).to(device).contiguous()
        a = GridArrays()
        a.tree_type = tree_type
        for i in range(3):
            a.lo[i] = lo[i]
        a.side = side
        a.n_nodes = fc.numel()
        a.n_leaves = r.numel()
        a.first_child = fc.data_ptr()
        a.rho = r.data_ptr()
        if gm is not None:
            a.geom = gm.data_ptr()
        h = C.c_void_p()
        rc = lib().grid_import(C.byref(a), _stream(stream), C.byref(h))
        _check(rc, "grid_import")
        return cls(h, device)

    def free(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().grid_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- queries -------------------------------------------------------------
    def locate(self, points, stream=None) -> torch.Tensor:
        p = _dev_f64x3(points, self.device)
        out = torch.empty(p.shape[0], dtype=torch.int32, device=self.device)
        _check(lib().grid_locate(self._h, _ptr(p), p.shape[0], _ptr(out), _stream(stream)),
               "grid_locate")
        return out

    def trace(self, origins, dirs, precision: int = FP64, mode: int = RECORDS,
              kappa: float = 1.0, capacity: Optional[int] = None, timing: bool = False,
              count_rechecks: bool = False, stream=None, out: Optional[dict] = None,
              block: int = 0, persistent: int = -1, chunk: int = 0, refill_min: int = 0,
              lds_bytes: int = 0, tuned: Optional[dict] = None, passes: int = 0,
              slab: int = 0, noalloc: bool = False) -> dict:
        """Trace paths; returns tau, count (and offsets, leaf, ds in records
        mode) as device tensors plus needed / rechecks / kernel_ms.  With
        noalloc the call goes to grid_trace_noalloc (no device allocation by
        the library; output buffers are still allocated here unless `out`
        holds them at the right size)."""
        o = _dev_f64x3(origins, self.device)
        k = _dev_f64x3(dirs, self.device)
        n = o.shape[0]
        res = out if out is not None else {}
        if "tau" not in res or res["tau"].numel() != n:
            res["tau"] = torch.empty(n, dtype=torch.float64, device=self.device)
            res["count"] = torch.empty(n, dtype=torch.int32, device=self.device)
        if mode == RECORDS and ("offsets" not in res or res["offsets"].numel() != n + 1):
            res["offsets"] = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        opts = TraceOpts()
        opts.precision = precision
        opts.mode = mode
        opts.kappa = kappa
        opts.flags = (FLAG_TIMING if timing else 0) | (FLAG_RECHECKS if count_rechecks else 0)
        opts.block = block
        opts.persistent = persistent
        opts.chunk = chunk
        opts.refill_min = refill_min
        opts.lds_bytes = lds_bytes
        opts.passes = passes
        opts.slab = slab
        if tuned is not None:
            for key in ("block", "lds_bytes", "chunk", "refill_min"):
                setattr(opts, key, int(tuned[key]))
            opts.persistent = 3
        dsdt = torch.float64 if precision == FP64 else torch.float32
        for attempt in range(2):
            to = TraceOut()
            to.tau = res["tau"].data_ptr()
            to.count = res["count"].data_ptr()
            if mode == RECORDS:
                cap = capacity if capacity is not None else (
                    res["leaf"].numel() if "leaf" in res else 64 * max(n, 1))
                if "leaf" not in res or res["leaf"].numel() < cap or res["ds"].dtype != dsdt:
                    res["leaf"] = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
                    res["ds"] = torch.empty(max(cap, 1), dtype=dsdt, device=self.device)
                to.offsets = res["offsets"].data_ptr()
                to.leaf = res["leaf"].data_ptr()
                to.ds = res["ds"].data_ptr()
                to.capacity = res["leaf"].numel()
            fn = lib().grid_trace_noalloc if noalloc else lib().grid_trace
            rc = fn(self._h, _ptr(o), _ptr(k), n, C.byref(opts), C.byref(to), _stream(stream))
            if rc == HG_E_CAPACITY and attempt == 0 and capacity is None:
                capacity = int(to.needed)
                res.pop("leaf", None)
                res.pop("ds", None)
                continue
            _check(rc, "grid_trace")
            break
        res["needed"] = int(to.needed)
        res["rechecks"] = int(to.rechecks)
        res["descents"] = int(to.descents)
        res["kernel_ms"] = list(to.kernel_ms)
        return res

    def tune(self, origins, dirs, precision: int = FP32_RECHECK, mode: int = RECORDS,
             kappa: float = 1.0, stream=None, passes: int = 0) -> dict:
        """Autotuned launch shape of the walk for these paths (grid_tune):
        dict(block, lds_bytes, chunk, refill_min, ms); pass it to trace(tuned=)."""
        o = _dev_f64x3(origins, self.device)
        k = _dev_f64x3(dirs, self.device)
        opts = TraceOpts()
        opts.precision = precision
        opts.mode = mode
        opts.kappa = kappa
        opts.passes = passes
        ms = C.c_float()
        _check(lib().grid_tune(self._h, _ptr(o), _ptr(k), o.shape[0], C.byref(opts), C.byref(ms),
                               _stream(stream)), "grid_tune")
        return dict(block=opts.block, lds_bytes=opts.lds_bytes, chunk=opts.chunk,
                    refill_min=opts.refill_min, ms=float(ms.value))

    # -- consumers of the walk (Sect. 3.2 measures, interaction point) -------
    @staticmethod
    def _records(res):
        to = TraceOut()
        to.offsets = res["offsets"].data_ptr()
        to.leaf = res["leaf"].data_ptr()
        to.ds = res["ds"].data_ptr()
        to.capacity = res["leaf"].numel()
        prec = FP64 if res["ds"].dtype == torch.float64 else FP32_RECHECK
        return to, prec

    def density_diff(self, density, points, stream=None) -> torch.Tensor:
        """rho_t(x) - rho_g(x) at the points (grid_density_diff)."""
        p = _dev_f64x3(points, self.device)
        out = torch.empty(p.shape[0], dtype=torch.float64, device=self.device)
        st, keep = _density_struct(density)
        rc = lib().grid_density_diff(self._h, C.byref(st), _ptr(p), p.shape[0], _ptr(out),
                                     _stream(stream))
        del keep
        _check(rc, "grid_density_diff")
        return out

    def segment_tau(self, res: dict, s_max, kappa: float = 1.0, stream=None) -> torch.Tensor:
        """Grid optical depth of every traced path up to s_max (grid_segment_tau)."""
        to, prec = self._records(res)
        n = res["count"].numel()
        sm = torch.as_tensor(s_max, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().grid_segment_tau(self._h, C.byref(to), prec, n, _ptr(sm), kappa, _ptr(out),
                                      _stream(stream)), "grid_segment_tau")
        return out

    def true_tau(self, density, origins, dirs, res: dict, s_max, kappa: float = 1.0, m: int = 16,
                 stream=None) -> torch.Tensor:
        """Gauss-Legendre integral of kappa rho_t along the traced paths up to
        s_max (grid_true_tau)."""
        to, prec = self._records(res)
        o = _dev_f64x3(origins, self.device)
        k = _dev_f64x3(dirs, self.device)
        n = o.shape[0]
        sm = torch.as_tensor(s_max, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        st, keep = _density_struct(density)
        rc = lib().grid_true_tau(self._h, C.byref(st), _ptr(o), _ptr(k), C.byref(to), prec, n,
                                 _ptr(sm), kappa, m, _ptr(out), _stream(stream))
        del keep
        _check(rc, "grid_true_tau")
        return out

    def interact(self, res: dict, tau_star, kappa: float = 1.0, stream=None):
        """(leaf, s) of the interaction point of every traced path (grid_interact)."""
        to, prec = self._records(res)
        n = res["count"].numel()
        ts = torch.as_tensor(tau_star, dtype=torch.float64).to(self.device).contiguous()
        leaf = torch.empty(n, dtype=torch.int32, device=self.device)
        s = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().grid_interact(self._h, C.byref(to), prec, n, _ptr(ts), kappa, _ptr(leaf),
                                   _ptr(s), _stream(stream)), "grid_interact")
        return leaf, s

    def _early_opts(self, precision, kappa, tuned):
        opts = TraceOpts()
        opts.precision = precision
        opts.kappa = kappa
        if tuned is not None:
            for key in ("block", "chunk", "refill_min"):
                setattr(opts, key, int(tuned[key]))
        return opts

    def trace_segment(self, origins, dirs, s_max, precision: int = FP64, kappa: float = 1.0,
                      stream=None, tuned: Optional[dict] = None):
        """Early-exit walk (grid_trace_segment): (tau, count) of every path
        up to length s_max, without records."""
        o = _dev_f64x3(origins, self.device)
        k = _dev_f64x3(dirs, self.device)
        n = o.shape[0]
        sm = torch.as_tensor(s_max, dtype=torch.float64).to(self.device).contiguous()
        tau = torch.empty(n, dtype=torch.float64, device=self.device)
        cnt = torch.empty(n, dtype=torch.int32, device=self.device)
        opts = self._early_opts(precision, kappa, tuned)
        _check(lib().grid_trace_segment(self._h, _ptr(o), _ptr(k), _ptr(sm), n, C.byref(opts), _ptr(tau),
                                        _ptr(cnt), _stream(stream)), "grid_trace_segment")
        return tau, cnt

    def trace_interact(self, origins, dirs, tau_star, precision: int = FP64, kappa: float = 1.0,
                       stream=None, tuned: Optional[dict] = None):
        """Early-exit walk (grid_trace_interact): (leaf, s) of the interaction
        point of every path, without records."""
        o = _dev_f64x3(origins, self.device)
        k = _dev_f64x3(dirs, self.device)
        n = o.shape[0]
        ts = torch.as_tensor(tau_star, dtype=torch.float64).to(self.device).contiguous()
        leaf = torch.empty(n, dtype=torch.int32, device=self.device)
        s = torch.empty(n, dtype=torch.float64, device=self.device)
        opts = self._early_opts(precision, kappa, tuned)
        _check(lib().grid_trace_interact(self._h, _ptr(o), _ptr(k), _ptr(ts), n, C.byref(opts), _ptr(leaf),
                                         _ptr(s), _stream(stream)), "grid_trace_interact")
        return leaf, s

    # -- arrays ----------------------------------------------------------------
    def export(self) -> dict:
        """Copies of the grid's flat arrays as device tensors."""
        a = GridArrays()
        _check(lib().grid_export(self._h, C.byref(a)), "grid_export")
        N, L = a.n_nodes, a.n_leaves
        torch.cuda.synchronize(self.device)

        def cp(ptr, shape, dt):
            t = torch.empty(shape, dtype=dt, device=self.device)
            if t.numel():
                rc = _hip().hipMemcpy(C.c_void_p(t.data_ptr()), C.c_void_p(ptr),
                                      t.numel() * t.element_size(), 3)
                if rc != 0:
                    raise RuntimeError(f"hipMemcpy failed ({rc})")
            return t

        return dict(
            tree_type=a.tree_type, max_level=a.max_level, lo=tuple(a.lo), side=a.side,
            n_nodes=N, n_leaves=L,
            first_child=cp(a.first_child, (N,), torch.int32),
            rho=cp(a.rho, (L,), torch.float64),
            level=cp(a.level, (N,), torch.uint8),
            coord=cp(a.coord, (N, 3), torch.int32),
            S=cp(a.S, (N,), torch.float64),
            rho_min=cp(a.rho_min, (N,), torch.float64),
            rho_max=cp(a.rho_max, (N,), torch.float64),
            leaf_of=cp(a.leaf_of, (N,), torch.int32),
            node_of=cp(a.node_of, (L,), torch.int32),
            rope=cp(a.rope, (N, 6), torch.int32),
            geom=cp(a.geom, (N,), torch.int32) if a.geom else None,
        )

    @staticmethod
    def split_axes(geom) -> torch.Tensor:
        """Split axis of every node from exported geom (-1: not split)."""
        ax = (geom.to(torch.int64) >> 24) & 3
        return torch.where(ax == 3, torch.full_like(ax, -1), ax).to(torch.int8)


def tune_cached(grid: "Grid", origins, dirs, precision: int = FP32_RECHECK, mode: int = RECORDS,
                kappa: float = 1.0, path: Optional[str] = None) -> dict:
    """Grid.tune memoised in a JSON file (HGRID_TUNE_CACHE, else
    ~/.cache/hgrid_tune.json), keyed by device architecture, tree type,
    precision, mode and the grid's size class (rounded log2 of its leaf count)."""
    import json
    import math
    path = path or os.environ.get("HGRID_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "hgrid_tune.json")
    arch = torch.cuda.get_device_properties(grid.device).gcnArchName
    key = "|".join(str(x) for x in (arch, grid.tree_type, precision, mode,
                                     int(round(math.log2(max(grid.n_leaves, 1))))))
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    if key in cache:
        return cache[key]
    t = grid.tune(origins, dirs, precision=precision, mode=mode, kappa=kappa)
    cache[key] = t
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return t


def trace_batched(grids, origins, dirs, precision: int = FP64, mode: int = RECORDS,
                  kappa: float = 1.0, capacities=None, timing: bool = False,
                  count_rechecks: bool = False, chunk: int = 0, refill_min: int = 0,
                  stream=None, outs=None, block: int = 0):
    """Trace len(grids) path batches in one batched call; returns one result
    dict per grid (as Grid.trace) and the batch's kernel_ms / rechecks in the
    first."""
    ng = len(grids)
    dev = grids[0].device
    os_ = [_dev_f64x3(o, dev) for o in origins]
    ks_ = [_dev_f64x3(k, dev) for k in dirs]
    ns = [o.shape[0] for o in os_]
    res = outs if outs is not None else [dict() for _ in range(ng)]
    dsdt = torch.float64 if precision == FP64 else torch.float32
    opts = TraceOpts()
    opts.precision = precision
    opts.mode = mode
    opts.kappa = kappa
    opts.flags = (FLAG_TIMING if timing else 0) | (FLAG_RECHECKS if count_rechecks else 0)
    opts.chunk = chunk
    opts.refill_min = refill_min
    opts.block = block
    for attempt in range(2):
        tos = (TraceOut * ng)()
        for i in range(ng):
            r = res[i]
            n = ns[i]
            if "tau" not in r or r["tau"].numel() != n:
                r["tau"] = torch.empty(n, dtype=torch.float64, device=dev)
                r["count"] = torch.empty(n, dtype=torch.int32, device=dev)
            to = tos[i]
            to.tau = r["tau"].data_ptr()
            to.count = r["count"].data_ptr()
            if mode == RECORDS:
                if "offsets" not in r or r["offsets"].numel() != n + 1:
                    r["offsets"] = torch.empty(n + 1, dtype=torch.int64, device=dev)
                cap = capacities[i] if capacities is not None else (
                    r["leaf"].numel() if "leaf" in r else 64 * max(n, 1))
                if "leaf" not in r or r["leaf"].numel() < cap or r["ds"].dtype != dsdt:
                    r["leaf"] = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
                    r["ds"] = torch.empty(max(cap, 1), dtype=dsdt, device=dev)
                to.offsets = r["offsets"].data_ptr()
                to.leaf = r["leaf"].data_ptr()
                to.ds = r["ds"].data_ptr()
                to.capacity = r["leaf"].numel()
        gp = (C.c_void_p * ng)(*[g._h.value if isinstance(g._h, C.c_void_p) else g._h for g in grids])
        op = (C.c_void_p * ng)(*[o.data_ptr() for o in os_])
        kp = (C.c_void_p * ng)(*[k.data_ptr() for k in ks_])
        np_ = (C.c_int64 * ng)(*ns)
        rc = lib().grid_trace_batched(ng, gp, op, kp, np_, C.byref(opts), tos, _stream(stream))
        if rc == HG_E_CAPACITY and attempt == 0 and capacities is None:
            capacities = [int(tos[i].needed) for i in range(ng)]
            for r in res:
                r.pop("leaf", None)
                r.pop("ds", None)
            continue
        _check(rc, "grid_trace_batched")
        break
    for i in range(ng):
        res[i]["needed"] = int(tos[i].needed)
        res[i]["rechecks"] = int(tos[i].rechecks)
        res[i]["descents"] = int(tos[i].descents)
        res[i]["kernel_ms"] = list(tos[i].kernel_ms)
    return res


def release_scratch(device="cuda") -> None:
    """Free the device memory the library keeps for reuse: the records-mode
    trace scratch and the array blocks of freed grids (grid_release_scratch)."""
    with torch.cuda.device(torch.device(device)):
        _check(lib().grid_release_scratch(), "grid_release_scratch")


def build(density, criteria, tree_type, stream=None, device="cuda", max_nodes=0) -> Grid:
    return Grid.build(density, criteria, tree_type, stream, device, max_nodes)


def import_grid(tree_type, first_child, rho, lo=(-1.0, -1.0, -1.0), side=2.0, stream=None,
                device="cuda", axis=None) -> Grid:
    return Grid.from_arrays(tree_type, first_child, rho, lo, side, stream, device, axis)


class Batch:
    """Many grids built and traced with no host synchronisation (the batch_*
    calls): construction of every grid level by level in shared launches,
    then the batched walk over the bound path batches; run() enqueues it,
    capture() records it into a HIP graph that replay() launches."""

    def __init__(self, densities, criteria, tree_types, max_nodes, device="cuda"):
        ng = len(densities)
        ds = (Density * ng)()
        keep = []
        for i, d in enumerate(densities):
            st, k = _density_struct(d)
            ds[i] = st
            keep += k
        cs = (Criteria * ng)(*[_criteria_struct(c, int(m)) for c, m in zip(criteria, max_nodes)])
        tt = (C.c_int * ng)(*[int(t) for t in tree_types])
        h = C.c_void_p()
        with torch.cuda.device(device):
            rc = lib().batch_create(ng, ds, cs, tt, C.byref(h))
        del keep
        _check(rc, "batch_create")
        self._h = h
        self.ng = ng
        self.device = device
        self.tree_types = [int(t) for t in tree_types]
        self.results = None
        self._keep = None
        self._outs = None
        self._capture_stream = None

    def bind(self, origins, dirs, precision: int = FP32_RECHECK, mode: int = RECORDS,
             kappa: float = 1.0, capacities=None, chunk: int = 0, refill_min: int = 0,
             count_rechecks: bool = False, block: int = 0, passes: int = 0, slab: int = 0):
        """Bind path batches (one per grid) and allocate their outputs; the
        returned result dicts are filled by each later run or replay.
        Records mode walks once into per-path rows of `slab` records (0: the
        library's choice) unless passes=2 asks for a counting and a filling
        walk."""
        dev = self.device
        os_ = [_dev_f64x3(o, dev) for o in origins]
        ks_ = [_dev_f64x3(k, dev) for k in dirs]
        ns = [o.shape[0] for o in os_]
        dsdt = torch.float64 if precision == FP64 else torch.float32
        res = []
        tos = (TraceOut * self.ng)()
        for i, n in enumerate(ns):
            r = {"tau": torch.empty(n, dtype=torch.float64, device=dev),
                 "count": torch.empty(n, dtype=torch.int32, device=dev)}
            tos[i].tau = r["tau"].data_ptr()
            tos[i].count = r["count"].data_ptr()
            if mode == RECORDS:
                cap = int(capacities[i]) if capacities is not None else 64 * max(n, 1)
                r["offsets"] = torch.empty(n + 1, dtype=torch.int64, device=dev)
                r["leaf"] = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
                r["ds"] = torch.empty(max(cap, 1), dtype=dsdt, device=dev)
                tos[i].offsets = r["offsets"].data_ptr()
                tos[i].leaf = r["leaf"].data_ptr()
                tos[i].ds = r["ds"].data_ptr()
                tos[i].capacity = r["leaf"].numel()
            res.append(r)
        opts = TraceOpts()
        opts.precision = precision
        opts.mode = mode
        opts.kappa = kappa
        opts.flags = FLAG_RECHECKS if count_rechecks else 0
        opts.chunk = chunk
        opts.refill_min = refill_min
        opts.block = block
        opts.passes = passes
        opts.slab = slab
        op = (C.c_void_p * self.ng)(*[o.data_ptr() for o in os_])
        kp = (C.c_void_p * self.ng)(*[k.data_ptr() for k in ks_])
        np_ = (C.c_int64 * self.ng)(*ns)
        with torch.cuda.device(dev):
            _check(lib().batch_bind(self._h, op, kp, np_, C.byref(opts), tos), "batch_bind")
        self._keep = (os_, ks_)
        self._outs = tos
        self.results = res
        return res

    def run(self, stages: int = STAGE_ALL, stream=None):
        _check(lib().batch_run(self._h, stages, _stream(stream)), "batch_run")

    def tune(self, stream=None) -> dict:
        """Autotune the bound trace (batch_tune; needs a built batch, drops a
        captured graph): dict(block, chunk, refill_min, ms) of the winner."""
        ms = C.c_float()
        o = TraceOpts()
        _check(lib().batch_tune(self._h, C.byref(o), C.byref(ms), _stream(stream)), "batch_tune")
        return dict(block=o.block, chunk=o.chunk, refill_min=o.refill_min, ms=float(ms.value))

    def capture(self, stages: int = STAGE_ALL, stream=None):
        """Record the stages into a graph (on a side stream unless one is
        given: the legacy default stream cannot be captured)."""
        if stream is None:
            if self._capture_stream is None:
                self._capture_stream = torch.cuda.Stream(self.device)
            stream = self._capture_stream
        torch.cuda.synchronize(self.device)
        _check(lib().batch_capture(self._h, stages, _stream(stream)), "batch_capture")

    def replay(self, stream=None):
        _check(lib().batch_replay(self._h, _stream(stream)), "batch_replay")

    def result(self, stream=None):
        """Wait for the stream; per-grid node and leaf counts; sets needed and
        rechecks in the bound result dicts.  Raises HGError on a failed grid."""
        nn = (C.c_int64 * self.ng)()
        nl = (C.c_int64 * self.ng)()
        rc = lib().batch_result(self._h, _stream(stream), nn, nl, self._outs)
        if self.results is not None:
            for i, r in enumerate(self.results):
                r["needed"] = int(self._outs[i].needed)
                r["rechecks"] = int(self._outs[i].rechecks)
                r["descents"] = int(self._outs[i].descents)
        _check(rc, "batch_result")
        return list(nn), list(nl)

    def grid(self, i: int) -> Grid:
        """Grid i as a Grid (borrowing the batch's arrays; free it first)."""
        h = C.c_void_p()
        _check(lib().batch_grid(self._h, int(i), C.byref(h)), "batch_grid")
        return Grid(h, self.device)

    def free(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

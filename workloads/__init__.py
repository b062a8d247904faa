"""Seeded synthetic inputs for the hierarchical-grid build and trace.

This module is shared by the CPU oracle's tests and by the GPU benchmarks.
It holds no part of the method itself (no sampling, no stopping criteria, no
tree, no walk): only

* the parameters of the synthetic density fields that stand in for the
  paper's test models (the three-armed spiral, the clumpy AGN torus and the
  SPH galaxy of Sect. 3.1 are not available, so an exponential disk, a
  sharp-edged torus plus Gaussian clumps, and hierarchically clustered
  clumps take their place),
* the total dust mass of each field over the domain (the M_tot of the mass
  criterion, Sect. 4.1), computed by quadrature of the model's own formula,
  independently of any grid,
* ray origins and directions (photon-packet emission points and isotropic
  directions, Sect. 2.3).

Every generator is driven by ``numpy.random.Generator(PCG64(seed))`` so the
same seed gives the same arrays on every machine.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Optional

import numpy as np
from scipy import special

OCTREE = 0
KDTREE = 1

# Face-on optical depth through the centre of the exponential disk equals 1
# for the full column z in [-1, 1]:  rho0 * 2 hz (1 - exp(-1/hz)) = 1.
DISK_HR = 0.25
DISK_HZ = 0.03
DISK_RHO0 = 1.0 / (2.0 * DISK_HZ * (1.0 - math.exp(-1.0 / DISK_HZ)))

GRID_SEED_BASE = 0x1311070500
RAY_SEED_XOR = 0x5DEECE66D


@dataclasses.dataclass
class Density:
    """Parametric density field: the sum of the enabled components.

    Components are added in this order: box, disk, clumps (ascending index),
    torus.  Domain is the cube ``[lo, lo+side]^3``.
    """
    lo: tuple = (-1.0, -1.0, -1.0)
    side: float = 2.0
    # constant density inside an axis-aligned box (closed), 0 outside
    box: Optional[tuple] = None          # (lo0,lo1,lo2, hi0,hi1,hi2, rho)
    # exponential disk rho0 * exp(-R/hR - |z|/hz)
    disk: Optional[tuple] = None         # (rho0, hR, hz)
    # ring torus about the z axis: rho inside (R-R0)^2 + z^2 <= a^2
    torus: Optional[tuple] = None        # (R0, a, rho)
    # truncated Gaussian clumps A exp(-r^2 / 2 sigma^2) for r <= t sigma
    clump_c: Optional[np.ndarray] = None     # [n,3] float64
    clump_sigma: Optional[np.ndarray] = None  # [n]
    clump_amp: Optional[np.ndarray] = None    # [n]
    clump_trunc: float = 3.0

    @property
    def n_clumps(self) -> int:
        return 0 if self.clump_c is None else int(self.clump_c.shape[0])

    @property
    def hi(self):
        return tuple(l + self.side for l in self.lo)

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(repr((self.lo, self.side, self.box, self.disk, self.torus,
                       self.clump_trunc)).encode())
        for a in (self.clump_c, self.clump_sigma, self.clump_amp):
            if a is not None:
                h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class Criteria:
    """Stopping criteria of the subdivision (Sect. 4.1, 4.2).

    A node at level l is split when l < min_level, or when l < max_level and
    any of delta > delta_max, tau > tau_max, q > q_max holds.
    """
    total_mass: float
    delta_max: float = 1e-4
    tau_max: float = math.inf
    q_max: float = 1.0
    kappa: float = 1.0
    min_level: int = 0
    max_level: int = 6
    n_samples: int = 64
    seed: int = GRID_SEED_BASE


@dataclasses.dataclass
class Workload:
    name: str
    tree_type: int
    density: Density
    criteria: Criteria
    n_rays: int
    ray_kind: str          # "uniform" or "disk"
    ray_seed: int


# ----------------------------------------------------------------------------
# Total mass of each component over the domain, by quadrature of its formula.
# ----------------------------------------------------------------------------

def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _gl_interval(a, b, n):
    x, w = _gl(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def mass_box(d: Density) -> float:
    if d.box is None:
        return 0.0
    lo = np.maximum(np.array(d.box[:3]), np.array(d.lo))
    hi = np.minimum(np.array(d.box[3:6]), np.array(d.hi))
    ext = np.clip(hi - lo, 0.0, None)
    return float(d.box[6] * ext.prod())


def mass_disk(d: Density, n_phi: int = 96) -> float:
    """Exponential disk over the cube centred on the origin.

    z part analytic; the xy part uses the closed radial integral
    int_0^U R exp(-R/h) dR = h^2 (1 - exp(-U/h)(1 + U/h)) along each azimuth
    of one eighth of the square, by Gauss-Legendre in azimuth.
    """
    if d.disk is None:
        return 0.0
    rho0, hR, hz = d.disk
    half = 0.5 * d.side
    if any(abs(l + half) > 1e-15 for l in d.lo):
        raise ValueError("disk mass needs a domain centred on the origin")
    zpart = 2.0 * hz * (1.0 - math.exp(-half / hz))
    phi, w = _gl_interval(0.0, math.pi / 4, n_phi)
    u = half / (hR * np.cos(phi))
    inner = hR * hR * (1.0 - np.exp(-u) * (1.0 + u))
    ixy = 8.0 * float((w * inner).sum())
    return rho0 * zpart * ixy


def mass_torus(d: Density) -> float:
    if d.torus is None:
        return 0.0
    R0, a, rho = d.torus
    half = 0.5 * d.side
    if R0 + a > half or a > half:
        raise ValueError("torus must lie inside the domain")
    return rho * 2.0 * math.pi ** 2 * R0 * a * a


def _chi3_cdf(t: float) -> float:
    """P(|X| <= t) for a standard 3-D Gaussian."""
    return float(special.erf(t / math.sqrt(2.0))
                 - math.sqrt(2.0 / math.pi) * t * math.exp(-0.5 * t * t))


def mass_clumps(d: Density, n_q: int = 96) -> float:
    """Truncated Gaussian clumps: closed form when the truncation ball lies in
    the domain, nested quadrature (trigonometric substitution, analytic
    innermost erf) when the domain clips it."""
    if d.n_clumps == 0:
        return 0.0
    t = d.clump_trunc
    c = d.clump_c
    s = d.clump_sigma
    A = d.clump_amp
    lo = np.array(d.lo)
    hi = np.array(d.hi)
    R = t * s
    inside = np.all((c - R[:, None] >= lo) & (c + R[:, None] <= hi), axis=1)
    full = A * (2.0 * math.pi) ** 1.5 * s ** 3 * _chi3_cdf(t)
    total = float(full[inside].sum())
    xg, wg = _gl(n_q)
    for i in np.nonzero(~inside)[0]:
        total += _clipped_clump_mass(c[i], s[i], A[i], R[i], lo, hi, xg, wg)
    return total


def _clipped_clump_mass(c, s, A, R, lo, hi, xg, wg):
    # x = cx + R sin(th1), th1 in [th_a, th_b] (clipped by the domain)
    xa = max(lo[0], c[0] - R)
    xb = min(hi[0], c[0] + R)
    if xb <= xa:
        return 0.0
    ta = math.asin(max(-1.0, min(1.0, (xa - c[0]) / R)))
    tb = math.asin(max(-1.0, min(1.0, (xb - c[0]) / R)))
    th = 0.5 * (tb - ta) * xg + 0.5 * (tb + ta)
    wth = 0.5 * (tb - ta) * wg
    total = 0.0
    sq2s = math.sqrt(2.0) * s
    for x_th, w_th in zip(th, wth):
        dx = R * math.sin(x_th)
        r1 = R * math.cos(x_th)
        jac_x = R * math.cos(x_th)
        if r1 <= 0.0:
            continue
        ya = max(lo[1], c[1] - r1)
        yb = min(hi[1], c[1] + r1)
        if yb <= ya:
            continue
        pa = math.asin(max(-1.0, min(1.0, (ya - c[1]) / r1)))
        pb = math.asin(max(-1.0, min(1.0, (yb - c[1]) / r1)))
        ph = 0.5 * (pb - pa) * xg + 0.5 * (pb + pa)
        wph = 0.5 * (pb - pa) * wg
        dy = r1 * np.sin(ph)
        r2 = r1 * np.cos(ph)
        jac_y = r1 * np.cos(ph)
        za = np.maximum(lo[2], c[2] - r2)
        zb = np.minimum(hi[2], c[2] + r2)
        zint = s * math.sqrt(math.pi / 2.0) * (
            special.erf((zb - c[2]) / sq2s) - special.erf((za - c[2]) / sq2s))
        zint = np.where(zb > za, zint, 0.0)
        g = np.exp(-(dx * dx + dy * dy) / (2.0 * s * s))
        total += w_th * jac_x * float((wph * jac_y * g * zint).sum())
    return A * total


def total_mass(d: Density) -> float:
    return mass_box(d) + mass_disk(d) + mass_clumps(d) + mass_torus(d)


# ----------------------------------------------------------------------------
# Density-field parameters
# ----------------------------------------------------------------------------

def exp_disk() -> Density:
    return Density(disk=(DISK_RHO0, DISK_HR, DISK_HZ))


def uniform(rho: float = 1.0) -> Density:
    return Density(box=(-1.0, -1.0, -1.0, 1.0, 1.0, 1.0, rho))


def clumps_uniform(rng, n, sigma_lo, sigma_hi, amp_sigma, lo=-1.0, hi=1.0):
    c = rng.uniform(lo, hi, size=(n, 3))
    s = rng.uniform(sigma_lo, sigma_hi, size=n)
    a = rng.lognormal(0.0, amp_sigma, size=n)
    return c, s, a


def clumps_hierarchical(rng, n_per=46, levels=3, shrink=0.1):
    """Clustered centres: n_per points uniform in the cube, each spawning
    n_per children uniformly in a ball of radius shrink*scale, the scale
    starting at 1 and shrinking by `shrink` per generation."""
    pts = rng.uniform(-1.0, 1.0, size=(n_per, 3))
    scale = 1.0
    for _ in range(levels - 1):
        r = shrink * scale
        m = pts.shape[0]
        v = rng.normal(size=(m, n_per, 3))
        v /= np.linalg.norm(v, axis=2, keepdims=True)
        rad = r * rng.uniform(0.0, 1.0, size=(m, n_per, 1)) ** (1.0 / 3.0)
        pts = (pts[:, None, :] + v * rad).reshape(-1, 3)
        scale *= shrink
    return pts


# ----------------------------------------------------------------------------
# Rays
# ----------------------------------------------------------------------------

def isotropic(rng, n):
    mu = 2.0 * rng.uniform(size=n) - 1.0
    phi = 2.0 * math.pi * rng.uniform(size=n)
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([st * np.cos(phi), st * np.sin(phi), mu], axis=1)


def origins_uniform(rng, n, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, size=(n, 3))


def origins_stellar_disk(rng, n, hR=0.3, hz=0.05, lo=-1.0, hi=1.0):
    """Emission points of a stellar disk exp(-R/hR - |z|/hz): the radius
    follows Gamma(2, hR), the height Laplace(0, hz), the azimuth is uniform.
    Draws outside the cube are redrawn."""
    out = np.empty((n, 3))
    got = 0
    while got < n:
        m = int((n - got) * 1.3) + 16
        R = -hR * np.log(rng.uniform(size=m) * rng.uniform(size=m))
        z = rng.laplace(0.0, hz, size=m)
        ph = 2.0 * math.pi * rng.uniform(size=m)
        p = np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)
        ok = np.all((p >= lo) & (p <= hi), axis=1)
        p = p[ok][: n - got]
        out[got:got + p.shape[0]] = p
        got += p.shape[0]
    return out


def rays(kind: str, n: int, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "uniform":
        o = origins_uniform(rng, n)
    elif kind == "disk":
        o = origins_stellar_disk(rng, n)
    else:
        raise ValueError(kind)
    k = isotropic(rng, n)
    return np.ascontiguousarray(o), np.ascontiguousarray(k)


def array_digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ----------------------------------------------------------------------------
# The five benchmark workloads
# ----------------------------------------------------------------------------

def grid_seed(c: int, g: int = 0) -> int:
    return GRID_SEED_BASE + 16 * c + g


def workload(c: int, g: int = 0, tree_type: Optional[int] = None,
             n_rays: Optional[int] = None) -> Workload:
    """Workload c in 1..5 (g selects the grid of workload 4; tree_type picks
    the octree or k-d half of workload 3)."""
    gs = grid_seed(c, g)
    rs = gs ^ RAY_SEED_XOR
    if c == 1:
        d = exp_disk()
        cr = Criteria(total_mass=total_mass(d), delta_max=1e-4,
                      max_level=6, seed=gs)
        w = Workload("disk-octree-5e3", OCTREE, d, cr, 10_000, "uniform", rs)
    elif c == 2:
        d = exp_disk()
        cr = Criteria(total_mass=total_mass(d), delta_max=1e-6,
                      max_level=24, seed=gs)
        w = Workload("disk-kd-1e6", KDTREE, d, cr, 10_000_000, "disk", rs)
    elif c == 3:
        rng = np.random.Generator(np.random.PCG64(gs))
        cc, s, a = clumps_uniform(rng, 500, 0.005, 0.02, 1.0)
        d = Density(torus=(0.5, 0.1, 1.0), clump_c=cc, clump_sigma=s,
                    clump_amp=a, clump_trunc=3.0)
        tt = KDTREE if tree_type is None else tree_type
        if tt == OCTREE:
            cr = Criteria(total_mass=total_mass(d), delta_max=1e-6,
                          tau_max=0.1, q_max=0.9, min_level=3, max_level=10,
                          seed=gs)
            name = "torus-clumps-octree-4e6"
        else:
            cr = Criteria(total_mass=total_mass(d), delta_max=1e-6,
                          tau_max=0.1, q_max=0.9, min_level=9, max_level=30,
                          seed=gs)
            name = "torus-clumps-kd-4e6"
        w = Workload(name, tt, d, cr, 100_000_000, "uniform", rs)
    elif c == 4:
        rng = np.random.Generator(np.random.PCG64(gs))
        n = int(rng.integers(10, 2001))
        cc, s, a = clumps_uniform(rng, n, 0.005, 0.05, 1.0)
        dmax = 10.0 ** rng.uniform(-6.0, -3.0)
        nr = int(round(10.0 ** rng.uniform(3.0, 6.0)))
        d = Density(clump_c=cc, clump_sigma=s, clump_amp=a, clump_trunc=3.0)
        tt = OCTREE if g % 2 == 0 else KDTREE
        cr = Criteria(total_mass=total_mass(d), delta_max=dmax,
                      min_level=3 if tt == OCTREE else 9,
                      max_level=10 if tt == OCTREE else 30, seed=gs)
        w = Workload(f"clumps-batch-{g}", tt, d, cr, nr, "uniform", rs)
    elif c == 5:
        rng = np.random.Generator(np.random.PCG64(gs))
        cc = clumps_hierarchical(rng)
        s = np.full(cc.shape[0], 0.003)
        a = rng.lognormal(0.0, 1.5, size=cc.shape[0])
        d = Density(clump_c=cc, clump_sigma=s, clump_amp=a, clump_trunc=3.0)
        cr = Criteria(total_mass=total_mass(d), delta_max=1e-8, min_level=9,
                      max_level=40, seed=gs)
        w = Workload("hier-clumps-kd-2e7", KDTREE, d, cr, 1_000_000_000,
                     "disk", rs)
    else:
        raise ValueError(c)
    if n_rays is not None:
        w.n_rays = n_rays
    return w

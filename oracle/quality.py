"""Oracle for the consumers of the walk: the grid-quality measures of
Sect. 3.2 and the Monte Carlo interaction point along a path.

Test infrastructure only (as the rest of oracle/): plain numpy over the
oracle's own density, locate and trace; nothing here is used by the GPU
library.

* density_diff -- Sect. 3.2, first measure: rho_t(x) - rho_g(x) at given
  points, rho_g the uniform density of the leaf holding x.
* segment_tau -- Sect. 3.2, second measure, grid side: the optical depth
  tau_g of a path from its start up to a length s_max, i.e. the sum of
  kappa rho ds over its crossings with the last crossing cut at s_max.
* true_tau -- Sect. 3.2, second measure, true side: tau_t, the integral of
  kappa rho_t along the same stretch, by Gauss-Legendre quadrature with m
  nodes on every piece between consecutive cell boundaries of the path.
* interaction -- the Monte Carlo use of the walk (Sect. 1 and 2.3): the first
  crossing at which the cumulative optical depth reaches a target tau*, and
  the distance along the path where it does (tau grows linearly inside a
  cell).
"""
from __future__ import annotations

import numpy as np

from . import density as _density


def density_diff(grid, d, points) -> np.ndarray:
    """rho_t(x) - rho_g(x) for every point (points outside the grid: NaN)."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    leaf = grid.locate(pts)
    rho_leaf = grid.leaves()["rho"]
    out = np.full(pts.shape[0], np.nan)
    ok = leaf >= 0
    out[ok] = _density(d, pts[ok]) - rho_leaf[leaf[ok]]
    return out


def _paths(rec):
    off = np.asarray(rec["offsets"], dtype=np.int64)
    for i in range(off.size - 1):
        yield i, slice(int(off[i]), int(off[i + 1]))


def segment_tau(rec, rho_leaf, s_max, kappa=1.0) -> np.ndarray:
    """tau_g over [0, s_max[i]] of every path of a records-mode trace."""
    leaf = np.asarray(rec["leaf"])
    ds = np.asarray(rec["ds"], dtype=np.float64)
    out = np.zeros(len(rec["offsets"]) - 1)
    for i, sl in _paths(rec):
        s = 0.0
        t = 0.0
        for l, d in zip(leaf[sl], ds[sl]):
            if s >= s_max[i]:
                break
            step = min(d, s_max[i] - s)
            t += kappa * rho_leaf[l] * step
            s += d
        out[i] = t
    return out


def true_tau(d, origins, dirs, rec, s_max, kappa=1.0, m=16) -> np.ndarray:
    """tau_t over [0, s_max[i]] by m-node Gauss-Legendre on every cell piece."""
    xg, wg = np.polynomial.legendre.leggauss(m)
    ds = np.asarray(rec["ds"], dtype=np.float64)
    o = np.asarray(origins, dtype=np.float64).reshape(-1, 3)
    k = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(o.shape[0])
    for i, sl in _paths(rec):
        s = 0.0
        t = 0.0
        for d_ in ds[sl]:
            if s >= s_max[i]:
                break
            b = min(s + d_, s_max[i])
            half = 0.5 * (b - s)
            mid = 0.5 * (b + s)
            pts = o[i] + np.outer(mid + half * xg, k[i])
            t += kappa * half * float(np.dot(wg, _density(d, pts)))
            s += d_
        out[i] = t
    return out


def interaction(rec, rho_leaf, tau_star, kappa=1.0):
    """(leaf, s) per path: the crossing where the cumulative tau first reaches
    tau_star[i] and the distance along the path where it does; (-1, total
    length) when the path's whole tau stays below tau_star[i]."""
    leaf = np.asarray(rec["leaf"])
    ds = np.asarray(rec["ds"], dtype=np.float64)
    n = len(rec["offsets"]) - 1
    out_leaf = np.full(n, -1, dtype=np.int32)
    out_s = np.zeros(n)
    for i, sl in _paths(rec):
        s = 0.0
        t = 0.0
        for l, d_ in zip(leaf[sl], ds[sl]):
            dt = kappa * rho_leaf[l] * d_
            if t + dt >= tau_star[i] and dt > 0.0:
                out_leaf[i] = l
                out_s[i] = s + (tau_star[i] - t) / (kappa * rho_leaf[l])
                break
            t += dt
            s += d_
        else:
            out_s[i] = s
    return out_leaf, out_s

"""Oracle for the optical-depth recipe of Sect. 4.1: build with the mass
criterion only, take the optical depth of every cell (Eq. 2 with the cell's
sampled mass), sort the values ascending and set tau_max to the value at
position floor(0.9 N_cells) (0-based), then build again with both criteria.

Test infrastructure only (as the rest of oracle/).  The position rounding is
not stated in the paper: floor, counted from 0, is the reading used.
"""
from __future__ import annotations

import copy
import math

import numpy as np

from . import Grid


def leaf_tau(grid, kappa: float, n_samples: int) -> np.ndarray:
    """Eq. (2) per leaf, in leaf order: kappa M sqrt(a^2+b^2+c^2) / (a b c)
    with M = S (V / N) the leaf's sampled mass (Eq. 1)."""
    nd = grid.nodes()
    no = grid.leaves()["node_of"]
    lv = nd["level"][no].astype(np.int64)
    S = nd["S"][no]
    if grid.tree == 0:   # octree: depth = level on every axis
        dep = np.stack([lv, lv, lv], axis=1)
    else:                # k-d: axis d has depth floor((level + 2 - d) / 3)
        dep = np.stack([(lv + 2 - d) // 3 for d in range(3)], axis=1)
    w = np.ldexp(np.full(dep.shape, grid.side), -dep)
    a, b, c = w[:, 0], w[:, 1], w[:, 2]
    V = a * b * c
    M = S * (V / float(n_samples))
    diag = np.sqrt(a * a + b * b + c * c)
    return kappa * M * diag / (a * b * c)


def tau_percentile(grid, kappa: float, n_samples: int, fraction: float = 0.9) -> float:
    t = np.sort(leaf_tau(grid, kappa, n_samples))
    return float(t[min(t.size - 1, int(math.floor(fraction * t.size)))])


def build_with_recipe(d, cr, tree, fraction: float = 0.9):
    """(grid, tau_max): the second build, with tau_max from the first."""
    c1 = copy.copy(cr)
    c1.tau_max = math.inf
    g1 = Grid.build(d, c1, tree)
    tmax = tau_percentile(g1, cr.kappa, cr.n_samples, fraction)
    del g1
    c2 = copy.copy(cr)
    c2.tau_max = tmax
    return Grid.build(d, c2, tree), tmax

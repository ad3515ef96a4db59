"""Seeded coefficient fields and right-hand sides.

alpha is the piecewise-constant coefficient of the curl-curl term (mu^{-1} in
the paper's equation for the model problem), one value per element.
"""
from __future__ import annotations

import numpy as np


def _cell_index(mesh):
    """(i, j[, k]) cell coordinates of each element (hex: one cell; tri/tet: the
    square/cube the simplex lies in)."""
    c = mesh.coords[mesh.elems].mean(axis=1)           # centroid
    n = np.array(mesh.shape)
    # centroids of jittered tets stay inside their cube (jitter < 0.25 h)
    idx = np.floor(c * n).astype(np.int64)
    return np.minimum(idx, n - 1)


def subdomain_log_uniform(mesh, sub: int, seed: int, lo: float = -4.0, hi: float = 4.0):
    """alpha = 10^U(lo,hi), constant on each of sub^d equal subdomains.

    The draw is one array of shape (sub,)*d indexed [k][j][i] (x fastest).
    """
    rng = np.random.default_rng(seed)
    d = mesh.dim
    logs = rng.uniform(lo, hi, size=(sub,) * d)
    cell = _cell_index(mesh)
    s = cell * sub // np.array(mesh.shape)
    if d == 3:
        la = logs[s[:, 2], s[:, 1], s[:, 0]]
    else:
        la = logs[s[:, 1], s[:, 0]]
    return 10.0 ** la


def checkerboard(mesh, sub: int, lo: float = 1e-4, hi: float = 1e4):
    """Binary checkerboard on sub^d subdomains: lo where the subdomain index sum is even."""
    cell = _cell_index(mesh)
    s = cell * sub // np.array(mesh.shape)
    par = s.sum(axis=1) % 2
    return np.where(par == 0, lo, hi)


def stripes_2d(mesh, a_even: float = 10.0, a_odd: float = 0.1):
    """alpha alternating per vertical column of elements (x index parity)."""
    cell = _cell_index(mesh)
    return np.where(cell[:, 0] % 2 == 0, a_even, a_odd)


def rhs_uniform(n: int, seed: int):
    """f ~ U[-1, 1]^n from numpy's default generator (PCG64)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)

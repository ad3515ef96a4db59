"""Geometric Nedelec interpolation ("Geo", the comparison method of Section 5).

For nested structured meshes (a mesh and its coarsening by two in every
direction) the coarse lowest-order Nedelec space lies inside the fine one,
and the geometric interpolation writes each coarse basis function in the
fine basis: P[e, E] = int_e w_E . t_e ds, the fine edge degree of freedom of
the coarse basis function w_E.  The basis functions are linear along every
fine edge, so the midpoint rule gives the integral exactly:
P[e, E] = w_E(midpoint of e) . (x_head(e) - x_tail(e)).

  * triangles: Whitney functions w_E = l_a grad(l_b) - l_b grad(l_a) of the
    coarse triangle holding the fine edge (a fine edge on a coarse edge may
    take either neighbour: the tangential trace is continuous);
  * hexahedra: first-kind tensor-product functions, e.g. for an x-edge of the
    coarse cell at transverse offsets (j, k): w = phi_j(eta) phi_k(zeta) e_x / H.

This is an input generator: it builds a transfer operator from mesh
coordinates and holds none of the paper's method (no coarsening, matching
or harmonic extension).  Both the CPU oracle and the GPU library take its
matrices as given (the library's AMG_INTERP_USER mode).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import hex_mesh, simplex_mesh_2d


def _kept_maps(mesh, dirichlet=True):
    ke = ~mesh.bnd_edge if dirichlet else np.ones(mesh.edges.shape[0], dtype=bool)
    emap = np.full(mesh.edges.shape[0], -1, dtype=np.int64)
    emap[ke] = np.arange(int(ke.sum()))
    return ke, emap


def _edge_lookup(mesh):
    nn = mesh.coords.shape[0]
    key = mesh.edges[:, 0] * nn + mesh.edges[:, 1]
    order = np.argsort(key)
    return nn, key[order], order


def _find_edges(lookup, a, b):
    nn, skey, order = lookup
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    k = lo * nn + hi
    pos = np.searchsorted(skey, k)
    pos = np.minimum(pos, len(skey) - 1)
    if not np.all(skey[pos] == k):
        raise ValueError("coarse edge not found")
    return order[pos]


def _assemble(rows, cols, vals, shape):
    keep = (rows >= 0) & (cols >= 0) & (vals != 0.0)
    P = sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=shape)
    P.sum_duplicates()
    P.sort_indices()
    return P


def geo_interpolation_tri(L: int, dirichlet: bool = True):
    """P (fine kept edges x coarse kept edges) from the level L-1 triangular
    mesh to the level L mesh (Dirichlet edges eliminated on both, unless
    dirichlet=False)."""
    fine, coarse = simplex_mesh_2d(L), simplex_mesh_2d(L - 1)
    kf, emap_f = _kept_maps(fine, dirichlet)
    kc, emap_c = _kept_maps(coarse, dirichlet)
    lookup = _edge_lookup(coarse)
    M = 2 ** (L - 1)
    H = 1.0 / M
    x0 = fine.coords[fine.edges[:, 0]]
    x1 = fine.coords[fine.edges[:, 1]]
    mid = 0.5 * (x0 + x1)
    t = x1 - x0
    I = np.clip(np.floor(mid[:, 0] / H).astype(np.int64), 0, M - 1)
    J = np.clip(np.floor(mid[:, 1] / H).astype(np.int64), 0, M - 1)
    xi = mid[:, 0] / H - I
    eta = mid[:, 1] / H - J
    lower = xi >= eta                                  # triangle (I,J),(I+1,J),(I+1,J+1)
    nx = M + 1
    v0 = I + nx * J
    v1 = np.where(lower, (I + 1) + nx * J, I + nx * (J + 1))
    v2 = (I + 1) + nx * (J + 1)
    V = np.stack([v0, v1, v2], axis=1)
    X = coarse.coords[V]                               # (ne, 3, 2)
    # barycentric coordinates and their gradients
    T = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]], axis=2)     # columns: edge vectors
    Tinv = np.linalg.inv(T)                            # rows: grad l1, grad l2
    g1, g2 = Tinv[:, 0, :], Tinv[:, 1, :]
    g0 = -(g1 + g2)
    d = mid - X[:, 0]
    l1 = np.einsum("ed,ed->e", g1, d)
    l2 = np.einsum("ed,ed->e", g2, d)
    lam = np.stack([1.0 - l1 - l2, l1, l2], axis=1)
    grads = np.stack([g0, g1, g2], axis=1)
    rows, cols, vals = [], [], []
    for a, b in ((0, 1), (0, 2), (1, 2)):
        na, nb = V[:, a], V[:, b]
        # orient the coarse edge from its lower to its higher node id
        swap = na > nb
        aa = np.where(swap, b, a)
        bb = np.where(swap, a, b)
        idx = np.arange(len(mid))
        w = lam[idx, aa][:, None] * grads[idx, bb] - lam[idx, bb][:, None] * grads[idx, aa]
        val = np.einsum("ed,ed->e", w, t)
        E = _find_edges(lookup, na, nb)
        rows.append(emap_f)
        cols.append(emap_c[E])
        vals.append(val)
    return _assemble(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                     (int(kf.sum()), int(kc.sum())))


def geo_interpolation_hex(N: int, dirichlet: bool = True):
    """P from the (N/2)^3 hexahedral mesh to the N^3 mesh (N even)."""
    if N % 2:
        raise ValueError("N must be even")
    fine, coarse = hex_mesh(N), hex_mesh(N // 2)
    kf, emap_f = _kept_maps(fine, dirichlet)
    kc, emap_c = _kept_maps(coarse, dirichlet)
    lookup = _edge_lookup(coarse)
    Nc = N // 2
    H = 1.0 / Nc
    x0 = fine.coords[fine.edges[:, 0]]
    x1 = fine.coords[fine.edges[:, 1]]
    mid = 0.5 * (x0 + x1)
    t = x1 - x0
    axis = np.argmax(np.abs(t), axis=1)
    cell = np.clip(np.floor(mid / H).astype(np.int64), 0, Nc - 1)
    loc = mid / H - cell                              # local coordinates in [0, 1]
    n1 = Nc + 1
    step = np.array([1, n1, n1 * n1])
    base = cell @ step
    idx = np.arange(len(mid))
    ax_b = (axis + 1) % 3
    ax_c = (axis + 2) % 3
    rows, cols, vals = [], [], []
    for j in (0, 1):
        for k in (0, 1):
            tail = base + j * step[ax_b] + k * step[ax_c]
            head = tail + step[axis]
            pj = np.where(j == 1, loc[idx, ax_b], 1.0 - loc[idx, ax_b])
            pk = np.where(k == 1, loc[idx, ax_c], 1.0 - loc[idx, ax_c])
            # w . t = phi_j phi_k (t . e_axis) / H
            val = pj * pk * t[idx, axis] / H
            E = _find_edges(lookup, tail, head)
            rows.append(emap_f)
            cols.append(emap_c[E])
            vals.append(val)
    return _assemble(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                     (int(kf.sum()), int(kc.sum())))


def geo_hierarchy(kind: str, size: int, nlevels: int):
    """(Ps, Gs) of the geometric hierarchy with `nlevels` levels: Ps[l] maps
    level l+1 (coarser) to level l, and Gs[l] is the Dirichlet discrete
    gradient of level l's mesh (Gs[0] is the finest problem's G)."""
    from .mesh import make_problem
    Ps, Gs = [], []
    for l in range(nlevels):
        s = size - l if kind == "tri" else size // 2 ** l
        Gs.append(make_problem(kind, s).G)
        if l + 1 < nlevels:
            Ps.append(geo_interpolation_tri(s) if kind == "tri" else geo_interpolation_hex(s))
    return Ps, Gs

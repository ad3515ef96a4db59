"""Meshes and lowest-order Nedelec assembly (Section 2 of the paper).

Conventions (the paper only names "lowest-order Nedelec elements"; the
textbook construction is used):

* Nodes are numbered row-major (x fastest).  Every edge is oriented from its
  lower to its higher global node id; the degree of freedom is the line
  integral of the tangential component along that orientation.
* Edges are numbered lexicographically by (tail node, head node).
* Dirichlet condition u x n = 0: every edge lying in the boundary is
  eliminated, and so is every boundary node (columns of G).  The surviving
  edges and nodes keep their relative order.
* G (edges x nodes) holds -1 at the tail and +1 at the head of each edge,
  restricted to the surviving nodes, so boundary-touching edges keep one entry.
* Hexahedra: tensor-product first-kind Nedelec functions on axis-aligned cubes,
  integrated with 2-point Gauss rules per direction (exact for these
  integrands).  Simplices (triangles, tetrahedra): Whitney forms
  lambda_a grad(lambda_b) - lambda_b grad(lambda_a) with exact integrals of
  products of barycentric coordinates.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# mesh containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    kind: str                 # "hex", "tri", "tet"
    dim: int
    coords: np.ndarray        # (nnodes, dim) float64
    elems: np.ndarray         # (nelem, nv) node ids; simplices sorted ascending
    edges: np.ndarray         # (nedges, 2) int64 (tail < head), lexicographic
    elem_edges: np.ndarray    # (nelem, nle) global edge ids in local edge order
    bnd_node: np.ndarray      # (nnodes,) bool
    bnd_edge: np.ndarray      # (nedges,) bool
    shape: tuple              # cells per direction
    h: float


def _structured_coords(shape, dim):
    axes = [np.linspace(0.0, 1.0, s + 1) for s in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    # row-major with x fastest: node id = i + (nx+1)*(j + (ny+1)*k)
    cols = [g.transpose(tuple(reversed(range(dim)))).reshape(-1) for g in grids]
    return np.stack(cols, axis=1)


def _node_index(shape):
    """Return a function (i, j[, k]) -> node id for a structured grid."""
    if len(shape) == 2:
        nx = shape[0] + 1
        return lambda i, j: i + nx * j
    nx, ny = shape[0] + 1, shape[1] + 1
    return lambda i, j, k: i + nx * (j + ny * k)


def _edges_from_pairs(pairs):
    """Unique lexicographic edge list and the inverse map for (tail, head) pairs."""
    nmax = int(pairs.max()) + 1
    key = pairs[:, 0].astype(np.int64) * nmax + pairs[:, 1].astype(np.int64)
    ukey, inv = np.unique(key, return_inverse=True)
    edges = np.stack([ukey // nmax, ukey % nmax], axis=1)
    return edges, inv


def hex_mesh(N: int) -> Mesh:
    """Uniform N^3 hexahedral mesh of the unit cube."""
    shape = (N, N, N)
    coords = _structured_coords(shape, 3)
    nid = _node_index(shape)
    n1 = N + 1
    nn = n1 ** 3
    # edges enumerated per tail node in id order: x, then y, then z
    i = np.arange(nn) % n1
    j = (np.arange(nn) // n1) % n1
    k = np.arange(nn) // (n1 * n1)
    has = np.stack([i < N, j < N, k < N], axis=1)            # (nn, 3)
    flat = has.reshape(-1)
    eid_flat = np.cumsum(flat) - 1                            # id of each existing (node, dir)
    eid = np.where(has, eid_flat.reshape(nn, 3), -1)
    step = np.array([1, n1, n1 * n1])
    tails = np.repeat(np.arange(nn), 3).reshape(nn, 3)[has]
    dirs = np.tile(np.arange(3), nn).reshape(nn, 3)[has]
    edges = np.stack([tails, tails + step[dirs]], axis=1).astype(np.int64)
    # elements (ei, ej, ek); corner (a,b,c) node = nid(ei+a, ej+b, ek+c)
    ei, ej, ek = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ei = ei.transpose(2, 1, 0).reshape(-1)
    ej = ej.transpose(2, 1, 0).reshape(-1)
    ek = ek.transpose(2, 1, 0).reshape(-1)
    corners = np.stack([nid(ei + a, ej + b, ek + c)
                        for c in (0, 1) for b in (0, 1) for a in (0, 1)], axis=1)
    # local edges: x-edges at (b,c), y-edges at (a,c), z-edges at (a,b); each
    # ordered with the varying transverse index fastest
    le = []
    for c in (0, 1):
        for b in (0, 1):
            le.append(eid[nid(ei, ej + b, ek + c), 0])
    for c in (0, 1):
        for a in (0, 1):
            le.append(eid[nid(ei + a, ej, ek + c), 1])
    for b in (0, 1):
        for a in (0, 1):
            le.append(eid[nid(ei + a, ej + b, ek), 2])
    elem_edges = np.stack(le, axis=1)
    bnd_node = (i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N)
    # an edge lies in the boundary iff a transverse coordinate is 0 or N
    ti, tj, tk = i[edges[:, 0]], j[edges[:, 0]], k[edges[:, 0]]
    d = dirs
    onb = np.zeros(len(edges), dtype=bool)
    for ax, t in enumerate((ti, tj, tk)):
        onb |= (d != ax) & ((t == 0) | (t == N))
    return Mesh("hex", 3, coords, corners, edges, elem_edges, bnd_node, onb,
                shape, 1.0 / N)


def simplex_mesh_2d(L: int) -> Mesh:
    """Uniform triangular mesh: 2^L x 2^L squares, each cut by the (i,j)-(i+1,j+1) diagonal."""
    M = 2 ** L
    shape = (M, M)
    coords = _structured_coords(shape, 2)
    nid = _node_index(shape)
    ii, jj = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    ii = ii.T.reshape(-1)
    jj = jj.T.reshape(-1)
    t1 = np.stack([nid(ii, jj), nid(ii + 1, jj), nid(ii + 1, jj + 1)], axis=1)
    t2 = np.stack([nid(ii, jj), nid(ii, jj + 1), nid(ii + 1, jj + 1)], axis=1)
    elems = np.sort(np.concatenate([t1, t2]), axis=1)
    return _simplex_finish("tri", 2, coords, elems, shape, 1.0 / M)


def kuhn_tet_mesh(N: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """N^3 cubes, each split into 6 tetrahedra sharing the (0,0,0)-(1,1,1) diagonal.

    Interior nodes are moved by U(-jitter*h, jitter*h) per coordinate (seeded);
    every tetrahedron must keep a positive volume.
    """
    shape = (N, N, N)
    coords = _structured_coords(shape, 3)
    nid = _node_index(shape)
    g = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ei, ej, ek = (x.transpose(2, 1, 0).reshape(-1) for x in g)
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        p0 = np.zeros(3, dtype=np.int64)
        p1 = p0 + unit[perm[0]]
        p2 = p1 + unit[perm[1]]
        p3 = np.ones(3, dtype=np.int64)
        tets.append(np.stack([nid(ei + p[0], ej + p[1], ek + p[2]) for p in (p0, p1, p2, p3)], axis=1))
    elems = np.sort(np.concatenate(tets), axis=1)
    h = 1.0 / N
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        n1 = N + 1
        ids = np.arange(n1 ** 3)
        i, j, k = ids % n1, (ids // n1) % n1, ids // (n1 * n1)
        inner = (i > 0) & (i < N) & (j > 0) & (j < N) & (k > 0) & (k < N)
        disp = rng.uniform(-jitter * h, jitter * h, size=(n1 ** 3, 3))
        coords = coords + np.where(inner[:, None], disp, 0.0)
    m = _simplex_finish("tet", 3, coords, elems, shape, h)
    vol = _simplex_volumes(m.coords, m.elems)
    if np.any(np.abs(vol) <= 0.0):
        raise ValueError("degenerate tetrahedron after jitter")
    # all Kuhn tets of a cube share one handedness only up to the permutation
    # parity; what must hold is that no tet flips relative to the unjittered mesh
    ref = _simplex_volumes(_structured_coords(shape, 3), m.elems)
    if np.any(np.sign(vol) != np.sign(ref)):
        raise ValueError("jitter inverted a tetrahedron")
    return m


def _simplex_volumes(coords, elems):
    d = coords.shape[1]
    v0 = coords[elems[:, 0]]
    J = np.stack([coords[elems[:, a + 1]] - v0 for a in range(d)], axis=2)
    return np.linalg.det(J) / (2.0 if d == 2 else 6.0)


def _simplex_finish(kind, dim, coords, elems, shape, h):
    nv = dim + 1
    loc = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    pairs = np.concatenate([np.stack([elems[:, a], elems[:, b]], axis=1) for a, b in loc])
    edges, inv = _edges_from_pairs(pairs)
    elem_edges = inv.reshape(len(loc), -1).T.copy()
    nn = coords.shape[0]
    tol = 1e-12
    bnd_node = np.any((coords < tol) | (coords > 1 - tol), axis=1)
    # an edge is in the boundary iff both endpoints share a boundary plane
    x0, x1 = coords[edges[:, 0]], coords[edges[:, 1]]
    same_plane = np.zeros(len(edges), dtype=bool)
    for ax in range(dim):
        for val in (0.0, 1.0):
            same_plane |= (np.abs(x0[:, ax] - val) < tol) & (np.abs(x1[:, ax] - val) < tol)
    return Mesh(kind, dim, coords, elems, edges, elem_edges, bnd_node, same_plane,
                shape, h)


# ----------------------------------------------------------------------------
# element matrices
# ----------------------------------------------------------------------------
def _hex_local(h):
    """12x12 curl-curl (S) and mass (M) matrices of an axis-aligned cube of side h."""
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    gw = np.array([0.5, 0.5])
    ell = [lambda t: 1.0 - t, lambda t: t]
    dell = [-1.0, 1.0]
    S = np.zeros((12, 12))
    M = np.zeros((12, 12))
    for qx, wx in zip(gp, gw):
        for qy, wy in zip(gp, gw):
            for qz, wz in zip(gp, gw):
                q = (qx, qy, qz)
                w = wx * wy * wz * h ** 3
                val = np.zeros((12, 3))
                cur = np.zeros((12, 3))
                idx = 0
                for ax in range(3):
                    t1, t2 = [a for a in range(3) if a != ax]
                    for b2 in (0, 1):
                        for b1 in (0, 1):
                            # phi = (1/h) ell_b1(x_t1) ell_b2(x_t2) e_ax
                            f = ell[b1](q[t1]) * ell[b2](q[t2]) / h
                            val[idx, ax] = f
                            # partial derivatives of the component along ax
                            dt1 = dell[b1] * ell[b2](q[t2]) / h / h
                            dt2 = ell[b1](q[t1]) * dell[b2] / h / h
                            grad = np.zeros(3)
                            grad[t1] = dt1
                            grad[t2] = dt2
                            # curl(phi e_ax) = grad(phi) x e_ax
                            e = np.zeros(3)
                            e[ax] = 1.0
                            cur[idx] = np.cross(grad, e)
                            idx += 1
                S += w * cur @ cur.T
                M += w * val @ val.T
    return S, M


def _whitney_local(coords, elems):
    """Per-element Whitney curl-curl and mass matrices, vectorised over elements."""
    ne, nv = elems.shape
    d = nv - 1
    X = coords[elems]                                   # (ne, nv, d)
    J = np.stack([X[:, a + 1] - X[:, 0] for a in range(d)], axis=2)   # (ne, d, d) cols = edges
    detJ = np.linalg.det(J)
    vol = np.abs(detJ) / (2.0 if d == 2 else 6.0)
    Jinv = np.linalg.inv(J)                             # rows: grad lambda_1..d
    grads = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)  # (ne, nv, d)
    loc = [(a, b) for a in range(nv) for b in range(a + 1, nv)]
    nle = len(loc)
    # integrals of lambda_i lambda_j: vol (1+delta_ij) / ((d+1)(d+2))
    mass_ll = lambda i, j: (1.0 + (i == j)) / ((d + 1) * (d + 2))
    gg = np.einsum("eid,ejd->eij", grads, grads)        # grad.grad
    if d == 2:
        cr = lambda a, b: grads[:, a, 0] * grads[:, b, 1] - grads[:, a, 1] * grads[:, b, 0]
        curls = np.stack([2.0 * cr(a, b) for a, b in loc], axis=1)[:, :, None]
    else:
        curls = np.stack([2.0 * np.cross(grads[:, a], grads[:, b]) for a, b in loc], axis=1)
    S = np.einsum("eik,ejk->eij", curls, curls) * vol[:, None, None]
    M = np.zeros((ne, nle, nle))
    for p, (a, b) in enumerate(loc):
        for q, (c, e) in enumerate(loc):
            # (l_a g_b - l_b g_a).(l_c g_e - l_e g_c)
            M[:, p, q] = vol * (mass_ll(a, c) * gg[:, b, e] - mass_ll(a, e) * gg[:, b, c]
                                - mass_ll(b, c) * gg[:, a, e] + mass_ll(b, e) * gg[:, a, c])
    return S, M


# ----------------------------------------------------------------------------
# assembly
# ----------------------------------------------------------------------------
def _coo_to_csr(rows, cols, vals, n):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def assemble(mesh: Mesh, alpha: np.ndarray, beta: float, dirichlet: bool = True,
             parts: bool = False):
    """Assemble A = A^s(alpha) + beta A^m and G.

    alpha: per-element coefficient of the curl-curl term (mu^{-1}).
    Returns (A, G, keep_edges, keep_nodes) or, with parts=True,
    (A, As, Am, G, keep_edges, keep_nodes) where As = A^s(alpha), Am = A^m.
    """
    ne = mesh.elems.shape[0]
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (ne,))
    ned = mesh.edges.shape[0]
    nn = mesh.coords.shape[0]
    if dirichlet:
        keep_e = ~mesh.bnd_edge
        keep_n = ~mesh.bnd_node
    else:
        keep_e = np.ones(ned, dtype=bool)
        keep_n = np.ones(nn, dtype=bool)
    emap = np.full(ned, -1, dtype=np.int64)
    emap[keep_e] = np.arange(int(keep_e.sum()))
    nmap = np.full(nn, -1, dtype=np.int64)
    nmap[keep_n] = np.arange(int(keep_n.sum()))
    n = int(keep_e.sum())
    EE = emap[mesh.elem_edges]                              # (ne, nle)
    nle = EE.shape[1]
    if mesh.kind == "hex":
        S0, M0 = _hex_local(mesh.h)
        Sl = None
    else:
        Sl, Ml = _whitney_local(mesh.coords, mesh.elems)
    outs = []
    which = ("A", "S", "M") if parts else ("A",)
    rr = np.repeat(EE, nle, axis=1).reshape(-1)
    cc = np.tile(EE, (1, nle)).reshape(-1)
    ok = (rr >= 0) & (cc >= 0)
    rr = rr[ok].astype(np.int32)
    cc = cc[ok].astype(np.int32)
    for w in which:
        if mesh.kind == "hex":
            if w == "A":
                v = alpha[:, None] * S0.reshape(1, -1) + beta * M0.reshape(1, -1)
            elif w == "S":
                v = alpha[:, None] * S0.reshape(1, -1)
            else:
                v = np.broadcast_to(M0.reshape(1, -1), (ne, nle * nle))
        else:
            if w == "A":
                v = alpha[:, None] * Sl.reshape(ne, -1) + beta * Ml.reshape(ne, -1)
            elif w == "S":
                v = alpha[:, None] * Sl.reshape(ne, -1)
            else:
                v = Ml.reshape(ne, -1)
        v = np.ascontiguousarray(v).reshape(-1)[ok]
        outs.append(_coo_to_csr(rr, cc, v, n))
        del v
    # discrete gradient
    tails = nmap[mesh.edges[keep_e, 0]]
    heads = nmap[mesh.edges[keep_e, 1]]
    rows = np.concatenate([np.arange(n), np.arange(n)])
    cols = np.concatenate([tails, heads])
    vals = np.concatenate([-np.ones(n), np.ones(n)])
    m = cols >= 0
    G = sp.csr_matrix((vals[m], (rows[m], cols[m])), shape=(n, int(keep_n.sum())))
    G.sort_indices()
    return (*outs, G, keep_e, keep_n)


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    A: sp.csr_matrix
    G: sp.csr_matrix
    f: np.ndarray
    mesh: Mesh
    keep_edges: np.ndarray
    keep_nodes: np.ndarray
    alpha: np.ndarray
    beta: float

    def ref_coarse_nodes(self, levels: int):
        """Coarse node lists of the geometric (refinement) hierarchy, per level.

        Level l's nodes are the surviving lattice nodes whose coordinates are
        multiples of 2^l (numbered in ascending fine id, which is how the
        algebraic coarse nodes are numbered too); its coarse set is the subset
        that are multiples of 2^(l+1), given as indices into level l's nodes.
        """
        shape = self.mesh.shape
        nn = self.mesh.coords.shape[0]
        ids = np.arange(nn)
        dim = self.mesh.dim
        sub = []
        rem = ids.copy()
        for ax in range(dim):
            sub.append(rem % (shape[ax] + 1))
            rem = rem // (shape[ax] + 1)
        out = []
        for l in range(levels):
            s, s2 = 2 ** l, 2 ** (l + 1)
            lvl = self.keep_nodes.copy()
            crs = self.keep_nodes.copy()
            for ax in range(dim):
                lvl &= sub[ax] % s == 0
                crs &= sub[ax] % s2 == 0
            lvl_ids = np.nonzero(lvl)[0]
            pos = np.searchsorted(lvl_ids, np.nonzero(crs)[0])
            out.append(pos.astype(np.int32))
        return out


def make_problem(kind: str, size: int, alpha=1.0, beta: float = 1.0, f=None,
                 dirichlet: bool = True, jitter: float = 0.0, mesh_seed: int = 0,
                 parts: bool = False):
    """Build a mesh, assemble it, and attach a right-hand side.

    kind: "hex" (size = N cells per side), "tri" (size = refinement level L),
    "tet" (size = N cubes per side, Kuhn split).  alpha: scalar, per-element
    array, or a callable mesh -> per-element array.
    """
    if kind == "hex":
        mesh = hex_mesh(size)
    elif kind == "tri":
        mesh = simplex_mesh_2d(size)
    elif kind == "tet":
        mesh = kuhn_tet_mesh(size, jitter, mesh_seed)
    else:
        raise ValueError(kind)
    a = alpha(mesh) if callable(alpha) else alpha
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (mesh.elems.shape[0],)).copy()
    res = assemble(mesh, a, beta, dirichlet, parts=parts)
    A, G, ke, kn = res[0], res[-3], res[-2], res[-1]
    n = A.shape[0]
    if f is None:
        f = np.ones(n)
    elif callable(f):
        f = f(n)
    p = Problem(A, G, np.asarray(f, dtype=np.float64), mesh, ke, kn, a, beta)
    if parts:
        p.As, p.Am = res[1], res[2]
    return p

"""FP64 CPU oracle of the H(curl) AMG method -- test infrastructure only.

Each function follows one step of the paper (arXiv 2602.23613):

  augment_g            Algorithm 1 (Section 4.1)
  nodal_graph          nodal dual operator A_G~ = G~^T A G~ (Section 4.1), as a graph
  coarse_nodal_graph   the same graph on coarser levels (distance-two rule, see below)
  rs_first_pass        classical C/F splitting, first pass (Section 4.1)
  nodal_cf             Algorithm 2
  form_r               Algorithm 3 (coarse edge variables R, interior set S_I)
  coarse_gradient      G_c = R G I_C, eq. (Gc) in Section 3.1 and the end of Section 4.2
  extension_blocks     local blocks of A_II used for the harmonic extension
  interpolation        P_app = (I - S_I A_II^{-1} S_I^T A) R^T, eq. (sparseP)
  patch_sets,          the same extension column by column on overlapping
  interpolation_patch  patches of interior DoFs (a 3D variant)
  galerkin             A_c = P^T A P (Section 1)
  smoother_setup       blocks, colours and factors of the OSS-l1 smoother (Section 5)
  vcycle, pcg          V(1,1) cycle and preconditioned CG (Section 5)

Readings of points the paper leaves open (each documented where it is used):
  * graph of A_G~: symbolic pattern of |G~|^T |A| |G~| on level 0, all
    connections strong; on coarser levels, coarse nodes are joined when their
    fine counterparts are within graph distance two;
  * C/F splitting: Ruge-Stueben first pass, measure |N_U|+2|N_F|, ties to the
    smallest id, F_ini = N(B) minus B;
  * "distance-two neighbours" and the path i -> k -> j are measured in the
    edge graph of G~ (nodes joined by an edge DoF); k = smallest mutual
    neighbour; R entries +-1 with r G~ = -e_i + e_j;
  * A_II^{-1}: when every connected component of graph(A_II) is small the
    blocks are the components (exact, as in the paper's 2D setting);
    otherwise blocks are owner groups ordered by BFS depth from the coarse
    and path-middle nodes, each solved with the already-extended shallower
    rows as data (parity unpinned: the paper has no 3D construction);
  * smoother: multiplicative Schwarz over node stars (the edges of one column
    of G), coloured greedily so that a colour's blocks are uncoupled; pre =
    forward + backward sweep then l1-Jacobi, post = l1-Jacobi then forward +
    backward sweep.
"""
from __future__ import annotations

import dataclasses
import heapq
from collections import deque

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def _ones(M):
    M = sp.csr_matrix(M, copy=True)
    M.data = np.ones_like(M.data, dtype=np.float64)
    return M


def structural_product(X, Y):
    """X @ Y keeping every structurally nonzero entry (no cancellation drops).

    The pattern is that of |X| |Y| computed on all-ones data (no cancellation is
    possible); the values come from the numeric product.
    """
    X = sp.csr_matrix(X)
    Y = sp.csr_matrix(Y)
    pat = (_ones(X) @ _ones(Y)).tocsr()
    pat.sort_indices()
    num = (X @ Y).tocsr()
    num.sort_indices()
    out = pat.copy()
    out.data = np.zeros_like(pat.data)
    ncol = Y.shape[1]
    pr = np.repeat(np.arange(pat.shape[0], dtype=np.int64), np.diff(pat.indptr))
    nr = np.repeat(np.arange(num.shape[0], dtype=np.int64), np.diff(num.indptr))
    pkey = pr * ncol + pat.indices
    nkey = nr * ncol + num.indices
    pos = np.searchsorted(pkey, nkey)
    out.data[pos] = num.data
    return out


def _rows_of(M, i):
    return M.indices[M.indptr[i]:M.indptr[i + 1]]


# ----------------------------------------------------------------------------
# Algorithm 1: augment G with boundary-node columns
# ----------------------------------------------------------------------------
def augment_g(G):
    """Algorithm 1: for each row of G holding a single nonzero delta, append a
    new column with -delta in that row.  Returns (G~, B) where B lists the new
    column ids m, m+1, ... in row order."""
    G = sp.csr_matrix(G)
    n, m = G.shape
    rows, cols, vals, B = [], [], [], []
    k = 0
    nnz_row = np.diff(G.indptr)
    for i in np.nonzero(nnz_row == 1)[0]:          # rows in increasing order
        delta = G.data[G.indptr[i]]
        rows.append(i)
        cols.append(m + k)
        vals.append(-delta)
        B.append(m + k)
        k += 1
    Gx = sp.csr_matrix((np.array(vals, dtype=np.float64), (np.array(rows, dtype=np.int64),
                        np.array(cols, dtype=np.int64) - m)), shape=(n, k))
    Gt = sp.hstack([G, Gx], format="csr")
    Gt.sort_indices()
    return Gt, np.array(B, dtype=np.int64)


# ----------------------------------------------------------------------------
# nodal dual graph
# ----------------------------------------------------------------------------
def nodal_graph(A, Gt):
    """Graph of A_G~ = G~^T A G~ (Section 4.1): nodes u != v are joined iff the
    symbolic product |G~|^T |A| |G~| has an entry (u, v).  All connections are
    strong (the values of G~^T A G~ are beta times a mass-Laplacian, whose
    structural zeros would remove the mesh edges the matching needs)."""
    Gt1 = _ones(Gt)
    S = (Gt1.T @ _ones(A) @ Gt1).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    S.data[:] = 1.0
    S.sort_indices()
    return S


def coarse_nodal_graph(S_fine, fine_of):
    """Nodal graph of the next level: coarse nodes u != v are joined iff their
    fine counterparts fine_of[u], fine_of[v] are within distance two in the
    fine nodal graph (coefficient-free; keeps the coarse graph as local as the
    fine one)."""
    nf = S_fine.shape[0]
    nc = len(fine_of)
    T = (_ones(S_fine) + sp.identity(nf, format="csr")).tocsr()
    Sel = sp.csr_matrix((np.ones(nc), (np.arange(nc), np.asarray(fine_of))), shape=(nc, nf))
    left = (Sel @ T).tocsr()
    right = (T @ Sel.T).tocsr()
    S = (left @ right).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    S.data[:] = 1.0
    S.sort_indices()
    return S


# ----------------------------------------------------------------------------
# C/F splitting (Algorithm 2)
# ----------------------------------------------------------------------------
U_, C_, F_ = 0, 1, 2


def rs_first_pass(S, C_ini, F_ini):
    """Classical (Ruge-Stueben) first-pass C/F splitting on the symmetric graph
    S, started from prescribed C and F sets (Algorithm 2).

    Measure of an undecided node: |N(i) in U| + 2 |N(i) in F|.  Repeatedly the
    undecided node of largest measure (ties: smallest id) becomes C and all its
    undecided neighbours become F ("mark all nearest neighbours of coarse nodes
    as fine"); every undecided neighbour of a new F node gains one.  Returns
    the state array (1 = C, 2 = F)."""
    n = S.shape[0]
    st = np.zeros(n, dtype=np.int8)
    st[np.asarray(C_ini, dtype=np.int64)] = C_
    st[np.asarray(F_ini, dtype=np.int64)] = F_
    ip, ix = S.indptr, S.indices
    lam = np.zeros(n, dtype=np.int64)
    for i in range(n):
        if st[i] == U_:
            nb = st[ix[ip[i]:ip[i + 1]]]
            lam[i] = int(np.sum(nb == U_)) + 2 * int(np.sum(nb == F_))
    heap = [(-int(lam[i]), i) for i in range(n) if st[i] == U_]
    heapq.heapify(heap)
    while heap:
        neg, i = heapq.heappop(heap)
        if st[i] != U_ or -neg != lam[i]:
            continue
        st[i] = C_
        new_f = [j for j in ix[ip[i]:ip[i + 1]] if st[j] == U_]
        for j in new_f:
            st[j] = F_
        for j in new_f:
            for m in ix[ip[j]:ip[j + 1]]:
                if st[m] == U_:
                    lam[m] += 1
                    heapq.heappush(heap, (-int(lam[m]), int(m)))
    return st


def nodal_cf(S, B):
    """Algorithm 2: C starts as the boundary nodes B, F as their neighbours
    (minus B), the C/F splitting runs on the rest; c_G = C minus B."""
    B = np.asarray(B, dtype=np.int64)
    nbr = set()
    for b in B:
        nbr.update(int(x) for x in _rows_of(S, b))
    F_ini = np.array(sorted(nbr - set(int(b) for b in B)), dtype=np.int64)
    st = rs_first_pass(S, B, F_ini)
    isB = np.zeros(S.shape[0], dtype=bool)
    isB[B] = True
    cG = np.nonzero((st == C_) & ~isB)[0]
    return cG, st


# ----------------------------------------------------------------------------
# Algorithm 3: coarse edge variables
# ----------------------------------------------------------------------------
def edge_graph(Gt):
    """Adjacency of nodes joined by an edge DoF (a row of G~ with two entries)
    and the map (u, v) -> row."""
    Gt = sp.csr_matrix(Gt)
    n = Gt.shape[0]
    nn = Gt.shape[1]
    cnt = np.diff(Gt.indptr)
    two = np.nonzero(cnt == 2)[0]
    u = Gt.indices[Gt.indptr[two]]
    v = Gt.indices[Gt.indptr[two] + 1]
    E = sp.csr_matrix((np.ones(2 * len(two)), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(nn, nn))
    E.sum_duplicates()
    E.sort_indices()
    row_of = {}
    for r, a, b in zip(two, u, v):
        row_of[(int(a), int(b))] = int(r)
        row_of[(int(b), int(a))] = int(r)
    return E, row_of


@dataclasses.dataclass
class RRows:
    dof1: np.ndarray
    dof2: np.ndarray
    s1: np.ndarray
    s2: np.ndarray
    i: np.ndarray
    j: np.ndarray
    k: np.ndarray

    def __len__(self):
        return len(self.dof1)


def form_r(Gt, Cp, B, n, skip_bb=True):
    """Algorithm 3 (coarse and fine variables).

    Cp: the coarse node set c_G united with the boundary nodes B.  Pairs (i, j)
    of Cp with i < j are visited in lexicographic order; a pair is used when i
    and j are at distance exactly two in the edge graph of G~ and not both in
    B.  k is their smallest mutual neighbour; if k was already the middle of a
    path the pair is skipped.  Otherwise the two edge DoFs i-k and k-j form a
    row r of R with entries +-1 chosen so that r G~ = -e_i + e_j.  All other
    DoFs are the interior set S_I (ascending)."""
    E, row_of = edge_graph(Gt)
    Gt = sp.csr_matrix(Gt)
    Cp = np.array(sorted(set(int(x) for x in Cp)), dtype=np.int64)
    inCp = np.zeros(Gt.shape[1], dtype=bool)
    inCp[Cp] = True
    inB = np.zeros(Gt.shape[1], dtype=bool)
    inB[np.asarray(B, dtype=np.int64)] = True
    used = np.zeros(n, dtype=bool)
    K = set()
    out = {x: [] for x in ("dof1", "dof2", "s1", "s2", "i", "j", "k")}

    def g(r, c):
        s, e = Gt.indptr[r], Gt.indptr[r + 1]
        idx = np.nonzero(Gt.indices[s:e] == c)[0]
        return Gt.data[s + idx[0]]

    for i in Cp:
        n1 = set(int(x) for x in _rows_of(E, i))
        d2 = set()
        for kk in n1:
            for jj in _rows_of(E, kk):
                jj = int(jj)
                if jj != i and jj not in n1:
                    d2.add(jj)
        for j in sorted(d2):
            if j <= i or not inCp[j]:
                continue
            if skip_bb and inB[i] and inB[j]:
                continue
            common = sorted(n1 & set(int(x) for x in _rows_of(E, j)))
            k = common[0]
            if k in K:
                continue
            d1 = row_of[(int(i), k)]
            dd2 = row_of[(k, int(j))]
            assert not used[d1] and not used[dd2]
            used[d1] = used[dd2] = True
            K.add(k)
            out["dof1"].append(d1)
            out["dof2"].append(dd2)
            out["s1"].append(-g(d1, i))
            out["s2"].append(g(dd2, j))
            out["i"].append(int(i))
            out["j"].append(int(j))
            out["k"].append(k)
    rr = RRows(*(np.array(out[x], dtype=np.float64 if x in ("s1", "s2") else np.int64)
                 for x in ("dof1", "dof2", "s1", "s2", "i", "j", "k")))
    interior = np.nonzero(~used)[0]
    return rr, interior


def r_transpose(rr, n):
    """R^T as an n x n_c sparse matrix."""
    nc = len(rr)
    rows = np.concatenate([rr.dof1, rr.dof2])
    cols = np.concatenate([np.arange(nc), np.arange(nc)])
    vals = np.concatenate([rr.s1, rr.s2])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def coarse_gradient(G, rr):
    """G_c = R G I_C: I_C keeps the nonzero columns of R G (ascending).
    Returns (G_c, kept columns as level-l node ids)."""
    R = r_transpose(rr, G.shape[0]).T.tocsr()
    RG = (R @ sp.csr_matrix(G)).tocsr()
    RG.eliminate_zeros()
    cols = np.unique(RG.indices)
    Gc = RG[:, cols].tocsr()
    Gc.sort_indices()
    return Gc, cols


# ----------------------------------------------------------------------------
# interpolation P_app by local harmonic extension
# ----------------------------------------------------------------------------
def extension_blocks(A, Gt, interior, sources, max_block=64):
    """Blocks of A_II for the local harmonic extension.

    If every connected component of graph(A_II) has at most max_block DoFs the
    blocks are the components (A_II is then block diagonal and the extension is
    exact).  Otherwise each interior DoF is owned by the deeper endpoint of its
    edge (ties: larger id), depth being the BFS distance in the edge graph of
    G~ from `sources` (the nodes of c_G, B and the path middles K); blocks are
    the owner groups, processed by ascending depth.

    Returns (blocks, depths, exact) with blocks a list of ascending DoF arrays."""
    A = sp.csr_matrix(A)
    interior = np.asarray(interior, dtype=np.int64)
    if len(interior) == 0:
        return [], np.zeros(0, dtype=np.int64), True
    AII = _ones(A[interior][:, interior])
    ncomp, lab = connected_components(AII, directed=False)
    sizes = np.bincount(lab, minlength=ncomp)
    if sizes.max() <= max_block:
        blocks = [interior[lab == c] for c in range(ncomp)]
        blocks.sort(key=lambda b: int(b[0]))
        return blocks, np.zeros(len(blocks), dtype=np.int64), True
    E, _ = edge_graph(Gt)
    nn = Gt.shape[1]
    INF = np.iinfo(np.int64).max
    depth = np.full(nn, INF, dtype=np.int64)
    dq = deque()
    for s in sorted(set(int(x) for x in sources)):
        depth[s] = 0
        dq.append(s)
    while dq:
        u = dq.popleft()
        for v in _rows_of(E, u):
            if depth[v] == INF:
                depth[v] = depth[u] + 1
                dq.append(int(v))
    Gt = sp.csr_matrix(Gt)
    groups = {}
    for e in interior:
        nodes = Gt.indices[Gt.indptr[e]:Gt.indptr[e + 1]]
        if len(nodes) == 0:
            key = (0, -1 - int(e))           # isolated DoF: its own block
        else:
            best = None
            for v in nodes:
                cand = (int(depth[v]), int(v))
                if best is None or cand > best:
                    best = cand
            key = best
        groups.setdefault(key, []).append(int(e))
    keys = sorted(groups)
    blocks = [np.array(sorted(groups[k]), dtype=np.int64) for k in keys]
    depths = np.array([k[0] for k in keys], dtype=np.int64)
    return blocks, depths, False


def interpolation(A, Rt, blocks, depths):
    """P_app = (I - S_I A_II^{-1} S_I^T A) R^T, eq. (sparseP), with A_II^{-1}
    replaced by the block solves: exterior rows are R^T; for each block B (by
    ascending depth) X_B = -A_BB^{-1} A_B,: P_done, where P_done holds R^T and
    the rows of all blocks of smaller depth.  The stored pattern of a block's
    rows is the union of the structural column patterns of A_B,: P_done."""
    A = sp.csr_matrix(A)
    n, nc = Rt.shape
    done = sp.csr_matrix(Rt)
    order = np.argsort(depths, kind="stable")
    uniq = np.unique(depths)
    rows_all, cols_all, vals_all = [], [], []
    for d in uniq:
        idx = [b for b in order if depths[b] == d]
        r_d, c_d, v_d = [], [], []
        for b in idx:
            blk = blocks[b]
            rhs = structural_product(A[blk], done)
            cols = np.unique(rhs.indices)
            R = rhs[:, cols].toarray()
            ABB = A[blk][:, blk].toarray()
            X = -np.linalg.solve(ABB, R) if len(cols) else np.zeros((len(blk), 0))
            for a, e in enumerate(blk):
                r_d.append(np.full(len(cols), e, dtype=np.int64))
                c_d.append(cols)
                v_d.append(X[a])
        if r_d:
            r_d = np.concatenate(r_d)
            c_d = np.concatenate(c_d)
            v_d = np.concatenate(v_d)
            done = _csr_union(done, r_d, c_d, v_d, n, nc)
    done.sort_indices()
    return done


def patch_sets(A, Rt, interior, hops=2, cap=128):
    """Interior support S_c of every column c of P for the patch extension.

    Column c of eq. (sparseP) is the A-harmonic extension of R^T e_c: the
    vector with exterior values R^T e_c and least energy, whose interior part
    solves A_II x = -A_IE (R^T e_c)_E on the whole interior set.  The patch
    form (an addition for 3D, where A_II does not split into small blocks)
    keeps the support of the interior part near the column's exterior DoFs:
    starting from S = {}, each of `hops` rounds counts, for every interior DoF
    j outside S, the DoFs of (exterior support of c) + S it is coupled to in
    A, and adds the coupled ones in order of that count (largest first, ties
    to the smaller id) until S holds `cap` DoFs.  Returns a list of ascending
    DoF arrays, one per column."""
    A = _ones(sp.csr_matrix(A))
    Rt = sp.csc_matrix(Rt)
    n, nc = Rt.shape
    isint = np.zeros(n, dtype=bool)
    isint[np.asarray(interior, dtype=np.int64)] = True
    out = []
    for c in range(nc):
        ext = [int(e) for e in Rt.indices[Rt.indptr[c]:Rt.indptr[c + 1]]]
        S = set()
        for _ in range(hops):
            if len(S) >= cap:
                break
            count = {}
            for e in ext + sorted(S):
                for j in _rows_of(A, e):
                    j = int(j)
                    if isint[j] and j not in S:
                        count[j] = count.get(j, 0) + 1
            ranked = sorted(count, key=lambda j: (-count[j], j))
            S.update(ranked[:max(cap - len(S), 0)])
        out.append(np.array(sorted(S), dtype=np.int64))
    return out


def interpolation_patch(A, Rt, patches):
    """P with column c = R^T e_c + X_c, where X_c is supported on patches[c]
    and solves A_SS X_c = -A_S,: R^T e_c with S = patches[c] (the least-energy
    extension of the column's exterior values into its patch).  When A_II is
    block diagonal and every patch holds the whole blocks coupled to the
    column, this is eq. (sparseP) exactly."""
    A = sp.csr_matrix(A)
    Rt = sp.csc_matrix(Rt)
    n, nc = Rt.shape
    rows, cols, vals = [], [], []
    for c in range(nc):
        S = patches[c]
        if len(S) == 0:
            continue
        rhs = (A[S] @ Rt[:, c]).toarray().ravel()
        x = -np.linalg.solve(A[S][:, S].toarray(), rhs)
        rows.append(S)
        cols.append(np.full(len(S), c, dtype=np.int64))
        vals.append(x)
    # exterior rows (R^T) and interior rows (X) do not overlap; the COO route
    # keeps every structural entry, including a solve's exact zeros
    E = Rt.tocoo()
    rows = np.concatenate([E.row.astype(np.int64)] + rows)
    cols = np.concatenate([E.col.astype(np.int64)] + cols)
    vals = np.concatenate([E.data] + vals)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(n, nc)).tocsr()
    P.sort_indices()
    return P


def _csr_union(M, r, c, v, n, nc):
    coo = sp.csr_matrix(M).tocoo()
    rr = np.concatenate([coo.row.astype(np.int64), r])
    cc = np.concatenate([coo.col.astype(np.int64), c])
    vv = np.concatenate([coo.data, v])
    order = np.lexsort((cc, rr))
    rr, cc, vv = rr[order], cc[order], vv[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rr + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.csr_matrix((vv, cc, indptr), shape=(n, nc))


def truncate_interior(P, interior, tau):
    """Optional sparsification (not in the paper): on interior rows drop the
    entries with |p_ij| < tau * max_j |p_ij|; exterior rows (R^T) are kept."""
    if tau <= 0.0:
        return P
    P = sp.csr_matrix(P, copy=True)
    rowmax = np.asarray(abs(P).max(axis=1).todense()).ravel()
    rows = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr))
    isint = np.zeros(P.shape[0], dtype=bool)
    isint[np.asarray(interior, dtype=np.int64)] = True
    keep = ~isint[rows] | (np.abs(P.data) >= tau * rowmax[rows])
    indptr = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=P.shape[0]))])
    return sp.csr_matrix((P.data[keep], P.indices[keep], indptr), shape=P.shape)


def galerkin(A, P):
    """A_c = P^T (A P), keeping every structural nonzero."""
    AP = structural_product(A, P)
    return structural_product(sp.csr_matrix(P.T), AP)


# ----------------------------------------------------------------------------
# smoother: multiplicative Schwarz over node stars + l1-Jacobi
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Smoother:
    blocks: list            # ascending DoF arrays (one per node star)
    color: np.ndarray       # colour of each block
    ncolors: int
    chol: list              # lower Cholesky factor of A_BB for each block (fp64)
    l1: np.ndarray          # sum_j |a_ij|


def smoother_setup(A, G, extra_blocks=None):
    """Node-star blocks supp(G[:, v]) for every column v, greedy colouring in
    block order of the conflict graph (two blocks conflict if they share a DoF
    or a DoF of one is coupled in A to a DoF of the other), Cholesky factors of
    the diagonal blocks and the l1 diagonal.  extra_blocks (the alternative
    reading "stars+interior") are appended after the stars: the interior
    blocks of the level's splitting, the decoupled fine-variable blocks that
    a compatible-relaxation smoother relaxes."""
    A = sp.csr_matrix(A)
    Gc = sp.csc_matrix(G)
    n = A.shape[0]
    blocks = []
    for v in range(Gc.shape[1]):
        rows = np.sort(Gc.indices[Gc.indptr[v]:Gc.indptr[v + 1]]).astype(np.int64)
        if len(rows):
            blocks.append(rows)
    for b in extra_blocks or []:
        if len(b):
            blocks.append(np.sort(np.asarray(b, dtype=np.int64)))
    nb = len(blocks)
    if nb:
        Bm = sp.csr_matrix((np.ones(sum(len(b) for b in blocks)),
                            (np.repeat(np.arange(nb), [len(b) for b in blocks]),
                             np.concatenate(blocks))), shape=(nb, n))
        Conf = (Bm @ (_ones(A) + sp.identity(n, format="csr")) @ Bm.T).tocsr()
    color = np.full(nb, -1, dtype=np.int64)
    for b in range(nb):
        taken = set(int(color[c]) for c in _rows_of(Conf, b) if c < b)
        c = 0
        while c in taken:
            c += 1
        color[b] = c
    chol = [np.linalg.cholesky(A[blk][:, blk].toarray()) for blk in blocks]
    l1 = np.asarray(abs(A).sum(axis=1)).ravel()
    return Smoother(blocks, color, int(color.max()) + 1 if nb else 0, chol, l1)


def _block_solve(L, r):
    """Solve (L L^T) y = r for a stack of factors L (nb, s, s) and r (nb, s)."""
    s = L.shape[1]
    y = np.zeros_like(r)
    for a in range(s):
        y[:, a] = (r[:, a] - np.einsum("bk,bk->b", L[:, a, :a], y[:, :a])) / L[:, a, a]
    x = np.zeros_like(r)
    for a in range(s - 1, -1, -1):
        x[:, a] = (y[:, a] - np.einsum("bk,bk->b", L[:, a + 1:, a], x[:, a + 1:])) / L[:, a, a]
    return x


# ----------------------------------------------------------------------------
# hierarchy
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    G: sp.csr_matrix
    Gt: sp.csr_matrix = None
    B: np.ndarray = None
    S: sp.csr_matrix = None
    cf: np.ndarray = None          # node states of the C/F splitting
    cG: np.ndarray = None
    rr: RRows = None
    interior: np.ndarray = None
    blocks: list = None
    depths: np.ndarray = None
    exact_blocks: bool = None
    patches: list = None           # per-column supports of the patch extension
    P: sp.csr_matrix = None
    Gc_cols: np.ndarray = None
    smoother: Smoother = None
    # per-block stacks grouped by colour, built lazily
    _groups: dict = None


@dataclasses.dataclass
class Hierarchy:
    levels: list
    coarse_chol: np.ndarray
    opts: dict

    @property
    def nlevels(self):
        return len(self.levels)

    def oc(self):
        return sum(l.A.nnz for l in self.levels) / self.levels[0].A.nnz

    def gc(self):
        return sum(l.A.shape[0] for l in self.levels) / self.levels[0].A.shape[0]


DEFAULTS = dict(interp="alg", max_levels=20, min_coarse=32, ext_block_max=64,
                ref_select=None, stall_ratio=0.9, p_trunc=0.0, schwarz="adjoint", user=None,
                ext_mode="blocks", patch_hops=2, patch_cap=128, smoother_blocks="stars")


def setup(A, G, **opts):
    """Build the multilevel hierarchy (Sections 3-5).

    Level l: G~ = augmentG(G_l); nodal graph; c_G by nodalCF (or, in the
    refinement-based mode, given by opts['ref_select'](l, level) returning
    (coarse real nodes, coarse artificial nodes)); R and S_I by Algorithm 3;
    P by local harmonic extension; A_{l+1} = P^T A_l P; G_{l+1} = R G_l I_C.
    Coarsening stops at max_levels, when n <= min_coarse, when R is empty or
    when n_{l+1} > stall_ratio * n_l.  p_trunc > 0 drops small interior
    entries of P (an option outside the paper, off by default).  The coarsest level is solved by a dense
    Cholesky factorisation."""
    o = dict(DEFAULTS)
    o.update(opts)
    A = sp.csr_matrix(A)
    A.sort_indices()
    G = sp.csr_matrix(G)
    levels = [Level(A=A, G=G)]
    S_prev = None
    fine_of = None
    user = o["user"]
    while True:
        lv = levels[-1]
        n = lv.A.shape[0]
        lv.smoother = smoother_setup(lv.A, lv.G)
        if user is not None:
            # caller-given interpolation (the geometric "Geo" comparison of
            # Section 5): P_l and G_{l+1} per level, Galerkin coarse operators
            Ps, Gs = user
            lvl = len(levels) - 1
            if lvl >= len(Ps) or len(levels) >= o["max_levels"]:
                break
            lv.P = sp.csr_matrix(Ps[lvl])
            lv.P.sort_indices()
            levels.append(Level(A=galerkin(lv.A, lv.P), G=sp.csr_matrix(Gs[lvl + 1])))
            continue
        if len(levels) >= o["max_levels"] or n <= o["min_coarse"]:
            break
        lv.Gt, lv.B = augment_g(lv.G)
        if len(levels) == 1:
            lv.S = nodal_graph(lv.A, lv.Gt)
        else:
            lv.S = coarse_nodal_graph(S_prev, fine_of)
        lvl = len(levels) - 1
        if o["interp"] == "ref" and o["ref_select"] is not None:
            sel = o["ref_select"](lvl, lv)
        else:
            sel = None
        if sel is not None:
            cG, Bc = (np.asarray(x, dtype=np.int64) for x in sel)
            lv.cG = np.sort(cG)
            Cp = np.concatenate([lv.cG, Bc])
        else:
            lv.cG, lv.cf = nodal_cf(lv.S, lv.B)
            Cp = np.concatenate([lv.cG, lv.B])
        lv.rr, lv.interior = form_r(lv.Gt, Cp, lv.B, n, skip_bb=sel is None)
        nc = len(lv.rr)
        if nc == 0 or nc > o["stall_ratio"] * n:
            lv.rr = None
            break
        Rt = r_transpose(lv.rr, n)
        sources = np.concatenate([Cp, lv.rr.k])
        lv.blocks, lv.depths, lv.exact_blocks = extension_blocks(
            lv.A, lv.Gt, lv.interior, sources, o["ext_block_max"])
        if o["ext_mode"] == "patch":
            lv.patches = patch_sets(lv.A, Rt, lv.interior, o["patch_hops"], o["patch_cap"])
            lv.P = interpolation_patch(lv.A, Rt, lv.patches)
        else:
            lv.P = interpolation(lv.A, Rt, lv.blocks, lv.depths)
        if o["smoother_blocks"] == "stars+interior":
            lv.smoother = smoother_setup(lv.A, lv.G, extra_blocks=lv.blocks)
        lv.P = truncate_interior(lv.P, lv.interior, o["p_trunc"])
        Ac = galerkin(lv.A, lv.P)
        Gc, cols = coarse_gradient(lv.G, lv.rr)
        lv.Gc_cols = cols
        # fine counterparts of the next level's nodes: real nodes are the kept
        # columns; artificial nodes (one per single-entry row of G_c, in row
        # order) stand for the boundary node of that row's path
        m_real = lv.G.shape[1]
        single = np.nonzero(np.diff(Gc.indptr) == 1)[0]
        b_end = np.where(lv.rr.i >= m_real, lv.rr.i, lv.rr.j)
        fine_of = np.concatenate([cols, b_end[single]])
        S_prev = lv.S
        levels.append(Level(A=Ac, G=Gc))
    Ad = levels[-1].A.toarray()
    coarse_chol = np.linalg.cholesky(Ad)
    return Hierarchy(levels, coarse_chol, o)


# ----------------------------------------------------------------------------
# solve phase
# ----------------------------------------------------------------------------
def _cast(H, dtype):
    key = np.dtype(dtype).name
    cache = H.opts.setdefault("_cast", {})
    if key in cache:
        return cache[key]
    out = []
    for lv in H.levels:
        sm = lv.smoother
        groups = []
        for c in range(sm.ncolors):
            ids = [b for b in range(len(sm.blocks)) if sm.color[b] == c]
            by_size = {}
            for b in ids:
                by_size.setdefault(len(sm.blocks[b]), []).append(b)
            g = []
            for s, bl in sorted(by_size.items()):
                dofs = np.stack([sm.blocks[b] for b in bl])
                L = np.stack([sm.chol[b] for b in bl]).astype(dtype)
                g.append((dofs, L))
            groups.append(g)
        out.append(dict(A=lv.A.astype(dtype), P=None if lv.P is None else lv.P.astype(dtype),
                        PT=None if lv.P is None else sp.csr_matrix(lv.P.T).astype(dtype),
                        l1=sm.l1.astype(dtype), groups=groups))
    cache[key] = out
    return out


def _schwarz(M, x, b, colors):
    for c in colors:
        r = b - M["A"] @ x
        for dofs, L in M["groups"][c]:
            x[dofs] += _block_solve(L, r[dofs])
    return x


# Above this value of eps_32 * rho_l (gradient_ratio) a level of the FP32
# form keeps FP64: FP32 storage of A_l or of the iterate then perturbs the
# level's gradient near-kernel by more than 1e-3 of its own energy.
FP32_RHO_TOL = 1e-3


def gradient_ratio(A, G):
    """rho = max over nodes v of (|G|^T |A| |G|)_vv / (G^T A G)_vv.

    (G^T A G)_vv is the energy of the gradient of node v's hat function and
    the numerator the scale of the entries it is summed from, so a relative
    perturbation eps of A's entries (or of a vector on the star of v) changes
    that energy by about eps * rho times itself.  On the finest level rho is
    about alpha / (beta h^2) (Section 2: A^s annihilates gradients, only
    beta A^m sees them)."""
    G = sp.csr_matrix(G)
    num = (abs(G).T @ abs(A) @ abs(G)).diagonal()
    den = (G.T @ A @ G).diagonal()
    ok = den > 0
    return float(np.max(num[ok] / den[ok])) if ok.any() else 1.0


def level_dtypes(H, dtype):
    """Value type of every level's V-cycle work.  FP64 everywhere for the FP64
    cycle; for the FP32 form each level runs in FP32 unless
    eps_32 * gradient_ratio exceeds FP32_RHO_TOL (then FP64).  The coarsest
    solve is FP64 in both."""
    if np.dtype(dtype) == np.float64:
        return [np.float64] * H.nlevels
    key = "_level_dtypes"
    if key not in H.opts:
        eps32 = float(np.finfo(np.float32).eps)
        H.opts[key] = [np.float64 if eps32 * gradient_ratio(lv.A, lv.G) > FP32_RHO_TOL else np.float32
                       for lv in H.levels]
    return H.opts[key]


def vcycle(H, b, dtype=np.float64, level=0):
    """One V(1,1) cycle with zero initial guess: returns x ~ A_l^{-1} b.

    Section 5 smooths with one pre- and one post-step of symmetrised
    multiplicative Schwarz followed by l1-Jacobi.  The order of the post step
    is H.opts['schwarz']:
      'adjoint' (default): pre = forward sweep (colours ascending), backward
          sweep (descending), l1-Jacobi; post = l1-Jacobi, forward, backward,
          the adjoint of pre, so the cycle is symmetric (for CG);
      'repeat': post = pre (forward, backward, l1-Jacobi);
      'split': pre = forward, l1-Jacobi; post = l1-Jacobi, backward.
    Coarse correction with P^T / P.  The coarsest level is solved exactly in
    FP64.  With dtype=float32 each level runs in the type level_dtypes
    gives it (FP32 unless its gradient near-kernel needs FP64); a vector
    crossing between levels of different types is converted."""
    mode = H.opts.get("schwarz", "adjoint")
    dts = level_dtypes(H, dtype)
    if level == H.nlevels - 1:
        L = H.coarse_chol
        y = np.linalg.solve(L, np.asarray(b, dtype=np.float64))
        return np.linalg.solve(L.T, y)
    dt = dts[level]
    M = _cast(H, dt)[level]
    b = np.asarray(b, dtype=dt)
    nc = H.levels[level].smoother.ncolors
    x = np.zeros_like(b)
    up, down = list(range(nc)), list(range(nc - 1, -1, -1))
    x = _schwarz(M, x, b, up)
    if mode != "split":
        x = _schwarz(M, x, b, down)
    x = x + (b - M["A"] @ x) / M["l1"]
    r = b - M["A"] @ x
    xc = vcycle(H, M["PT"] @ r, dtype, level + 1)
    x = x + M["P"] @ np.asarray(xc, dtype=dt)
    if mode == "repeat":
        x = _schwarz(M, x, b, up)
        x = _schwarz(M, x, b, down)
        return x + (b - M["A"] @ x) / M["l1"]
    x = x + (b - M["A"] @ x) / M["l1"]
    if mode != "split":
        x = _schwarz(M, x, b, up)
    x = _schwarz(M, x, b, down)
    return x


def pcg(H, A, f, x0=None, rtol=1e-8, maxit=500, dtype=np.float64, flexible=None):
    """Preconditioned CG (FP64) with one V-cycle as preconditioner; stops when
    ||f - A x_k|| <= rtol ||f - A x_0|| (R14: the test is on the residual of
    the system).  CG updates its residual recursively; when that one meets
    the tolerance, f - A x_k is formed, and if it does not meet it CG goes on
    from it with a fresh direction (rounding makes the two drift apart over
    long runs), until it does or a restart no longer halves it (the
    attainable accuracy of FP64 on the system).  With an FP32 V-cycle the
    Polak-Ribiere (flexible) beta is used.  Returns (x, iterations,
    residual-norm history)."""
    A = sp.csr_matrix(A)
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    if flexible is None:
        flexible = np.dtype(dtype) != np.float64
    r = f - A @ x
    r0 = np.linalg.norm(r)
    hist = [r0]
    if r0 == 0.0:
        return x, 0, hist
    z = vcycle(H, r, dtype).astype(np.float64)
    p = z.copy()
    rz = r @ z
    it = 0
    restarts, t_last = 0, 0.0
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        nr = np.linalg.norm(r)
        hist.append(nr)
        if nr <= rtol * r0:
            r = f - A @ x
            t = np.linalg.norm(r)
            if t <= rtol * r0 or it >= maxit or (restarts > 0 and t > 0.5 * t_last):
                break
            restarts, t_last = restarts + 1, t
            z = vcycle(H, r, dtype).astype(np.float64)
            rz = r @ z
            p = z.copy()
            continue
        z = vcycle(H, r, dtype).astype(np.float64)
        rz_new = r @ z
        beta = ((r - r_old) @ z) / rz if flexible else rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, it, hist


def amg_solve(H, A, f, x0=None, rtol=1e-8, maxit=400, dtype=np.float64):
    """Stand-alone AMG iteration x <- x + V(f - A x) (Section 5)."""
    A = sp.csr_matrix(A)
    x = np.zeros(A.shape[0]) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - A @ x
    r0 = np.linalg.norm(r)
    hist = [r0]
    it = 0
    while it < maxit and hist[-1] > rtol * r0:
        x += vcycle(H, r, dtype).astype(np.float64)
        r = f - A @ x
        hist.append(np.linalg.norm(r))
        it += 1
    return x, it, hist

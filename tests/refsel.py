"""Refinement-based coarse node selection for structured meshes (test helper).

The refinement-based interpolation of Section 3 takes its coarse nodes from
the geometric hierarchy.  This helper tracks the coordinates of every node of
every level (real nodes are kept coarse nodes; an artificial node of level l
stands for the eliminated boundary node of its edge) and marks as coarse the
nodes lying on the lattice of spacing 2^(l+1) h.
"""
import numpy as np


class RefSelector:
    def __init__(self, problem):
        mesh = problem.mesh
        self.h = mesh.h
        self.real0 = mesh.coords[problem.keep_nodes]
        # eliminated endpoint of every surviving edge with one surviving node
        edges = mesh.edges[problem.keep_edges]
        kept = problem.keep_nodes
        self.edge_bnd = np.where(~kept[edges[:, 0]], edges[:, 0], edges[:, 1])
        self.all_coords = mesh.coords
        self.prev = None
        self.coords = None

    def _level_coords(self, lvl, lv):
        if lvl == 0:
            real = self.real0
            single = np.nonzero(np.diff(lv.G.indptr) == 1)[0]
            art = self.all_coords[self.edge_bnd[single]]
            return np.concatenate([real, art])
        plv, pc = self.prev
        m_real = plv.G.shape[1]
        real = pc[plv.Gc_cols]
        single = np.nonzero(np.diff(lv.G.indptr) == 1)[0]
        b_end = np.where(plv.rr.i >= m_real, plv.rr.i, plv.rr.j)
        art = pc[b_end[single]]
        return np.concatenate([real, art])

    def __call__(self, lvl, lv):
        c = self._level_coords(lvl, lv)
        self.prev = (lv, c)
        s = self.h * 2 ** (lvl + 1)
        q = c / s
        on = np.all(np.abs(q - np.round(q)) < 1e-9, axis=1)
        m_real = lv.G.shape[1]
        ids = np.nonzero(on)[0]
        return ids[ids < m_real], ids[ids >= m_real]

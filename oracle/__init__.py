"""CPU oracle for the H(curl) AMG method -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 (plus an FP32-V-cycle mode) NumPy/SciPy implementation
of the paper's algebraic multigrid method, written to be checked against the
paper by eye.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  The GPU library never calls it, shares no
code with it, and must fail loudly when its own compiled extension is missing.

Parity pins: every function is checked in tests/ against values the paper
prints (the structural operator/grid complexities of Tables 1-2), closed
forms, invariants and brute force.  Parts without a pin from the paper are
marked "parity unpinned" in their docstrings: the 3D extension order of the
local harmonic extension (depth-ordered blocks), the FP32 V-cycle mode and
the learned-setup surrogate.
"""
from .amg import (augment_g, nodal_graph, coarse_nodal_graph, rs_first_pass,
                  nodal_cf, edge_graph, form_r, coarse_gradient, extension_blocks,
                  interpolation, galerkin, smoother_setup, Level, Hierarchy,
                  setup, vcycle, pcg, amg_solve, structural_product)

__all__ = ["augment_g", "nodal_graph", "coarse_nodal_graph", "rs_first_pass",
           "nodal_cf", "edge_graph", "form_r", "coarse_gradient",
           "extension_blocks", "interpolation", "galerkin", "smoother_setup",
           "Level", "Hierarchy", "setup", "vcycle", "pcg", "amg_solve",
           "structural_product"]

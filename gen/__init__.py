"""Seeded synthetic inputs for the H(curl) AMG solver.

This package builds the linear systems the method is applied to: meshes of the
unit square/cube, lowest-order Nedelec (edge element) discretisations of the
shifted curl-curl problem curl(alpha curl u) + beta u = f with Dirichlet
condition u x n = 0 (Section 2 of the paper), the discrete gradient G, and
seeded coefficient fields and right-hand sides.

It holds none of the multigrid method's arithmetic: both the CPU oracle and the
GPU library take its arrays as plain inputs.
"""
from .mesh import (hex_mesh, simplex_mesh_2d, kuhn_tet_mesh, assemble, Problem,
                   make_problem)
from .fields import subdomain_log_uniform, stripes_2d, checkerboard, rhs_uniform
from .geo import geo_interpolation_tri, geo_interpolation_hex, geo_hierarchy

__all__ = ["hex_mesh", "simplex_mesh_2d", "kuhn_tet_mesh", "assemble", "Problem",
           "make_problem", "subdomain_log_uniform", "stripes_2d", "checkerboard",
           "rhs_uniform", "geo_interpolation_tri", "geo_interpolation_hex", "geo_hierarchy"]

"""ctypes binding of libhcurlamg.so (argument marshalling only).

Every computation happens inside the compiled library: the host integer
setup in C++ and every floating-point step in HIP kernels.  There is no
Python or CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhcurlamg.so")

AMG_OK = 0
AMG_NOT_CONVERGED = 1
AMG_INTERP_ALG = 0
AMG_INTERP_REF = 1
AMG_INTERP_USER = 2
AMG_EXT_BLOCKS = 0
AMG_EXT_PATCH = 1
SCHWARZ_MODES = {"adjoint": 0, "repeat": 1, "split": 2}

STATUS = {0: "AMG_OK", 1: "AMG_NOT_CONVERGED", -1: "AMG_ERR_ARG", -2: "AMG_ERR_SHAPE",
          -3: "AMG_ERR_CSR", -4: "AMG_ERR_G_NOT_INCIDENCE", -5: "AMG_ERR_NOT_SPD",
          -6: "AMG_ERR_COARSEN", -7: "AMG_ERR_HIP", -8: "AMG_ERR_OOM", -9: "AMG_ERR_LIMIT",
          -10: "AMG_ERR_NOT_FINITE"}

EXPORTED = ["amg_default_options", "amg_setup", "amg_resetup_numeric", "amg_vcycle",
            "amg_pcg_solve", "amg_smoother_sweep", "amg_spmv", "amg_hier_info", "amg_export_integers",
            "amg_export_level", "amg_level0_integers", "amg_free_integers", "amg_destroy",
            "amg_last_error", "amg_mlp_nparams", "amg_mlp_train", "amg_mlp_use", "amg_mlp_stats_get",
            "amg_mlp_params", "amg_mlp_forward", "amg_mlp_backward", "amg_mlp_loss_grad", "amg_check",
            "amg_cycle_solve", "amg_complexity", "amg_spmv_dot", "amg_spmv_dot_noalloc"]


class AmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class amg_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("val", C.c_void_p),
                ("on_device", C.c_int)]


class amg_options(C.Structure):
    _fields_ = [("interp", C.c_int), ("max_levels", C.c_int), ("min_coarse", C.c_int64),
                ("vcycle_prec", C.c_int), ("ext_block_max", C.c_int), ("stall_ratio", C.c_double),
                ("p_trunc", C.c_double),
                ("ref_nlevels", C.c_int),
                ("ref_coarse_nodes", C.POINTER(C.POINTER(C.c_int32))),
                ("ref_ncoarse", C.POINTER(C.c_int64)),
                ("ref_coarse_bnd", C.POINTER(C.POINTER(C.c_int32))),
                ("ref_nbnd", C.POINTER(C.c_int64)),
                ("schwarz_mode", C.c_int), ("seed", C.c_uint64),
                ("user_nlevels", C.c_int), ("user_P", C.POINTER(amg_csr)),
                ("user_G", C.POINTER(amg_csr)), ("fp32_rho_tol", C.c_double),
                ("ext_mode", C.c_int), ("patch_hops", C.c_int), ("patch_cap", C.c_int),
                ("borrow_a", C.c_int)]


class amg_solve_stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("relres", C.c_double), ("true_relres", C.c_double),
                ("seconds", C.c_double), ("history", C.POINTER(C.c_double)),
                ("replacements", C.c_int), ("floor_relres", C.c_double),
                ("conv_factor", C.c_double)]


class amg_level_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("p_nnz", C.c_int64),
                ("nblocks", C.c_int64), ("ncolors", C.c_int), ("exact_blocks", C.c_int),
                ("star_rows", C.c_int64), ("star_row_nnz", C.c_int64), ("fac_entries", C.c_int64),
                ("sweep_form", C.c_int), ("sweep_lanes", C.c_int), ("prec", C.c_int),
                ("grad_ratio", C.c_double), ("sweep_pairs", C.c_int)]


class amg_int_export(C.Structure):
    _fields_ = [("n", C.c_int64), ("m_real", C.c_int64), ("n_art", C.c_int64),
                ("cf", C.POINTER(C.c_int8)),
                ("n_cg", C.c_int64), ("cg", C.POINTER(C.c_int32)),
                ("nc", C.c_int64),
                ("r_dof1", C.POINTER(C.c_int32)), ("r_dof2", C.POINTER(C.c_int32)),
                ("r_i", C.POINTER(C.c_int32)), ("r_j", C.POINTER(C.c_int32)),
                ("r_k", C.POINTER(C.c_int32)),
                ("r_s1", C.POINTER(C.c_int8)), ("r_s2", C.POINTER(C.c_int8)),
                ("n_interior", C.c_int64), ("interior", C.POINTER(C.c_int32)),
                ("nblocks", C.c_int64), ("block_ptr", C.POINTER(C.c_int64)),
                ("block_dofs", C.POINTER(C.c_int32)), ("block_key_depth", C.POINTER(C.c_int64)),
                ("exact_blocks", C.c_int),
                ("nstars", C.c_int64), ("star_ptr", C.POINTER(C.c_int64)),
                ("star_dofs", C.POINTER(C.c_int32)), ("star_color", C.POINTER(C.c_int32)),
                ("ncolors", C.c_int),
                ("gc_nrows", C.c_int64), ("gc_ncols", C.c_int64),
                ("gc_ptr", C.POINTER(C.c_int64)), ("gc_col", C.POINTER(C.c_int32)),
                ("gc_val", C.POINTER(C.c_int8)), ("gc_cols", C.POINTER(C.c_int32)),
                ("npatch_entries", C.c_int64), ("patch_ptr", C.POINTER(C.c_int64)),
                ("patch_dofs", C.POINTER(C.c_int32))]


class amg_mlp_train_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("seed", C.c_uint64),
                ("eligible_max", C.c_double), ("init", C.POINTER(C.c_float)),
                ("global_iters", C.c_int)]


class amg_mlp_use_cfg(C.Structure):
    _fields_ = [("refine_steps", C.c_int), ("accept_tol", C.c_double), ("global_iters", C.c_int),
                ("global_slack", C.c_double)]


class amg_mlp_stats(C.Structure):
    _fields_ = [("blocks", C.c_int64), ("eligible", C.c_int64), ("accepted", C.c_int64),
                ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("train_seconds", C.c_double), ("infer_seconds", C.c_double),
                ("exact_seconds", C.c_double), ("rho_reference", C.c_double),
                ("rho_learned", C.c_double), ("global_fallback", C.c_int)]


_lib = None


def load():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} not found: build it with __graft_entry__.build() "
                          "(python paper_2602_23613_amd/build.py)")
    lib = C.CDLL(LIBPATH)
    P = C.c_void_p
    lib.amg_default_options.argtypes = [C.POINTER(amg_options)]
    lib.amg_default_options.restype = None
    lib.amg_setup.argtypes = [C.POINTER(amg_csr), C.POINTER(amg_csr), C.POINTER(amg_options), P,
                              C.POINTER(P)]
    lib.amg_resetup_numeric.argtypes = [P, C.POINTER(amg_csr), P]
    lib.amg_vcycle.argtypes = [P, P, P, P]
    lib.amg_pcg_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.POINTER(amg_solve_stats), P]
    lib.amg_cycle_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.POINTER(amg_solve_stats), P]
    lib.amg_complexity.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.amg_spmv.argtypes = [C.POINTER(amg_csr), P, P, P]
    lib.amg_spmv_dot.argtypes = [C.POINTER(amg_csr), P, P, P, P]
    lib.amg_spmv_dot_noalloc.argtypes = [C.POINTER(amg_csr), P, P, P, P]
    lib.amg_smoother_sweep.argtypes = [P, C.c_int, C.c_int, P, P, C.c_int, P]
    lib.amg_check.argtypes = [P, P]
    lib.amg_hier_info.argtypes = [P, C.POINTER(amg_level_info), C.c_int, C.POINTER(C.c_int)]
    lib.amg_export_integers.argtypes = [P, C.c_int, C.POINTER(amg_int_export)]
    lib.amg_export_level.argtypes = [P, C.c_int, P, P, P, P, P, P]
    lib.amg_level0_integers.argtypes = [C.POINTER(amg_csr), C.POINTER(amg_csr),
                                        C.POINTER(amg_options), C.POINTER(amg_int_export),
                                        C.POINTER(P)]
    lib.amg_free_integers.argtypes = [P]
    lib.amg_free_integers.restype = None
    lib.amg_destroy.argtypes = [P]
    lib.amg_destroy.restype = None
    lib.amg_last_error.restype = C.c_char_p
    lib.amg_mlp_nparams.restype = C.c_int64
    lib.amg_mlp_nparams.argtypes = []
    lib.amg_mlp_train.argtypes = [P, C.POINTER(amg_mlp_train_cfg), C.POINTER(amg_mlp_stats), P]
    lib.amg_mlp_use.argtypes = [P, C.POINTER(amg_mlp_use_cfg)]
    lib.amg_mlp_stats_get.argtypes = [P, C.POINTER(amg_mlp_stats)]
    lib.amg_mlp_params.argtypes = [P, P, P]
    lib.amg_mlp_forward.argtypes = [P, P, C.c_int64, P, P]
    lib.amg_mlp_backward.argtypes = [P, P, C.c_int64, P, P, P]
    lib.amg_mlp_loss_grad.argtypes = [P, P, P, C.c_int64, C.c_int64, P, P, P]
    for name in ("amg_setup", "amg_resetup_numeric", "amg_vcycle", "amg_pcg_solve", "amg_spmv",
                 "amg_spmv_dot", "amg_spmv_dot_noalloc",
                 "amg_cycle_solve", "amg_complexity",
                 "amg_smoother_sweep", "amg_check",
                 "amg_hier_info", "amg_export_integers", "amg_export_level",
                 "amg_level0_integers", "amg_mlp_train", "amg_mlp_use", "amg_mlp_stats_get",
                 "amg_mlp_params", "amg_mlp_forward", "amg_mlp_backward", "amg_mlp_loss_grad"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def check(status):
    if status < 0:
        raise AmgError(status, load().amg_last_error().decode())
    return status


def _ptr(a):
    """Address of a numpy array or a torch tensor."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _is_dev(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def make_csr(rowptr, colidx, val, nrows, ncols):
    """amg_csr over numpy arrays (host) or torch tensors (device).  The
    arrays must stay alive while the struct is in use."""
    dev = _is_dev(rowptr)
    return amg_csr(nrows, ncols, int(colidx.shape[0]), _ptr(rowptr), _ptr(colidx), _ptr(val),
                   1 if dev else 0)


def host_csr(M):
    """(rowptr int64, colidx int32, val float64) numpy arrays of a scipy CSR matrix."""
    return (np.ascontiguousarray(M.indptr, dtype=np.int64),
            np.ascontiguousarray(M.indices, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


def default_options():
    o = amg_options()
    load().amg_default_options(C.byref(o))
    return o


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(int(n),)).astype(dtype, copy=True)


def export_to_dict(e: amg_int_export):
    nb, ns = e.nblocks, e.nstars
    d = dict(n=e.n, m_real=e.m_real, n_art=e.n_art,
             cf=_arr(e.cf, e.m_real + e.n_art, np.int8) if e.cf else None,
             cg=_arr(e.cg, e.n_cg, np.int64), nc=e.nc,
             r_dof1=_arr(e.r_dof1, e.nc, np.int64), r_dof2=_arr(e.r_dof2, e.nc, np.int64),
             r_i=_arr(e.r_i, e.nc, np.int64), r_j=_arr(e.r_j, e.nc, np.int64),
             r_k=_arr(e.r_k, e.nc, np.int64), r_s1=_arr(e.r_s1, e.nc, np.int64),
             r_s2=_arr(e.r_s2, e.nc, np.int64),
             interior=_arr(e.interior, e.n_interior, np.int64),
             block_ptr=_arr(e.block_ptr, nb + 1, np.int64) if nb else np.zeros(1, np.int64),
             exact_blocks=bool(e.exact_blocks),
             star_ptr=_arr(e.star_ptr, ns + 1, np.int64) if ns else np.zeros(1, np.int64),
             ncolors=e.ncolors, gc_nrows=e.gc_nrows, gc_ncols=e.gc_ncols)
    d["block_dofs"] = _arr(e.block_dofs, d["block_ptr"][-1], np.int64)
    d["block_depth"] = _arr(e.block_key_depth, nb, np.int64)
    d["star_dofs"] = _arr(e.star_dofs, d["star_ptr"][-1], np.int64)
    d["star_color"] = _arr(e.star_color, ns, np.int64)
    d["gc_ptr"] = _arr(e.gc_ptr, e.gc_nrows + 1, np.int64)
    d["gc_col"] = _arr(e.gc_col, d["gc_ptr"][-1] if e.gc_nrows else 0, np.int64)
    d["gc_val"] = _arr(e.gc_val, d["gc_ptr"][-1] if e.gc_nrows else 0, np.int64)
    d["gc_cols"] = _arr(e.gc_cols, e.gc_ncols, np.int64)
    if e.patch_ptr:
        d["patch_ptr"] = _arr(e.patch_ptr, e.nc + 1, np.int64)
        d["patch_dofs"] = _arr(e.patch_dofs, e.npatch_entries, np.int64)
    return d

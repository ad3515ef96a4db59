"""MI355X-native H(curl) algebraic multigrid (arXiv 2602.23613).

Python front end of libhcurlamg.so: argument marshalling only.  Inputs are
scipy CSR matrices (host) or torch CUDA tensors (device); vectors passed to
the solve phase are torch CUDA tensors of float64.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import AmgError, load  # noqa: F401

# amg_level_info.sweep_form values
SWEEP_FORMS = {0: "colour", 1: "one", 2: "pipe", 3: "dense", 4: "panel"}

__all__ = ["Hierarchy", "level0_integers", "spmv", "spmv_dot", "mlp_loss_grad", "load", "AmgError"]


def _stream(stream):
    if stream is not None:
        return stream
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _check_csr_arrays(rp, ci, va, nrows, name="A"):
    """What the C ABI assumes of a CSR triple it gets as raw pointers: row
    pointers int64 with nrows + 1 entries, column ids int32, values float64
    with as many entries as column ids, all contiguous, and either all three
    host numpy arrays or all three CUDA tensors on one device.  A library
    that borrows A keeps reading these arrays, so a wrong type or length
    would make its kernels read past them."""
    if all(isinstance(a, np.ndarray) for a in (rp, ci, va)):
        kinds = [(a.dtype, a.flags.c_contiguous, a.size) for a in (rp, ci, va)]
        want = (np.dtype(np.int64), np.dtype(np.int32), np.dtype(np.float64))
    else:
        import torch
        if not all(isinstance(a, torch.Tensor) and a.is_cuda for a in (rp, ci, va)):
            raise TypeError(f"{name}: rowptr, colidx and val must be all numpy arrays or all CUDA tensors")
        if len({a.device for a in (rp, ci, va)}) != 1:
            raise ValueError(f"{name}: rowptr, colidx and val are on different devices")
        kinds = [(a.dtype, a.is_contiguous(), a.numel()) for a in (rp, ci, va)]
        want = (torch.int64, torch.int32, torch.float64)
    for (dt, contig, _), w, part in zip(kinds, want, ("rowptr", "colidx", "val")):
        if dt != w:
            raise TypeError(f"{name}.{part} must be {w}, got {dt}")
        if not contig:
            raise ValueError(f"{name}.{part} must be contiguous")
    if kinds[0][2] != nrows + 1:
        raise ValueError(f"{name}.rowptr has {kinds[0][2]} entries, expected nrows + 1 = {nrows + 1}")
    if kinds[1][2] != kinds[2][2]:
        raise ValueError(f"{name}: colidx has {kinds[1][2]} entries and val {kinds[2][2]}")


def _csr_arg(M, keep):
    """amg_csr for a scipy matrix (host) or a (rowptr, colidx, val, nrows, ncols) tuple of tensors."""
    if isinstance(M, tuple):
        rp, ci, va, nr, nc = M
        _check_csr_arrays(rp, ci, va, nr)
        keep.extend([rp, ci, va])
        return _lib.make_csr(rp, ci, va, nr, nc)
    rp, ci, va = _lib.host_csr(M)
    keep.extend([rp, ci, va])
    return _lib.make_csr(rp, ci, va, M.shape[0], M.shape[1])


def _options(keep, interp="alg", max_levels=20, min_coarse=32, vcycle_prec=64, ext_block_max=64,
             stall_ratio=0.9, p_trunc=0.0, ref=None, schwarz="adjoint", seed=None, user=None,
             fp32_rho_tol=None, ext_mode="blocks", patch_hops=2, patch_cap=128, borrow_a=False):
    o = _lib.default_options()
    o.ext_mode = {"blocks": _lib.AMG_EXT_BLOCKS, "patch": _lib.AMG_EXT_PATCH}[ext_mode]
    o.patch_hops = patch_hops
    o.patch_cap = patch_cap
    o.borrow_a = 1 if borrow_a else 0
    o.interp = {"alg": _lib.AMG_INTERP_ALG, "ref": _lib.AMG_INTERP_REF,
                "user": _lib.AMG_INTERP_USER}[interp]
    o.max_levels = max_levels
    o.min_coarse = min_coarse
    o.vcycle_prec = vcycle_prec
    o.ext_block_max = ext_block_max
    o.stall_ratio = stall_ratio
    o.p_trunc = p_trunc
    o.schwarz_mode = _lib.SCHWARZ_MODES[schwarz]
    if seed is not None:
        o.seed = seed
    if fp32_rho_tol is not None:
        o.fp32_rho_tol = fp32_rho_tol
    if user:
        # user: (list of P_l, list of G_l with G_0 unused) as scipy CSR matrices
        Ps, Gs = user
        nl = len(Ps)
        pa = (_lib.amg_csr * nl)(*[_csr_arg(P, keep) for P in Ps])
        ga = (_lib.amg_csr * (nl + 1))(*[_csr_arg(G, keep) if G is not None else _lib.amg_csr()
                                         for G in Gs[:nl + 1]])
        keep.extend([pa, ga])
        o.user_nlevels = nl
        o.user_P = C.cast(pa, C.POINTER(_lib.amg_csr))
        o.user_G = C.cast(ga, C.POINTER(_lib.amg_csr))
    if ref:
        # ref: list of (coarse real nodes, coarse artificial nodes) per level
        nl = len(ref)
        cn = [np.ascontiguousarray(r[0], dtype=np.int32) for r in ref]
        cb = [np.ascontiguousarray(r[1], dtype=np.int32) for r in ref]
        keep.extend(cn + cb)
        P32 = C.POINTER(C.c_int32)
        arr_n = (P32 * nl)(*[a.ctypes.data_as(P32) for a in cn])
        arr_b = (P32 * nl)(*[a.ctypes.data_as(P32) for a in cb])
        cnt_n = (C.c_int64 * nl)(*[len(a) for a in cn])
        cnt_b = (C.c_int64 * nl)(*[len(a) for a in cb])
        keep.extend([arr_n, arr_b, cnt_n, cnt_b])
        o.ref_nlevels = nl
        o.ref_coarse_nodes = C.cast(arr_n, C.POINTER(P32))
        o.ref_coarse_bnd = C.cast(arr_b, C.POINTER(P32))
        o.ref_ncoarse = C.cast(cnt_n, C.POINTER(C.c_int64))
        o.ref_nbnd = C.cast(cnt_b, C.POINTER(C.c_int64))
    return o


def _vec(t, n, name, dtype="float64"):
    """Pointer of a device vector after checking what the kernels assume: a
    CUDA tensor of the given dtype, contiguous, with exactly n entries."""
    import torch
    want = torch.float64 if dtype == "float64" else torch.float32
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != want:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, the level has {n}")
    return t.data_ptr()


class Hierarchy:
    """AMG hierarchy owned by the library (amg_setup / amg_destroy)."""

    def __init__(self, A, G, stream=None, **opts):
        lib = load()
        keep = []
        a = _csr_arg(A, keep)
        g = _csr_arg(G, keep)
        o = _options(keep, **opts)
        h = C.c_void_p()
        _lib.check(lib.amg_setup(C.byref(a), C.byref(g), C.byref(o), _stream(stream), C.byref(h)))
        self._h = h
        self.prec = opts.get("vcycle_prec", 64)
        self.n = A[3] if isinstance(A, tuple) else A.shape[0]
        # borrow_a with device tensors: the library reads them in place, so
        # the hierarchy holds them until a re-setup borrows another A
        self._borrow = bool(opts.get("borrow_a")) and isinstance(A, tuple)
        self._a_ref = A if self._borrow else None
        # level sizes never change after setup (a numeric re-setup keeps them)
        self._sizes = [li["n"] for li in self.info()]

    def close(self):
        if getattr(self, "_h", None):
            load().amg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def resetup(self, A, stream=None):
        keep = []
        a = _csr_arg(A, keep)
        _lib.check(load().amg_resetup_numeric(self._h, C.byref(a), _stream(stream)))
        if self._borrow:
            self._a_ref = A

    def vcycle(self, r, z, stream=None):
        """z = B r (device float64 tensors), asynchronous on the stream."""
        _lib.check(load().amg_vcycle(self._h, _vec(r, self.n, "r"), _vec(z, self.n, "z"),
                                     _stream(stream)))

    def _solve(self, fn, f, u, rtol, maxit, history, stream):
        st = _lib.amg_solve_stats()
        hist = None
        if history:
            hist = np.zeros(maxit + 1)
            st.history = hist.ctypes.data_as(C.POINTER(C.c_double))
        status = _lib.check(fn(self._h, _vec(f, self.n, "f"), _vec(u, self.n, "u"), rtol, maxit,
                               C.byref(st), _stream(stream)))
        out = dict(status=status, converged=status == _lib.AMG_OK, iterations=st.iterations,
                   relres=st.relres, true_relres=st.true_relres, seconds=st.seconds,
                   replacements=st.replacements, floor_relres=st.floor_relres,
                   conv_factor=st.conv_factor)
        if history:
            out["history"] = hist[:st.iterations + 1].copy()
        return out

    def pcg(self, f, u, rtol=1e-8, maxit=500, history=False, stream=None):
        """amg_pcg_solve: status AMG_OK only if the true residual meets rtol."""
        return self._solve(load().amg_pcg_solve, f, u, rtol, maxit, history, stream)

    def cycle_solve(self, f, u, rtol=1e-8, maxit=400, history=False, stream=None):
        """amg_cycle_solve: the stand-alone iteration u <- u + B (f - A u)."""
        return self._solve(load().amg_cycle_solve, f, u, rtol, maxit, history, stream)

    def complexity(self):
        """(operator complexity, grid complexity) of the hierarchy."""
        oc, gc = C.c_double(), C.c_double()
        _lib.check(load().amg_complexity(self._h, C.byref(oc), C.byref(gc)))
        return oc.value, gc.value

    def info(self):
        cap = 32
        arr = (_lib.amg_level_info * cap)()
        nl = C.c_int()
        _lib.check(load().amg_hier_info(self._h, arr, cap, C.byref(nl)))
        return [dict(n=x.n, nnz=x.nnz, p_nnz=x.p_nnz, nblocks=x.nblocks, ncolors=x.ncolors,
                     exact_blocks=bool(x.exact_blocks), star_rows=x.star_rows,
                     star_row_nnz=x.star_row_nnz, fac_entries=x.fac_entries,
                     sweep_form=SWEEP_FORMS[x.sweep_form], sweep_lanes=x.sweep_lanes,
                     prec=x.prec, grad_ratio=x.grad_ratio, sweep_pairs=x.sweep_pairs)
                for x in arr[:nl.value]]

    def sweep(self, level, b, x, backward=False, stream=None):
        """One multiplicative Schwarz sweep on `level` (x updated in place)."""
        import torch
        prec = 32 if b.dtype == torch.float32 else 64
        if not 0 <= level < len(self._sizes) - 1:
            raise ValueError("level has no smoother")
        n, dt = self._sizes[level], "float32" if prec == 32 else "float64"
        _lib.check(load().amg_smoother_sweep(self._h, level, prec, _vec(b, n, "b", dt),
                                             _vec(x, n, "x", dt), 1 if backward else 0,
                                             _stream(stream)))

    def check(self, stream=None):
        """Synchronize and raise if a pipelined smoother sweep gave up a wait."""
        _lib.check(load().amg_check(self._h, _stream(stream)))

    # --- learned setup ---------------------------------------------------
    def mlp_train(self, epochs=4, batch=1024, lr=1e-3, seed=0, eligible_max=50.0, init=None,
                  global_iters=0, stream=None):
        """Train the surrogate on the exact finest-level local solves of the
        current A.  init: initial parameters (float32 array) or None to continue."""
        cfg = _lib.amg_mlp_train_cfg(epochs, batch, lr, seed, eligible_max, None, global_iters)
        keep = None
        if init is not None:
            keep = np.ascontiguousarray(init, dtype=np.float32)
            cfg.init = keep.ctypes.data_as(C.POINTER(C.c_float))
        st = _lib.amg_mlp_stats()
        _lib.check(load().amg_mlp_train(self._h, C.byref(cfg), C.byref(st), _stream(stream)))
        return _stats_dict(st)

    def mlp_use(self, refine_steps=3, accept_tol=1e-10, global_iters=0, global_slack=0.02,
                enable=True):
        if not enable:
            _lib.check(load().amg_mlp_use(self._h, None))
            return
        cfg = _lib.amg_mlp_use_cfg(refine_steps, accept_tol, global_iters, global_slack)
        _lib.check(load().amg_mlp_use(self._h, C.byref(cfg)))

    def mlp_stats(self):
        st = _lib.amg_mlp_stats()
        _lib.check(load().amg_mlp_stats_get(self._h, C.byref(st)))
        return _stats_dict(st)

    def mlp_params(self, set=None):
        n = load().amg_mlp_nparams()
        if set is not None:
            arr = np.ascontiguousarray(set, dtype=np.float32)
            assert arr.size == n
            _lib.check(load().amg_mlp_params(self._h, None, arr.ctypes.data))
            return None
        out = np.zeros(n, dtype=np.float32)
        _lib.check(load().amg_mlp_params(self._h, out.ctypes.data, None))
        return out

    def mlp_forward(self, x_bf16, y, stream=None):
        n = x_bf16.shape[0]
        _lib.check(load().amg_mlp_forward(self._h, x_bf16.data_ptr(), n, y.data_ptr(), _stream(stream)))

    def mlp_backward(self, x_bf16, dy, grad, stream=None):
        n = x_bf16.shape[0]
        _lib.check(load().amg_mlp_backward(self._h, x_bf16.data_ptr(), n, dy.data_ptr(),
                                           grad.data_ptr(), _stream(stream)))

    def integers(self, level):
        e = _lib.amg_int_export()
        _lib.check(load().amg_export_integers(self._h, level, C.byref(e)))
        return _lib.export_to_dict(e)

    def level(self, level):
        """(A_l, P_l) as scipy CSR matrices copied from the device (P_l None on the coarsest)."""
        import scipy.sparse as sp
        info = self.info()
        li = info[level]
        n, nnz, pnnz = li["n"], li["nnz"], li["p_nnz"]
        ap = np.zeros(n + 1, np.int64)
        ac = np.zeros(max(nnz, 1), np.int32)
        av = np.zeros(max(nnz, 1), np.float64)
        coarsest = level == len(info) - 1
        pp = np.zeros(n + 1, np.int64)
        pc = np.zeros(max(pnnz, 1), np.int32)
        pv = np.zeros(max(pnnz, 1), np.float64)
        _lib.check(load().amg_export_level(self._h, level, ap.ctypes.data, ac.ctypes.data,
                                           av.ctypes.data, pp.ctypes.data, pc.ctypes.data,
                                           pv.ctypes.data))
        A = sp.csr_matrix((av[:nnz], ac[:nnz], ap), shape=(n, n))
        P = None
        if not coarsest:
            P = sp.csr_matrix((pv[:pnnz], pc[:pnnz], pp), shape=(n, info[level + 1]["n"]))
        return A, P


def _stats_dict(st):
    return {k: getattr(st, k) for k, _ in st._fields_}


def mlp_loss_grad(y, t, ahat, nvalid, dy, row_loss, stream=None):
    """Learned-form training loss ||Ahat (W - W*)||_F^2 per row and its gradient
    (device tensors: y, t, dy float32 (n, 64); ahat float64 (n, 36); row_loss (n,))."""
    n = y.shape[0]
    _lib.check(load().amg_mlp_loss_grad(y.data_ptr(), t.data_ptr(), ahat.data_ptr(), n, nvalid,
                                        dy.data_ptr(), row_loss.data_ptr(), _stream(stream)))


def level0_integers(A, G, **opts):
    """Host-only integer setup of the finest level (same code as amg_setup's)."""
    lib = load()
    keep = []
    a = _csr_arg(A, keep)
    g = _csr_arg(G, keep)
    o = _options(keep, **opts)
    e = _lib.amg_int_export()
    h = C.c_void_p()
    _lib.check(lib.amg_level0_integers(C.byref(a), C.byref(g), C.byref(o), C.byref(e), C.byref(h)))
    try:
        return _lib.export_to_dict(e)
    finally:
        lib.amg_free_integers(h)


def spmv(rowptr, colidx, val, x, y, stream=None):
    """y = A x with the library's CSR kernel (all device tensors)."""
    n = rowptr.shape[0] - 1
    _check_csr_arrays(rowptr, colidx, val, n)
    _vec(x, x.numel(), "x")
    _vec(y, n, "y")
    a = _lib.make_csr(rowptr, colidx, val, n, x.shape[0])
    _lib.check(load().amg_spmv(C.byref(a), x.data_ptr(), y.data_ptr(), _stream(stream)))


def spmv_dot(rowptr, colidx, val, x, y, dot, stream=None, noalloc=False):
    """y = A x and dot[0] = x^T y (device tensors; dot a float64 tensor of one
    entry).  noalloc=False: amg_spmv_dot (synchronizes the stream);
    noalloc=True: amg_spmv_dot_noalloc (static scratch, asynchronous)."""
    n = rowptr.shape[0] - 1
    _check_csr_arrays(rowptr, colidx, val, n)
    _vec(x, n, "x")
    _vec(y, n, "y")
    _vec(dot, 1, "dot")
    a = _lib.make_csr(rowptr, colidx, val, n, n)
    fn = load().amg_spmv_dot_noalloc if noalloc else load().amg_spmv_dot
    _lib.check(fn(C.byref(a), x.data_ptr(), y.data_ptr(), dot.data_ptr(), _stream(stream)))

/*
 * amg.h -- C ABI of the MI355X H(curl) algebraic multigrid library.
 *
 * The library solves A u = f for the lowest-order Nedelec discretisation of
 * curl(alpha curl u) + beta u = f with u x n = 0 (Section 2 of
 * arXiv 2602.23613, "Nodal Coarsening and Sparse Ideal Interpolation for
 * H(curl) Problems in Algebraic Multigrid").  Inputs are the sparse SPD
 * matrix A (Section 1, eq. (axb)) and the discrete gradient G from nodes to
 * edges (Section 2, eq. (deRham)).  The preconditioner is the paper's
 * algebraic multigrid hierarchy:
 *   - augmentG (Algorithm 1), nodal coarsening of the dual operator
 *     G~^T A G~ (Algorithm 2), coarse edge variables from length-two paths
 *     (Algorithm 3) and the coarse gradient G_c = R G I_C (eq. (Gc));
 *   - the sparse ideal interpolation P_app = (I - S_I A_II^{-1} S_I^T A) R^T
 *     (eq. (sparseP)) built by batched local harmonic extension on the GPU;
 *   - Galerkin coarse operators A_c = P^T A P (Section 1) by GPU SpGEMM;
 *   - V(1,1) cycles with the symmetrised multiplicative Schwarz + l1-Jacobi
 *     smoother (Section 5), used as a preconditioner for CG.
 *
 * Conventions
 *   - Every function returns amg_status; 0 (AMG_OK) is success.  On a
 *     negative status the caller's buffers are left untouched and
 *     amg_last_error() returns a message naming the level and the cause.
 *   - CSR inputs are borrowed for the duration of the call only (except a
 *     device A under amg_options.borrow_a): column
 *     indices sorted and unique within each row, int64 row pointers, int32
 *     column indices, FP64 values.  `on_device` = 1 means the three arrays
 *     are HIP device pointers, 0 means host pointers.
 *   - Vectors passed to amg_vcycle / amg_pcg_solve are caller-owned HIP
 *     device buffers (e.g. torch tensors' data_ptr()).
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  All
 *     device work of a call is enqueued in order on that stream.
 *     amg_vcycle returns without synchronising; amg_setup,
 *     amg_resetup_numeric and amg_pcg_solve synchronise before returning.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef HCURL_AMG_H
#define HCURL_AMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMG_OK = 0,
  AMG_NOT_CONVERGED = 1,       /* PCG hit maxit; u and stats hold the last iterate */
  AMG_ERR_ARG = -1,            /* NULL pointer, bad option value */
  AMG_ERR_SHAPE = -2,          /* inconsistent sizes (A not square, G rows != n, ...) */
  AMG_ERR_CSR = -3,            /* row pointers not monotone, column out of range, unsorted or duplicate */
  AMG_ERR_G_NOT_INCIDENCE = -4,/* a row of G is not {}, {+-1} or {+1, -1} */
  AMG_ERR_NOT_SPD = -5,        /* non-positive pivot in a block or coarse Cholesky factorisation */
  AMG_ERR_COARSEN = -6,        /* the first coarsening step produced no coarse variables */
  AMG_ERR_HIP = -7,            /* a HIP runtime call failed (message holds the HIP error string) */
  AMG_ERR_OOM = -8,            /* device allocation failed */
  AMG_ERR_LIMIT = -9,          /* a block or row exceeds a kernel's size limit (message names it) */
  AMG_ERR_NOT_FINITE = -10     /* NaN or Inf in the right-hand side */
} amg_status;

enum { AMG_INTERP_ALG = 0, AMG_INTERP_REF = 1, AMG_INTERP_USER = 2 };

/* Order of the smoothing steps in the V(1,1) cycle.  Section 5 uses one pre-
   and one post-smoothing step of "symmetrised multiplicative Schwarz
   followed by l1-Jacobi" (OSS-l1); it does not say how the post step is
   ordered.
     AMG_SCHWARZ_ADJOINT (default): pre = forward sweep, backward sweep,
       l1-Jacobi; post = l1-Jacobi, forward sweep, backward sweep -- the
       adjoint of the pre step, so that the cycle is a symmetric
       preconditioner for CG;
     AMG_SCHWARZ_REPEAT: post = pre (forward, backward, l1-Jacobi twice);
       the literal reading, not symmetric;
     AMG_SCHWARZ_SPLIT: pre = forward sweep, l1-Jacobi; post = l1-Jacobi,
       backward sweep (half the sweeps; symmetric). */
enum { AMG_SCHWARZ_ADJOINT = 0, AMG_SCHWARZ_REPEAT = 1, AMG_SCHWARZ_SPLIT = 2 };

/* Compressed sparse row view (borrowed). */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t *rowptr;   /* nrows + 1 */
  const int32_t *colidx;   /* nnz */
  const double *val;       /* nnz */
  int on_device;           /* 0: host pointers, 1: HIP device pointers */
} amg_csr;

/* Setup options; amg_default_options() fills the paper's values (Section 5). */
typedef struct {
  int interp;              /* AMG_INTERP_ALG (Algorithms 1-3) or AMG_INTERP_REF */
  int max_levels;          /* 20: maximum number of levels (Section 5) */
  int64_t min_coarse;      /* 32: stop coarsening at or below this many DoFs (Section 5) */
  int vcycle_prec;         /* 64: FP64 V-cycle; 32: FP32 V-cycle (FP64 coarsest solve) */
  int ext_block_max;       /* 64: largest connected component of graph(A_II) solved as one exact block */
  double stall_ratio;      /* 0.9: stop when n_{l+1} > stall_ratio * n_l */
  double p_trunc;          /* 0: the paper's P.  > 0: after the local solves, drop interior-row
                              entries of P below p_trunc * (row max |p|) (an option outside the
                              paper that bounds the growth of the coarse operators) */
  /* AMG_INTERP_REF only: for levels 0 .. ref_nlevels-1 the coarse nodes come
     from the geometric refinement instead of Algorithm 2.  Per level l:
     ref_coarse_nodes[l] (ref_ncoarse[l] entries) lists coarse real nodes
     (columns of G_l); ref_coarse_bnd[l] (ref_nbnd[l] entries) lists the coarse
     artificial nodes, as ids in augmentG's numbering (columns m_l, m_l+1, ...
     of G~_l).  Host pointers, read during amg_setup only. */
  int ref_nlevels;
  const int32_t *const *ref_coarse_nodes;
  const int64_t *ref_ncoarse;
  const int32_t *const *ref_coarse_bnd;
  const int64_t *ref_nbnd;
  int schwarz_mode;        /* AMG_SCHWARZ_ADJOINT (default), AMG_SCHWARZ_REPEAT or AMG_SCHWARZ_SPLIT */
  uint64_t seed;           /* seed of the counter-based start vector of the measured convergence
                              factor (the learned setup's global check); nothing else is random */
  /* AMG_INTERP_USER only: the caller gives the interpolation of every level
     (for example the geometric Nedelec interpolation "Geo" of Section 5,
     the paper's comparison method) instead of Algorithms 1-3 and
     eq. (sparseP).  user_nlevels transfer operators: user_P[l] is
     n_l x n_{l+1} and user_G[l + 1] the discrete gradient of level l + 1
     (n_{l+1} rows; it defines that level's node-star smoother blocks);
     user_G[0] is ignored (G is the argument of amg_setup).  Coarse
     operators are the Galerkin products A_{l+1} = P_l^T A_l P_l.  Host or
     device CSR views, read during amg_setup only. */
  int user_nlevels;
  const amg_csr *user_P;
  const amg_csr *user_G;
  /* vcycle_prec = 32 only: a level runs in FP32 unless eps_32 * rho_l exceeds
     this tolerance (default 1e-3), where rho_l = max over node stars B of
     sum |A_BB| / (s^T A_BB s), s = the signs of the star's column of G_l.
     The gradient of a hat function is the near-kernel of the curl-curl
     operator (A^s G = 0, Section 2); rounding A_l or a vector to FP32
     perturbs that gradient's energy by about eps_32 * rho_l times itself,
     so such a level keeps FP64 matrices, smoother and vectors.  A huge
     value runs every level in FP32. */
  double fp32_rho_tol;
  /* How the interior rows of P are formed (eq. (sparseP) localised):
     AMG_EXT_BLOCKS (default): blocks of A_II, solved one block at a time (the
     connected components when all have at most ext_block_max DoFs, as in the
     paper's 2D setting; otherwise owner groups in depth order).
     AMG_EXT_PATCH: each column c of P is R^T e_c plus its least-energy
     extension into a patch S_c of interior DoFs, A_SS x = -A_S,ext (R^T e_c),
     the patch grown from the column's two exterior DoFs over patch_hops
     rounds of A-couplings (most couplings first, ties to the smaller id), at
     most patch_cap DoFs (1..192).  Overlapping patches reach across the
     3D interior blocks that the block form decouples; with block-diagonal
     A_II and enough hops it equals the block form. */
  int ext_mode;
  int patch_hops;          /* default 2 */
  int patch_cap;           /* default 128 */
  /* 0 (default): the hierarchy keeps its own device copy of A.  1, with a
     device A (on_device = 1): the hierarchy reads the caller's rowptr, colidx
     and val in place and copies nothing; the caller keeps them allocated and
     unchanged until amg_destroy, or until an amg_resetup_numeric whose A (also
     on the device, same pattern) is then borrowed in its place.  A host A is
     copied whatever this says. */
  int borrow_a;
} amg_options;

enum { AMG_EXT_BLOCKS = 0, AMG_EXT_PATCH = 1 };

typedef struct amg_hier amg_hier;   /* opaque; owns all device memory of the hierarchy */

typedef struct {
  int iterations;          /* CG iterations performed */
  double relres;           /* final ||f - A u|| / ||f - A u0|| (recursive residual) */
  double true_relres;      /* final true residual recomputed with one extra SpMV */
  double seconds;          /* wall time of the solve on the host clock */
  double *history;         /* optional caller buffer (maxit + 1 doubles) of residual norms, or NULL */
  int replacements;        /* times CG continued from the true residual (see amg_pcg_solve) */
  double floor_relres;     /* 64 eps || |A| |u| || / ||f - A u0||: the rounding level of an FP64
                              residual at the final iterate; a true_relres near it cannot be
                              reduced further in FP64 */
  double conv_factor;      /* amg_pcg_solve: (relres)^(1/iterations); amg_cycle_solve: ratio of
                              the last two residual norms (Section 5's "AMG conv") */
} amg_solve_stats;

typedef struct {
  int64_t n, nnz;          /* DoFs and stored entries of A_l */
  int64_t p_nnz;           /* stored entries of P_l (0 on the coarsest level) */
  int64_t nblocks;         /* smoother blocks (node stars) */
  int ncolors;             /* colours of the multiplicative Schwarz sweep */
  int exact_blocks;        /* 1 if P_l used exact component blocks of A_II */
  int64_t star_rows;       /* sum of block sizes: rows visited by one Schwarz sweep */
  int64_t star_row_nnz;    /* stored entries of A_l in those rows (with repetition) */
  int64_t fac_entries;     /* packed lower-triangular factor entries of all blocks */
  int sweep_form;          /* how a sweep runs: 0 one launch per colour, 1 one workgroup,
                              2 colours pipelined in one launch, 3 dense residual-update form
                              in one workgroup, 4 panel residual-update form (wide levels) */
  int sweep_lanes;         /* lanes per row of the row forms (0 for the dense and panel forms) */
  int prec;                /* 64 or 32: value type of this level's V-cycle work */
  double grad_ratio;       /* rho_l of fp32_rho_tol (computed on every level but the coarsest) */
  int sweep_pairs;         /* pipelined form: (column, value) pairs per lane loaded before a
                              chunk waits for the colour before it (0 for the other forms) */
} amg_level_info;

/* Integer results of one level's setup, for bit-exact comparison.  All
   arrays are host memory owned by the handle (valid until amg_destroy). */
typedef struct {
  int64_t n, m_real, n_art;                 /* DoFs, columns of G_l, artificial nodes of G~_l */
  const int8_t *cf;                         /* m_real + n_art node states (1 = C, 2 = F), NULL in REF levels */
  int64_t n_cg; const int32_t *cg;          /* coarse real nodes c_G (ascending) */
  int64_t nc;                               /* coarse DoFs = rows of R */
  const int32_t *r_dof1, *r_dof2, *r_i, *r_j, *r_k;
  const int8_t *r_s1, *r_s2;
  int64_t n_interior; const int32_t *interior;
  int64_t nblocks; const int64_t *block_ptr; const int32_t *block_dofs; const int64_t *block_key_depth;
  int exact_blocks;
  int64_t nstars; const int64_t *star_ptr; const int32_t *star_dofs; const int32_t *star_color;
  int ncolors;
  int64_t gc_nrows, gc_ncols; const int64_t *gc_ptr; const int32_t *gc_col; const int8_t *gc_val;
  const int32_t *gc_cols;                   /* level-l node id of each column of G_{l+1} */
  /* AMG_EXT_PATCH levels (else 0 / NULL): interior support of every column
     of P_l, patch_ptr[nc] + 1 offsets into patch_dofs (ascending per column) */
  int64_t npatch_entries; const int64_t *patch_ptr; const int32_t *patch_dofs;
} amg_int_export;

/* Fill *opt with the paper's defaults (Section 5). */
void amg_default_options(amg_options *opt);

/* Build the hierarchy for A (n x n, SPD) and G (n x m discrete gradient)
   (Sections 3-4): per level, augmentG (Algorithm 1), the nodal C/F
   splitting (Algorithm 2), the matching of length-two paths and R, S_I
   (Algorithm 3), G_c = R G I_C (eq. (Gc)), P by local harmonic extension
   (eq. (sparseP): block solves of A_II, or per-column patch solves with
   ext_mode AMG_EXT_PATCH), A_c = P^T A P (Section 1), and the
   node-star Schwarz smoother with its l1 diagonal (Section 5); coarsening
   stops as in Section 5 (20 levels, 32 DoFs).  The integer phase runs on the
   host, every floating-point step on the GPU.  A and G are borrowed for the
   call; everything kept is copied (with borrow_a = 1, a device A is read in
   place for the life of the handle instead).  On success *out owns a new handle; on
   failure *out is NULL and nothing is left allocated. */
amg_status amg_setup(const amg_csr *A, const amg_csr *G, const amg_options *opt,
                     void *stream, amg_hier **out);

/* Recompute every floating-point part of the hierarchy (P, A_c, smoother
   factors, l1 diagonals, coarsest factor) for a new A with exactly the
   pattern of the one given to amg_setup (e.g. a new coefficient field on the
   same mesh); the integer setup is reused unchanged.  A handle set up with
   borrow_a = 1 borrows this A in place of the earlier one (it must be a
   device A: a host A returns AMG_ERR_ARG).  A different pattern returns
   AMG_ERR_CSR, a different size AMG_ERR_SHAPE, before anything changes. */
amg_status amg_resetup_numeric(amg_hier *h, const amg_csr *A, void *stream);

/* z = B r: one V(1,1) cycle with zero initial guess (Section 1, eq. (tl)
   applied recursively; smoothing as in Section 5 with the order of
   amg_options.schwarz_mode; exact dense solve on the coarsest level).  r and
   z are caller-owned device buffers of n doubles (the FP32 form converts at
   the boundary) and must not alias.  Asynchronous on `stream`; the cycle is
   captured once per (r, z) pair as a HIP graph and replayed. */
amg_status amg_vcycle(amg_hier *h, const double *r, double *z, void *stream);

/* Preconditioned CG on A u = f with one V-cycle as the preconditioner
   (Section 5: "PCG", relative residual tolerance 1e-8).  FP64 vectors,
   reductions and updates; the V-cycle in the handle's precision, with the
   flexible Polak-Ribiere beta for the FP32 form.  f, u: caller-owned device
   buffers of n doubles; u holds the initial guess on entry and the iterate
   on exit.  When the recursively updated residual meets
   ||r|| <= rtol ||f - A u0||, the true residual f - A u is formed; if it
   misses the tolerance (rounding makes the two drift apart on
   ill-conditioned systems), CG continues from it with a fresh direction
   until it meets the tolerance or a restart no longer halves it.
   Returns AMG_OK only if the final true residual meets the tolerance, and
   AMG_NOT_CONVERGED otherwise (maxit reached, or the true residual stuck
   near the FP64 rounding level stats->floor_relres); u and stats then hold
   the last iterate.  Synchronises. */
amg_status amg_pcg_solve(amg_hier *h, const double *f, double *u, double rtol, int maxit,
                         amg_solve_stats *stats, void *stream);

/* The stand-alone multigrid iteration u <- u + B (f - A u) (Section 5:
   "standalone AMG V-cycle iteration counts"), until
   ||f - A u|| <= rtol ||f - A u0|| (AMG_OK) or maxit cycles
   (AMG_NOT_CONVERGED).  Same buffers and statistics as amg_pcg_solve;
   stats->conv_factor is the ratio of the last two residual norms.
   Synchronises. */
amg_status amg_cycle_solve(amg_hier *h, const double *f, double *u, double rtol, int maxit,
                           amg_solve_stats *stats, void *stream);

/* Operator complexity sum_l nnz(A_l) / nnz(A_0) and grid complexity
   sum_l n_l / n_0 of the hierarchy (the OC of Section 5's tables).  Either
   pointer may be NULL. */
amg_status amg_complexity(const amg_hier *h, double *oc, double *gc);

/* One multiplicative Schwarz sweep of the smoother on level `level`
   (Section 5): for every colour in ascending order (backward = 0) or
   descending order (backward = 1), x_B += A_BB^{-1} (b - A x)_B for all
   node-star blocks B of that colour.  prec must be the level's precision
   (amg_level_info.prec): 64 = device doubles and FP64 factors, 32 = device
   floats and the FP32 copies.  Asynchronous;
   used for kernel tests and measurement.  A sweep whose colours run
   pipelined in one launch (levels with many colours) bounds each of its
   waits for the previous colour; a wait that gives up leaves x wrong and
   raises a flag that amg_check and amg_pcg_solve report. */
amg_status amg_smoother_sweep(amg_hier *h, int level, int prec, const void *b, void *x,
                              int backward, void *stream);

/* Synchronizes `stream` and reports whether any smoother sweep of this
   handle gave up a wait (AMG_ERR_HIP; the flag stays set for the handle's
   lifetime, and every result computed since is suspect).  AMG_OK otherwise. */
amg_status amg_check(amg_hier *h, void *stream);

/* y = A x with the CSR SpMV kernel of the solve phase (device CSR and
   vectors, FP64).  Used for measurement and kernel tests. */
amg_status amg_spmv(const amg_csr *A, const double *x, double *y, void *stream);

/* y = A x and *dot = x^T y in one pass: the SpMV with the dot product that
   each PCG iteration forms for its step length (q = A p and p^T q, Section 5),
   for callers that run their own Krylov loop.  A: square device CSR (FP64);
   x, y: device vectors of A->nrows entries (y is overwritten, x and y must not
   overlap); dot: one device double.  The dot product sums one partial per
   workgroup in a fixed order, so repeated calls give the same bits.  The call
   allocates a partial-sum buffer of one double per 256/lanes rows, runs on
   `stream` and synchronizes it before returning.  AMG_ERR_ARG / AMG_ERR_SHAPE
   for bad arguments (nothing launched), AMG_ERR_HIP / AMG_ERR_OOM from HIP. */
amg_status amg_spmv_dot(const amg_csr *A, const double *x, double *y, double *dot, void *stream);

/* amg_spmv_dot for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same kernels and the same bits, with the partial sums in a static
   2 MiB device array that the library holds on every device it runs on until
   the process ends.  Allocates nothing and does not synchronize: the results
   are ready when `stream` reaches them.  At most 262,144 partial sums, one per
   256/lanes rows (lanes 4, 8, 16, 32 or 64 from the mean row length), e.g.
   8.4M rows of 9-40 entries; larger A fails with AMG_ERR_LIMIT before any
   launch.  All calls on one device share that array: calls that overlap on
   one device (other streams, other threads) race and must be serialized by
   the caller.  Other errors as amg_spmv_dot. */
amg_status amg_spmv_dot_noalloc(const amg_csr *A, const double *x, double *y, double *dot,
                                void *stream);

/* Per-level sizes; writes min(cap, levels) entries and the level count. */
amg_status amg_hier_info(const amg_hier *h, amg_level_info *lv, int cap, int *nlevels);

/* Integer results of level `level` (0 .. nlevels-2). */
amg_status amg_export_integers(const amg_hier *h, int level, amg_int_export *out);

/* Copy level `level`'s matrices to caller host buffers: A_l (nnz values,
   rowptr, colidx) and, unless `level` is the coarsest, P_l.  Any pointer
   may be NULL to skip it.  Sizes come from amg_hier_info. */
amg_status amg_export_level(const amg_hier *h, int level,
                            int64_t *a_ptr, int32_t *a_col, double *a_val,
                            int64_t *p_ptr, int32_t *p_col, double *p_val);

/* Host-only integer setup of the finest level (no GPU needed): the same
   code path amg_setup runs for level 0.  *out is owned by *handle; release
   it with amg_free_integers. */
amg_status amg_level0_integers(const amg_csr *A, const amg_csr *G, const amg_options *opt,
                               amg_int_export *out, void **handle);
void amg_free_integers(void *handle);

/* ---------------------------------------------------------------------------
   Learned setup (an addition outside the paper).  A small network
   (64 -> 128 -> 128 -> 64, ReLU, BF16 weights with FP32 master copies and
   FP32 accumulation on MFMA) maps each finest-level extension block of at
   most 8 DoFs, normalised as D^{-1/2} A_BB D^{-1/2}, to that matrix's
   inverse, i.e. to the weights of the local harmonic extension
   X_B = -A_BB^{-1} A_B,: P (eq. (sparseP)).  It is trained on the exact local
   solves of the current hierarchy.  When enabled, amg_resetup_numeric
   predicts the eligible finest-level blocks, refines each prediction by
   Newton-Schulz steps in FP64 and accepts it only if
   ||Ahat W - I||_F <= accept_tol; every other block is solved exactly.  A
   global check then compares the stand-alone V-cycle convergence factor with
   the one measured on the exact hierarchy at training time and redoes the
   whole numeric setup exactly if it is worse by more than global_slack.
   --------------------------------------------------------------------------- */
typedef struct {
  int epochs;              /* passes over the eligible blocks */
  int batch;               /* rows per optimisation step (multiple of 16) */
  double lr;               /* Adam step size */
  uint64_t seed;           /* order of the samples */
  double eligible_max;     /* blocks whose normalised inverse has an entry above this are not learned */
  const float *init;       /* host array of amg_mlp_nparams() initial parameters, or NULL to
                              continue from the current ones (required on first use) */
  int global_iters;        /* stand-alone cycles used to measure the reference convergence factor */
} amg_mlp_train_cfg;

typedef struct {
  int refine_steps;        /* Newton-Schulz steps after each prediction */
  double accept_tol;       /* per-block bound on ||Ahat W - I||_F */
  int global_iters;        /* stand-alone cycles of the global check (0 = no global check) */
  double global_slack;     /* the learned hierarchy passes if rho <= rho_reference + slack */
} amg_mlp_use_cfg;

typedef struct {
  int64_t blocks, eligible, accepted;   /* finest-level extension blocks in the last learned setup */
  double loss_first, loss_last;         /* training MSE of the first and last epoch */
  double train_seconds;                 /* last amg_mlp_train */
  double infer_seconds;                 /* features + network + refinement + learned extension */
  double exact_seconds;                 /* finest-level extension with exact solves (last exact setup) */
  double rho_reference, rho_learned;    /* global check (stand-alone V-cycle convergence factors) */
  int global_fallback;                  /* 1 if the global check rejected the learned setup */
} amg_mlp_stats;

/* Number of network parameters (FP32, layout W1, b1, W2, b2, W3, b3 row-major). */
int64_t amg_mlp_nparams(void);

/* Train on the exact finest-level local solves of the hierarchy's current A
   (the blocks' exact inverses are the targets).  Synchronises. */
amg_status amg_mlp_train(amg_hier *h, const amg_mlp_train_cfg *cfg, amg_mlp_stats *stats,
                         void *stream);

/* Enable (cfg != NULL) or disable (cfg == NULL) the learned setup in later
   amg_resetup_numeric calls. */
amg_status amg_mlp_use(amg_hier *h, const amg_mlp_use_cfg *cfg);

/* Statistics of the last training and learned setup. */
amg_status amg_mlp_stats_get(const amg_hier *h, amg_mlp_stats *stats);

/* Read (get != NULL) and/or overwrite (set != NULL) the FP32 master
   parameters (host arrays of amg_mlp_nparams() floats). */
amg_status amg_mlp_params(amg_hier *h, float *get, const float *set);

/* Raw network passes for checking the kernels: x = n rows (n a multiple of
   16) of 64 BF16 features (device, raw 16-bit patterns); y = n x 64 FP32
   outputs (device).  amg_mlp_backward takes dy = dL/dy (device, n x 64) and
   writes the gradient of all parameters (device, amg_mlp_nparams() floats). */
amg_status amg_mlp_forward(amg_hier *h, const uint16_t *x, int64_t n, float *y, void *stream);
amg_status amg_mlp_backward(amg_hier *h, const uint16_t *x, int64_t n, const float *dy, float *grad,
                            void *stream);

/* Training loss of the learned form, for checking the kernel: for each of the
   n rows (device arrays) y = prediction, t = exact target (64 FP32 values,
   the first 36 being packed lower triangles of symmetric 8 x 8 matrices) and
   ahat = the normalised block (36 FP64 values, packed the same way),
   row_loss[r] = ||Ahat (W - W*)||_F^2 and dy[r] = its gradient with respect
   to y divided by nvalid; rows r >= nvalid (batch padding) get zeros.
   Asynchronous on the stream. */
amg_status amg_mlp_loss_grad(const float *y, const float *t, const double *ahat, int64_t n,
                             int64_t nvalid, float *dy, float *row_loss, void *stream);

/* Release a hierarchy and all its device memory.  NULL is ignored. */
void amg_destroy(amg_hier *h);

/* Message of the last failure on the calling thread ("" if none). */
const char *amg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HCURL_AMG_H */

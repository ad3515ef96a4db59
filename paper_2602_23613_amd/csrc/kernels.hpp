// Device data structures and kernel launchers of the H(curl) AMG solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hamg {

// Device CSR matrix (values of type T); lpr = lanes per row of the row kernels.
template <class T>
struct CsrDev {
  int64_t n = 0, m = 0, nnz = 0;
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const T* val = nullptr;
  int lpr = 8;
};

// Device pattern only.
struct CsrPat {
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
};

// Counters of the one-launch sweeps sit SYNC_STRIDE ints (128 bytes) apart,
// one cache line each.
constexpr int SYNC_STRIDE = 32;

// Smoother blocks sorted by colour and packed into chunks: the device side (a
// plain struct, passed to the kernels by value) ...
template <class T>
struct SmootherArgs {
  int ncolours = 0;
  const int32_t* colour_chunk = nullptr;  // chunk range of each colour (+ sentinel)
  const int32_t* chunk_colour = nullptr;  // colour of each chunk
  const int32_t* chunk_blk = nullptr;     // first block of each chunk (+ sentinel)
  const int64_t* sb_ptr = nullptr;        // rows of each block (colour order)
  const int32_t* sb_dofs = nullptr;
  const int64_t* fac_off = nullptr;       // packed lower factor offset of each block
  const T* fac = nullptr;                 // Cholesky factors (dense form)
  const T* binv = nullptr;                // symmetric inverses, packed like fac (row forms)
  const int32_t* row_blk = nullptr;       // block of each star row
  const int32_t* ck_row0 = nullptr;       // first star row of each chunk (+ sentinel)
  // per chunk, padded to WGS / LPR row slots: the row copy's entry range of
  // every slot (rpb + 1 offsets; slots past the chunk's rows are empty) and
  // every slot's {DoF, block start in the chunk, block size, factor offset
  // in the chunk}, so that a chunk reaches its rows' entries and blocks in
  // one dependent load
  const int64_t* ck_q = nullptr;
  const int4* ck_row = nullptr;
  const int64_t* ck_fac0 = nullptr;       // first factor entry of each chunk (+ sentinel)
  const int64_t* srow_ptr = nullptr;      // the smoother's copy of A's rows in star order
  const int32_t* scol = nullptr;
  const T* sval = nullptr;
  int* sync = nullptr;                    // pipelined sweep: ticket + per-colour counters (SYNC_STRIDE apart)
  int* err = nullptr;                     // pipelined sweep: set when a wait gave up
  int spin_max = 0;
};

// ... and the host side: launch shape and the dense-level form.
enum { SWEEP_COLOUR = 0, SWEEP_ONE = 1, SWEEP_PIPE = 2, SWEEP_DENSE = 3, SWEEP_PANEL = 4 };
constexpr int PANEL_GROUP_SLOTS = 64;
constexpr int PANEL_ROW_WIDTH = 16;   // largest block of the panel form; width of its inverse rows

// Panel form of a level: groups of consecutive blocks in colour order with at
// most PANEL_GROUP_SLOTS star rows ("slots") each; every per-group table is
// padded to PANEL_GROUP_SLOTS slots so that its address follows from the
// group index.
template <class T>
struct PanelDev {
  int n = 0, ngroups = 0;
  const int32_t* gdof = nullptr;   // per group slot: its DoF, -1 past the group's rows
  const int32_t* gsl = nullptr;    // per group slot: first slot of its block | (slot of the same DoF
                                   // in group g-1, + 1) << 8 | (in group g+1, + 1) << 16
  const int32_t* gblk = nullptr;   // per group block: first slot | size << 8 | first << 16 and
                                   // last << 24 block of its run of one colour; -1 past the blocks
  const int32_t* dgrp = nullptr;   // per DoF: the (at most two) groups holding it, -1 if none
  const int32_t* docc = nullptr;   // per DoF: its (at most two) slots g * 64 + t, ascending, -1 if none
  const T* gslc = nullptr;         // per group: A(D_g, D_g), 64 x 64, entry l * 64 + k = A(dof_k, dof_l)
  const T* gcf = nullptr;          // per group: A(D_g+1, D_g), entry k * 64 + kn = A(dof_{g+1,kn}, dof_{g,k})
  const T* gcb = nullptr;          // per group: A(D_g-1, D_g), the same layout
  const T* gbinv = nullptr;        // per group slot: its row of the block inverse, 16 wide
  const T* Acm = nullptr;          // A(i, j) at Acm[j n + i]
  T* dsl = nullptr;                // per sweep position: the published d of each slot
  int* sync = nullptr;             // per sweep position: flag, then tile counter (SYNC_STRIDE apart)
};

template <class T>
struct SmootherDev : SmootherArgs<T> {
  std::vector<int> colour_chunk_h;      // host copy of colour_chunk
  int mode = SWEEP_COLOUR;
  int wg = 256;                         // threads per chunk (rows per chunk = wg / lpr)
  int lpr = 8;
  int pipe_grid = 0;                    // workgroups of the pipelined sweep
  int pipe_u = 8;                       // (column, value) pairs per lane loaded before the wait
  // dense level (nnz = n^2, one block per colour): the sweep keeps r and x in
  // LDS and updates r from a column-major dense copy of A
  int n = 0;
  int nblocks = 0;
  int max_block = 0;
  const T* Acm = nullptr;
  T* rtmp = nullptr;                    // level-sized scratch for b - A x
  PanelDev<T> pn;                       // panel form (wide levels)
};

// scalar slots of the CG state vector
enum { SC_RZ = 0, SC_PQ = 1, SC_ALPHA = 2, SC_BETA = 3, SC_RR = 4, SC_RZNEW = 5, SC_ROLDZ = 6,
       SC_COUNT = 8 };

template <class T> void spmv(const CsrDev<T>& A, const T* x, T* y, hipStream_t st);
template <class T> void residual(const CsrDev<T>& A, const T* x, const T* b, T* r, hipStream_t st);
template <class T>
void jacobi(const CsrDev<T>& A, const T* x, const T* b, const T* dinv, T* xn, hipStream_t st);
template <class T> void spmv_add(const CsrDev<T>& A, const T* x, T* y, hipStream_t st);
void spmv_dot(const CsrDev<double>& A, const double* x, double* y, double* partial, hipStream_t st);
int64_t spmv_dot_partials(int lpr, int64_t n);

bool schwarz_shape_ok(int lpr, int wg);
template <class T>
void schwarz_colour(const SmootherDev<T>& S, int colour, const T* b, T* x, hipStream_t st);
template <class T>
void schwarz_sweep_small(const SmootherDev<T>& S, int backward, const T* b, T* x, hipStream_t st);
template <class T>
void schwarz_pipe(const SmootherDev<T>& S, int backward, const T* b, T* x, hipStream_t st);
void star_cols(int64_t nrows, const int32_t* sb_dofs, const int64_t* Aptr, const int32_t* Acol,
               const int64_t* srow_ptr, int32_t* scol, hipStream_t st);
void star_rows(int64_t nrows, const int32_t* sb_dofs, const int64_t* Aptr, const double* Aval,
               const int64_t* srow_ptr, double* sval, hipStream_t st);
bool panel_sweep_ok(int n, int max_block);
int panel_tiles(int n);
int panel_resident_per_cu(int prec);
template <class T>
void panel_sweep(const PanelDev<T>& D, int backward, T* r, T* x, int* err, int spin_max, hipStream_t st);
void panel_slices(int ngroups, int64_t n, const int32_t* gdof, const double* Acm, double* gslc,
                  double* gcf, double* gcb, hipStream_t st);

template <class T> bool dense_sweep_ok(int n, int max_block);
template <class T>
void dense_sweep(int n, int nblocks, int max_block, int backward, const int64_t* sb_ptr,
                 const int32_t* sb_dofs, const int64_t* fac_off, const T* fac, const T* Acm,
                 const T* r_in, T* x, hipStream_t st);
void csr_to_dense_cm(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                     double* D, hipStream_t st);

// one multiplicative Schwarz sweep (all colours) with the launch shape the level uses
template <class T>
void schwarz_sweep(const SmootherDev<T>& S, const CsrDev<T>& A, int backward, const T* b, T* x,
                   hipStream_t st) {
  switch (S.mode) {
    case SWEEP_DENSE:
      residual<T>(A, x, b, S.rtmp, st);
      dense_sweep<T>(S.n, S.nblocks, S.max_block, backward, S.sb_ptr, S.sb_dofs, S.fac_off, S.fac,
                     S.Acm, S.rtmp, x, st);
      return;
    case SWEEP_ONE:
      schwarz_sweep_small<T>(S, backward, b, x, st);
      return;
    case SWEEP_PIPE:
      schwarz_pipe<T>(S, backward, b, x, st);
      return;
    case SWEEP_PANEL:
      residual<T>(A, x, b, S.rtmp, st);
      panel_sweep<T>(S.pn, backward, S.rtmp, x, S.err, S.spin_max, st);
      return;
    default:
      for (int k = 0; k < S.ncolours; ++k)
        schwarz_colour<T>(S, backward ? S.ncolours - 1 - k : k, b, x, st);
  }
}
template <class T>
void dense_solve(int n, const double* L, const T* b, T* x, double* work, hipStream_t st);
void dense_factor(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, double* D,
                  int* flag, hipStream_t st);

template <class T> void fill(int64_t n, T v, T* x, hipStream_t st);
template <class A, class B> void cast(int64_t n, const A* a, B* b, hipStream_t st);

void cg_update(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
               double* r_old, double* partial, hipStream_t st);
void dot2(int64_t n, const double* a, const double* b, const double* c, double* partial,
          hipStream_t st);
void reduce(int64_t count, const double* partial, double* sc, int slot, int slot2, hipStream_t st);
void cg_scalar(double* sc, int mode, int flexible, hipStream_t st);
void cg_dir(int64_t n, const double* sc, const double* z, double* p, int first, hipStream_t st);
int red_grid();

// patch extension: one workgroup per column of P (patch of at most mmax DoFs)
size_t ext_patch_lds(int mmax);
// The padded per-chunk tables of SmootherArgs (ck_q, ck_row) from the
// smoother's star-order arrays: one thread per (chunk, row slot).
void chunk_tables(int64_t nchunks, int rpb, const int32_t* ck_row0, const int64_t* ck_fac0,
                  const int64_t* srow_ptr, const int32_t* sb_dofs, const int32_t* row_blk,
                  const int64_t* sb_ptr, const int64_t* fac_off, int64_t* ck_q, int4* ck_row,
                  hipStream_t st);

// P^T's pattern on the device (transpose.hip): row pointers tptr (nc + 1),
// column ids tcol (nnz) and perm[q] = position of P's entry q in P^T.
// Needs nnz and nc below 2^31; returns the first HIP error.
hipError_t transpose_pattern(int64_t n, int64_t nc, int64_t nnz, const int64_t* ptr,
                             const int32_t* col, int64_t* tptr, int32_t* tcol, int64_t* perm,
                             hipStream_t st);
void ext_patches(int64_t nc, const int64_t* pptr, const int32_t* pdofs, const int64_t* Pptr,
                 const int32_t* Pcol, const int32_t* rd1, const int32_t* rd2, const int8_t* rs1,
                 const int8_t* rs2, const CsrDev<double>& A, double* Pval, int mmax, int* flag,
                 hipStream_t st);
size_t ext_block_lds(int smax, int ctile);
int ext_block_tile(int smax);
void ext_blocks(int64_t b0, int64_t nb, const int64_t* bptr, const int32_t* bdofs,
                const int32_t* dof_stage, int stage, const CsrDev<double>& A,
                const int64_t* Pptr, const int32_t* Pcol, double* Pval, int smax, int cmax,
                int prow_max, int* flag, hipStream_t st, const double* Wl = nullptr,
                const int8_t* accepted = nullptr, const double* dsq = nullptr);
void hash_fill(int64_t n, uint64_t seed, double* x, hipStream_t st);
void axpy(int64_t n, double a, const double* x, double* y, hipStream_t st);
void sign_to_val(int64_t n, const int8_t* s, double* v, hipStream_t st);
void permute(int64_t n, const int64_t* perm, const double* a, double* b, hipStream_t st);

void mm_count(int64_t nrows, const CsrPat& X, const CsrPat& Y, int64_t* cnt, int* overflow,
              hipStream_t st);
void mm_fill(int64_t nrows, const CsrPat& X, const CsrPat& Y, const int64_t* Cptr, int32_t* Ccol,
             int* overflow, hipStream_t st);
void mm_vals(int64_t nrows, const CsrPat& X, const double* Xval, const CsrPat& Y,
             const double* Yval, const int64_t* Cptr, const int32_t* Ccol, double* Cval, int mmax,
             hipStream_t st);
int mm_hash_cap();
int mm_wide_at();
size_t mm_wide_lds(int64_t ncols);
void mm_count_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const CsrPat& Y, int64_t ncols,
                   int64_t* cnt, hipStream_t st);
void mm_fill_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const CsrPat& Y, int64_t ncols,
                  const int64_t* Cptr, int32_t* Ccol, hipStream_t st);
void mm_vals_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const double* Xval,
                  const CsrPat& Y, const double* Yval, int64_t ncols, const int64_t* Cptr,
                  const int32_t* Ccol, double* Cval, hipStream_t st);

void pad_inv(int64_t nrows, const int32_t* row_blk, const int32_t* row_slot, const int64_t* sb_ptr,
             const int64_t* fac_off, const double* binv, double* out, hipStream_t st);
void star_inv(int64_t nrows, const int32_t* row_blk, const int64_t* sb_ptr, const int64_t* fac_off,
              const double* fac, double* binv, hipStream_t st);
void star_chol(int64_t nb, const int64_t* sb_ptr, const int32_t* sb_dofs, const int64_t* fac_off,
               const CsrDev<double>& A, double* fac, int* flag, hipStream_t st);
void l1inv(const CsrDev<double>& A, double* dinv, hipStream_t st);
void spmv_abs(const CsrDev<double>& A, const double* x, double* y, hipStream_t st);
void star_rho(int64_t nb, const int64_t* sb_ptr, const int32_t* sb_dofs, const int8_t* ssign,
              const int64_t* srow_ptr, const int32_t* scol, const double* sval, double* rho,
              hipStream_t st);

}  // namespace hamg

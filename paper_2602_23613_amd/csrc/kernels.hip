// HIP kernels (gfx950) of the H(curl) AMG solver.
//
// Solve phase (memory-bound; CSR rows are streamed by groups of LPR lanes of
// a 64-wide wavefront, reduced with cross-lane shuffles):
//   k_spmv        y = A x and fused epilogues (residual, l1-Jacobi step,
//                 prolongation add, dot-product partials)
//   k_schwarz     one colour of the multiplicative Schwarz sweep over
//                 node-star blocks (residual rows -> LDS, block Cholesky
//                 solve, update); k_schwarz_pipe runs a whole sweep with
//                 the colours pipelined across workgroups
//   k_dense_solve coarsest-level FP64 Cholesky solve (one workgroup)
//   PCG helpers   deterministic two-stage reductions and vector updates
// Setup phase:
//   k_ext_block   local harmonic extension X_B = -A_BB^{-1} A_B,: P_done
//                 (one wavefront per block, LDS-resident dense block)
//   k_mm_*        sparse products by row merge (A P, then P^T (A P)): LDS
//                 hash symbolic pass, sorted column fill, deterministic
//                 numeric pass
//   k_star_chol   Cholesky factors of the smoother's diagonal blocks
//   k_l1inv, casts, dense coarsest factorisation
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

namespace hamg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <int LPR, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_down(v, off, LPR);
  return v;
}

// sum_q val[q] x[col[q]] over q = b + lane, b + lane + LPR, ... < e, in that
// order; the loads of four consecutive terms are issued before their sums so
// that several gathers are in flight per lane
template <int LPR, class T>
__device__ __forceinline__ T row_dot(int64_t b, int64_t e, int lane, const int32_t* __restrict__ col,
                                     const T* __restrict__ val, const T* __restrict__ x) {
  T s = 0;
  int64_t q = b + lane;
  for (; q + 3 * LPR < e; q += 4 * LPR) {
    const int32_t c0 = col[q], c1 = col[q + LPR], c2 = col[q + 2 * LPR], c3 = col[q + 3 * LPR];
    const T v0 = val[q], v1 = val[q + LPR], v2 = val[q + 2 * LPR], v3 = val[q + 3 * LPR];
    const T x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; q < e; q += LPR) s += val[q] * x[col[q]];
  return s;
}

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <class T> void fill(int64_t n, T v, T* x, hipStream_t st);

// ---------------------------------------------------------------------------
// SpMV family
// ---------------------------------------------------------------------------
enum { EPI_Y = 0, EPI_RES = 1, EPI_JAC = 2, EPI_ADD = 3, EPI_DOT = 4 };

template <class T, int LPR, int EPI>
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ x,
                                              const T* __restrict__ b, const T* __restrict__ dinv,
                                              T* __restrict__ y, double* __restrict__ partial) {
  constexpr int RPB = 256 / LPR;
  const int lane = threadIdx.x % LPR;
  const int grp = threadIdx.x / LPR;
  const int64_t row = (int64_t)blockIdx.x * RPB + grp;
  T s = 0;
  if (row < n) s = row_dot<LPR, T>(ptr[row], ptr[row + 1], lane, col, val, x);
  s = group_sum<LPR>(s);
  double d = 0.0;
  if (row < n && lane == 0) {
    if (EPI == EPI_Y) y[row] = s;
    if (EPI == EPI_RES) y[row] = b[row] - s;
    if (EPI == EPI_JAC) y[row] = x[row] + (b[row] - s) * dinv[row];
    if (EPI == EPI_ADD) y[row] += s;
    if (EPI == EPI_DOT) {
      y[row] = s;
      d = (double)s * (double)x[row];
    }
  }
  if (EPI == EPI_DOT) {
    __shared__ double red[RPB];
    if (lane == 0) red[grp] = d;
    __syncthreads();
    for (int w = RPB / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  }
}

template <class T, int EPI>
static void spmv_lpr(int lpr, hipStream_t st, int64_t n, const int64_t* ptr, const int32_t* col,
                     const T* val, const T* x, const T* b, const T* dinv, T* y, double* partial) {
  if (n <= 0) return;
#define LAUNCH_SPMV(L)                                                                        \
  {                                                                                           \
    int64_t grid = (n + (256 / L) - 1) / (256 / L);                                           \
    hipLaunchKernelGGL((k_spmv<T, L, EPI>), dim3((unsigned)grid), dim3(256), 0, st, n, ptr, col, \
                       val, x, b, dinv, y, partial);                                          \
  }
  switch (lpr) {
    case 4: LAUNCH_SPMV(4); break;
    case 8: LAUNCH_SPMV(8); break;
    case 16: LAUNCH_SPMV(16); break;
    case 32: LAUNCH_SPMV(32); break;
    default: LAUNCH_SPMV(64); break;
  }
#undef LAUNCH_SPMV
}

int64_t spmv_dot_partials(int lpr, int64_t n) {
  int64_t rpb = 256 / lpr;
  return (n + rpb - 1) / rpb;
}

template <class T>
void spmv(const CsrDev<T>& A, const T* x, T* y, hipStream_t st) {
  spmv_lpr<T, EPI_Y>(A.lpr, st, A.n, A.ptr, A.col, A.val, x, nullptr, nullptr, y, nullptr);
}
template <class T>
void residual(const CsrDev<T>& A, const T* x, const T* b, T* r, hipStream_t st) {
  spmv_lpr<T, EPI_RES>(A.lpr, st, A.n, A.ptr, A.col, A.val, x, b, nullptr, r, nullptr);
}
template <class T>
void jacobi(const CsrDev<T>& A, const T* x, const T* b, const T* dinv, T* xn, hipStream_t st) {
  spmv_lpr<T, EPI_JAC>(A.lpr, st, A.n, A.ptr, A.col, A.val, x, b, dinv, xn, nullptr);
}
template <class T>
void spmv_add(const CsrDev<T>& A, const T* x, T* y, hipStream_t st) {
  spmv_lpr<T, EPI_ADD>(A.lpr, st, A.n, A.ptr, A.col, A.val, x, nullptr, nullptr, y, nullptr);
}
void spmv_dot(const CsrDev<double>& A, const double* x, double* y, double* partial,
              hipStream_t st) {
  spmv_lpr<double, EPI_DOT>(A.lpr, st, A.n, A.ptr, A.col, A.val, x, nullptr, nullptr, y, partial);
}

// ---------------------------------------------------------------------------
// multiplicative Schwarz over node-star blocks
// ---------------------------------------------------------------------------
// A chunk is a run of blocks of one colour with at most WGS / LPR rows in all.
// The smoother keeps its own copy of A's rows in star order (srow_ptr, scol,
// sval: star row r is row sb_dofs[r] of A), so a chunk streams one contiguous
// range.  A group of WGS threads does one chunk in two phases:
//   chunk_load    chunk bounds, row bounds, DoFs, each row's block, the
//                 blocks' packed inverses and the first U (column, value)
//                 pairs per lane of every row: everything that does not
//                 depend on x;
//   chunk_finish  b and x entries, row sums (lane sums in entry order, then a
//                 shuffle tree), residuals in LDS, d = A_BB^{-1} r_B (one
//                 thread per row: its row of the block's symmetric inverse
//                 times the block's residuals), x_B += d.
// Blocks of one colour share no DoF and no coupling, so the chunks of a colour
// update x independently and in any order.

// LDS of one chunk: residuals of its rows, per-wave partial sums when a row
// spans several wavefronts (LPR > 64), and the chunk's packed block inverses.
// A chunk holds at most RPB rows in blocks of at most min(RPB, 32) rows, so
// its packed inverses take at most RPB (min(RPB, 32) + 1) / 2 entries.
template <class T, int LPR, int WGS>
struct ChunkLds {
  static constexpr int RPB = WGS / LPR;
  static constexpr int WPR = LPR > 64 ? LPR / 64 : 1;
  static constexpr int SMAX = RPB < 32 ? RPB : 32;
  static constexpr int FL = RPB * (SMAX + 1) / 2;
  T res[RPB];
  T part[WPR > 1 ? RPB * WPR : 1];
  T fl[FL];
};

// Per-thread state of a loaded chunk.
template <class T, int LPR, int WGS, int U>
struct ChunkRegs {
  static constexpr int FPT = (ChunkLds<T, LPR, WGS>::FL + WGS - 1) / WGS;
  int blk0, nblk, r0, nrows, nf;
  int64_t f0, q0, q1;
  int bp, bs, bfo;        // this thread's row: its block's first row (in the chunk), size, inverse offset
  int32_t rdof, mydof;
  T fv[FPT];
  int32_t c[U];
  T v[U];
};

template <class T, int LPR, int WGS, int U>
__device__ __forceinline__ void chunk_load(bool act, int c, int tid, const SmootherArgs<T>& D,
                                           ChunkRegs<T, LPR, WGS, U>& R) {
  constexpr int FPT = ChunkRegs<T, LPR, WGS, U>::FPT;
  R.blk0 = R.nblk = R.r0 = R.nrows = R.nf = 0;
  R.f0 = 0;
  if (act) {
    R.blk0 = D.chunk_blk[c];
    R.nblk = D.chunk_blk[c + 1] - R.blk0;
    R.r0 = D.ck_row0[c];
    R.nrows = D.ck_row0[c + 1] - R.r0;
    R.f0 = D.ck_fac0[c];
    R.nf = (int)(D.ck_fac0[c + 1] - R.f0);
  }
  const int grp = tid / LPR, lane = tid % LPR;
  R.q0 = R.q1 = 0;
  R.rdof = R.mydof = 0;
  if (grp < R.nrows) {
    const int64_t r = (int64_t)R.r0 + grp;
    R.q0 = D.srow_ptr[r];
    R.q1 = D.srow_ptr[r + 1];
    if (lane == 0) R.rdof = D.sb_dofs[r];
  }
  R.bp = R.bs = R.bfo = 0;
  if (tid < R.nrows) {
    R.mydof = D.sb_dofs[R.r0 + tid];
    const int rb = D.row_blk[R.r0 + tid];
    const int64_t p0 = D.sb_ptr[rb];
    R.bp = (int)(p0 - R.r0);
    R.bs = (int)(D.sb_ptr[rb + 1] - p0);
    R.bfo = (int)(D.fac_off[rb] - R.f0);
  }
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int t = tid + k * WGS;
    R.fv[k] = t < R.nf ? D.binv[R.f0 + t] : T(0);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t q = R.q0 + lane + (int64_t)u * LPR;
    const bool in = q < R.q1;
    R.c[u] = in ? D.scol[q] : -1;
    R.v[u] = in ? D.sval[q] : T(0);
  }
}

// Accesses of x.  COH: x is written by other workgroups while the kernel
// runs (the pipelined sweep), so its loads and stores are agent-scope
// relaxed atomics: coherent across the XCDs' L2 caches without cache-wide
// write-back or invalidation.
template <class T, bool COH>
__device__ __forceinline__ T ld_x(const T* p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <class T, bool COH>
__device__ __forceinline__ void st_x(T* p, T v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

template <class T, int LPR, int WGS, int U, bool COH = false>
__device__ __forceinline__ void chunk_finish(int tid, const ChunkRegs<T, LPR, WGS, U>& R,
                                             ChunkLds<T, LPR, WGS>& S, const SmootherArgs<T>& D,
                                             const T* b, T* x) {
  constexpr int WPR = ChunkLds<T, LPR, WGS>::WPR;
  constexpr int FPT = ChunkRegs<T, LPR, WGS, U>::FPT;
  const int grp = tid / LPR, lane = tid % LPR;
  const bool row_act = grp < R.nrows;
  T bv = 0, myx = 0;
  if (row_act && lane == 0) bv = b[R.rdof];
  if (tid < R.nrows) myx = ld_x<T, COH>(x + R.mydof);   // only this chunk changes these in its colour
  T s = 0;
  if (row_act) {
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = R.c[u] >= 0 ? ld_x<T, COH>(x + R.c[u]) : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u) s += R.v[u] * xv[u];
    for (int64_t q0 = R.q0 + lane + (int64_t)U * LPR; q0 < R.q1; q0 += (int64_t)U * LPR) {
      int32_t c[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = q0 + (int64_t)u * LPR;
        const bool in = q < R.q1;
        c[u] = in ? D.scol[q] : -1;
        v[u] = in ? D.sval[q] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = c[u] >= 0 ? ld_x<T, COH>(x + c[u]) : T(0);
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u] * xv[u];
    }
  }
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int t = tid + k * WGS;
    if (t < R.nf) S.fl[t] = R.fv[k];
  }
  if (row_act) {
    if constexpr (LPR <= 64) {
      s = group_sum<LPR>(s);
      if (lane == 0) S.res[grp] = bv - s;
    } else {
      s = group_sum<64>(s);
      if (lane % 64 == 0) S.part[grp * WPR + lane / 64] = s;
      if (lane == 0) S.res[grp] = bv;
    }
  }
  __syncthreads();
  if constexpr (WPR > 1) {
    if (tid < R.nrows) {
      T p = 0;
      for (int w = 0; w < WPR; ++w) p += S.part[tid * WPR + w];
      S.res[tid] -= p;
    }
    __syncthreads();
  }
  if (tid < R.nrows) {
    // d_i = sum_j (A_BB^{-1})_ij r_j, the inverse stored packed (lower half)
    const int i = tid - R.bp;
    const T* Bi = S.fl + R.bfo;
    const T* v = S.res + R.bp;
    T d = 0;
    for (int j = 0; j < R.bs; ++j) {
      const int hi = i > j ? i : j, lo = i > j ? j : i;
      d += Bi[hi * (hi + 1) / 2 + lo] * v[j];
    }
    st_x<T, COH>(x + R.mydof, myx + d);
  }
}

template <int LPR>
constexpr int unroll_for() { return LPR >= 64 ? 16 : 8; }

// one colour: chunk chunk0 + blockIdx.x per workgroup
template <class T, int LPR, int WG>
__global__ __launch_bounds__(WG) void k_schwarz(SmootherArgs<T> D, int chunk0, const T* b, T* x) {
  constexpr int U = unroll_for<LPR>();
  __shared__ ChunkLds<T, LPR, WG> S;
  ChunkRegs<T, LPR, WG, U> R;
  chunk_load<T, LPR, WG, U>(true, chunk0 + blockIdx.x, threadIdx.x, D, R);
  chunk_finish<T, LPR, WG, U>(threadIdx.x, R, S, D, b, x);
}

// Whole sweep of a small level in one workgroup: the 1024 threads walk the
// colours in order, their 1024 / WGS groups taking the chunks of the current
// colour in turn.  The barriers inside chunk_finish and the one after each
// round make the x updates of a colour visible before the next colour reads x.
template <class T, int LPR, int WGS>
__global__ __launch_bounds__(1024) void k_schwarz_sweep1(SmootherArgs<T> D, int backward,
                                                         const T* b, T* x) {
  constexpr int U = unroll_for<LPR>();
  constexpr int NSUB = 1024 / WGS;
  __shared__ ChunkLds<T, LPR, WGS> S_all[NSUB];
  const int sub = threadIdx.x / WGS;
  const int tid = threadIdx.x % WGS;
  for (int ci = 0; ci < D.ncolours; ++ci) {
    const int colour = backward ? D.ncolours - 1 - ci : ci;
    const int c0 = D.colour_chunk[colour], c1 = D.colour_chunk[colour + 1];
    for (int base = c0; base < c1; base += NSUB) {
      const int c = base + sub;
      ChunkRegs<T, LPR, WGS, U> R;
      chunk_load<T, LPR, WGS, U>(c < c1, c, tid, D, R);
      chunk_finish<T, LPR, WGS, U>(tid, R, S_all[sub], D, b, x);
      __syncthreads();
    }
  }
}

// Whole sweep in one launch with the colours pipelined across workgroups.
// Chunks are numbered in sweep order (colour by colour) and handed out by a
// ticket counter, sync[0]; sync[SYNC_STRIDE (1 + c)] counts the finished
// chunks of colour c (each counter on a cache line of its own: they are
// polled by many workgroups at once).
// A workgroup loads its chunk's structure at once and starts the x-dependent
// work when every chunk of the colour before it in sweep order has finished;
// those chunks waited in turn for theirs, so every earlier colour is done and
// the sweep computes what the colour-by-colour launches compute.
// Progress: tickets are taken in increasing order and a workgroup finishes its
// chunks in ticket order, so the unfinished chunk with the smallest ticket
// only waits on finished chunks and always belongs to a running workgroup; no
// assumption on how many workgroups are resident is needed.
// Visibility: x is loaded and stored with agent-scope (all XCDs) coherent
// accesses; a chunk's stores have completed (each storing thread waits for
// its memory counter) before the workgroup barrier that precedes the raise
// of its count, and a waiting chunk loads x only after the barrier that
// follows its wait.  Every wait is bounded: after spin_max polls the wait
// sets *err and gives up (the sweep result is then wrong and the caller
// reports the error), and once *err is set no wait blocks, so the grid always
// drains.  The caller zeroes sync before each sweep.
template <class T, int LPR>
__global__ __launch_bounds__(1024) void k_schwarz_pipe(SmootherArgs<T> D, int backward,
                                                       const T* b, T* x) {
  constexpr int U = unroll_for<LPR>();
  __shared__ ChunkLds<T, LPR, 1024> S;
  __shared__ int ticket[2];
  int* sync = D.sync;
  const int nchunks = D.colour_chunk[D.ncolours];
  const int tid = threadIdx.x;
  if (tid == 0) ticket[0] = __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  int t = ticket[0];
  while (t < nchunks) {
    int next = 0;
    if (tid == 0) next = __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int c = backward ? nchunks - 1 - t : t;
    const int colour = D.chunk_colour[c];
    const int prev = backward ? colour + 1 : colour - 1;
    ChunkRegs<T, LPR, 1024, U> R;
    chunk_load<T, LPR, 1024, U>(true, c, tid, D, R);
    if (tid == 0 && prev >= 0 && prev < D.ncolours) {
      const int need = D.colour_chunk[prev + 1] - D.colour_chunk[prev];
      int spins = 0;
      while (__hip_atomic_load(&sync[SYNC_STRIDE * (1 + prev)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if ((++spins & 255) == 0 &&
            __hip_atomic_load(D.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
          break;
        if (spins > D.spin_max) {
          __hip_atomic_store(D.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    chunk_finish<T, LPR, 1024, U, true>(tid, R, S, D, b, x);
    __builtin_amdgcn_s_waitcnt(0);   // this thread's x stores have completed
    __syncthreads();
    if (tid == 0) {
      __hip_atomic_fetch_add(&sync[SYNC_STRIDE * (1 + colour)], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ticket[1] = next;
    }
    __syncthreads();
    t = ticket[1];
  }
}

// (lanes per row, threads per chunk) pairs of the colour and one-launch forms
bool schwarz_shape_ok(int lpr, int wg) {
  if (wg == 256) return lpr == 4 || lpr == 8 || lpr == 16 || lpr == 32 || lpr == 64;
  if (wg == 512) return lpr == 16 || lpr == 32 || lpr == 64 || lpr == 128;
  if (wg == 1024) return lpr == 8 || lpr == 16 || lpr == 32 || lpr == 64 || lpr == 128 || lpr == 256;
  return false;
}

#define SCHWARZ_SHAPES(X)                                                                        \
  X(4, 256) X(8, 256) X(16, 256) X(32, 256) X(64, 256) X(16, 512) X(32, 512) X(64, 512)         \
  X(128, 512) X(8, 1024) X(16, 1024) X(32, 1024) X(64, 1024) X(128, 1024) X(256, 1024)

template <class T>
void schwarz_sweep_small(const SmootherDev<T>& S, int backward, const T* b, T* x, hipStream_t st) {
  const SmootherArgs<T> D = S;
#define LAUNCH_SW1(L, W)                                                                         \
  if (S.lpr == L && S.wg == W) {                                                                 \
    hipLaunchKernelGGL((k_schwarz_sweep1<T, L, W>), dim3(1), dim3(1024), 0, st, D, backward, b,   \
                       x);                                                                       \
    return;                                                                                      \
  }
  SCHWARZ_SHAPES(LAUNCH_SW1)
#undef LAUNCH_SW1
}

template <class T>
void schwarz_colour(const SmootherDev<T>& S, int colour, const T* b, T* x, hipStream_t st) {
  int c0 = S.colour_chunk_h[colour], c1 = S.colour_chunk_h[colour + 1];
  if (c1 <= c0) return;
  const SmootherArgs<T> D = S;
#define LAUNCH_SW(L, W)                                                                          \
  if (S.lpr == L && S.wg == W) {                                                                 \
    hipLaunchKernelGGL((k_schwarz<T, L, W>), dim3(c1 - c0), dim3(W), 0, st, D, c0, b, x);         \
    return;                                                                                      \
  }
  SCHWARZ_SHAPES(LAUNCH_SW)
#undef LAUNCH_SW
}

__global__ void k_zero_i32(int n, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <class T>
void schwarz_pipe(const SmootherDev<T>& S, int backward, const T* b, T* x, hipStream_t st) {
  const int nsync = SYNC_STRIDE * (S.ncolours + 1);
  hipLaunchKernelGGL(k_zero_i32, dim3((nsync + 255) / 256), dim3(256), 0, st, nsync, S.sync);
  const SmootherArgs<T> D = S;
#define LAUNCH_PIPE(L)                                                                           \
  if (S.lpr == L) {                                                                              \
    hipLaunchKernelGGL((k_schwarz_pipe<T, L>), dim3(S.pipe_grid), dim3(1024), 0, st, D, backward, \
                       b, x);                                                                    \
    return;                                                                                      \
  }
  LAUNCH_PIPE(8) LAUNCH_PIPE(16) LAUNCH_PIPE(32) LAUNCH_PIPE(64) LAUNCH_PIPE(128) LAUNCH_PIPE(256)
#undef LAUNCH_PIPE
}

// values of the smoother's row copy: star row r is row sb_dofs[r] of A
__global__ void k_star_rows(int64_t nrows, const int32_t* __restrict__ sb_dofs,
                            const int64_t* __restrict__ Aptr, const double* __restrict__ Aval,
                            const int64_t* __restrict__ srow_ptr, double* __restrict__ sval) {
  const int64_t r = (int64_t)blockIdx.x * 8 + threadIdx.x / 32;
  const int lane = threadIdx.x % 32;
  if (r >= nrows) return;
  const int64_t a0 = Aptr[sb_dofs[r]];
  const int64_t s0 = srow_ptr[r], len = srow_ptr[r + 1] - s0;
  for (int64_t q = lane; q < len; q += 32) sval[s0 + q] = Aval[a0 + q];
}
void star_rows(int64_t nrows, const int32_t* sb_dofs, const int64_t* Aptr, const double* Aval,
               const int64_t* srow_ptr, double* sval, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_star_rows, dim3((unsigned)((nrows + 7) / 8)), dim3(256), 0, st, nrows,
                       sb_dofs, Aptr, Aval, srow_ptr, sval);
}

// ---------------------------------------------------------------------------
// multiplicative Schwarz on a dense level
// ---------------------------------------------------------------------------
// At the bottom of the hierarchy the Galerkin operators are dense or nearly
// so: almost every pair of blocks conflicts, each colour holds about one
// block, and a sweep is a sequential chain over the blocks.  One 1024-thread
// workgroup keeps r = b - A x and x in LDS; for each block B in colour order
// (blocks of one colour in any order: they are uncoupled, so their updates
// commute exactly) it solves d = A_BB^{-1} r_B from the packed Cholesky
// factor, sets x_B += d and updates r -= A_{:,B} d from a column-major dense
// copy of A.  This is the sweep of the row form; only the rounding differs,
// because r is updated instead of recomputed.  Everything a block needs from
// global memory (its DoFs, factor and the columns A_{:,B}) is fetched one
// block ahead, so the chain between blocks stays in LDS and registers.
// Limits (checked by the caller): n <= 1024 * RPT <= 2048, blocks of at most
// SM <= 16 DoFs.
constexpr int DENSE_SMAX = 16;
constexpr int DENSE_FMAX = DENSE_SMAX * (DENSE_SMAX + 1) / 2;

size_t dense_sweep_lds(int n, size_t tsize) {
  return tsize * (2 * (size_t)n + DENSE_SMAX + DENSE_FMAX) + sizeof(int32_t) * DENSE_SMAX;
}

template <class T, int RPT, int SM>
__global__ __launch_bounds__(1024) void k_dense_sweep(int n, int nblocks, int backward,
                                                      const int64_t* __restrict__ sb_ptr,
                                                      const int32_t* __restrict__ sb_dofs,
                                                      const int64_t* __restrict__ fac_off,
                                                      const T* __restrict__ fac,
                                                      const T* __restrict__ Acm,
                                                      const T* __restrict__ r_in, T* __restrict__ x) {
  extern __shared__ unsigned char lds_raw[];
  T* r = (T*)lds_raw;                 // n
  T* xs = r + n;                      // n
  T* d = xs + n;                      // DENSE_SMAX
  T* fl = d + DENSE_SMAX;             // DENSE_FMAX
  int32_t* dofs = (int32_t*)(fl + DENSE_FMAX);   // DENSE_SMAX
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += 1024) {
    r[i] = r_in[i];
    xs[i] = x[i];
  }
  // one block ahead: its size, this thread's DoF and factor entry, and the
  // thread's rows of the block's columns
  int nx_s = 0;
  int32_t nx_dof = 0;
  T nx_f = 0;
  T nx_col[RPT][SM];
  auto fetch = [&](int bi) {
    const int blk = backward ? nblocks - 1 - bi : bi;
    const int64_t p0 = sb_ptr[blk];
    const int sz = (int)(sb_ptr[blk + 1] - p0);
    const int64_t f0 = fac_off[blk];
    nx_s = sz;
    nx_dof = tid < sz ? sb_dofs[p0 + tid] : 0;
    nx_f = tid < sz * (sz + 1) / 2 ? fac[f0 + tid] : T(0);
#pragma unroll
    for (int k = 0; k < SM; ++k) {
      const int32_t dk = k < sz ? sb_dofs[p0 + k] : 0;
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) {
        const int i = tid + rr * 1024;
        nx_col[rr][k] = (k < sz && i < n) ? Acm[(int64_t)dk * n + i] : T(0);
      }
    }
  };
  if (nblocks > 0) fetch(0);
  for (int bi = 0; bi < nblocks; ++bi) {
    const int sz = nx_s;
    T col[RPT][SM];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr)
#pragma unroll
      for (int k = 0; k < SM; ++k) col[rr][k] = nx_col[rr][k];
    if (tid < sz) dofs[tid] = nx_dof;
    if (tid < sz * (sz + 1) / 2) fl[tid] = nx_f;
    __syncthreads();   // dofs, factor (and, on the first block, r and xs) in LDS
    if (bi + 1 < nblocks) fetch(bi + 1);
    if (tid == 0) {
      for (int i = 0; i < sz; ++i) {
        T a = r[dofs[i]];
        const T* Li = fl + i * (i + 1) / 2;
        for (int j = 0; j < i; ++j) a -= Li[j] * d[j];
        d[i] = a / Li[i];
      }
      for (int i = sz - 1; i >= 0; --i) {
        T a = d[i];
        for (int j = i + 1; j < sz; ++j) a -= fl[j * (j + 1) / 2 + i] * d[j];
        d[i] = a / fl[i * (i + 1) / 2 + i];
      }
    }
    __syncthreads();   // d ready
    if (tid < sz) xs[dofs[tid]] += d[tid];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int i = tid + rr * 1024;
      if (i < n) {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < SM; ++k)
          if (k < sz) acc += col[rr][k] * d[k];
        r[i] -= acc;
      }
    }
    __syncthreads();   // r, xs updated; dofs, fl and d free for the next block
  }
  for (int i = tid; i < n; i += 1024) x[i] = xs[i];
}

// The same sweep for larger nearly dense levels (2048 < n <= 16384): r and x
// stay in global memory (one workgroup touches them, so they stay in its
// CU's cache path), the block's DoFs and factor are fetched one block ahead,
// and each thread updates its rows of r from the block's columns.
template <class T, int SM>
__global__ __launch_bounds__(1024) void k_dense_sweep_big(int n, int nblocks, int backward,
                                                          const int64_t* __restrict__ sb_ptr,
                                                          const int32_t* __restrict__ sb_dofs,
                                                          const int64_t* __restrict__ fac_off,
                                                          const T* __restrict__ fac,
                                                          const T* __restrict__ Acm,
                                                          T* __restrict__ r, T* __restrict__ x) {
  __shared__ T d[SM];
  __shared__ T fl[SM * (SM + 1) / 2];
  __shared__ int32_t dofs[SM];
  const int tid = threadIdx.x;
  int nx_s = 0;
  int32_t nx_dof = 0;
  T nx_f = 0;
  auto fetch = [&](int bi) {
    const int blk = backward ? nblocks - 1 - bi : bi;
    const int64_t p0 = sb_ptr[blk];
    const int sz = (int)(sb_ptr[blk + 1] - p0);
    nx_s = sz;
    nx_dof = tid < sz ? sb_dofs[p0 + tid] : 0;
    nx_f = tid < sz * (sz + 1) / 2 ? fac[fac_off[blk] + tid] : T(0);
  };
  if (nblocks > 0) fetch(0);
  for (int bi = 0; bi < nblocks; ++bi) {
    const int sz = nx_s;
    if (tid < sz) dofs[tid] = nx_dof;
    if (tid < sz * (sz + 1) / 2) fl[tid] = nx_f;
    __syncthreads();   // dofs and factor in LDS; r and x of the previous block visible
    if (bi + 1 < nblocks) fetch(bi + 1);
    if (tid == 0) {
      T v[SM];
#pragma unroll
      for (int i = 0; i < SM; ++i) v[i] = i < sz ? r[dofs[i]] : T(0);
      for (int i = 0; i < sz; ++i) {
        T a = v[i];
        const T* Li = fl + i * (i + 1) / 2;
        for (int j = 0; j < i; ++j) a -= Li[j] * d[j];
        d[i] = a / Li[i];
      }
      for (int i = sz - 1; i >= 0; --i) {
        T a = d[i];
        for (int j = i + 1; j < sz; ++j) a -= fl[j * (j + 1) / 2 + i] * d[j];
        d[i] = a / fl[i * (i + 1) / 2 + i];
      }
    }
    __syncthreads();   // d ready
    if (tid < sz) x[dofs[tid]] += d[tid];
    T dk[SM];
    int32_t ck[SM];
#pragma unroll
    for (int k = 0; k < SM; ++k) {
      dk[k] = k < sz ? d[k] : T(0);
      ck[k] = k < sz ? dofs[k] : 0;
    }
    for (int i = tid; i < n; i += 1024) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < SM; ++k)
        if (k < sz) acc += Acm[(int64_t)ck[k] * n + i] * dk[k];
      r[i] -= acc;
    }
    __syncthreads();   // r and x updated; dofs, fl and d free for the next block
  }
}

template <class T>
bool dense_sweep_ok(int n, int max_block) {
  if (n <= 0 || max_block > DENSE_SMAX) return false;
  if (n <= 2048) return dense_sweep_lds(n, sizeof(T)) <= 64 * 1024;
  return n <= 16384;
}

template <class T>
void dense_sweep(int n, int nblocks, int max_block, int backward, const int64_t* sb_ptr,
                 const int32_t* sb_dofs, const int64_t* fac_off, const T* fac, const T* Acm,
                 const T* r_in, T* x, hipStream_t st) {
  // HCURL_AMG_DENSE_BIG=1 takes the global-memory form at any size (for tests)
  const char* big_env = std::getenv("HCURL_AMG_DENSE_BIG");
  if (n > 2048 || (big_env && big_env[0] == '1')) {   // r_in (the level's scratch) is updated in place
    if (max_block <= 8)
      hipLaunchKernelGGL((k_dense_sweep_big<T, 8>), dim3(1), dim3(1024), 0, st, n, nblocks, backward,
                         sb_ptr, sb_dofs, fac_off, fac, Acm, const_cast<T*>(r_in), x);
    else
      hipLaunchKernelGGL((k_dense_sweep_big<T, 16>), dim3(1), dim3(1024), 0, st, n, nblocks,
                         backward, sb_ptr, sb_dofs, fac_off, fac, Acm, const_cast<T*>(r_in), x);
    return;
  }
  const size_t lds = dense_sweep_lds(n, sizeof(T));
#define LAUNCH_DS(R, M)                                                                          \
  hipLaunchKernelGGL((k_dense_sweep<T, R, M>), dim3(1), dim3(1024), lds, st, n, nblocks, backward, \
                     sb_ptr, sb_dofs, fac_off, fac, Acm, r_in, x)
  if (n <= 1024) {
    if (max_block <= 8) LAUNCH_DS(1, 8); else LAUNCH_DS(1, 16);
  } else {
    if (max_block <= 8) LAUNCH_DS(2, 8); else LAUNCH_DS(2, 16);
  }
#undef LAUNCH_DS
}

// ---------------------------------------------------------------------------
// multiplicative Schwarz on a wide level: the panel sweep
// ---------------------------------------------------------------------------
// Coarse Galerkin operators near the bottom of the hierarchy have rows of
// thousands of entries and hundreds to thousands of colours with a few blocks
// each, so a sweep is a long chain of small steps.  The panel form keeps
// r = b - A x and follows the blocks in sweep order in groups of consecutive
// blocks with at most PANEL_SLOTS rows in all (a row of a group is a "slot";
// a DoF in two blocks of one group has two slots).  Workgroup 0 (the chain)
// takes the groups in turn: it loads the group's slice A(D_g, D_g) and
// residual entries, and for each block B in sweep order forms
// d = A_BB^{-1} r_B (the lanes of B's slots, each with its row of the
// block's symmetric inverse) and updates the residual of every slot of the
// group, all in one wavefront; x_B += d follows at the end of the group.  The other workgroups own tiles of PANEL_TILE rows
// and apply each group's update r_i -= sum_k A(i, dof_k) d_k to their rows,
// reading A from a column-major dense copy.  Exactly-once rule for the update
// of group h on row i: the chain applies it when i is in D_h (inside the
// group) or in the next group D_h' (as a correction it carries to h'), the
// tiles otherwise.  The chain reads the residual of D_g after the tiles have
// applied every group two or more positions back (they skip rows of D_g for
// the group just before it), so the chain only waits when the tiles fall
// more than a group behind.  The result is the multiplicative Schwarz sweep
// in residual-update form (only the rounding differs from the row form).
// Shared data (r, the published d) use agent-coherent accesses; a stored
// value is complete (memory counter drained) before the barrier that precedes
// its flag.  Every wait is bounded as in the pipelined sweep.  All
// workgroups of the grid must be able to run at once (1 + n / PANEL_TILE of
// 256 threads, n <= PANEL_NMAX, on an otherwise idle device).
constexpr int PANEL_SLOTS = PANEL_GROUP_SLOTS;
constexpr int PANEL_TILE = 256;
constexpr int PANEL_NMAX = 32768;
constexpr int PANEL_SMAX = PANEL_ROW_WIDTH;
constexpr int PANEL_FMAX = PANEL_SLOTS * (PANEL_SMAX + 1) / 2;

template <class T>
struct PanelArgs {
  int n = 0, ngroups = 0, ntiles = 0, backward = 0, spin_max = 0;
  const int32_t* grp_blk = nullptr;   // first block of each group (+ sentinel), colour order
  const int64_t* sb_ptr = nullptr;
  const int32_t* sb_dofs = nullptr;
  const int64_t* fac_off = nullptr;
  const T* binv_pad = nullptr;        // per star row: its row of the block inverse, 16 wide, zero-padded
  const T* Acm = nullptr;             // A(i, j) at Acm[j n + i]
  const T* slc = nullptr;             // per group: A(D_g, D_g), column-major m_g x m_g
  const T* cor = nullptr;             // per group g < G-1: A(D_g+1, D_g), column-major
  const int64_t* slc_off = nullptr;
  const int64_t* cor_off = nullptr;
  const int32_t* dgrp = nullptr;      // the (at most two) groups holding each DoF, -1 if none
  const int32_t* sdup = nullptr;      // per slot: the group's other slot of the same DoF, or -1
  T* r = nullptr;                     // b - A x on entry, kept equal to it
  T* x = nullptr;
  T* dsl = nullptr;                   // per sweep position: d of each slot of the group
  int* flag = nullptr;                // per sweep position (stride SYNC_STRIDE): dsl is published
  int* done = nullptr;                // per sweep position (stride SYNC_STRIDE): tiles that applied it
  int* err = nullptr;
};

__device__ __forceinline__ void panel_wait(const int* p, int need, int* err, int spin_max) {
  int spins = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if ((++spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return;
    if (spins > spin_max) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// value of a uniform lane, broadcast through the scalar unit
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Structure of one group, as the chain workgroup stages it: DoFs, the other
// slot of a repeated DoF, block offsets / sizes / factor offsets, packed
// factors and the slice A(D_g, D_g).
struct PanelGroup {
  int g, bb0, nbk, m, nf;
  int64_t q0, f0;
};

template <class T>
__device__ __forceinline__ PanelGroup panel_group(const PanelArgs<T>& P, int pos) {
  PanelGroup q;
  q.g = P.backward ? P.ngroups - 1 - pos : pos;
  q.bb0 = P.grp_blk[q.g];
  const int bb1 = P.grp_blk[q.g + 1];
  q.nbk = bb1 - q.bb0;
  q.q0 = P.sb_ptr[q.bb0];
  q.m = (int)(P.sb_ptr[bb1] - q.q0);
  q.f0 = P.fac_off[q.bb0];
  q.nf = (int)(P.fac_off[bb1] - q.f0);
  return q;
}

// One block B (slots p .. p+s-1, s <= SB) of the panel chain, in one
// wavefront (lane k = slot k): the lanes of B form d_k = sum_j
// (A_BB^{-1})_{k-p, j} r_{p+j}, then every slot's residual drops by
// sum_j A(slot, p+j) d_j.  Operands come into registers first; the values
// of other lanes are broadcast through the scalar unit, all independent of
// each other; each sum is a fixed pairwise tree, so the dependent chain is
// two tree depths instead of 2 s multiply-adds.
template <class T, int SB>
__device__ __forceinline__ T tree_sum(T (&v)[SB]) {
#pragma unroll
  for (int w = SB / 2; w > 0; w /= 2)
#pragma unroll
    for (int j = 0; j < w; ++j) v[j] = v[j] + v[j + w];
  return v[0];
}

template <class T, int SB>
__device__ __forceinline__ void panel_step(int k, int m, int p, int s, const T* brow, const T* Aloc,
                                           T& rk, T& dk) {
  // brow: this lane's row of its block's inverse, zero beyond the block
  // (meaningful for the lanes of B only; the others' d is never used)
  T v[SB];
#pragma unroll
  for (int j = 0; j < SB; ++j) v[j] = brow[j] * (j < s ? lane_bcast(rk, p + j) : T(0));
  const T d = tree_sum<T, SB>(v);
  if (k >= p && k < p + s) dk = d;
  const T* acol = Aloc + p * PANEL_SLOTS + k;
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    const T a = acol[j * PANEL_SLOTS];
    v[j] = (j < s && k < m ? a : T(0)) * (j < s ? lane_bcast(d, p + j) : T(0));
  }
  rk -= tree_sum<T, SB>(v);
}

// entries of the 64 x 64 slot matrices that one of the 192 staging threads
// holds: e = t + 192 j
constexpr int PANEL_STAGE = 192;
constexpr int PANEL_PER = (PANEL_SLOTS * PANEL_SLOTS + PANEL_STAGE - 1) / PANEL_STAGE;   // 22
constexpr int PANEL_FPER = (PANEL_SLOTS * PANEL_SMAX + PANEL_STAGE - 1) / PANEL_STAGE;  // 6

template <class T>
__global__ __launch_bounds__(256) void k_schwarz_panel(PanelArgs<T> P) {
  __shared__ T Aloc[PANEL_SLOTS * PANEL_SLOTS];   // Aloc[l * 64 + k] = A(dof_k, dof_l)
  __shared__ T fl[PANEL_SLOTS * PANEL_SMAX];   // per slot: its row of the block inverse (padded)
  __shared__ T part[3][PANEL_SLOTS];
  __shared__ T ds_s[PANEL_SLOTS];
  __shared__ T corr[PANEL_SLOTS];
  __shared__ int dof_s[PANEL_SLOTS];
  __shared__ int sdup_s[PANEL_SLOTS];
  __shared__ int inprev_s[PANEL_SLOTS];
  __shared__ int blk_p[PANEL_SLOTS], blk_s[PANEL_SLOTS], blk_f[PANEL_SLOTS];
  const int tid = threadIdx.x;
  const int G = P.ngroups;
  const int64_t n = P.n;
  if (blockIdx.x == 0) {
    // ---------------- the chain ----------------
    // prologue: stage group 0
    {
      const PanelGroup q = panel_group(P, 0);
      if (tid < q.m) {
        dof_s[tid] = P.sb_dofs[q.q0 + tid];
        sdup_s[tid] = P.sdup[q.q0 + tid];
        inprev_s[tid] = 0;
      }
      if (tid < q.nbk) {
        const int blk = q.bb0 + tid;
        const int bp = (int)(P.sb_ptr[blk] - q.q0), bs = (int)(P.sb_ptr[blk + 1] - P.sb_ptr[blk]);
        const int64_t bf = P.fac_off[blk];
        blk_p[tid] = bp;
        blk_s[tid] = bs;
        blk_f[tid] = (int)(bf - q.f0);
      }
      for (int t = tid; t < PANEL_SLOTS * PANEL_SMAX; t += 256)
        fl[t] = t < q.m * PANEL_SMAX ? P.binv_pad[q.q0 * PANEL_SMAX + t] : T(0);
      __syncthreads();
      for (int e = tid; e < PANEL_SLOTS * PANEL_SLOTS; e += 256) {
        const int l = e / PANEL_SLOTS, k = e % PANEL_SLOTS;
        if (l < q.m && k < q.m) Aloc[e] = P.slc[P.slc_off[q.g] + l * q.m + k];
      }
      __syncthreads();
    }
    for (int pos = 0; pos < G; ++pos) {
      const PanelGroup q = panel_group(P, pos);
      const int m = q.m;
      const bool more = pos + 1 < G;
      PanelGroup qn{};
      if (more) qn = panel_group(P, pos + 1);
      // the tiles have applied every group two or more positions back
      if (tid == 0 && pos >= 2) panel_wait(&P.done[SYNC_STRIDE * (pos - 2)], P.ntiles, P.err, P.spin_max);
      __syncthreads();
      // staging registers of waves 1-3 (next group's structure and slice,
      // and the entries A(D_next, D_g) of the correction)
      T an[PANEL_PER], cn[PANEL_PER], fn[PANEL_FPER];
      int dn = 0, sn = 0, ipn = 0, bpn = 0, bsn = 0, bfn = 0;
      if (tid < 64) {
        // wave 0: the chain over the group's blocks; lane k holds slot k
        const int k = tid;
        const int dofk = k < m ? dof_s[k] : 0;
        T rk = 0, dk = 0;
        if (k < m) {
          rk = ld_x<T, true>(P.r + dofk);
          if (pos >= 1 && !inprev_s[k]) rk += corr[k];
        }
        for (int jb = 0; jb < q.nbk; ++jb) {
          const int ib = P.backward ? q.nbk - 1 - jb : jb;
          // uniform across the wavefront: keeps the broadcasts on the scalar unit
          const int p = __builtin_amdgcn_readfirstlane(blk_p[ib]);
          const int s = __builtin_amdgcn_readfirstlane(blk_s[ib]);
          const T* brow = fl + (k < m ? k : 0) * PANEL_SMAX;
          if (s <= PANEL_SMAX / 2)
            panel_step<T, PANEL_SMAX / 2>(k, m, p, s, brow, Aloc, rk, dk);
          else
            panel_step<T, PANEL_SMAX>(k, m, p, s, brow, Aloc, rk, dk);
        }
        // x_B += d for the group's blocks in sweep order: a DoF in two blocks
        // of the group (slots k and dup) gets both updates from the lower slot's lane
        const int dup = k < m ? sdup_s[k] : -1;
        const T ddup = __shfl(dk, dup & 63);
        if (k < m) {
          if (dup < 0) {
            st_x<T, true>(P.x + dofk, ld_x<T, true>(P.x + dofk) + dk);
          } else if (k < dup) {
            const T x0 = ld_x<T, true>(P.x + dofk);
            st_x<T, true>(P.x + dofk, P.backward ? (x0 + ddup) + dk : (x0 + dk) + ddup);
          }
          st_x<T, true>(P.r + dofk, rk);
          st_x<T, true>(P.dsl + (int64_t)pos * PANEL_SLOTS + k, dk);
          ds_s[k] = dk;
        }
        __builtin_amdgcn_s_waitcnt(0);
      } else if (more) {
        // waves 1-3: load the next group while the chain runs
        const int t = tid - 64;
        const int mn = qn.m;
        const int64_t dq = qn.q0;
        if (t < mn) {
          dn = P.sb_dofs[dq + t];
          sn = P.sdup[dq + t];
          const int d = dn;
          ipn = P.dgrp[2 * d] == q.g || P.dgrp[2 * d + 1] == q.g;
        }
        if (t < qn.nbk) {
          const int blk = qn.bb0 + t;
          bpn = (int)(P.sb_ptr[blk] - dq);
          bsn = (int)(P.sb_ptr[blk + 1] - P.sb_ptr[blk]);
          bfn = (int)(P.fac_off[blk] - qn.f0);
        }
#pragma unroll
        for (int j = 0; j < PANEL_FPER; ++j) {
          const int e = t + PANEL_STAGE * j;
          fn[j] = e < qn.m * PANEL_SMAX ? P.binv_pad[qn.q0 * PANEL_SMAX + e] : T(0);
        }
        // slice of the next group (stored contiguously): entry e = l * 64 + k
        const T* Sn = P.slc + P.slc_off[qn.g];
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int e = t + PANEL_STAGE * j;
          const int l = e / PANEL_SLOTS, k = e % PANEL_SLOTS;
          an[j] = (l < mn && k < mn) ? Sn[l * mn + k] : T(0);
        }
        // correction entries: thread (kn, part) holds A(dof_n[kn], dof_s[k])
        // for k = part, part + 3, ...; the block between two consecutive
        // groups is stored once (forward order) and read transposed backward
        const int kn = t % PANEL_SLOTS, pt = t / PANEL_SLOTS;
        const T* Cg = P.cor + P.cor_off[P.backward ? qn.g : q.g];
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int k = pt + 3 * j;
          cn[j] = T(0);
          if (kn < mn && k < m) cn[j] = P.backward ? Cg[kn * m + k] : Cg[k * mn + kn];
        }
      }
      __syncthreads();
      if (tid == 0) __hip_atomic_store(&P.flag[SYNC_STRIDE * pos], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!more) break;
      // correction partial sums (this group's d is in ds_s) and the next group's staging
      if (tid >= 64) {
        const int t = tid - 64;
        const int kn = t % PANEL_SLOTS, pt = t / PANEL_SLOTS;
        T acc = 0;
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int k = pt + 3 * j;
          if (k < m) acc += cn[j] * ds_s[k];
        }
        part[pt][kn] = acc;
      }
      __syncthreads();
      if (tid < qn.m) corr[tid] = -((part[0][tid] + part[1][tid]) + part[2][tid]);
      if (tid >= 64) {
        const int t = tid - 64;
        if (t < qn.m) {
          dof_s[t] = dn;
          sdup_s[t] = sn;
          inprev_s[t] = ipn;
        }
        if (t < qn.nbk) {
          blk_p[t] = bpn;
          blk_s[t] = bsn;
          blk_f[t] = bfn;
        }
#pragma unroll
        for (int j = 0; j < PANEL_FPER; ++j) {
          const int e = t + PANEL_STAGE * j;
          if (e < PANEL_SLOTS * PANEL_SMAX) fl[e] = fn[j];
        }
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int e = t + PANEL_STAGE * j;
          const int l = e / PANEL_SLOTS, k = e % PANEL_SLOTS;
          if (l < qn.m && k < qn.m) Aloc[e] = an[j];
        }
      }
      __syncthreads();
    }
    return;
  }
  // ---------------- the tiles ----------------
  // Each thread owns row i; for every group it loads the group's columns of
  // its row (and the row's residual) before waiting for the group's d.
  const int64_t i = (int64_t)(blockIdx.x - 1) * PANEL_TILE + tid;
  const bool row = i < n;
  const int ga = row ? P.dgrp[2 * i] : -1, gb = row ? P.dgrp[2 * i + 1] : -1;
  for (int pos = 0; pos < G; ++pos) {
    const int g = P.backward ? G - 1 - pos : pos;
    const int gn = pos + 1 < G ? (P.backward ? g - 1 : g + 1) : -2;
    const int64_t q0 = P.sb_ptr[P.grp_blk[g]];
    const int m = (int)(P.sb_ptr[P.grp_blk[g + 1]] - q0);
    const bool upd = row && ga != g && ga != gn && gb != g && gb != gn;
    if (tid < m) dof_s[tid] = P.sb_dofs[q0 + tid];
    __syncthreads();
    T a[PANEL_SLOTS];
#pragma unroll
    for (int k = 0; k < PANEL_SLOTS; ++k) a[k] = (upd && k < m) ? P.Acm[(int64_t)dof_s[k] * n + i] : T(0);
    // the tile wrote r_i last itself, or the chain did before an earlier flag
    const T ri = upd ? ld_x<T, true>(P.r + i) : T(0);
    if (tid == 0) panel_wait(&P.flag[SYNC_STRIDE * pos], 1, P.err, P.spin_max);
    __syncthreads();
    if (tid < m) ds_s[tid] = ld_x<T, true>(P.dsl + (int64_t)pos * PANEL_SLOTS + tid);
    __syncthreads();
    if (upd) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < PANEL_SLOTS; ++k)
        if (k < m) acc += a[k] * ds_s[k];
      st_x<T, true>(P.r + i, ri - acc);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&P.done[SYNC_STRIDE * pos], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

bool panel_sweep_ok(int n, int max_block) {
  return n > 0 && n <= PANEL_NMAX && max_block <= PANEL_SMAX;
}

int panel_tiles(int n) { return (n + PANEL_TILE - 1) / PANEL_TILE; }

// The panel form's per-group slices A(D_g, D_g) and inter-group blocks
// A(D_g+1, D_g), gathered from the dense copy once per numeric setup.
template <class T>
__global__ void k_panel_slices(int ngroups, int64_t n, const int32_t* __restrict__ grp_blk,
                               const int64_t* __restrict__ sb_ptr, const int32_t* __restrict__ sb_dofs,
                               const T* __restrict__ Acm, const int64_t* __restrict__ slc_off,
                               const int64_t* __restrict__ cor_off, T* __restrict__ slc,
                               T* __restrict__ cor) {
  const int g = blockIdx.x;
  const int64_t q0 = sb_ptr[grp_blk[g]];
  const int m = (int)(sb_ptr[grp_blk[g + 1]] - q0);
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int l = e / m, k = e % m;
    slc[slc_off[g] + e] = Acm[(int64_t)sb_dofs[q0 + l] * n + sb_dofs[q0 + k]];
  }
  if (g + 1 < ngroups) {
    const int64_t q1 = sb_ptr[grp_blk[g + 1]];
    const int mn = (int)(sb_ptr[grp_blk[g + 2]] - q1);
    for (int e = threadIdx.x; e < m * mn; e += blockDim.x) {
      const int k = e / mn, kn = e % mn;
      cor[cor_off[g] + e] = Acm[(int64_t)sb_dofs[q0 + k] * n + sb_dofs[q1 + kn]];
    }
  }
}

template <class T>
void panel_slices(int ngroups, int64_t n, const int32_t* grp_blk, const int64_t* sb_ptr,
                  const int32_t* sb_dofs, const T* Acm, const int64_t* slc_off, const int64_t* cor_off,
                  T* slc, T* cor, hipStream_t st) {
  if (ngroups > 0)
    hipLaunchKernelGGL((k_panel_slices<T>), dim3(ngroups), dim3(256), 0, st, ngroups, n, grp_blk,
                       sb_ptr, sb_dofs, Acm, slc_off, cor_off, slc, cor);
}

template <class T>
void panel_sweep(int n, int ngroups, int backward, const int32_t* grp_blk, const int64_t* sb_ptr,
                 const int32_t* sb_dofs, const int64_t* fac_off, const T* binv, const T* Acm,
                 const T* slc, const T* cor, const int64_t* slc_off, const int64_t* cor_off,
                 const int32_t* dgrp, const int32_t* sdup, T* r, T* x, T* dsl, int* sync, int* err,
                 int spin_max, hipStream_t st) {
  if (ngroups <= 0) return;
  const int nsync = 2 * SYNC_STRIDE * ngroups;
  hipLaunchKernelGGL(k_zero_i32, dim3((nsync + 255) / 256), dim3(256), 0, st, nsync, sync);
  PanelArgs<T> P;
  P.n = n;
  P.ngroups = ngroups;
  P.ntiles = panel_tiles(n);
  P.backward = backward;
  P.spin_max = spin_max;
  P.grp_blk = grp_blk;
  P.sb_ptr = sb_ptr;
  P.sb_dofs = sb_dofs;
  P.fac_off = fac_off;
  P.binv_pad = binv;
  P.Acm = Acm;
  P.slc = slc;
  P.cor = cor;
  P.slc_off = slc_off;
  P.cor_off = cor_off;
  P.dgrp = dgrp;
  P.sdup = sdup;
  P.r = r;
  P.x = x;
  P.dsl = dsl;
  P.flag = sync;
  P.done = sync + SYNC_STRIDE * ngroups;
  P.err = err;
  hipLaunchKernelGGL((k_schwarz_panel<T>), dim3(1 + P.ntiles), dim3(256), 0, st, P);
}

// column-major dense copy of a CSR matrix (D(i, j) at D[j n + i])
__global__ void k_csr_to_dense_cm(int64_t n, const int64_t* __restrict__ ptr,
                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                  double* __restrict__ D) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) D[(int64_t)col[q] * n + i] = val[q];
}
void csr_to_dense_cm(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                     double* D, hipStream_t st) {
  fill<double>(n * n, 0.0, D, st);
  hipLaunchKernelGGL(k_csr_to_dense_cm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ptr,
                     col, val, D);
}

// ---------------------------------------------------------------------------
// coarsest level: x = (L L^T)^{-1} b with a dense FP64 factor, one workgroup
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_dense_solve(int n, const double* __restrict__ L,
                                                     const T* __restrict__ b, T* __restrict__ x,
                                                     double* __restrict__ work) {
  // work: n doubles (global scratch for the running right-hand side)
  for (int i = threadIdx.x; i < n; i += blockDim.x) work[i] = (double)b[i];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double yk = work[k] / L[(int64_t)k * n + k];
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) work[i] -= L[(int64_t)i * n + k] * yk;
    if (threadIdx.x == 0) work[k] = yk;
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    double xk = work[k] / L[(int64_t)k * n + k];
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) work[i] -= L[(int64_t)k * n + i] * xk;
    if (threadIdx.x == 0) work[k] = xk;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (T)work[i];
}

template <class T>
void dense_solve(int n, const double* L, const T* b, T* x, double* work, hipStream_t st) {
  hipLaunchKernelGGL((k_dense_solve<T>), dim3(1), dim3(256), 0, st, n, L, b, x, work);
}

// dense gather of a (small) CSR matrix into row-major n x n
__global__ void k_csr_to_dense(int64_t n, const int64_t* __restrict__ ptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ D) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) D[i * n + col[q]] = val[q];
}

// right-looking dense Cholesky (lower, row-major; upper part left as is)
__global__ __launch_bounds__(256) void k_dense_chol(int n, double* __restrict__ D,
                                                    int* __restrict__ flag) {
  for (int k = 0; k < n; ++k) {
    __shared__ double dk;
    if (threadIdx.x == 0) {
      double a = D[(int64_t)k * n + k];
      if (!(a > 0.0)) {
        *flag = 1;
        a = 1.0;
      }
      dk = sqrt(a);
      D[(int64_t)k * n + k] = dk;
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) D[(int64_t)i * n + k] /= dk;
    __syncthreads();
    // trailing update of the lower triangle: rows i > k, cols k < j <= i
    int64_t m = n - k - 1;
    for (int64_t t = threadIdx.x; t < m * m; t += blockDim.x) {
      int64_t i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) D[i * n + j] -= D[i * n + k] * D[j * n + k];
    }
    __syncthreads();
  }
}

void dense_factor(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, double* D,
                  int* flag, hipStream_t st) {
  fill<double>(n * n, 0.0, D, st);
  hipLaunchKernelGGL(k_csr_to_dense, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ptr,
                     col, val, D);
  hipLaunchKernelGGL(k_dense_chol, dim3(1), dim3(256), 0, st, (int)n, D, flag);
}

// ---------------------------------------------------------------------------
// vector kernels (FP64 PCG, casts, fills)
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(int64_t n, T v, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
template <class A, class B>
__global__ void k_cast(int64_t n, const A* __restrict__ a, B* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (B)a[i];
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <class T>
void fill(int64_t n, T v, T* x, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(256), 0, st, n, v, x);
}
template <class A, class B>
void cast(int64_t n, const A* a, B* b, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL((k_cast<A, B>), dim3(grid_for(n)), dim3(256), 0, st, n, a, b);
}

// Deterministic reductions: a fixed grid of RED_GRID blocks, each summing a
// fixed strided subset in a fixed order, then one block summing the partials.
constexpr int RED_GRID = 1024;

__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// x += alpha p; r -= alpha q; partial[b] = sum r.r
__global__ __launch_bounds__(256) void k_cg_update(int64_t n, const double* __restrict__ sc,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ r_old,
                                                   double* __restrict__ partial) {
  const double alpha = sc[SC_ALPHA];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)RED_GRID * 256) {
    x[i] += alpha * p[i];
    double ri = r[i];
    if (r_old) r_old[i] = ri;
    ri -= alpha * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  acc = block_sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// partial sums of a.b (and, if c != NULL, of c.b)
__global__ __launch_bounds__(256) void k_dot2(int64_t n, const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const double* __restrict__ c,
                                              double* __restrict__ partial) {
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)RED_GRID * 256) {
    s0 += a[i] * b[i];
    if (c) s1 += c[i] * b[i];
  }
  s0 = block_sum256(s0);
  s1 = block_sum256(s1);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[RED_GRID + blockIdx.x] = s1;
  }
}

// sum `count` partials into sc[slot] (and a second set into sc[slot2])
__global__ __launch_bounds__(256) void k_reduce(int64_t count, const double* __restrict__ partial,
                                                double* __restrict__ sc, int slot, int slot2) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += partial[i];
  s = block_sum256(s);
  double s2 = 0.0;
  if (slot2 >= 0) {
    for (int64_t i = threadIdx.x; i < count; i += 256) s2 += partial[RED_GRID + i];
    s2 = block_sum256(s2);
  }
  if (threadIdx.x == 0) {
    sc[slot] = s;
    if (slot2 >= 0) sc[slot2] = s2;
  }
}

// scalar step of CG: mode 0: alpha = rz / pq; mode 1: beta (FR or PR), rz = rz_new
__global__ void k_cg_scalar(double* sc, int mode, int flexible) {
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    sc[SC_ALPHA] = sc[SC_RZ] / sc[SC_PQ];
  } else {
    double beta = flexible ? (sc[SC_RZNEW] - sc[SC_ROLDZ]) / sc[SC_RZ] : sc[SC_RZNEW] / sc[SC_RZ];
    sc[SC_BETA] = beta;
    sc[SC_RZ] = sc[SC_RZNEW];
  }
}

// p = z + beta p; on the first iteration p = z (p is not read: it may hold
// anything, and 0 * NaN would poison the direction)
__global__ __launch_bounds__(256) void k_cg_dir(int64_t n, const double* __restrict__ sc,
                                                const double* __restrict__ z,
                                                double* __restrict__ p, int first) {
  if (first) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
      p[i] = z[i];
    return;
  }
  const double beta = sc[SC_BETA];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = z[i] + beta * p[i];
}

void cg_update(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
               double* r_old, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_update, dim3(RED_GRID), dim3(256), 0, st, n, sc, p, q, x, r, r_old,
                     partial);
}
void dot2(int64_t n, const double* a, const double* b, const double* c, double* partial,
          hipStream_t st) {
  hipLaunchKernelGGL(k_dot2, dim3(RED_GRID), dim3(256), 0, st, n, a, b, c, partial);
}
void reduce(int64_t count, const double* partial, double* sc, int slot, int slot2, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, count, partial, sc, slot, slot2);
}
void cg_scalar(double* sc, int mode, int flexible, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(64), 0, st, sc, mode, flexible);
}
void cg_dir(int64_t n, const double* sc, const double* z, double* p, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_dir, dim3(grid_for(n)), dim3(256), 0, st, n, sc, z, p, first);
}
int red_grid() { return RED_GRID; }

// ---------------------------------------------------------------------------
// setup: local harmonic extension (eq. (sparseP))
// ---------------------------------------------------------------------------
// One 64-lane workgroup per block B (|B| <= 64): lane a gathers row a of
// A_BB and of the right-hand side A_B,: P_done (sequentially, so the sum
// order is fixed), the block is Cholesky-factored in LDS and every
// right-hand-side column is solved by one lane; P rows get -X.
__global__ __launch_bounds__(64) void k_ext_block(
    int64_t b0, const int64_t* __restrict__ bptr, const int32_t* __restrict__ bdofs,
    const int32_t* __restrict__ dof_stage, int stage, const int64_t* __restrict__ Aptr,
    const int32_t* __restrict__ Acol, const double* __restrict__ Aval,
    const int64_t* __restrict__ Pptr, const int32_t* __restrict__ Pcol, double* __restrict__ Pval,
    int smax, int ctile, int wide, int* __restrict__ flag, const double* __restrict__ Wl,
    const int8_t* __restrict__ accepted, const double* __restrict__ dsq) {
  extern __shared__ unsigned char lds_raw[];
  double* Abb = (double*)lds_raw;                 // smax * smax
  double* R = Abb + smax * smax;                   // smax * ctile
  int32_t* cols = (int32_t*)(R + smax * ctile);    // ctile
  int32_t* dofs = cols + ctile;                    // smax
  const int64_t blk = b0 + blockIdx.x;
  const int64_t d0 = bptr[blk];
  const int s = (int)(bptr[blk + 1] - d0);
  const int32_t first = bdofs[d0];
  const int64_t cbeg = Pptr[first];
  const int ctot = (int)(Pptr[first + 1] - cbeg);
  // this workgroup's tile of the block's P columns: [t0, t0 + c)
  const int t0 = (int)blockIdx.y * ctile;
  if (t0 >= ctot) return;   // the whole workgroup: this block has fewer tiles
  const int c = min(ctile, ctot - t0);
  const int64_t c0 = cbeg + t0;
  const int lane = threadIdx.x;
  for (int t = lane; t < c; t += 64) cols[t] = Pcol[c0 + t];
  for (int t = lane; t < s; t += 64) dofs[t] = bdofs[d0 + t];
  for (int t = lane; t < s * s; t += 64) Abb[t] = 0.0;
  for (int t = lane; t < s * c; t += 64) R[t] = 0.0;
  __syncthreads();
  const int32_t clo = cols[0], chi = cols[c - 1];
  // Right-hand side R = A_B,done P_done.  Every R entry sums its terms in the
  // order of A's row (one term per A entry at most, as a P row has distinct
  // columns), so both ways below give the same bits:
  // narrow P rows: lane i gathers row i of the block;
  // wide P rows (wide != 0): the rows one after the other, the 64 lanes over
  // the distinct columns of one P row at a time.
  auto gather_entry = [&](int i, int64_t q, int u0, int du) {
    const int32_t j = Acol[q];
    const double a = Aval[q];
    const int pos = lower_bound_i32(dofs, s, j);
    if (pos < s && dofs[pos] == j) {
      if (u0 == 0) Abb[i * s + pos] = a;
      return;
    }
    const int sj = dof_stage[j];
    if (sj >= 0 && sj >= stage) return;  // not extended yet
    double* Rr = R + i * c;
    for (int64_t u = Pptr[j] + u0; u < Pptr[j + 1]; u += du) {
      const int32_t pc = Pcol[u];
      if (pc < clo || pc > chi) continue;   // another tile's column
      const int cp = lower_bound_i32(cols, c, pc);
      if (cp < c && cols[cp] == pc) {
        Rr[cp] += a * Pval[u];
      } else {
        atomicExch(flag, 2);   // pattern mismatch (cannot happen for host-built patterns)
      }
    }
  };
  if (!wide) {
    if (lane < s)
      for (int64_t q = Aptr[dofs[lane]]; q < Aptr[dofs[lane] + 1]; ++q) gather_entry(lane, q, 0, 1);
  } else {
    for (int i = 0; i < s; ++i)
      for (int64_t q = Aptr[dofs[i]]; q < Aptr[dofs[i] + 1]; ++q) gather_entry(i, q, lane, 64);
  }
  __syncthreads();
  if (Wl && accepted[blk]) {
    // learned block: X = -D^{-1/2} W D^{-1/2} R with the accepted, refined
    // normalised inverse W (packed lower triangle)
    const double* w = Wl + blk * 36;
    const double* dq = dsq + blk * 8;
    for (int t = lane; t < c; t += 64) {
      double y[8];
      for (int i = 0; i < s; ++i) {
        double v = 0.0;
        for (int j = 0; j < s; ++j) {
          const double wij = i >= j ? w[i * (i + 1) / 2 + j] : w[j * (j + 1) / 2 + i];
          v += wij / dq[j] * R[j * c + t];
        }
        y[i] = v / dq[i];
      }
      for (int i = 0; i < s; ++i) Pval[Pptr[dofs[i]] + t0 + t] = -y[i];
    }
    return;
  }
  // Cholesky (lower) of Abb in place, lane i owns row i
  for (int k = 0; k < s; ++k) {
    if (lane == 0) {
      double a = Abb[k * s + k];
      if (!(a > 0.0)) {
        atomicExch(flag, 1);
        a = 1.0;
      }
      Abb[k * s + k] = sqrt(a);
    }
    __syncthreads();
    const double dk = Abb[k * s + k];
    if (lane > k && lane < s) Abb[lane * s + k] /= dk;
    __syncthreads();
    if (lane > k && lane < s)
      for (int j = k + 1; j <= lane; ++j) Abb[lane * s + j] -= Abb[lane * s + k] * Abb[j * s + k];
    __syncthreads();
  }
  // solve L L^T X = R column by column; write P = -X
  for (int t = lane; t < c; t += 64) {
    for (int i = 0; i < s; ++i) {
      double v = R[i * c + t];
      for (int j = 0; j < i; ++j) v -= Abb[i * s + j] * R[j * c + t];
      R[i * c + t] = v / Abb[i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {
      double v = R[i * c + t];
      for (int j = i + 1; j < s; ++j) v -= Abb[j * s + i] * R[j * c + t];
      R[i * c + t] = v / Abb[i * s + i];
    }
    for (int i = 0; i < s; ++i) Pval[Pptr[dofs[i]] + t0 + t] = -R[i * c + t];
  }
}

size_t ext_block_lds(int smax, int ctile) {
  return sizeof(double) * ((size_t)smax * smax + (size_t)smax * ctile) +
         sizeof(int32_t) * ((size_t)ctile + (size_t)smax);
}

// the widest column tile whose block fits 64 KiB of LDS (0 if none does)
int ext_block_tile(int smax) {
  const int64_t room = 65536 - (int64_t)sizeof(double) * smax * smax - (int64_t)sizeof(int32_t) * smax;
  const int64_t per = (int64_t)sizeof(double) * smax + (int64_t)sizeof(int32_t);
  return room > 0 ? (int)(room / per) : 0;
}

void ext_blocks(int64_t b0, int64_t nb, const int64_t* bptr, const int32_t* bdofs,
                const int32_t* dof_stage, int stage, const CsrDev<double>& A,
                const int64_t* Pptr, const int32_t* Pcol, double* Pval, int smax, int cmax,
                int prow_max, int* flag, hipStream_t st, const double* Wl,
                const int8_t* accepted, const double* dsq) {
  if (nb <= 0 || cmax <= 0) return;
  // columns in tiles of ctile (one tile when the widest block fits LDS whole;
  // HCURL_AMG_EXT_TILE caps the tile width)
  int ctile = std::min(cmax, ext_block_tile(smax));
  if (const char* e = std::getenv("HCURL_AMG_EXT_TILE")) ctile = std::max(1, std::min(ctile, std::atoi(e)));
  const int ntiles = (cmax + ctile - 1) / ctile;
  size_t lds = ext_block_lds(smax, ctile);
  // lanes over P's columns once the P rows of the done DoFs are wide enough
  // to keep 64 lanes busy (HCURL_AMG_EXT_WIDE=0/1 forces either way)
  int wide = prow_max > 64 ? 1 : 0;
  if (const char* e = std::getenv("HCURL_AMG_EXT_WIDE")) wide = e[0] == '1' ? 1 : 0;
  hipLaunchKernelGGL(k_ext_block, dim3((unsigned)nb, (unsigned)ntiles), dim3(64), lds, st, b0, bptr,
                     bdofs, dof_stage, stage, A.ptr, A.col, A.val, Pptr, Pcol, Pval, smax, ctile,
                     wide, flag, Wl, accepted, dsq);
}

// x_i = a pseudo-random value in [-1, 1) from a counter-based hash (SplitMix64)
__global__ void k_hash_fill(int64_t n, uint64_t seed, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}
// y += a x
__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
void hash_fill(int64_t n, uint64_t seed, double* x, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_hash_fill, dim3(grid_for(n)), dim3(256), 0, st, n, seed, x);
}
void axpy(int64_t n, double a, const double* x, double* y, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, st, n, a, x, y);
}

// P values from the exterior signs (interior entries start at 0)
__global__ void k_sign_to_val(int64_t n, const int8_t* __restrict__ s, double* __restrict__ v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (double)s[i];
}
void sign_to_val(int64_t n, const int8_t* s, double* v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_sign_to_val, dim3(grid_for(n)), dim3(256), 0, st, n, s, v);
}

// PT values by a precomputed permutation
__global__ void k_permute(int64_t n, const int64_t* __restrict__ perm, const double* __restrict__ a,
                          double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[perm[i]] = a[i];
}
void permute(int64_t n, const int64_t* perm, const double* a, double* b, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_permute, dim3(grid_for(n)), dim3(256), 0, st, n, perm, a, b);
}

// ---------------------------------------------------------------------------
// setup: sparse products C = X Y (row merge), used for A P and P^T (A P)
// ---------------------------------------------------------------------------
constexpr int HCAP = 8192;   // LDS hash slots of the symbolic passes (32 KiB)

// insert the columns of row i of X Y into an LDS hash; the 256 threads take
// the entries of X's row in turn and walk the matching rows of Y
__device__ void mm_insert(int64_t i, const int64_t* Xptr, const int32_t* Xcol, const int64_t* Yptr,
                          const int32_t* Ycol, int32_t* hash, int* count, int* overflow) {
  for (int64_t t = Xptr[i] + threadIdx.x; t < Xptr[i + 1]; t += blockDim.x) {
    const int32_t k = Xcol[t];
    for (int64_t u = Yptr[k]; u < Yptr[k + 1]; ++u) {
      if (*(volatile int*)overflow) return;   // the row goes to the wide passes anyway
      const int32_t J = Ycol[u];
      uint32_t h = ((uint32_t)J * 2654435761u) & (HCAP - 1);
      int probes = 0;
      while (true) {
        int32_t old = atomicCAS(&hash[h], -1, J);
        if (old == -1) {
          atomicAdd(count, 1);
          break;
        }
        if (old == J) break;
        h = (h + 1) & (HCAP - 1);
        if (++probes >= HCAP) {
          atomicExch(overflow, 1);
          break;
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mm_count(int64_t nrows, const int64_t* __restrict__ Xptr,
                                                  const int32_t* __restrict__ Xcol,
                                                  const int64_t* __restrict__ Yptr,
                                                  const int32_t* __restrict__ Ycol,
                                                  int64_t* __restrict__ cnt,
                                                  int* __restrict__ overflow, int wide_at) {
  __shared__ int32_t hash[HCAP];
  __shared__ int count;
  __shared__ int full;
  const int64_t i = blockIdx.x;
  for (int t = threadIdx.x; t < HCAP; t += blockDim.x) hash[t] = -1;
  if (threadIdx.x == 0) {
    count = 0;
    full = 0;
  }
  __syncthreads();
  mm_insert(i, Xptr, Xcol, Yptr, Ycol, hash, &count, &full);
  __syncthreads();
  // a row too wide for the hash passes (more than wide_at <= HCAP / 2
  // columns) is marked -1 and counted again by k_mm_count_wide
  if (threadIdx.x == 0) cnt[i] = (full || count > wide_at) ? -1 : count;
}

// sorted columns of row i (its length, from k_mm_count, is at most HCAP / 2)
__global__ __launch_bounds__(256) void k_mm_fill(int64_t nrows, const int64_t* __restrict__ Xptr,
                                                 const int32_t* __restrict__ Xcol,
                                                 const int64_t* __restrict__ Yptr,
                                                 const int32_t* __restrict__ Ycol,
                                                 const int64_t* __restrict__ Cptr,
                                                 int32_t* __restrict__ Ccol,
                                                 int* __restrict__ overflow, int wide_at) {
  __shared__ int32_t hash[HCAP];
  __shared__ int count;
  __shared__ int nfill;
  __shared__ int full;
  const int64_t i = blockIdx.x;
  if (Cptr[i + 1] - Cptr[i] > wide_at) return;   // wide row: k_mm_fill_wide
  for (int t = threadIdx.x; t < HCAP; t += blockDim.x) hash[t] = -1;
  if (threadIdx.x == 0) {
    count = 0;
    nfill = 0;
    full = 0;
  }
  __syncthreads();
  mm_insert(i, Xptr, Xcol, Yptr, Ycol, hash, &count, &full);
  __syncthreads();
  if (full) {   // cannot happen: the row was counted to fit
    if (threadIdx.x == 0) atomicExch(overflow, 1);
    return;
  }
  // gather the keys into registers, then compact them to the front
  int32_t keys[HCAP / 256];
  int nk = 0;
  for (int t = threadIdx.x; t < HCAP; t += blockDim.x)
    if (hash[t] >= 0) keys[nk++] = hash[t];
  __syncthreads();
  for (int t = threadIdx.x; t < HCAP; t += blockDim.x) hash[t] = 0x7fffffff;
  __syncthreads();
  for (int t = 0; t < nk; ++t) hash[atomicAdd(&nfill, 1)] = keys[t];
  __syncthreads();
  const int m = nfill;
  int P2 = 1;
  while (P2 < m) P2 <<= 1;
  // bitonic sort of hash[0 .. P2) (padding holds INT_MAX)
  for (int k = 2; k <= P2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < P2; q += blockDim.x) {
        int qj = q ^ j;
        if (qj > q) {
          int32_t a = hash[q], b = hash[qj];
          bool up = (q & k) == 0;
          if ((a > b) == up) {
            hash[q] = b;
            hash[qj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const int64_t o = Cptr[i];
  for (int t = threadIdx.x; t < m; t += blockDim.x) Ccol[o + t] = hash[t];
}

// numeric pass of row i: C[i,:] = sum_t X[i,t] Y[t,:] in the stored order of
// X's row; lanes own distinct columns of one Y row at a time, so every
// accumulator slot is updated in a fixed order (deterministic)
__global__ __launch_bounds__(64) void k_mm_vals(
    int64_t nrows, const int64_t* __restrict__ Xptr, const int32_t* __restrict__ Xcol,
    const double* __restrict__ Xval, const int64_t* __restrict__ Yptr,
    const int32_t* __restrict__ Ycol, const double* __restrict__ Yval,
    const int64_t* __restrict__ Cptr, const int32_t* __restrict__ Ccol, double* __restrict__ Cval,
    int mmax) {
  extern __shared__ unsigned char lds_raw[];
  double* acc = (double*)lds_raw;          // mmax
  int32_t* cols = (int32_t*)(acc + mmax);  // mmax
  const int64_t i = blockIdx.x;
  const int64_t o = Cptr[i];
  const int m = (int)(Cptr[i + 1] - o);
  if (m > mmax) return;   // wide row: k_mm_vals_wide
  const int lane = threadIdx.x;
  for (int t = lane; t < m; t += 64) {
    cols[t] = Ccol[o + t];
    acc[t] = 0.0;
  }
  __syncthreads();
  for (int64_t t = Xptr[i]; t < Xptr[i + 1]; ++t) {
    const int32_t k = Xcol[t];
    const double x = Xval[t];
    for (int64_t u = Yptr[k] + lane; u < Yptr[k + 1]; u += 64) {
      const int pos = lower_bound_i32(cols, m, Ycol[u]);
      if (pos < m && cols[pos] == Ycol[u]) acc[pos] += x * Yval[u];
    }
    __syncthreads();
  }
  for (int t = lane; t < m; t += 64) Cval[o + t] = acc[t];
}

// Wide rows (more distinct columns than the LDS hash holds): the row's
// column set is a bitset over the ncols columns of Y in LDS (set bits are
// order-free, so the result is deterministic), counted by popcount,
// listed in order by a scan, and addressed in the numeric pass by rank
// (prefix popcount), with the sums accumulated in place in C's row.
// (each wavefront takes X entries in turn, its lanes the entries of the Y row)
__device__ void mm_mark_wide(int64_t i, const int64_t* Xptr, const int32_t* Xcol,
                             const int64_t* Yptr, const int32_t* Ycol, uint32_t* bits) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwave = blockDim.x / 64;
  for (int64_t t = Xptr[i] + wave; t < Xptr[i + 1]; t += nwave) {
    const int32_t k = Xcol[t];
    for (int64_t u = Yptr[k] + lane; u < Yptr[k + 1]; u += 64) {
      const int32_t J = Ycol[u];
      atomicOr(&bits[J >> 5], 1u << (J & 31));
    }
  }
}

__device__ int block_exclusive_scan256(int v, int* tmp, int* total) {
  // Hillis-Steele over 256 threads in LDS
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int a = threadIdx.x >= off ? tmp[threadIdx.x - off] : 0;
    __syncthreads();
    tmp[threadIdx.x] += a;
    __syncthreads();
  }
  const int incl = tmp[threadIdx.x];
  if (total) *total = tmp[255];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_mm_count_wide(const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ Xptr,
                                                       const int32_t* __restrict__ Xcol,
                                                       const int64_t* __restrict__ Yptr,
                                                       const int32_t* __restrict__ Ycol, int nwords,
                                                       int64_t* __restrict__ cnt) {
  extern __shared__ uint32_t bits[];   // nwords
  __shared__ int tmp[256];
  const int64_t i = rows[blockIdx.x];
  for (int w = threadIdx.x; w < nwords; w += 256) bits[w] = 0u;
  __syncthreads();
  mm_mark_wide(i, Xptr, Xcol, Yptr, Ycol, bits);
  __syncthreads();
  int c = 0;
  for (int w = threadIdx.x; w < nwords; w += 256) c += __popc(bits[w]);
  int total = 0;
  block_exclusive_scan256(c, tmp, &total);
  if (threadIdx.x == 0) cnt[i] = total;
}

__global__ __launch_bounds__(256) void k_mm_fill_wide(const int32_t* __restrict__ rows,
                                                      const int64_t* __restrict__ Xptr,
                                                      const int32_t* __restrict__ Xcol,
                                                      const int64_t* __restrict__ Yptr,
                                                      const int32_t* __restrict__ Ycol, int nwords,
                                                      const int64_t* __restrict__ Cptr,
                                                      int32_t* __restrict__ Ccol) {
  extern __shared__ uint32_t bits[];   // nwords
  __shared__ int tmp[256];
  const int64_t i = rows[blockIdx.x];
  for (int w = threadIdx.x; w < nwords; w += 256) bits[w] = 0u;
  __syncthreads();
  mm_mark_wide(i, Xptr, Xcol, Yptr, Ycol, bits);
  __syncthreads();
  // thread t lists the set bits of words [w0, w1) in order
  const int per = (nwords + 255) / 256;
  const int w0 = min(nwords, (int)threadIdx.x * per), w1 = min(nwords, w0 + per);
  int c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
  int pos = block_exclusive_scan256(c, tmp, nullptr);
  int32_t* out = Ccol + Cptr[i];
  for (int w = w0; w < w1; ++w) {
    uint32_t b = bits[w];
    while (b) {
      const int lsb = __ffs(b) - 1;
      out[pos++] = w * 32 + lsb;
      b &= b - 1;
    }
  }
}

constexpr int MM_WIDE_VALS_WG = 1024;
__global__ __launch_bounds__(MM_WIDE_VALS_WG) void k_mm_vals_wide(
    const int32_t* __restrict__ rows, const int64_t* __restrict__ Xptr,
    const int32_t* __restrict__ Xcol, const double* __restrict__ Xval,
    const int64_t* __restrict__ Yptr, const int32_t* __restrict__ Ycol,
    const double* __restrict__ Yval, int nwords, const int64_t* __restrict__ Cptr,
    const int32_t* __restrict__ Ccol, double* __restrict__ Cval) {
  extern __shared__ uint32_t bits[];   // nwords bits, then nwords prefix counts
  int32_t* rank0 = (int32_t*)(bits + nwords);
  const int64_t i = rows[blockIdx.x];
  const int64_t o = Cptr[i];
  const int m = (int)(Cptr[i + 1] - o);
  const int lane = threadIdx.x;
  for (int w = lane; w < nwords; w += MM_WIDE_VALS_WG) bits[w] = 0u;
  __syncthreads();
  for (int t = lane; t < m; t += MM_WIDE_VALS_WG) {
    const int32_t J = Ccol[o + t];
    atomicOr(&bits[J >> 5], 1u << (J & 31));
    Cval[o + t] = 0.0;
  }
  __syncthreads();
  if (lane == 0) {
    int run = 0;
    for (int w = 0; w < nwords; ++w) {
      rank0[w] = run;
      run += __popc(bits[w]);
    }
  }
  __syncthreads();
  // same order as k_mm_vals: X's entries in stored order, threads over the
  // distinct columns of one Y row, so each C entry is summed in a fixed
  // order (the barrier after each X entry orders the updates of C's row)
  for (int64_t t = Xptr[i]; t < Xptr[i + 1]; ++t) {
    const int32_t k = Xcol[t];
    const double x = Xval[t];
    for (int64_t u = Yptr[k] + lane; u < Yptr[k + 1]; u += MM_WIDE_VALS_WG) {
      const int32_t J = Ycol[u];
      const uint32_t w = bits[J >> 5];
      if (w & (1u << (J & 31))) {
        const int pos = rank0[J >> 5] + __popc(w & ((1u << (J & 31)) - 1u));
        Cval[o + pos] += x * Yval[u];
      }
    }
    __syncthreads();
  }
}

size_t mm_wide_lds(int64_t ncols) { return (size_t)((ncols + 31) / 32) * 2 * sizeof(uint32_t); }

void mm_count_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const CsrPat& Y, int64_t ncols,
                   int64_t* cnt, hipStream_t st) {
  if (nw <= 0) return;
  const int nwords = (int)((ncols + 31) / 32);
  hipLaunchKernelGGL(k_mm_count_wide, dim3((unsigned)nw), dim3(256), nwords * sizeof(uint32_t), st,
                     rows, X.ptr, X.col, Y.ptr, Y.col, nwords, cnt);
}
void mm_fill_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const CsrPat& Y, int64_t ncols,
                  const int64_t* Cptr, int32_t* Ccol, hipStream_t st) {
  if (nw <= 0) return;
  const int nwords = (int)((ncols + 31) / 32);
  hipLaunchKernelGGL(k_mm_fill_wide, dim3((unsigned)nw), dim3(256), nwords * sizeof(uint32_t), st,
                     rows, X.ptr, X.col, Y.ptr, Y.col, nwords, Cptr, Ccol);
}
void mm_vals_wide(int64_t nw, const int32_t* rows, const CsrPat& X, const double* Xval,
                  const CsrPat& Y, const double* Yval, int64_t ncols, const int64_t* Cptr,
                  const int32_t* Ccol, double* Cval, hipStream_t st) {
  if (nw <= 0) return;
  const int nwords = (int)((ncols + 31) / 32);
  hipLaunchKernelGGL(k_mm_vals_wide, dim3((unsigned)nw), dim3(MM_WIDE_VALS_WG), mm_wide_lds(ncols), st, rows,
                     X.ptr, X.col, Xval, Y.ptr, Y.col, Yval, nwords, Cptr, Ccol, Cval);
}

// rows with more columns than this take the wide passes (HCAP / 2, or less
// with HCURL_AMG_MM_WIDE, which also caps the numeric pass's LDS rows)
int mm_wide_at() {
  int w = HCAP / 2;
  if (const char* e = std::getenv("HCURL_AMG_MM_WIDE")) w = std::max(1, std::min(w, std::atoi(e)));
  return w;
}
void mm_count(int64_t nrows, const CsrPat& X, const CsrPat& Y, int64_t* cnt, int* overflow,
              hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_mm_count, dim3((unsigned)nrows), dim3(256), 0, st, nrows, X.ptr, X.col,
                       Y.ptr, Y.col, cnt, overflow, mm_wide_at());
}
void mm_fill(int64_t nrows, const CsrPat& X, const CsrPat& Y, const int64_t* Cptr, int32_t* Ccol,
             int* overflow, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_mm_fill, dim3((unsigned)nrows), dim3(256), 0, st, nrows, X.ptr, X.col,
                       Y.ptr, Y.col, Cptr, Ccol, overflow, mm_wide_at());
}
void mm_vals(int64_t nrows, const CsrPat& X, const double* Xval, const CsrPat& Y,
             const double* Yval, const int64_t* Cptr, const int32_t* Ccol, double* Cval, int mmax,
             hipStream_t st) {
  if (nrows <= 0) return;
  size_t lds = (size_t)std::max(mmax, 1) * (sizeof(double) + sizeof(int32_t));
  hipLaunchKernelGGL(k_mm_vals, dim3((unsigned)nrows), dim3(64), lds, st, nrows, X.ptr, X.col,
                     Xval, Y.ptr, Y.col, Yval, Cptr, Ccol, Cval, mmax);
}
int mm_hash_cap() { return HCAP; }

// ---------------------------------------------------------------------------
// setup: smoother factors and l1 diagonal
// ---------------------------------------------------------------------------
constexpr int MAXS = 32;

// one thread per block: gather the lower triangle of A_BB, factor, store packed
__global__ void k_star_chol(int64_t nb, const int64_t* __restrict__ sb_ptr,
                            const int32_t* __restrict__ sb_dofs, const int64_t* __restrict__ fac_off,
                            const int64_t* __restrict__ Aptr, const int32_t* __restrict__ Acol,
                            const double* __restrict__ Aval, double* __restrict__ fac,
                            int* __restrict__ flag) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t d0 = sb_ptr[b];
  const int s = (int)(sb_ptr[b + 1] - d0);
  double* L = fac + fac_off[b];
  for (int i = 0; i < s; ++i) {
    const int32_t e = sb_dofs[d0 + i];
    const int64_t q0 = Aptr[e];
    const int len = (int)(Aptr[e + 1] - q0);
    for (int j = 0; j <= i; ++j) {
      const int32_t d = sb_dofs[d0 + j];
      const int pos = lower_bound_i32(Acol + q0, len, d);
      L[i * (i + 1) / 2 + j] = (pos < len && Acol[q0 + pos] == d) ? Aval[q0 + pos] : 0.0;
    }
  }
  for (int j = 0; j < s; ++j) {
    double a = L[j * (j + 1) / 2 + j];
    for (int k = 0; k < j; ++k) a -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
    if (!(a > 0.0)) {
      atomicExch(flag, 1);
      a = 1.0;
    }
    const double d = sqrt(a);
    L[j * (j + 1) / 2 + j] = d;
    for (int i = j + 1; i < s; ++i) {
      double v = L[i * (i + 1) / 2 + j];
      for (int k = 0; k < j; ++k) v -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = v / d;
    }
  }
}

void star_chol(int64_t nb, const int64_t* sb_ptr, const int32_t* sb_dofs, const int64_t* fac_off,
               const CsrDev<double>& A, double* fac, int* flag, hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_star_chol, dim3((unsigned)((nb + 127) / 128)), dim3(128), 0, st, nb,
                       sb_ptr, sb_dofs, fac_off, A.ptr, A.col, A.val, fac, flag);
}

// Symmetric inverse of each block from its Cholesky factor, packed like the
// factor (lower half): thread r solves L L^T z = e_j for its row r, the j-th
// row of block row_blk[r], and writes entries (i >= j) of column j.
__global__ void k_star_inv(int64_t nrows, const int32_t* __restrict__ row_blk,
                           const int64_t* __restrict__ sb_ptr, const int64_t* __restrict__ fac_off,
                           const double* __restrict__ fac, double* __restrict__ binv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int b = row_blk[r];
  const int64_t p0 = sb_ptr[b];
  const int s = (int)(sb_ptr[b + 1] - p0);
  const int j = (int)(r - p0);
  const double* L = fac + fac_off[b];
  double* B = binv + fac_off[b];
  double y[32];
  for (int i = 0; i < s; ++i) {
    double a = i == j ? 1.0 : 0.0;
    for (int q = 0; q < i; ++q) a -= L[i * (i + 1) / 2 + q] * y[q];
    y[i] = a / L[i * (i + 1) / 2 + i];
  }
  for (int i = s - 1; i >= 0; --i) {
    double a = y[i];
    for (int q = i + 1; q < s; ++q) a -= L[q * (q + 1) / 2 + i] * y[q];
    y[i] = a / L[i * (i + 1) / 2 + i];
  }
  for (int i = j; i < s; ++i) B[i * (i + 1) / 2 + j] = y[i];
}

// Each star row's row of its block's inverse, PANEL_SMAX wide, zero beyond
// the block (the panel form's operand layout).
__global__ void k_pad_inv(int64_t nrows, const int32_t* __restrict__ row_blk,
                          const int64_t* __restrict__ sb_ptr, const int64_t* __restrict__ fac_off,
                          const double* __restrict__ binv, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int b = row_blk[r];
  const int s = (int)(sb_ptr[b + 1] - sb_ptr[b]);
  const int i = (int)(r - sb_ptr[b]);
  const double* B = binv + fac_off[b];
  for (int j = 0; j < PANEL_SMAX; ++j) {
    const int hi = i > j ? i : j, lo = i > j ? j : i;
    out[r * PANEL_SMAX + j] = j < s ? B[hi * (hi + 1) / 2 + lo] : 0.0;
  }
}

void pad_inv(int64_t nrows, const int32_t* row_blk, const int64_t* sb_ptr, const int64_t* fac_off,
             const double* binv, double* out, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_pad_inv, dim3((unsigned)((nrows + 127) / 128)), dim3(128), 0, st, nrows,
                       row_blk, sb_ptr, fac_off, binv, out);
}

void star_inv(int64_t nrows, const int32_t* row_blk, const int64_t* sb_ptr, const int64_t* fac_off,
              const double* fac, double* binv, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_star_inv, dim3((unsigned)((nrows + 127) / 128)), dim3(128), 0, st, nrows,
                       row_blk, sb_ptr, fac_off, fac, binv);
}

__global__ void k_l1inv(int64_t n, const int64_t* __restrict__ ptr, const double* __restrict__ val,
                        double* __restrict__ dinv) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) s += fabs(val[q]);
    dinv[i] = 1.0 / s;
  }
}
void l1inv(const CsrDev<double>& A, double* dinv, hipStream_t st) {
  if (A.n > 0)
    hipLaunchKernelGGL(k_l1inv, dim3(grid_for(A.n)), dim3(256), 0, st, A.n, A.ptr, A.val, dinv);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
template void spmv<double>(const CsrDev<double>&, const double*, double*, hipStream_t);
template void spmv<float>(const CsrDev<float>&, const float*, float*, hipStream_t);
template void residual<double>(const CsrDev<double>&, const double*, const double*, double*, hipStream_t);
template void residual<float>(const CsrDev<float>&, const float*, const float*, float*, hipStream_t);
template void jacobi<double>(const CsrDev<double>&, const double*, const double*, const double*, double*, hipStream_t);
template void jacobi<float>(const CsrDev<float>&, const float*, const float*, const float*, float*, hipStream_t);
template void spmv_add<double>(const CsrDev<double>&, const double*, double*, hipStream_t);
template void spmv_add<float>(const CsrDev<float>&, const float*, float*, hipStream_t);
template void schwarz_colour<double>(const SmootherDev<double>&, int, const double*, double*, hipStream_t);
template void schwarz_colour<float>(const SmootherDev<float>&, int, const float*, float*, hipStream_t);
template void schwarz_sweep_small<double>(const SmootherDev<double>&, int, const double*, double*, hipStream_t);
template void schwarz_sweep_small<float>(const SmootherDev<float>&, int, const float*, float*, hipStream_t);
template void schwarz_pipe<double>(const SmootherDev<double>&, int, const double*, double*, hipStream_t);
template void schwarz_pipe<float>(const SmootherDev<float>&, int, const float*, float*, hipStream_t);
template void panel_sweep<double>(int, int, int, const int32_t*, const int64_t*, const int32_t*,
                                  const int64_t*, const double*, const double*, const double*,
                                  const double*, const int64_t*, const int64_t*, const int32_t*,
                                  const int32_t*, double*, double*, double*, int*, int*, int,
                                  hipStream_t);
template void panel_sweep<float>(int, int, int, const int32_t*, const int64_t*, const int32_t*,
                                 const int64_t*, const float*, const float*, const float*,
                                 const float*, const int64_t*, const int64_t*, const int32_t*,
                                 const int32_t*, float*, float*, float*, int*, int*, int,
                                 hipStream_t);
template void panel_slices<double>(int, int64_t, const int32_t*, const int64_t*, const int32_t*,
                                   const double*, const int64_t*, const int64_t*, double*, double*,
                                   hipStream_t);
template bool dense_sweep_ok<double>(int, int);
template bool dense_sweep_ok<float>(int, int);
template void dense_sweep<double>(int, int, int, int, const int64_t*, const int32_t*, const int64_t*,
                                  const double*, const double*, const double*, double*, hipStream_t);
template void dense_sweep<float>(int, int, int, int, const int64_t*, const int32_t*, const int64_t*,
                                 const float*, const float*, const float*, float*, hipStream_t);
template void dense_solve<double>(int, const double*, const double*, double*, double*, hipStream_t);
template void dense_solve<float>(int, const double*, const float*, float*, double*, hipStream_t);
template void fill<double>(int64_t, double, double*, hipStream_t);
template void fill<float>(int64_t, float, float*, hipStream_t);
template void cast<double, float>(int64_t, const double*, float*, hipStream_t);
template void cast<float, double>(int64_t, const float*, double*, hipStream_t);

}  // namespace hamg

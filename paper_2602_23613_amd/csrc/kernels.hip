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

// A dispatch counts its work-items in 32 bits.  Launches whose workgroup
// count grows with the rows (one workgroup per row, block or column) go out
// in batches of at most MAX_WG_PER_LAUNCH workgroups (2^30 work-items at 256
// threads), each told the id of its first workgroup.  HCURL_AMG_MAX_WG
// lowers the batch size, so that small problems exercise the batching.
constexpr int64_t MAX_WG_PER_LAUNCH = int64_t(1) << 22;
static int64_t wg_per_launch() {
  static const int64_t v = [] {
    int64_t w = MAX_WG_PER_LAUNCH;
    if (const char* e = std::getenv("HCURL_AMG_MAX_WG"))
      w = std::max<int64_t>(1, std::min<int64_t>(w, std::atoll(e)));
    return w;
  }();
  return v;
}
template <class F>
static void in_batches(int64_t nwg, F launch) {
  const int64_t step = wg_per_launch();
  for (int64_t w0 = 0; w0 < nwg; w0 += step) launch(w0, (unsigned)std::min(step, nwg - w0));
}

// ---------------------------------------------------------------------------
// SpMV family
// ---------------------------------------------------------------------------
enum { EPI_Y = 0, EPI_RES = 1, EPI_JAC = 2, EPI_ADD = 3, EPI_DOT = 4 };

template <class T, int LPR, int EPI>
__global__ __launch_bounds__(256) void k_spmv(int64_t wg0, int64_t n, const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ x,
                                              const T* __restrict__ b, const T* __restrict__ dinv,
                                              T* __restrict__ y, double* __restrict__ partial) {
  constexpr int RPB = 256 / LPR;
  const int lane = threadIdx.x % LPR;
  const int grp = threadIdx.x / LPR;
  const int64_t wg = wg0 + blockIdx.x;
  const int64_t row = wg * RPB + grp;
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
    if (threadIdx.x == 0) partial[wg] = red[0];
  }
}

template <class T, int EPI>
static void spmv_lpr(int lpr, hipStream_t st, int64_t n, const int64_t* ptr, const int32_t* col,
                     const T* val, const T* x, const T* b, const T* dinv, T* y, double* partial) {
  if (n <= 0) return;
#define LAUNCH_SPMV(L)                                                                        \
  {                                                                                           \
    int64_t grid = (n + (256 / L) - 1) / (256 / L);                                           \
    in_batches(grid, [&](int64_t w0, unsigned g) {                                            \
      hipLaunchKernelGGL((k_spmv<T, L, EPI>), dim3(g), dim3(256), 0, st, w0, n, ptr, col, val, \
                         x, b, dinv, y, partial);                                             \
    });                                                                                       \
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

// everything of a chunk but its (column, value) pairs
template <class T, int LPR, int WGS, int U>
__device__ __forceinline__ void chunk_load_head(bool act, int c, int tid, const SmootherArgs<T>& D,
                                                ChunkRegs<T, LPR, WGS, U>& R) {
  constexpr int FPT = ChunkRegs<T, LPR, WGS, U>::FPT;
  constexpr int RPB = WGS / LPR;
  R.blk0 = R.nblk = R.r0 = R.nrows = R.nf = 0;
  R.f0 = 0;
  const int grp = tid / LPR, lane = tid % LPR;
  R.q0 = R.q1 = 0;
  R.rdof = R.mydof = 0;
  R.bp = R.bs = R.bfo = 0;
  if (act) {
    // everything below is indexed by the chunk and the thread alone
    R.r0 = D.ck_row0[c];
    R.nrows = D.ck_row0[c + 1] - R.r0;
    R.f0 = D.ck_fac0[c];
    R.nf = (int)(D.ck_fac0[c + 1] - R.f0);
    const int64_t* cq = D.ck_q + (int64_t)c * (RPB + 1);
    R.q0 = cq[grp];
    R.q1 = cq[grp + 1];
    if (lane == 0) R.rdof = D.ck_row[(int64_t)c * RPB + grp].x;
    if (tid < RPB) {
      const int4 info = D.ck_row[(int64_t)c * RPB + tid];
      R.mydof = info.x;
      R.bp = info.y;
      R.bs = info.z;
      R.bfo = info.w;
    }
  }
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int t = tid + k * WGS;
    R.fv[k] = t < R.nf ? D.binv[R.f0 + t] : T(0);
  }
}

// the first U (column, value) pairs of every lane of the chunk's rows
template <class T, int LPR, int WGS, int U>
__device__ __forceinline__ void chunk_load_pairs(int tid, const SmootherArgs<T>& D,
                                                 ChunkRegs<T, LPR, WGS, U>& R) {
  const int lane = tid % LPR;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t q = R.q0 + lane + (int64_t)u * LPR;
    const bool in = q < R.q1;
    R.c[u] = in ? D.scol[q] : -1;
    R.v[u] = in ? D.sval[q] : T(0);
  }
}

template <class T, int LPR, int WGS, int U>
__device__ __forceinline__ void chunk_load(bool act, int c, int tid, const SmootherArgs<T>& D,
                                           ChunkRegs<T, LPR, WGS, U>& R) {
  chunk_load_head<T, LPR, WGS, U>(act, c, tid, D, R);
  chunk_load_pairs<T, LPR, WGS, U>(tid, D, R);
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
template <class T, int LPR, int U>
__global__ __launch_bounds__(1024) void k_schwarz_pipe(SmootherArgs<T> D, int backward,
                                                       const T* b, T* x) {
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
    in_batches(c1 - c0, [&](int64_t w0, unsigned g) {                                            \
      hipLaunchKernelGGL((k_schwarz<T, L, W>), dim3(g), dim3(W), 0, st, D, (int)(c0 + w0), b, x); \
    });                                                                                          \
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
#define LAUNCH_PIPE(L, U)                                                                        \
  if (S.lpr == L && S.pipe_u == U) {                                                             \
    hipLaunchKernelGGL((k_schwarz_pipe<T, L, U>), dim3(S.pipe_grid), dim3(1024), 0, st, D,        \
                       backward, b, x);                                                          \
    return;                                                                                      \
  }
  LAUNCH_PIPE(8, 8) LAUNCH_PIPE(16, 8) LAUNCH_PIPE(32, 8) LAUNCH_PIPE(16, 16) LAUNCH_PIPE(32, 16)
  LAUNCH_PIPE(64, 16) LAUNCH_PIPE(128, 16) LAUNCH_PIPE(256, 16)
#undef LAUNCH_PIPE
}

static unsigned grid_for(int64_t n);

// slot i of chunk c is star row r0 + i (r0 = ck_row0[c]) while that is below
// the next chunk's first row; the entry range of a slot past the rows is empty
__global__ void k_chunk_tables(int64_t nchunks, int rpb, const int32_t* __restrict__ ck_row0,
                               const int64_t* __restrict__ ck_fac0, const int64_t* __restrict__ srow_ptr,
                               const int32_t* __restrict__ sb_dofs, const int32_t* __restrict__ row_blk,
                               const int64_t* __restrict__ sb_ptr, const int64_t* __restrict__ fac_off,
                               int64_t* __restrict__ ck_q, int4* __restrict__ ck_row) {
  const int64_t total = nchunks * (int64_t)(rpb + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / (rpb + 1);
    const int i = (int)(t % (rpb + 1));
    const int64_t r0 = ck_row0[c], r1 = ck_row0[c + 1];
    const int64_t r = r0 + i;
    ck_q[t] = srow_ptr[r < r1 ? r : r1];
    if (i < rpb) {
      int4 info = make_int4(0, 0, 0, 0);
      if (r < r1) {
        const int32_t b = row_blk[r];
        info.x = sb_dofs[r];
        info.y = (int)(sb_ptr[b] - r0);
        info.z = (int)(sb_ptr[b + 1] - sb_ptr[b]);
        info.w = (int)(fac_off[b] - ck_fac0[c]);
      }
      ck_row[c * rpb + i] = info;
    }
  }
}
void chunk_tables(int64_t nchunks, int rpb, const int32_t* ck_row0, const int64_t* ck_fac0,
                  const int64_t* srow_ptr, const int32_t* sb_dofs, const int32_t* row_blk,
                  const int64_t* sb_ptr, const int64_t* fac_off, int64_t* ck_q, int4* ck_row,
                  hipStream_t st) {
  if (nchunks > 0)
    hipLaunchKernelGGL(k_chunk_tables, dim3(grid_for(nchunks * (int64_t)(rpb + 1))), dim3(256), 0, st,
                       nchunks, rpb, ck_row0, ck_fac0, srow_ptr, sb_dofs, row_blk, sb_ptr, fac_off, ck_q,
                       ck_row);
}

// values of the smoother's row copy: star row r is row sb_dofs[r] of A
__global__ void k_star_rows(int64_t nrows, const int32_t* __restrict__ sb_dofs,
                            const int64_t* __restrict__ Aptr, const double* __restrict__ Aval,
                            const int64_t* __restrict__ srow_ptr, double* __restrict__ sval) {
  const int lane = threadIdx.x % 32;
  for (int64_t r = (int64_t)blockIdx.x * 8 + threadIdx.x / 32; r < nrows; r += (int64_t)gridDim.x * 8) {
    const int64_t a0 = Aptr[sb_dofs[r]];
    const int64_t s0 = srow_ptr[r], len = srow_ptr[r + 1] - s0;
    for (int64_t q = lane; q < len; q += 32) sval[s0 + q] = Aval[a0 + q];
  }
}
// the column ids of the same copy (once per pattern)
__global__ void k_star_cols(int64_t nrows, const int32_t* __restrict__ sb_dofs,
                            const int64_t* __restrict__ Aptr, const int32_t* __restrict__ Acol,
                            const int64_t* __restrict__ srow_ptr, int32_t* __restrict__ scol) {
  const int lane = threadIdx.x % 32;
  for (int64_t r = (int64_t)blockIdx.x * 8 + threadIdx.x / 32; r < nrows; r += (int64_t)gridDim.x * 8) {
    const int64_t a0 = Aptr[sb_dofs[r]];
    const int64_t s0 = srow_ptr[r], len = srow_ptr[r + 1] - s0;
    for (int64_t q = lane; q < len; q += 32) scol[s0 + q] = Acol[a0 + q];
  }
}
void star_cols(int64_t nrows, const int32_t* sb_dofs, const int64_t* Aptr, const int32_t* Acol,
               const int64_t* srow_ptr, int32_t* scol, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_star_cols, dim3((unsigned)std::min<int64_t>((nrows + 7) / 8, MAX_WG_PER_LAUNCH)), dim3(256), 0, st, nrows,
                       sb_dofs, Aptr, Acol, srow_ptr, scol);
}
void star_rows(int64_t nrows, const int32_t* sb_dofs, const int64_t* Aptr, const double* Aval,
               const int64_t* srow_ptr, double* sval, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_star_rows, dim3((unsigned)std::min<int64_t>((nrows + 7) / 8, MAX_WG_PER_LAUNCH)), dim3(256), 0, st, nrows,
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
// a DoF in two blocks of one group has two slots).
//
// Workgroup 0 (the chain) takes the groups in turn.  Its first wavefront
// holds slot k of the current group in lane k, with the group's slice
// A(D_g, D_g), the slots' rows of their block inverses and the residual
// entries in LDS, and for each block B in sweep order forms
// d = A_BB^{-1} r_B and updates the residual of every slot of the group.
// A run of consecutive blocks of one colour is one step (such blocks share
// no DoF and no entry of A).  It then publishes d and the group's residual
// entries and raises the group's flag.  Meanwhile its other three
// wavefronts load the next group (padded per-group tables, so every
// address follows from the group index alone) and the next group's
// residual entries, which are complete once the tiles have applied every
// group up to the one before the current, and stage all of it in the other
// half of double-buffered LDS tables; after the flag they only form the
// correction A(D_next, D_g) d.
//
// The other workgroups own tiles of PANEL_TROWS rows (two threads per row,
// 32 slots each) and apply each group's update r_i -= sum_k A(i, dof_k) d_k
// to their rows from a column-major dense copy of A, and x_i += d for each
// slot that holds DoF i.  Exactly-once rule for the update of group h on
// row i: the chain applies it when i is in D_h (inside the group) or in the
// next group D_h' (the correction it carries to h'), the tiles otherwise.
// A DoF in D_g that was also in the group before takes its residual from
// the chain's own final value of that slot.  The result is the
// multiplicative Schwarz sweep in residual-update form (only the rounding
// differs from the row form).
//
// Shared data (r, the published d) use agent-coherent accesses; a stored
// value is complete (memory counter drained) before its flag or counter is
// raised.  Every wait is bounded as in the pipelined sweep.  All workgroups
// of the grid must be able to run at once: 1 + n / PANEL_TROWS <= 129
// workgroups of 256 threads (n <= PANEL_NMAX), each holding more than half
// a CU's LDS, so one per CU of the 256, on an otherwise idle device.
constexpr int PANEL_SLOTS = PANEL_GROUP_SLOTS;
constexpr int PANEL_ELEMS = PANEL_SLOTS * PANEL_SLOTS;
constexpr int PANEL_TROWS = 128;
constexpr int PANEL_NMAX = 16384;
static_assert((long long)PANEL_NMAX * PANEL_NMAX < (1LL << 31), "dense-copy offsets in 32 bits");
constexpr int PANEL_SMAX = PANEL_ROW_WIDTH;

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

// fixed pairwise tree over SB values
template <class T, int SB>
__device__ __forceinline__ T tree_sum(T (&v)[SB]) {
#pragma unroll
  for (int w = SB / 2; w > 0; w /= 2)
#pragma unroll
    for (int j = 0; j < w; ++j) v[j] = v[j] + v[j + w];
  return v[0];
}

// Lane values shared through LDS inside the chain's wavefront: LDS
// operations of one wavefront are performed in order, so the fences only
// keep the compiler from reordering them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One block B (slots p .. p+s-1, s <= SB) of the chain, in one wavefront
// (lane k = slot k): the lanes of B form d_k = sum_j (A_BB^{-1})_{k-p, j}
// r_{p+j}, then every slot's residual drops by sum_j A(slot, p+j) d_j.
// br holds this lane's row of its block's inverse (zero beyond the block;
// meaningful for the lanes of B only).  The slice columns are read before
// the chain needs them; r_B comes through the scalar unit and d_B through
// LDS (dsh: d on the lanes of B, zero elsewhere and in PANEL_SMAX entries of
// padding), all reads independent of each other; each sum is a fixed
// pairwise tree, so the dependent chain is two tree depths instead of 2 s
// multiply-adds.  The slice is zero past the group's slots, with PANEL_SMAX
// rows of zero padding, so the step needs no masks and no branches.
template <class T, int SB>
__device__ __forceinline__ void panel_step(int k, int p, int s, const T (&br)[PANEL_SMAX],
                                           const T* Aloc, T* dsh, T& rk, T& dk) {
  T a[SB], v[SB];
  const T* acol = Aloc + p * PANEL_SLOTS + k;
#pragma unroll
  for (int j = 0; j < SB; ++j) a[j] = acol[j * PANEL_SLOTS];
#pragma unroll
  for (int j = 0; j < SB; ++j) v[j] = br[j] * lane_bcast(rk, (p + j) & (PANEL_SLOTS - 1));
  const T d = tree_sum<T, SB>(v);
  const bool inb = k >= p && k < p + s;
  if (inb) dk = d;
  dsh[k] = inb ? d : T(0);
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < SB; ++j) v[j] = a[j] * dsh[p + j];
  rk -= tree_sum<T, SB>(v);
}

// A run of consecutive blocks of one colour (slots P0 .. P1-1) in one step:
// such blocks share no DoF and no entry of A, so each block's d comes from
// the residual before the run, as it would after its predecessors in the
// run.  Lane k forms d_k from its own block (first slot pk; r through LDS,
// rsh, zero past the slots), then every slot's residual drops by
// sum_l A(slot, l) d_l over the run (d zero outside it), summed in trees of
// sixteen.
template <class T>
__device__ __forceinline__ void panel_run(int k, int P0, int P1, int pk, const T (&br)[PANEL_SMAX],
                                          const T* Aloc, T* rsh, T* dsh, T& rk, T& dk) {
  T v[PANEL_SMAX];
  rsh[k] = rk;
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < PANEL_SMAX; ++j) v[j] = br[j] * rsh[pk + j];
  const T d = tree_sum<T, PANEL_SMAX>(v);
  const bool inr = k >= P0 && k < P1;
  if (inr) dk = d;
  dsh[k] = inr ? d : T(0);
  wave_lds_sync();
  T acc = 0;
  for (int l0 = P0; l0 < P1; l0 += PANEL_SMAX) {
    const T* acol = Aloc + l0 * PANEL_SLOTS + k;
#pragma unroll
    for (int j = 0; j < PANEL_SMAX; ++j) v[j] = acol[j * PANEL_SLOTS] * dsh[l0 + j];
    acc += tree_sum<T, PANEL_SMAX>(v);
  }
  rk -= acc;
}

// entries of a 64 x 64 group matrix that one of the 192 staging threads
// holds: e = t + 192 j
constexpr int PANEL_STAGE = 192;
constexpr int PANEL_PER = (PANEL_ELEMS + PANEL_STAGE - 1) / PANEL_STAGE;                   // 22
constexpr int PANEL_FPER = (PANEL_SLOTS * PANEL_SMAX + PANEL_STAGE - 1) / PANEL_STAGE;     // 6
// all but the last entry of each thread fall inside the matrix
static_assert(PANEL_STAGE * (PANEL_PER - 1) <= PANEL_ELEMS, "staging layout");
static_assert(PANEL_STAGE * (PANEL_FPER - 1) <= PANEL_SLOTS * PANEL_SMAX, "staging layout");

template <class T>
__global__ __launch_bounds__(256) void k_schwarz_panel(PanelDev<T> P, int backward, T* r, T* x,
                                                       int* err, int spin_max, int ntiles) {
  // the current group's tables in buffer pos & 1 while the next group is
  // staged in the other
  __shared__ T Aloc2[2][PANEL_ELEMS + PANEL_SMAX * PANEL_SLOTS];   // Aloc[l * 64 + k] = A(dof_k, dof_l),
                                                                  // PANEL_SMAX zero rows past l = 63
  __shared__ T fl2[2][PANEL_SLOTS * PANEL_SMAX];  // per slot: its row of the block inverse (padded)
  __shared__ T part[3][PANEL_SLOTS];              // partial sums of the correction
  __shared__ T ds_s[PANEL_SLOTS];                 // the group's d (chain), the published d (tiles)
  __shared__ T rfin_s[PANEL_SLOTS];               // the chain's final residual of each slot
  __shared__ T rnx_s[2][PANEL_SLOTS];             // the group's residual entries before correction
  __shared__ T rsh[PANEL_SLOTS + PANEL_SMAX];     // lane values of the chain's wavefront (zero
  __shared__ T dsh[PANEL_SLOTS + PANEL_SMAX];     // past the slots)
  __shared__ int dof_s[2][PANEL_SLOTS];
  __shared__ int gsl_s[2][PANEL_SLOTS];
  __shared__ int gblk_s[2][PANEL_SLOTS];
  __shared__ int gmn_s[2][2];                     // the group's slots and blocks
  const int tid = threadIdx.x;
  const int G = P.ngroups;
  const int64_t n = P.n;
  int* flag = P.sync;
  int* done = P.sync + SYNC_STRIDE * G;
  if (blockIdx.x == 0) {
    // ---------------- the chain ----------------
    {
      const int g0 = backward ? G - 1 : 0;
      // all loads first, then the LDS stores
      T pa[PANEL_ELEMS / 256], pf[PANEL_SLOTS * PANEL_SMAX / 256];
#pragma unroll
      for (int j = 0; j < PANEL_ELEMS / 256; ++j) pa[j] = P.gslc[(int64_t)g0 * PANEL_ELEMS + tid + 256 * j];
#pragma unroll
      for (int j = 0; j < PANEL_SLOTS * PANEL_SMAX / 256; ++j)
        pf[j] = P.gbinv[(int64_t)g0 * PANEL_SLOTS * PANEL_SMAX + tid + 256 * j];
#pragma unroll
      for (int j = 0; j < PANEL_ELEMS / 256; ++j) Aloc2[0][tid + 256 * j] = pa[j];
#pragma unroll
      for (int j = 0; j < PANEL_SLOTS * PANEL_SMAX / 256; ++j) fl2[0][tid + 256 * j] = pf[j];
      if (tid < PANEL_SMAX) {
        rsh[PANEL_SLOTS + tid] = T(0);
        dsh[PANEL_SLOTS + tid] = T(0);
      }
#pragma unroll
      for (int j = 0; j < PANEL_SMAX * PANEL_SLOTS / 256; ++j) {
        Aloc2[0][PANEL_ELEMS + tid + 256 * j] = T(0);
        Aloc2[1][PANEL_ELEMS + tid + 256 * j] = T(0);
      }
      if (tid < 64) {
        const int d = P.gdof[g0 * PANEL_SLOTS + tid];
        const int bk = P.gblk[g0 * PANEL_SLOTS + tid];
        dof_s[0][tid] = d;
        gsl_s[0][tid] = P.gsl[g0 * PANEL_SLOTS + tid];
        gblk_s[0][tid] = bk;
        rnx_s[0][tid] = d >= 0 ? ld_x<T, true>(r + d) : T(0);
        const unsigned long long vm = __ballot(d >= 0), vb = __ballot(bk >= 0);
        if (tid == 0) {
          gmn_s[0][0] = __popcll(vm);
          gmn_s[0][1] = __popcll(vb);
        }
      }
      __syncthreads();
    }
    for (int pos = 0; pos < G; ++pos) {
      const int g = backward ? G - 1 - pos : pos;
      const bool more = pos + 1 < G;
      const int gn = backward ? g - 1 : g + 1;
      if (tid < 64) {
        // wave 0: the chain over the group's blocks; lane k holds slot k
        const int k = tid;
        const int b = pos & 1;
        const T* Aloc = Aloc2[b];
        const T* fl = fl2[b];
        const int m = gmn_s[b][0], nbk = gmn_s[b][1];
        const int dofk = dof_s[b][k];
        const int sl = gsl_s[b][k];
        const int pk = sl & 255;
        const int ips = ((backward ? sl >> 16 : sl >> 8) & 255) - 1;
        T rk = 0, dk = 0;
        if (k < m) {
          if (pos == 0) rk = rnx_s[b][k];
          else if (ips >= 0) rk = rfin_s[ips];
          else rk = rnx_s[b][k] - ((part[0][k] + part[1][k]) + part[2][k]);
        }
        // lane b holds block b's first slot, size and colour run
        const int bk = k < nbk ? gblk_s[b][k] : 0;
        T br[PANEL_SMAX];
#pragma unroll
        for (int j = 0; j < PANEL_SMAX; ++j) br[j] = fl[k * PANEL_SMAX + j];
        int ib = backward ? nbk - 1 : 0;
        while (backward ? ib >= 0 : ib < nbk) {
          const int e = __builtin_amdgcn_readlane(bk, ib);
          const int lo = (e >> 16) & 255, hi = (e >> 24) & 255;
          if (lo == hi) {
            const int p = e & 255, s = (e >> 8) & 255;
            if (s <= PANEL_SMAX / 2)
              panel_step<T, PANEL_SMAX / 2>(k, p, s, br, Aloc, dsh, rk, dk);
            else
              panel_step<T, PANEL_SMAX>(k, p, s, br, Aloc, dsh, rk, dk);
          } else {
            const int e0 = __builtin_amdgcn_readlane(bk, lo), e1 = __builtin_amdgcn_readlane(bk, hi);
            panel_run<T>(k, e0 & 255, (e1 & 255) + ((e1 >> 8) & 255), pk, br, Aloc, rsh, dsh, rk, dk);
          }
          ib = backward ? lo - 1 : hi + 1;
        }
        if (k < m) {
          st_x<T, true>(r + dofk, rk);
          st_x<T, true>(P.dsl + (int64_t)pos * PANEL_SLOTS + k, dk);
        }
        rfin_s[k] = rk;
        ds_s[k] = k < m ? dk : T(0);
        __builtin_amdgcn_s_waitcnt(0);
        if (k == 0) __hip_atomic_store(&flag[SYNC_STRIDE * pos], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!more) break;
      // waves 1-3: the next group's tables, slice and inverse rows, and the
      // entries A(D_next, D_g) of the correction, while the chain runs
      T an[PANEL_PER], cn[PANEL_PER], fn[PANEL_FPER];
      int dn = -1, sln = 0, bkn = -1;
      T rn = 0;
      const int t = tid - 64;
      const int kn = t % PANEL_SLOTS, pt = t / PANEL_SLOTS;
      if (tid >= 64) {
        const T* Sn = P.gslc + (int64_t)gn * PANEL_ELEMS;
#pragma unroll
        for (int j = 0; j < PANEL_PER - 1; ++j) an[j] = Sn[t + PANEL_STAGE * j];
        an[PANEL_PER - 1] = t + PANEL_STAGE * (PANEL_PER - 1) < PANEL_ELEMS
                                ? Sn[t + PANEL_STAGE * (PANEL_PER - 1)] : T(0);
        const T* Fn = P.gbinv + (int64_t)gn * PANEL_SLOTS * PANEL_SMAX;
#pragma unroll
        for (int j = 0; j < PANEL_FPER - 1; ++j) fn[j] = Fn[t + PANEL_STAGE * j];
        fn[PANEL_FPER - 1] = t + PANEL_STAGE * (PANEL_FPER - 1) < PANEL_SLOTS * PANEL_SMAX
                                 ? Fn[t + PANEL_STAGE * (PANEL_FPER - 1)] : T(0);
        // thread (kn, pt) holds A(dof_next[kn], dof_g[k]) for k = pt, pt + 3, ...
        const T* Cg = (backward ? P.gcb : P.gcf) + (int64_t)g * PANEL_ELEMS;
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int k = pt + 3 * j;
          cn[j] = k < PANEL_SLOTS ? Cg[k * PANEL_SLOTS + kn] : T(0);
        }
        if (tid < 128) {
          dn = P.gdof[gn * PANEL_SLOTS + t];
          sln = P.gsl[gn * PANEL_SLOTS + t];
          bkn = P.gblk[gn * PANEL_SLOTS + t];
          // residual entries of the next group's new DoFs, once the tiles
          // have applied every group before the current one
          if (pos >= 1) panel_wait(&done[SYNC_STRIDE * (pos - 1)], ntiles, err, spin_max);
          const int ipn = ((backward ? sln >> 16 : sln >> 8) & 255) - 1;
          if (dn >= 0 && ipn < 0) rn = ld_x<T, true>(r + dn);
        }
        // the next group into the other buffer (read by the chain one
        // iteration back, before the last barrier)
        const int bn = (pos + 1) & 1;
        // only the last of each set can fall past the end
#pragma unroll
        for (int j = 0; j < PANEL_PER - 1; ++j) Aloc2[bn][t + PANEL_STAGE * j] = an[j];
        if (t + PANEL_STAGE * (PANEL_PER - 1) < PANEL_ELEMS)
          Aloc2[bn][t + PANEL_STAGE * (PANEL_PER - 1)] = an[PANEL_PER - 1];
#pragma unroll
        for (int j = 0; j < PANEL_FPER - 1; ++j) fl2[bn][t + PANEL_STAGE * j] = fn[j];
        if (t + PANEL_STAGE * (PANEL_FPER - 1) < PANEL_SLOTS * PANEL_SMAX)
          fl2[bn][t + PANEL_STAGE * (PANEL_FPER - 1)] = fn[PANEL_FPER - 1];
        if (tid < 128) {
          dof_s[bn][t] = dn;
          gsl_s[bn][t] = sln;
          gblk_s[bn][t] = bkn;
          rnx_s[bn][t] = rn;
          const unsigned long long vm = __ballot(dn >= 0), vb = __ballot(bkn >= 0);
          if (t == 0) {
            gmn_s[bn][0] = __popcll(vm);
            gmn_s[bn][1] = __popcll(vb);
          }
        }
      }
      __syncthreads();
      if (tid >= 64) {
        // correction partial sums (this group's d is in ds_s)
        T acc = 0;
#pragma unroll
        for (int j = 0; j < PANEL_PER; ++j) {
          const int k = pt + 3 * j;
          if (k < PANEL_SLOTS) acc += cn[j] * ds_s[k];
        }
        part[pt][kn] = acc;
      }
      __syncthreads();
    }
    return;
  }
  // ---------------- the tiles ----------------
  // Two threads per row i (slots 0-31 and 32-63).  For every group a tile
  // loads the group's columns of its rows (and the rows' residuals) and the
  // next group's DoFs before it waits for the group's d.
  const int64_t i = (int64_t)(blockIdx.x - 1) * PANEL_TROWS + (tid >> 1);
  const int half = tid & 1;
  const bool row = i < n;
  const int ga = row ? P.dgrp[2 * i] : -1, gb = row ? P.dgrp[2 * i + 1] : -1;
  const int o0 = row ? P.docc[2 * i] : -1, o1 = row ? P.docc[2 * i + 1] : -1;
  const bool xown = row && half == 0 && o0 >= 0;
  T xi = xown ? x[i] : T(0);   // x_i changes only here during the sweep
  if (tid < 64) dof_s[0][tid] = P.gdof[(backward ? G - 1 : 0) * PANEL_SLOTS + tid];
  __syncthreads();
  for (int pos = 0; pos < G; ++pos) {
    const int b = pos & 1;
    const int g = backward ? G - 1 - pos : pos;
    const int gn = pos + 1 < G ? (backward ? g - 1 : g + 1) : -2;
    const bool upd = row && ga != g && ga != gn && gb != g && gb != gn;
    const int dnx = (tid < 64 && gn >= 0) ? P.gdof[gn * PANEL_SLOTS + tid] : -1;
    // every load is issued, from a clamped address and without a mask (the
    // published d is zero past the group's slots, and rows that take no
    // update store nothing), so the 32 loads are in flight together; n <=
    // PANEL_NMAX, so the offsets into the dense copy fit in 32 bits
    const int ic = row ? (int)i : 0, ni = (int)n;
    T a[PANEL_SLOTS / 2];
#pragma unroll
    for (int j = 0; j < PANEL_SLOTS / 2; ++j) {
      const int d = dof_s[b][half * (PANEL_SLOTS / 2) + j];
      a[j] = P.Acm[(d >= 0 ? d : 0) * ni + ic];
    }
    // the tile wrote r_i last itself, or the chain did before an earlier flag
    const T ri = (upd && half == 0) ? ld_x<T, true>(r + i) : T(0);
    if (tid == 0) panel_wait(&flag[SYNC_STRIDE * pos], 1, err, spin_max);
    __syncthreads();
    if (tid < 64) {
      ds_s[tid] = dof_s[b][tid] >= 0 ? ld_x<T, true>(P.dsl + (int64_t)pos * PANEL_SLOTS + tid) : T(0);
      dof_s[b ^ 1][tid] = dnx;
    }
    __syncthreads();
    T acc = 0;
#pragma unroll
    for (int j = 0; j < PANEL_SLOTS / 2; ++j) acc += a[j] * ds_s[half * (PANEL_SLOTS / 2) + j];
    acc += __shfl_xor(acc, 1);
    if (upd && half == 0) st_x<T, true>(r + i, ri - acc);
    if (xown) {
      // x_i += d of the slots that hold DoF i, in sweep order
      const int e0 = backward ? o1 : o0, e1 = backward ? o0 : o1;
      if (e0 >= 0 && (e0 >> 6) == g) xi += ds_s[e0 & 63];
      if (e1 >= 0 && (e1 >> 6) == g) xi += ds_s[e1 & 63];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&done[SYNC_STRIDE * pos], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (xown) x[i] = xi;
}

bool panel_sweep_ok(int n, int max_block) {
  return n > 0 && n <= PANEL_NMAX && max_block <= PANEL_SMAX;
}

int panel_tiles(int n) { return (n + PANEL_TROWS - 1) / PANEL_TROWS; }

// Dynamic LDS the panel launch adds so that its workgroups hold more than
// half a CU's 160 KB each (one workgroup per CU).
template <class T>
static size_t panel_pad() {
  static const size_t pad = [] {
    hipFuncAttributes fa{};
    const size_t want = 80 * 1024 + 1024;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_schwarz_panel<T>)) != hipSuccess) return size_t(0);
    return fa.sharedSizeBytes >= want ? size_t(0) : want - fa.sharedSizeBytes;
  }();
  return pad;
}

// Workgroups of the panel launch that one CU can hold at once (from the
// occupancy query with the launch's LDS padding), or -1 if the query fails.
int panel_resident_per_cu(int prec) {
  int blocks = -1;
  hipError_t e;
  if (prec == 32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_schwarz_panel<float>),
                                                     256, panel_pad<float>());
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_schwarz_panel<double>),
                                                     256, panel_pad<double>());
  return e == hipSuccess ? blocks : -1;
}

template <class T>
void panel_sweep(const PanelDev<T>& D, int backward, T* r, T* x, int* err, int spin_max, hipStream_t st) {
  if (D.ngroups <= 0) return;
  const int nsync = 2 * SYNC_STRIDE * D.ngroups;
  hipLaunchKernelGGL(k_zero_i32, dim3((nsync + 255) / 256), dim3(256), 0, st, nsync, D.sync);
  const int ntiles = panel_tiles(D.n);
  // Unused dynamic LDS up to more than half a CU's 160 KB, so that no two
  // workgroups share a CU: tiles on the chain's CU slow the chain.
  const size_t pad = panel_pad<T>();
  hipLaunchKernelGGL((k_schwarz_panel<T>), dim3(1 + ntiles), dim3(256), pad, st, D, backward, r, x, err,
                     spin_max, ntiles);
}

// The panel form's per-group matrices, gathered from the dense copy once per
// numeric setup: A(D_g, D_g) (entry l * 64 + k = A(dof_k, dof_l)) and the
// blocks to the neighbouring groups, A(D_g+1, D_g) and A(D_g-1, D_g) (entry
// k * 64 + kn = A(dof_{g+-1, kn}, dof_{g, k})), zero past the groups' slots.
template <class T>
__global__ void k_panel_slices(int ngroups, int64_t n, const int32_t* __restrict__ gdof,
                               const T* __restrict__ Acm, T* __restrict__ gslc, T* __restrict__ gcf,
                               T* __restrict__ gcb) {
  const int g = blockIdx.x;
  const int32_t* D = gdof + (int64_t)g * PANEL_SLOTS;
  const int32_t* Df = g + 1 < ngroups ? D + PANEL_SLOTS : nullptr;
  const int32_t* Db = g > 0 ? D - PANEL_SLOTS : nullptr;
  for (int e = threadIdx.x; e < PANEL_ELEMS; e += blockDim.x) {
    const int hi = e / PANEL_SLOTS, lo = e % PANEL_SLOTS;
    const int dh = D[hi], dl = D[lo];
    gslc[(int64_t)g * PANEL_ELEMS + e] = (dh >= 0 && dl >= 0) ? Acm[(int64_t)dh * n + dl] : T(0);
    const int df = Df ? Df[lo] : -1, db = Db ? Db[lo] : -1;
    gcf[(int64_t)g * PANEL_ELEMS + e] = (dh >= 0 && df >= 0) ? Acm[(int64_t)dh * n + df] : T(0);
    gcb[(int64_t)g * PANEL_ELEMS + e] = (dh >= 0 && db >= 0) ? Acm[(int64_t)dh * n + db] : T(0);
  }
}

void panel_slices(int ngroups, int64_t n, const int32_t* gdof, const double* Acm, double* gslc,
                  double* gcf, double* gcb, hipStream_t st) {
  if (ngroups > 0)
    hipLaunchKernelGGL((k_panel_slices<double>), dim3(ngroups), dim3(256), 0, st, ngroups, n, gdof, Acm,
                       gslc, gcf, gcb);
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
  in_batches(nb, [&](int64_t w0, unsigned g) {
    hipLaunchKernelGGL(k_ext_block, dim3(g, (unsigned)ntiles), dim3(64), lds, st, b0 + w0, bptr, bdofs,
                       dof_stage, stage, A.ptr, A.col, A.val, Pptr, Pcol, Pval, smax, ctile, wide,
                       flag, Wl, accepted, dsq);
  });
}

// Patch extension: one 256-thread workgroup per column c of P.  The column's
// patch S (m <= mmax interior DoFs, ascending) gives the dense SPD system
// A_SS x = -A_S,ext r_c, where r_c holds the column's two exterior values
// (the signs of its R row).
//  * gather: the entries of the patch's rows of A are spread over all
//    threads (a row-length prefix in LDS maps a flat index to (row, entry));
//    lower-triangle entries of A_SS go to a packed LDS matrix (row i at
//    i(i+1)/2), the two exterior couplings of each row to two LDS vectors;
//  * Cholesky in blocks of 16 columns: the diagonal block by 16 lanes of
//    wavefront 0 with shuffles (no barrier), the panel below it one row per
//    thread, the trailing update spread over all threads by (row, column);
//  * forward and back substitution in the same blocks;
// about 7 barriers per 16 columns.  x goes to P's entries of the column.
constexpr int EXT_NB = 16;
constexpr int EXT_GATHER = 4;   // entries of A per thread with their loads in flight together

__device__ __forceinline__ int tri_off(int i) { return i * (i + 1) / 2; }

__global__ __launch_bounds__(256) void k_ext_patch(
    const int64_t* __restrict__ pptr, const int32_t* __restrict__ pdofs,
    const int64_t* __restrict__ Pptr, const int32_t* __restrict__ Pcol, const int32_t* __restrict__ rd1,
    const int32_t* __restrict__ rd2, const int8_t* __restrict__ rs1,
    const int8_t* __restrict__ rs2, const int64_t* __restrict__ Aptr,
    const int32_t* __restrict__ Acol, const double* __restrict__ Aval, double* __restrict__ Pval,
    int mmax, int* __restrict__ flag, int64_t cfirst) {
  extern __shared__ unsigned char lds_raw[];
  double* L = (double*)lds_raw;                             // packed lower triangle
  double* y = L + (size_t)mmax * (mmax + 1) / 2;            // right-hand side, then x
  double* e1v = y + mmax;                                   // A(S_i, ext1)
  double* e2v = e1v + mmax;                                 // A(S_i, ext2)
  int64_t* rstart = (int64_t*)(e2v + mmax);                 // first A entry of each row
  double* rdiag = (double*)(rstart + mmax);                 // 1 / L(i, i)
  int32_t* pre = (int32_t*)(rdiag + mmax);                  // row-length prefix (m + 1)
  int32_t* dofs = pre + mmax + 1;
  const int64_t c = cfirst + blockIdx.x;
  const int64_t p0 = pptr[c];
  const int m = (int)(pptr[c + 1] - p0);
  if (m == 0) return;   // the whole workgroup: nothing to extend
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int32_t x1 = rd1[c], x2 = rd2[c];
  const double s1 = (double)rs1[c], s2 = (double)rs2[c];
  int32_t mylen[3] = {0, 0, 0};
  // rows 3 lane .. 3 lane + 2 of wavefront 0 (m <= 192)
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = 3 * lane + k;
      if (i < m) {
        const int32_t r = pdofs[p0 + i];
        dofs[i] = r;
        const int64_t a = Aptr[r];
        rstart[i] = a;
        mylen[k] = (int32_t)(Aptr[r + 1] - a);
      }
    }
    // exclusive prefix of the row lengths over the wavefront
    int32_t tot = mylen[0] + mylen[1] + mylen[2];
    int32_t inc = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    int32_t run = inc - tot;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = 3 * lane + k;
      if (i < m) pre[i] = run;
      run += mylen[k];
    }
    if (lane == 63) pre[m] = inc;
  }
  const int tri = m * (m + 1) / 2;
  for (int t = tid; t < tri; t += 256) L[t] = 0.0;
  for (int t = tid; t < m; t += 256) e1v[t] = e2v[t] = 0.0;
  __syncthreads();
  const int E = pre[m];
  // EXT_GATHER flat entries per thread and round, their loads issued together
  for (int e0 = tid; e0 < E; e0 += 256 * EXT_GATHER) {
    int ri[EXT_GATHER];
    int32_t jv[EXT_GATHER];
    double av[EXT_GATHER];
#pragma unroll
    for (int u = 0; u < EXT_GATHER; ++u) {
      const int e = e0 + u * 256;
      ri[u] = -1;
      if (e < E) {
        // row of flat entry e: the last i with pre[i] <= e
        int lo = 0, hi = m;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (pre[mid] <= e) lo = mid; else hi = mid;
        }
        ri[u] = lo;
      }
    }
#pragma unroll
    for (int u = 0; u < EXT_GATHER; ++u) {
      if (ri[u] >= 0) {
        const int64_t q = rstart[ri[u]] + (e0 + u * 256 - pre[ri[u]]);
        jv[u] = Acol[q];
        av[u] = Aval[q];
      }
    }
#pragma unroll
    for (int u = 0; u < EXT_GATHER; ++u) {
      const int i = ri[u];
      if (i < 0) continue;
      const int32_t j = jv[u];
      if (j == x1) {
        e1v[i] = av[u];
      } else if (j == x2) {
        e2v[i] = av[u];
      } else if (j <= dofs[i]) {
        const int pos = lower_bound_i32(dofs, i + 1, j);
        if (pos <= i && dofs[pos] == j) L[tri_off(i) + pos] = av[u];
      }
    }
  }
  __syncthreads();
  // two terms with exact +-1 factors: the sum does not depend on the order
  for (int i = tid; i < m; i += 256) y[i] = -(e1v[i] * s1 + e2v[i] * s2);
  // ---- blocked Cholesky ----
  for (int kb = 0; kb < m; kb += EXT_NB) {
    const int nb = min(EXT_NB, m - kb);
    if (wave == 0) {
      // lane r < nb holds row kb + r of the diagonal block
      double d[EXT_NB];
#pragma unroll
      for (int t = 0; t < EXT_NB; ++t)
        d[t] = (lane < nb && t <= lane && t < nb) ? L[tri_off(kb + lane) + kb + t] : (t == lane ? 1.0 : 0.0);
#pragma unroll
      for (int cc = 0; cc < EXT_NB; ++cc) {
        if (lane == cc) {
          double v = d[cc];
          if (cc < nb && !(v > 0.0)) {
            atomicExch(flag, 1);
            v = 1.0;
          }
          d[cc] = sqrt(v);
        }
        const double piv = __shfl(d[cc], cc, 64);
        if (lane > cc) d[cc] /= piv;
#pragma unroll
        for (int jj = cc + 1; jj < EXT_NB; ++jj) {
          const double ljc = __shfl(d[cc], jj, 64);
          if (lane >= jj) d[jj] -= d[cc] * ljc;
        }
      }
      if (lane < nb) {
#pragma unroll
        for (int t = 0; t < EXT_NB; ++t)
          if (t <= lane) L[tri_off(kb + lane) + kb + t] = d[t];
        rdiag[kb + lane] = 1.0 / d[lane];
      }
    }
    __syncthreads();
    const int r0 = kb + nb;
    // panel: rows i >= r0, columns kb .. kb + nb: x = a L_D^{-T}
    for (int i = r0 + tid; i < m; i += 256) {
      double* Li = L + tri_off(i) + kb;
      double xv[EXT_NB];
#pragma unroll
      for (int cc = 0; cc < EXT_NB; ++cc) {
        if (cc < nb) {
          double v = Li[cc];
          const double* Lc = L + tri_off(kb + cc) + kb;
#pragma unroll
          for (int t = 0; t < cc; ++t) v -= xv[t] * Lc[t];
          xv[cc] = v * rdiag[kb + cc];
        } else {
          xv[cc] = 0.0;
        }
      }
#pragma unroll
      for (int cc = 0; cc < EXT_NB; ++cc)
        if (cc < nb) Li[cc] = xv[cc];
    }
    __syncthreads();
    // trailing update: L(i, j) -= sum_t L(i, kb + t) L(j, kb + t), r0 <= j <= i < m,
    // the (i, j) pairs numbered row by row and dealt to threads in turn
    const int R = m - r0;
    if (R > 0) {
      const int T = R * (R + 1) / 2;
      int e = tid;
      // (i, j) of flat index e: i the largest with i(i+1)/2 <= e
      int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (tri_off(ii + 1) <= e) ++ii;
      while (tri_off(ii) > e) --ii;
      int jj = e - tri_off(ii);
      for (; e < T; e += 256) {
        const double* Li = L + tri_off(r0 + ii) + kb;
        const double* Lj = L + tri_off(r0 + jj) + kb;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < EXT_NB; ++t)
          if (t < nb) acc += Li[t] * Lj[t];
        L[tri_off(r0 + ii) + r0 + jj] -= acc;
        jj += 256;
        while (jj > ii && ii < R) {
          jj -= ii + 1;
          ++ii;
        }
      }
    }
    __syncthreads();
  }
  // ---- L z = y, then L^T x = z (in y), in the same blocks ----
  for (int kb = 0; kb < m; kb += EXT_NB) {
    const int nb = min(EXT_NB, m - kb);
    if (wave == 0) {
      double lr[EXT_NB];
#pragma unroll
      for (int t = 0; t < EXT_NB; ++t)
        lr[t] = (lane < nb && t <= lane) ? L[tri_off(kb + lane) + kb + t] : 1.0;
      double yr = lane < nb ? y[kb + lane] : 0.0;
      const double rd = lane < nb ? rdiag[kb + lane] : 1.0;
#pragma unroll
      for (int cc = 0; cc < EXT_NB; ++cc) {
        if (lane == cc) yr *= rd;
        const double zc = __shfl(yr, cc, 64);
        if (lane > cc) yr -= lr[cc] * zc;
      }
      if (lane < nb) y[kb + lane] = yr;
    }
    __syncthreads();
    for (int i = kb + nb + tid; i < m; i += 256) {
      const double* Li = L + tri_off(i) + kb;
      double v = y[i];
#pragma unroll
      for (int t = 0; t < EXT_NB; ++t)
        if (t < nb) v -= Li[t] * y[kb + t];
      y[i] = v;
    }
    __syncthreads();
  }
  const int nblk = (m + EXT_NB - 1) / EXT_NB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int kb = bi * EXT_NB;
    const int nb = min(EXT_NB, m - kb);
    if (wave == 0) {
      // lane r holds x_{kb+r} and column kb + r of the block: lc[t] = L(kb + t, kb + r)
      double lc[EXT_NB];
#pragma unroll
      for (int t = 0; t < EXT_NB; ++t)
        lc[t] = (lane < nb && t >= lane && t < nb) ? L[tri_off(kb + t) + kb + lane] : 1.0;
      double xr = lane < nb ? y[kb + lane] : 0.0;
      const double rd = lane < nb ? rdiag[kb + lane] : 1.0;
#pragma unroll
      for (int cc = EXT_NB - 1; cc >= 0; --cc) {
        if (lane == cc) xr *= rd;
        const double xc = __shfl(xr, cc, 64);
        if (lane < cc) xr -= lc[cc] * xc;
      }
      if (lane < nb) y[kb + lane] = xr;
    }
    __syncthreads();
    for (int i = tid; i < kb; i += 256) {
      double v = y[i];
#pragma unroll
      for (int t = 0; t < EXT_NB; ++t)
        if (t < nb) v -= L[tri_off(kb + t) + i] * y[kb + t];
      y[i] = v;
    }
    __syncthreads();
  }
  // x_i goes to P(S_i, c): row S_i of P lists its columns in ascending order
  for (int t = tid; t < m; t += 256) {
    const int64_t r0 = Pptr[dofs[t]];
    int lo = 0, hi = (int)(Pptr[dofs[t] + 1] - r0);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Pcol[r0 + mid] < (int32_t)c) lo = mid + 1; else hi = mid;
    }
    Pval[r0 + lo] = y[t];
  }
}

size_t ext_patch_lds(int mmax) {
  return sizeof(double) * ((size_t)mmax * (mmax + 1) / 2 + 4 * (size_t)mmax) +
         sizeof(int64_t) * (size_t)mmax + sizeof(int32_t) * (2 * (size_t)mmax + 1);
}

void ext_patches(int64_t nc, const int64_t* pptr, const int32_t* pdofs, const int64_t* Pptr,
                 const int32_t* Pcol, const int32_t* rd1, const int32_t* rd2, const int8_t* rs1,
                 const int8_t* rs2, const CsrDev<double>& A, double* Pval, int mmax, int* flag,
                 hipStream_t st) {
  if (nc <= 0 || mmax <= 0) return;
  in_batches(nc, [&](int64_t c0, unsigned g) {
    hipLaunchKernelGGL(k_ext_patch, dim3(g), dim3(256), ext_patch_lds(mmax), st, pptr, pdofs, Pptr,
                       Pcol, rd1, rd2, rs1, rs2, A.ptr, A.col, A.val, Pval, mmax, flag, c0);
  });
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
                          const int32_t* Ycol, int32_t* hash, int tsize, int* count, int* overflow) {
  const uint32_t mask = (uint32_t)tsize - 1u;
  for (int64_t t = Xptr[i] + threadIdx.x; t < Xptr[i + 1]; t += blockDim.x) {
    const int32_t k = Xcol[t];
    for (int64_t u = Yptr[k]; u < Yptr[k + 1]; ++u) {
      if (*(volatile int*)overflow) return;   // the row goes to the wide passes anyway
      const int32_t J = Ycol[u];
      uint32_t h = ((uint32_t)J * 2654435761u) & mask;
      int probes = 0;
      while (true) {
        int32_t old = atomicCAS(&hash[h], -1, J);
        if (old == -1) {
          atomicAdd(count, 1);
          break;
        }
        if (old == J) break;
        h = (h + 1) & mask;
        if (++probes >= tsize) {
          atomicExch(overflow, 1);
          break;
        }
      }
    }
  }
}

// Hash slots for row i: the sum of the lengths of the Y rows that X's row
// touches bounds its distinct columns; the table takes the power of two at
// or above twice that bound (at least 64, at most HCAP), so that a short row
// does not clear and scan all HCAP slots.  Every thread of the block returns
// the same size.
__device__ int mm_table_size(int64_t i, const int64_t* Xptr, const int32_t* Xcol,
                             const int64_t* Yptr, int* red) {
  if (threadIdx.x == 0) *red = 0;
  __syncthreads();
  int64_t u = 0;
  for (int64_t t = Xptr[i] + threadIdx.x; t < Xptr[i + 1]; t += blockDim.x) {
    const int32_t k = Xcol[t];
    u += Yptr[k + 1] - Yptr[k];
  }
  if (u > 0) atomicAdd(red, (int)(u < HCAP ? u : HCAP));
  __syncthreads();
  const int bound = *red;
  int tsize = 64;
  while (tsize < HCAP && tsize < 2 * bound) tsize <<= 1;
  return tsize;
}

__global__ __launch_bounds__(256) void k_mm_count(int64_t nrows, const int64_t* __restrict__ Xptr,
                                                  const int32_t* __restrict__ Xcol,
                                                  const int64_t* __restrict__ Yptr,
                                                  const int32_t* __restrict__ Ycol,
                                                  int64_t* __restrict__ cnt,
                                                  int* __restrict__ overflow, int wide_at, int64_t r0) {
  __shared__ int32_t hash[HCAP];
  __shared__ int count;
  __shared__ int full;
  __shared__ int red;
  const int64_t i = r0 + blockIdx.x;
  const int tsize = mm_table_size(i, Xptr, Xcol, Yptr, &red);
  for (int t = threadIdx.x; t < tsize; t += blockDim.x) hash[t] = -1;
  if (threadIdx.x == 0) {
    count = 0;
    full = 0;
  }
  __syncthreads();
  mm_insert(i, Xptr, Xcol, Yptr, Ycol, hash, tsize, &count, &full);
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
                                                 int* __restrict__ overflow, int wide_at, int64_t r0) {
  __shared__ int32_t hash[HCAP];
  __shared__ int count;
  __shared__ int nfill;
  __shared__ int full;
  __shared__ int red;
  const int64_t i = r0 + blockIdx.x;
  if (Cptr[i + 1] - Cptr[i] > wide_at) return;   // wide row: k_mm_fill_wide
  const int tsize = mm_table_size(i, Xptr, Xcol, Yptr, &red);
  for (int t = threadIdx.x; t < tsize; t += blockDim.x) hash[t] = -1;
  if (threadIdx.x == 0) {
    count = 0;
    nfill = 0;
    full = 0;
  }
  __syncthreads();
  mm_insert(i, Xptr, Xcol, Yptr, Ycol, hash, tsize, &count, &full);
  __syncthreads();
  if (full) {   // cannot happen: the row was counted to fit
    if (threadIdx.x == 0) atomicExch(overflow, 1);
    return;
  }
  // gather the keys into registers, then compact them to the front
  // (m <= tsize / 2, so the sort's padded length P2 stays inside the table)
  int32_t keys[HCAP / 256];
  int nk = 0;
  for (int t = threadIdx.x; t < tsize; t += blockDim.x)
    if (hash[t] >= 0) keys[nk++] = hash[t];
  __syncthreads();
  for (int t = threadIdx.x; t < tsize; t += blockDim.x) hash[t] = 0x7fffffff;
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
    int mmax, int64_t r0) {
  extern __shared__ unsigned char lds_raw[];
  double* acc = (double*)lds_raw;          // mmax
  int32_t* cols = (int32_t*)(acc + mmax);  // mmax
  const int64_t i = r0 + blockIdx.x;
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
  const int wide_at = mm_wide_at();
  in_batches(nrows, [&](int64_t r0, unsigned g) {
    hipLaunchKernelGGL(k_mm_count, dim3(g), dim3(256), 0, st, nrows, X.ptr, X.col, Y.ptr, Y.col, cnt,
                       overflow, wide_at, r0);
  });
}
void mm_fill(int64_t nrows, const CsrPat& X, const CsrPat& Y, const int64_t* Cptr, int32_t* Ccol,
             int* overflow, hipStream_t st) {
  const int wide_at = mm_wide_at();
  in_batches(nrows, [&](int64_t r0, unsigned g) {
    hipLaunchKernelGGL(k_mm_fill, dim3(g), dim3(256), 0, st, nrows, X.ptr, X.col, Y.ptr, Y.col, Cptr,
                       Ccol, overflow, wide_at, r0);
  });
}
void mm_vals(int64_t nrows, const CsrPat& X, const double* Xval, const CsrPat& Y,
             const double* Yval, const int64_t* Cptr, const int32_t* Ccol, double* Cval, int mmax,
             hipStream_t st) {
  if (nrows <= 0) return;
  size_t lds = (size_t)std::max(mmax, 1) * (sizeof(double) + sizeof(int32_t));
  in_batches(nrows, [&](int64_t r0, unsigned g) {
    hipLaunchKernelGGL(k_mm_vals, dim3(g), dim3(64), lds, st, nrows, X.ptr, X.col, Xval, Y.ptr, Y.col,
                       Yval, Cptr, Ccol, Cval, mmax, r0);
  });
}
int mm_hash_cap() { return HCAP; }

// ---------------------------------------------------------------------------
// setup: smoother factors and l1 diagonal
// ---------------------------------------------------------------------------

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
// the block, at its group slot (the panel form's operand layout).
__global__ void k_pad_inv(int64_t nrows, const int32_t* __restrict__ row_blk,
                          const int32_t* __restrict__ row_slot, const int64_t* __restrict__ sb_ptr,
                          const int64_t* __restrict__ fac_off, const double* __restrict__ binv,
                          double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int b = row_blk[r];
  const int s = (int)(sb_ptr[b + 1] - sb_ptr[b]);
  const int i = (int)(r - sb_ptr[b]);
  const double* B = binv + fac_off[b];
  for (int j = 0; j < PANEL_SMAX; ++j) {
    const int hi = i > j ? i : j, lo = i > j ? j : i;
    out[(int64_t)row_slot[r] * PANEL_SMAX + j] = j < s ? B[hi * (hi + 1) / 2 + lo] : 0.0;
  }
}

void pad_inv(int64_t nrows, const int32_t* row_blk, const int32_t* row_slot, const int64_t* sb_ptr,
             const int64_t* fac_off, const double* binv, double* out, hipStream_t st) {
  if (nrows > 0)
    hipLaunchKernelGGL(k_pad_inv, dim3((unsigned)((nrows + 127) / 128)), dim3(128), 0, st, nrows,
                       row_blk, row_slot, sb_ptr, fac_off, binv, out);
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

// y = |A| |x| (entrywise absolute values), one thread per row: the scale of
// the rounding error of a residual f - A x computed in FP64
__global__ void k_spmv_abs(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const double* __restrict__ x,
                           double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) s += fabs(val[q]) * fabs(x[col[q]]);
    y[i] = s;
  }
}
void spmv_abs(const CsrDev<double>& A, const double* x, double* y, hipStream_t st) {
  if (A.n > 0)
    hipLaunchKernelGGL(k_spmv_abs, dim3(grid_for(A.n)), dim3(256), 0, st, A.n, A.ptr, A.col, A.val, x, y);
}

// Gradient conditioning of every node-star block B (the DoFs of one column v
// of G, with signs s = G[B, v]): num = sum_{i,j in B} |a_ij| and
// den = s^T A_BB s, the energy of the gradient of v's hat function.  One
// thread per block, from the smoother's star-ordered copy of A's rows.
__global__ void k_star_rho(int64_t nb, const int64_t* __restrict__ sb_ptr, const int32_t* __restrict__ sb_dofs,
                           const int8_t* __restrict__ ssign, const int64_t* __restrict__ srow_ptr,
                           const int32_t* __restrict__ scol, const double* __restrict__ sval,
                           double* __restrict__ rho) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = sb_ptr[b], r1 = sb_ptr[b + 1];
    double num = 0.0, den = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double sr = (double)ssign[r];
      for (int64_t q = srow_ptr[r]; q < srow_ptr[r + 1]; ++q) {
        const int32_t c = scol[q];
        for (int64_t j = r0; j < r1; ++j)
          if (sb_dofs[j] == c) {
            num += fabs(sval[q]);
            den += sr * (double)ssign[j] * sval[q];
            break;
          }
      }
    }
    rho[b] = den > 0.0 ? num / den : 0.0;
  }
}
void star_rho(int64_t nb, const int64_t* sb_ptr, const int32_t* sb_dofs, const int8_t* ssign,
              const int64_t* srow_ptr, const int32_t* scol, const double* sval, double* rho,
              hipStream_t st) {
  if (nb > 0)
    hipLaunchKernelGGL(k_star_rho, dim3(grid_for(nb)), dim3(256), 0, st, nb, sb_ptr, sb_dofs, ssign,
                       srow_ptr, scol, sval, rho);
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
template void panel_sweep<double>(const PanelDev<double>&, int, double*, double*, int*, int, hipStream_t);
template void panel_sweep<float>(const PanelDev<float>&, int, float*, float*, int*, int, hipStream_t);
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
template void cast<double, double>(int64_t, const double*, double*, hipStream_t);
template void cast<float, float>(int64_t, const float*, float*, hipStream_t);

}  // namespace hamg

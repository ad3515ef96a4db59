// C ABI of the H(curl) AMG library: hierarchy construction (host integer
// phase + GPU numeric phase), V-cycle and PCG drivers.  See include/amg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/amg.h"
#include "host_setup.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

using namespace hamg;

namespace {

thread_local std::string g_err;

// HCURL_AMG_VERBOSE=1: per-phase wall times of the setup on stderr
bool verbose() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("HCURL_AMG_VERBOSE");
    v = (e && e[0] && e[0] != '0') ? 1 : 0;
  }
  return v == 1;
}

struct PhaseClock {
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(hipStream_t st, const char* what, int level) {
    if (!verbose()) return;
    (void)hipStreamSynchronize(st);
    auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[amg] level %d %-28s %8.3f s\n", level, what,
                 std::chrono::duration<double>(now - t).count());
    std::fflush(stderr);
    t = now;
  }
};

// HCURL_AMG_VERBOSE=2: the steps inside a phase (stream synchronised at each)
struct StepTimer {
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  bool on = false;
  StepTimer() {
    const char* e = std::getenv("HCURL_AMG_VERBOSE");
    on = e && std::atoi(e) >= 2;
  }
  void mark(hipStream_t st, const std::string& what) {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[amg]   %-40s %8.3f s\n", what.c_str(),
                 std::chrono::duration<double>(now - t).count());
    std::fflush(stderr);
    t = now;
  }
};

struct Fail {
  amg_status code;
  std::string msg;
};

[[noreturn]] void fail(amg_status c, const std::string& m) { throw Fail{c, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(AMG_ERR_OOM, std::string(what) + ": out of device memory");
    fail(AMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HIPC(x) hip_check((x), #x)

int lpr_for(int64_t n, int64_t nnz) {
  double avg = n > 0 ? (double)nnz / (double)n : 1.0;
  if (avg <= 6) return 4;
  if (avg <= 40) return 8;
  if (avg <= 100) return 16;
  if (avg <= 250) return 32;
  return 64;
}

// Device allocations owned by a hierarchy.
// Large copies between pageable host memory and the device go through two
// pinned 32 MiB buffers: the host fills (or drains) one while the DMA engine
// moves the other.  Pageable copies run at a few GB/s on these hosts; copies
// below 4 MiB stay plain.
struct Staging {
  static constexpr size_t CAP = size_t(32) << 20;
  static constexpr size_t SMALL = size_t(4) << 20;
  char* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};   // an upload may still read buf[b]
  void init() {
    if (buf[0]) return;
    for (int b = 0; b < 2; ++b) {
      HIPC(hipHostMalloc((void**)&buf[b], CAP, hipHostMallocDefault));
      HIPC(hipEventCreateWithFlags(&ev[b], hipEventDisableTiming));
    }
  }
  void drain(int b) {
    if (pending[b]) {
      HIPC(hipEventSynchronize(ev[b]));
      pending[b] = false;
    }
  }
  void h2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes < SMALL) {
      HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
      return;
    }
    init();
    for (size_t off = 0, k = 0; off < bytes; off += CAP, ++k) {
      const int b = (int)(k & 1);
      const size_t len = std::min(CAP, bytes - off);
      drain(b);
      std::memcpy(buf[b], (const char*)src + off, len);
      HIPC(hipMemcpyAsync((char*)dst + off, buf[b], len, hipMemcpyHostToDevice, st));
      HIPC(hipEventRecord(ev[b], st));
      pending[b] = true;
    }
  }
  // returns once dst holds the bytes
  void d2h(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes < SMALL) {
      HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      return;
    }
    init();
    const size_t n = (bytes + CAP - 1) / CAP;
    auto issue = [&](size_t k) {
      const int b = (int)(k & 1);
      drain(b);
      const size_t off = k * CAP, len = std::min(CAP, bytes - off);
      HIPC(hipMemcpyAsync(buf[b], (const char*)src + off, len, hipMemcpyDeviceToHost, st));
      HIPC(hipEventRecord(ev[b], st));
    };
    issue(0);
    for (size_t k = 0; k < n; ++k) {
      if (k + 1 < n) issue(k + 1);
      const int b = (int)(k & 1);
      HIPC(hipEventSynchronize(ev[b]));
      const size_t off = k * CAP, len = std::min(CAP, bytes - off);
      std::memcpy((char*)dst + off, buf[b], len);
    }
  }
  ~Staging() {
    for (int b = 0; b < 2; ++b) {
      if (ev[b]) {
        (void)hipEventSynchronize(ev[b]);
        (void)hipEventDestroy(ev[b]);
      }
      if (buf[b]) (void)hipHostFree(buf[b]);
    }
  }
};

struct Pool {
  std::vector<void*> ptrs;
  Staging stage;
  template <class T>
  T* get(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    HIPC(hipMalloc(&p, n * sizeof(T)));
    ptrs.push_back(p);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t st) {
    T* d = get<T>(v.size());
    if (!v.empty()) stage.h2d(d, v.data(), v.size() * sizeof(T), st);
    return d;
  }
  ~Pool() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// largest patch of the patch extension: its packed factor fits 160 KB of LDS
constexpr int PATCH_CAP_MAX = 192;

struct Stage {
  int64_t b0, nb;
  int smax, cmax;
};

struct Level {
  // host side
  Pattern Apat;
  Incidence G;
  Pattern S;
  LevelInts ints;
  bool coarsest = false;
  bool user_p = false;             // P given by the caller (AMG_INTERP_USER)
  int prec = 64;                   // value type of this level's V-cycle work (64 or 32)
  double grad_ratio = 0.0;         // max over node stars of sum |A_BB| / (s^T A_BB s)
  int8_t* ssign = nullptr;         // per star row: G[row, node of its star]
  // device: A
  int64_t n = 0, nnz = 0;
  int64_t* A_ptr = nullptr;
  int32_t* A_col = nullptr;
  double* A_val = nullptr;
  float* A_val32 = nullptr;
  int lpr_A = 8;
  // device: P and P^T
  int64_t nc = 0, p_nnz = 0;
  int64_t* P_ptr = nullptr;
  int32_t* P_col = nullptr;
  double* P_val = nullptr;
  float* P_val32 = nullptr;
  int8_t* P_sign = nullptr;
  int64_t* PT_ptr = nullptr;
  int32_t* PT_col = nullptr;
  double* PT_val = nullptr;
  float* PT_val32 = nullptr;
  int64_t* PT_perm = nullptr;
  int lpr_P = 4, lpr_PT = 8;
  int p_row_max = 0;               // widest row of P's structural pattern
  std::vector<int64_t> p_ptr_h;   // host copy of P's current pattern
  std::vector<int32_t> p_col_h;
  int32_t* dof_stage = nullptr;
  // patch extension: per-column interior supports, their P entries, R rows
  int64_t* patch_ptr = nullptr;
  int32_t* patch_dofs = nullptr;
  int32_t* r_d1 = nullptr;
  int32_t* r_d2 = nullptr;
  int8_t* r_sg1 = nullptr;
  int8_t* r_sg2 = nullptr;
  int64_t* blk_ptr = nullptr;
  int32_t* blk_dofs = nullptr;
  std::vector<Stage> stages;
  int rap_mmax = 0, ap_mmax = 0;
  int32_t* ap_wide = nullptr;    // rows of A P / P^T (A P) too long for the LDS numeric pass
  int32_t* rap_wide = nullptr;
  int64_t ap_nwide = 0, rap_nwide = 0;
  int64_t ap_nnz = 0;
  int64_t* AP_ptr = nullptr;     // A P (n x nc), kept for numeric re-setup
  int32_t* AP_col = nullptr;
  double* AP_val = nullptr;
  // device: smoother
  int64_t nstars = 0;
  int64_t star_rows = 0, star_row_nnz = 0;   // star rows and their A entries (for byte counts)
  int ncolours = 0;
  std::vector<int> colour_chunk;
  int32_t* colour_chunk_dev = nullptr;
  int32_t* chunk_colour = nullptr;
  int sweep_mode = SWEEP_COLOUR;
  int wg_S = 256;
  int pipe_grid = 0;
  int pipe_u = 8;
  int32_t* sweep_sync = nullptr;   // pipelined sweep: ticket + per-colour counters
  int32_t* chunk_blk = nullptr;
  int32_t* ck_row0 = nullptr;
  int64_t* ck_q = nullptr;
  int4* ck_row = nullptr;
  int64_t* ck_fac0 = nullptr;
  int64_t srow_nnz = 0;
  int64_t* srow_ptr = nullptr;     // the smoother's copy of A's rows in star order
  int32_t* scol = nullptr;
  double* sval = nullptr;
  float* sval32 = nullptr;
  int64_t* sb_ptr = nullptr;
  int32_t* sb_dofs = nullptr;
  int64_t* fac_off = nullptr;
  int64_t fac_total = 0;
  double* fac = nullptr;
  float* fac32 = nullptr;
  double* binv = nullptr;        // symmetric block inverses, packed like fac
  float* binv32 = nullptr;
  int32_t* row_blk = nullptr;    // block of each star row
  double* dinv = nullptr;
  float* dinv32 = nullptr;
  int lpr_S = 8;
  int max_block = 0;
  double* Acm = nullptr;         // column-major dense A (dense and panel forms)
  float* Acm32 = nullptr;
  int ngroups = 0;               // panel form: groups of consecutive blocks (PanelDev tables)
  int32_t *gdof = nullptr, *gsl = nullptr, *gblk = nullptr, *dgrp = nullptr, *docc = nullptr;
  int32_t* row_slot = nullptr;   // group slot g * 64 + t of each star row
  double *gslc = nullptr, *gcf = nullptr, *gcb = nullptr, *gbinv = nullptr, *dsl = nullptr;
  float *gslc32 = nullptr, *gcf32 = nullptr, *gcb32 = nullptr, *gbinv32 = nullptr, *dsl32 = nullptr;
  int* psync = nullptr;
  // device: cycle vectors
  double *x = nullptr, *t = nullptr, *b = nullptr, *r = nullptr;
  float *x32 = nullptr, *t32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  // coarsest factor
  double* Lc = nullptr;

  template <class T>
  CsrDev<T> A_dev() const {
    CsrDev<T> m;
    m.n = n; m.m = n; m.nnz = nnz; m.ptr = A_ptr; m.col = A_col; m.lpr = lpr_A;
    if constexpr (std::is_same<T, double>::value) m.val = A_val; else m.val = A_val32;
    return m;
  }
  template <class T>
  CsrDev<T> P_dev() const {
    CsrDev<T> m;
    m.n = n; m.m = nc; m.nnz = p_nnz; m.ptr = P_ptr; m.col = P_col; m.lpr = lpr_P;
    if constexpr (std::is_same<T, double>::value) m.val = P_val; else m.val = P_val32;
    return m;
  }
  template <class T>
  CsrDev<T> PT_dev() const {
    CsrDev<T> m;
    m.n = nc; m.m = n; m.nnz = p_nnz; m.ptr = PT_ptr; m.col = PT_col; m.lpr = lpr_PT;
    if constexpr (std::is_same<T, double>::value) m.val = PT_val; else m.val = PT_val32;
    return m;
  }
  template <class T>
  SmootherDev<T> S_dev(int* err, int spin_max) const {
    SmootherDev<T> s;
    s.ncolours = ncolours; s.colour_chunk = colour_chunk_dev; s.colour_chunk_h = colour_chunk;
    s.chunk_colour = chunk_colour; s.chunk_blk = chunk_blk;
    s.sb_ptr = sb_ptr; s.sb_dofs = sb_dofs; s.fac_off = fac_off;
    s.ck_row0 = ck_row0; s.ck_fac0 = ck_fac0; s.srow_ptr = srow_ptr; s.scol = scol;
    s.ck_q = ck_q; s.ck_row = ck_row;
    if constexpr (std::is_same<T, double>::value) {
      s.fac = fac;
      s.binv = binv;
      s.sval = sval;
    } else {
      s.fac = fac32;
      s.binv = binv32;
      s.sval = sval32;
    }
    s.row_blk = row_blk;
    s.sync = sweep_sync; s.err = err; s.spin_max = spin_max;
    s.mode = sweep_mode; s.wg = wg_S; s.lpr = lpr_S; s.pipe_grid = pipe_grid; s.pipe_u = pipe_u;
    s.n = (int)n;
    s.pn.n = (int)n;
    s.pn.ngroups = ngroups;
    s.pn.gdof = gdof; s.pn.gsl = gsl; s.pn.gblk = gblk; s.pn.dgrp = dgrp; s.pn.docc = docc;
    s.pn.sync = psync;
    if constexpr (std::is_same<T, double>::value) {
      s.pn.gslc = gslc; s.pn.gcf = gcf; s.pn.gcb = gcb; s.pn.gbinv = gbinv; s.pn.dsl = dsl;
      s.pn.Acm = Acm;
    } else {
      s.pn.gslc = gslc32; s.pn.gcf = gcf32; s.pn.gcb = gcb32; s.pn.gbinv = gbinv32; s.pn.dsl = dsl32;
      s.pn.Acm = Acm32;
    }
    s.nblocks = (int)nstars;
    s.max_block = max_block;
    if constexpr (std::is_same<T, double>::value) {
      s.Acm = Acm;
      s.rtmp = r;
    } else {
      s.Acm = Acm32;
      s.rtmp = r32;
    }
    return s;
  }
};

}  // namespace

struct amg_hier {
  amg_options opt;
  std::vector<Level> lv;
  Pool pool;
  int prec = 64;
  int* d_flag = nullptr;        // non-SPD / overflow flags
  int* d_sweep_err = nullptr;   // set by a pipelined smoother sweep whose wait gave up
  int spin_max = 1 << 20;       // polls before such a wait gives up
  int cu_count = 256;
  bool a_borrowed = false;      // level 0 reads the caller's A in place (amg_options.borrow_a)
  double* d_sc = nullptr;       // CG scalars
  double* d_partial = nullptr;  // reduction partials
  int64_t partial_cap = 0;
  double* h_sc = nullptr;       // pinned host mirror of the scalars
  double* dense_work = nullptr;
  // PCG vectors
  double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr, *prold = nullptr;
  // V-cycles captured as HIP graphs, one per (r, z) buffer pair, replayed on
  // a library stream ordered after / before the caller's stream by events
  struct Graph {
    const double* r;
    double* z;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  // learned setup (finest-level extension blocks)
  MlpDev mlp;
  MlpWork work;
  int64_t mlp_nb = 0, mlp_rows = 0;     // blocks, rows padded to a multiple of 16
  uint16_t* fX = nullptr;                // features (mlp_rows x 64, BF16)
  float* fT = nullptr;                   // exact targets (mlp_rows x 64)
  float* fY = nullptr;                   // predictions
  double* fAhat = nullptr;               // normalised blocks (36 packed)
  double* fdsq = nullptr;                // sqrt of the block diagonals (8)
  double* fW = nullptr;                  // refined accepted inverses (36 packed)
  int8_t* fel = nullptr;                 // eligible
  int8_t* facc = nullptr;                // accepted
  float* fres = nullptr;                 // refinement residual
  uint16_t* bX = nullptr;                // batch buffers
  float *bT = nullptr, *bY = nullptr, *bdY = nullptr, *bloss = nullptr;
  int32_t* bidx = nullptr;
  int64_t batch_cap = 0;
  bool learned = false;
  amg_mlp_use_cfg use_cfg{};
  amg_mlp_stats mstats{};
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool use_graphs = true;
  ~amg_hier() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (h_sc) (void)hipHostFree(h_sc);
  }
};

namespace {

void check_flag(amg_hier* h, hipStream_t st, amg_status code, const std::string& msg) {
  int f = 0;
  HIPC(hipMemcpyAsync(&f, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (f) {
    HIPC(hipMemsetAsync(h->d_flag, 0, sizeof(int), st));
    HIPC(hipStreamSynchronize(st));
    fail(code, msg);
  }
}

// A pipelined smoother sweep whose wait gave up leaves its result wrong and
// raises this flag (sticky for the handle's lifetime).
void check_sweep_err(amg_hier* h, hipStream_t st) {
  int f = 0;
  HIPC(hipMemcpyAsync(&f, h->d_sweep_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (f) fail(AMG_ERR_HIP, "a pipelined smoother sweep timed out waiting for the previous colour");
}

// Host copies of a CSR (pattern, and values if wanted).
// (sg: pinned staging for device arrays; NULL copies them directly)
void host_csr(const amg_csr* M, std::vector<int64_t>& ptr, std::vector<int32_t>& col,
              std::vector<double>* val, Staging* sg = nullptr) {
  auto d2h = [&](void* dst, const void* src, size_t bytes) {
    if (sg) sg->d2h(dst, src, bytes, nullptr);
    else HIPC(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  };
  ptr.resize(M->nrows + 1);
  if (M->on_device) {
    d2h(ptr.data(), M->rowptr, ptr.size() * sizeof(int64_t));
  } else {
    std::memcpy(ptr.data(), M->rowptr, ptr.size() * sizeof(int64_t));
  }
  int64_t nnz = ptr.back();
  if (nnz != M->nnz) fail(AMG_ERR_CSR, "rowptr[nrows] != nnz");
  col.resize(nnz);
  if (val) val->resize(nnz);
  if (M->on_device) {
    d2h(col.data(), M->colidx, nnz * sizeof(int32_t));
    if (val) d2h(val->data(), M->val, nnz * sizeof(double));
  } else {
    std::memcpy(col.data(), M->colidx, nnz * sizeof(int32_t));
    if (val) std::memcpy(val->data(), M->val, nnz * sizeof(double));
  }
}

// --- smoother: colour-sorted star blocks, chunks, factors, l1 diagonal ---
// Sweep form of a level (chosen from measurements on MI355X):
//   pipe    16 or more colours: one launch, colours pipelined across
//           workgroups (a launch per colour would leave the GPU idle between
//           short colours);
//   panel   16 or more colours, n <= 32768, and rows longer than 4096
//           entries, at most 1.5 blocks per colour, or no more groups of 64
//           star rows than colours (at most 60 star rows per colour): the
//           Galerkin operators near the bottom of the hierarchy are nearly
//           dense, a pipelined chunk would stream thousands of entries per
//           block, and every colour step of the pipe is a full round of
//           inter-workgroup signalling; instead one workgroup chains groups
//           of blocks (a group costs about what one pipelined colour does)
//           while the others apply each group's residual update to their
//           rows from a dense copy of A;
//   one     small level with fewer colours: the whole sweep in one workgroup;
//   colour  one launch per colour (the finest levels: few colours, many blocks);
//   dense   nearly sequential level (at most 1.5 blocks per colour): block by
//           block in one workgroup with the residual and a dense copy of A
//           in LDS (n <= 2048, or in global memory up to 16384 rows);
//           available on request.
// HCURL_AMG_SWEEP=colour|one|pipe|dense|panel forces a form where it applies
// (dense and panel need a level that fits their kernels); HCURL_AMG_DENSE_SWEEP=0
// turns the dense form off.
int sweep_mode_for(int64_t n, int64_t nnz, int64_t ns, int64_t nrows, int ncolours, int maxs) {
  const char* dense_env = std::getenv("HCURL_AMG_DENSE_SWEEP");
  const bool dense_any = !(dense_env && dense_env[0] == '0') && dense_sweep_ok<double>((int)n, maxs);
  const bool panel_ok = panel_sweep_ok((int)std::min<int64_t>(n, INT32_MAX), maxs);
  int mode = SWEEP_COLOUR;
  if (ncolours >= 16) {
    // one launch per colour while a colour holds 1,024 to 16,383 star rows:
    // enough rows to fill the device per launch, few enough that the
    // pipelined form's ticket and counter traffic does not pay (measured at
    // 128^3: 1,824 rows per colour 0.71 ms per sweep against 1.22 ms
    // pipelined; 26,300 rows 2.48 ms against 2.00 ms; 140 rows 0.76 against
    // 0.56 ms)
    const int64_t per = nrows / std::max(ncolours, 1);
    if (panel_ok && (nnz > 4096 * n || 2 * ns <= 3 * (int64_t)ncolours ||
                     nrows <= 60 * (int64_t)ncolours))
      mode = SWEEP_PANEL;
    else if (per >= 1024 && per < 16384)
      mode = SWEEP_COLOUR;
    else
      mode = SWEEP_PIPE;
  } else if (nnz <= 200000) {
    mode = SWEEP_ONE;
  }
  if (const char* e = std::getenv("HCURL_AMG_SWEEP")) {
    const std::string f(e);
    if (f == "colour") mode = SWEEP_COLOUR;
    else if (f == "one") mode = SWEEP_ONE;
    else if (f == "pipe") mode = SWEEP_PIPE;
    else if (f == "dense" && dense_any && 2 * ns <= 3 * (int64_t)ncolours) mode = SWEEP_DENSE;
    else if (f == "panel" && panel_ok) mode = SWEEP_PANEL;
  }
  return mode;
}

// Groups of the panel form: consecutive blocks (colour order) with at most
// PANEL_GROUP_SLOTS rows; each DoF's groups (at most two: a DoF lies in at
// most two node stars) and, per star row, the other row of the same DoF in
// its group.  False if a DoF lies in more than two groups, or in more than
// two rows of one group (the form then does not apply).
bool build_panel_groups(const std::vector<int64_t>& sb_ptr, const std::vector<int32_t>& sb_dofs,
                        int64_t n, std::vector<int32_t>& grp_blk, std::vector<int32_t>& dgrp,
                        std::vector<int32_t>& sdup) {
  const int64_t ns = (int64_t)sb_ptr.size() - 1;
  grp_blk.clear();
  int64_t t = 0;
  while (t < ns) {
    grp_blk.push_back((int32_t)t);
    int64_t rows = 0;
    while (t < ns && rows + (sb_ptr[t + 1] - sb_ptr[t]) <= PANEL_GROUP_SLOTS) {
      rows += sb_ptr[t + 1] - sb_ptr[t];
      ++t;
    }
    if (rows == 0) return false;   // a block larger than a group
  }
  grp_blk.push_back((int32_t)ns);
  dgrp.assign(2 * n, -1);
  sdup.assign(sb_dofs.size(), -1);
  std::vector<int32_t> seen(n, -1);   // row of the DoF inside the current group
  const int G = (int)grp_blk.size() - 1;
  for (int g = 0; g < G; ++g) {
    const int64_t q0 = sb_ptr[grp_blk[g]], q1 = sb_ptr[grp_blk[g + 1]];
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t d = sb_dofs[q];
      if (seen[d] >= 0) {
        const int64_t q2 = q0 + seen[d];
        if (sdup[q2] >= 0) return false;   // a third row of one DoF in a group
        sdup[q2] = (int32_t)(q - q0);
        sdup[q] = seen[d];
        continue;
      }
      seen[d] = (int32_t)(q - q0);
      if (dgrp[2 * d] < 0) dgrp[2 * d] = g;
      else if (dgrp[2 * d + 1] < 0) dgrp[2 * d + 1] = g;
      else return false;                   // a DoF in a third group
    }
    for (int64_t q = q0; q < q1; ++q) seen[sb_dofs[q]] = -1;
  }
  return true;
}

// Padded per-group tables of the panel form (layouts in PanelDev): per slot
// its DoF, its block's first slot and the slot of the same DoF in the
// neighbouring groups; per block its first slot, size and run of one colour
// inside the group; per DoF its slots; per star row its group slot.  False
// if a DoF has more than two slots (the form then does not apply).
bool build_panel_tables(const std::vector<int64_t>& sb_ptr, const std::vector<int32_t>& sb_dofs,
                        const std::vector<int32_t>& blk_col, const std::vector<int32_t>& grp_blk,
                        int64_t n, std::vector<int32_t>& gdof, std::vector<int32_t>& gsl,
                        std::vector<int32_t>& gblk, std::vector<int32_t>& docc,
                        std::vector<int32_t>& row_slot) {
  constexpr int S = PANEL_GROUP_SLOTS;
  const int G = (int)grp_blk.size() - 1;
  gdof.assign((size_t)G * S, -1);
  gsl.assign((size_t)G * S, 0);
  gblk.assign((size_t)G * S, -1);
  docc.assign(2 * n, -1);
  row_slot.assign(sb_dofs.size(), 0);
  for (int g = 0; g < G; ++g) {
    const int bb0 = grp_blk[g], bb1 = grp_blk[g + 1];
    const int64_t q0 = sb_ptr[bb0];
    for (int b = bb0; b < bb1; ++b) {
      int lo = b, hi = b;
      while (lo > bb0 && blk_col[lo - 1] == blk_col[b]) --lo;
      while (hi + 1 < bb1 && blk_col[hi + 1] == blk_col[b]) ++hi;
      const int p = (int)(sb_ptr[b] - q0), sz = (int)(sb_ptr[b + 1] - sb_ptr[b]);
      gblk[(size_t)g * S + (b - bb0)] = p | sz << 8 | (lo - bb0) << 16 | (hi - bb0) << 24;
      for (int t = p; t < p + sz; ++t) {
        const int32_t d = sb_dofs[q0 + t];
        gdof[(size_t)g * S + t] = d;
        gsl[(size_t)g * S + t] = p;
        row_slot[q0 + t] = g * S + t;
        if (docc[2 * d] < 0) docc[2 * d] = g * S + t;
        else if (docc[2 * d + 1] < 0) docc[2 * d + 1] = g * S + t;
        else return false;
      }
    }
  }
  for (int g = 0; g < G; ++g)
    for (int t = 0; t < S; ++t) {
      const int32_t d = gdof[(size_t)g * S + t];
      if (d < 0) continue;
      const int self = g * S + t;
      const int other = docc[2 * d] == self ? docc[2 * d + 1] : docc[2 * d];
      if (other < 0) continue;
      if (other / S == g - 1) gsl[(size_t)g * S + t] |= (other % S + 1) << 8;
      if (other / S == g + 1) gsl[(size_t)g * S + t] |= (other % S + 1) << 16;
    }
  return true;
}

void build_smoother(amg_hier* h, Level& L, hipStream_t st) {
  const LevelInts& I = L.ints;
  int64_t ns = (int64_t)I.star_ptr.size() - 1;
  L.nstars = ns;
  L.ncolours = I.ncolors;
  L.star_rows = I.star_ptr.empty() ? 0 : I.star_ptr.back();
  L.star_row_nnz = 0;
  for (int64_t q = 0; q < L.star_rows; ++q) {
    const int32_t e = I.star_dofs[q];
    L.star_row_nnz += L.Apat.ptr[e + 1] - L.Apat.ptr[e];
  }
  int maxs = 0;
  for (int64_t b = 0; b < ns; ++b) maxs = std::max<int>(maxs, (int)(I.star_ptr[b + 1] - I.star_ptr[b]));
  if (maxs > 32) fail(AMG_ERR_LIMIT, "smoother block with more than 32 DoFs");
  L.max_block = maxs;
  L.sweep_mode = sweep_mode_for(L.n, L.nnz, ns, (int64_t)I.star_dofs.size(), I.ncolors, maxs);
  // lanes per row from the row length; a chunk (wg / lpr rows) must hold a
  // whole block
  int lpr = L.lpr_A;
  int wg = 256;
  if (L.sweep_mode == SWEEP_PIPE) {
    // one chunk per 1024-thread workgroup.  Every lane loads its first 16
    // (column, value) pairs before the chunk waits for the colour before it
    // (8 at 8 lanes per row), so the fewest lanes whose 16 pairs hold an
    // average row (up to 17 entries per lane) give the most rows per chunk
    // with the whole row in flight: at 128^3, level 1 (266 entries per row)
    // sweeps in 1.74 ms at 16 lanes against 1.98 ms at 32 lanes with 8 pairs
    const double avg_row = L.n > 0 ? (double)L.nnz / (double)L.n : 0.0;
    wg = 1024;
    lpr = 8;
    while (lpr < 256 && avg_row > 17.0 * lpr && 1024 / (2 * lpr) >= std::max(maxs, 1)) lpr *= 2;
    if (const char* e = std::getenv("HCURL_AMG_PIPE_LPR")) lpr = std::max(8, std::min(256, std::atoi(e)));
    while (1024 / lpr < std::max(maxs, 1)) lpr /= 2;
  } else {
    if (const char* e = std::getenv("HCURL_AMG_COLOUR_LPR")) lpr = std::max(4, std::min(64, std::atoi(e)));
    while (wg / lpr < std::max(maxs, 1) && wg < 1024) wg *= 2;
    while (wg / lpr < std::max(maxs, 1) && lpr > 4) lpr /= 2;
    if (wg > 256 && lpr < 16) {   // wide workgroups only pay off with wide rows
      wg = 256;
      while (256 / lpr < std::max(maxs, 1)) lpr /= 2;
    }
  }
  if (!schwarz_shape_ok(lpr, wg) || wg / lpr < std::max(maxs, 1))
    fail(AMG_ERR_LIMIT, "no smoother launch shape for this level");
  L.lpr_S = lpr;
  L.wg_S = wg;
  // pairs per lane loaded before a pipelined chunk waits: 16 from 16 lanes
  // per row on, 8 at 8 lanes (HCURL_AMG_PIPE_U=8 selects 8 at 16 and 32)
  L.pipe_u = lpr >= 16 ? 16 : 8;
  if (const char* e = std::getenv("HCURL_AMG_PIPE_U"))
    if (std::atoi(e) == 8 && (lpr == 16 || lpr == 32)) L.pipe_u = 8;
  const int rpb = wg / lpr;
  // blocks in (colour, id) order
  std::vector<int64_t> order(ns);
  {
    std::vector<int64_t> cnt(I.ncolors + 1, 0);
    for (int64_t b = 0; b < ns; ++b) cnt[I.star_color[b] + 1]++;
    for (int c = 0; c < I.ncolors; ++c) cnt[c + 1] += cnt[c];
    for (int64_t b = 0; b < ns; ++b) order[cnt[I.star_color[b]]++] = b;
  }
  // node of each star (stars are built for the columns of G with a
  // non-empty support, in column order) and each star row's sign G[e, v]
  std::vector<int32_t> star_node;
  {
    std::vector<char> used(L.G.m, 0);
    for (int64_t e = 0; e < L.G.n; ++e) {
      if (L.G.a[e] >= 0) used[L.G.a[e]] = 1;
      if (L.G.b[e] >= 0) used[L.G.b[e]] = 1;
    }
    for (int64_t v = 0; v < L.G.m; ++v)
      if (used[v]) star_node.push_back((int32_t)v);
    if ((int64_t)star_node.size() != ns) fail(AMG_ERR_SHAPE, "star count differs from G's used columns");
  }
  std::vector<int64_t> sb_ptr(ns + 1, 0), fac_off(ns + 1, 0);
  std::vector<int32_t> sb_dofs;
  std::vector<int8_t> ssign;
  sb_dofs.reserve(I.star_dofs.size());
  ssign.reserve(I.star_dofs.size());
  for (int64_t t = 0; t < ns; ++t) {
    int64_t b = order[t];
    int64_t s = I.star_ptr[b + 1] - I.star_ptr[b];
    const int32_t v = star_node[b];
    for (int64_t q = I.star_ptr[b]; q < I.star_ptr[b + 1]; ++q) {
      const int32_t e = I.star_dofs[q];
      sb_dofs.push_back(e);
      ssign.push_back(L.G.a[e] == v ? L.G.sa[e] : L.G.sb[e]);
    }
    sb_ptr[t + 1] = sb_ptr[t] + s;
    fac_off[t + 1] = fac_off[t] + s * (s + 1) / 2;
  }
  if (sb_ptr[ns] > INT32_MAX) fail(AMG_ERR_LIMIT, "more than 2^31 smoother rows on one level");
  // chunks: consecutive blocks of one colour with at most rpb rows
  std::vector<int32_t> chunk_blk, chunk_colour;
  L.colour_chunk.assign(I.ncolors + 1, 0);
  bool every_colour = true;
  int64_t t = 0;
  for (int c = 0; c < I.ncolors; ++c) {
    L.colour_chunk[c] = (int)chunk_blk.size();
    while (t < ns && I.star_color[order[t]] == c) {
      chunk_blk.push_back((int32_t)t);
      chunk_colour.push_back(c);
      int64_t rows = 0;
      while (t < ns && I.star_color[order[t]] == c && rows + (sb_ptr[t + 1] - sb_ptr[t]) <= rpb) {
        rows += sb_ptr[t + 1] - sb_ptr[t];
        ++t;
      }
    }
    every_colour = every_colour && (int)chunk_blk.size() > L.colour_chunk[c];
  }
  L.colour_chunk[I.ncolors] = (int)chunk_blk.size();
  chunk_blk.push_back((int32_t)ns);
  const int nchunks = L.colour_chunk[I.ncolors];
  // the pipelined sweep waits on the colour before in sweep order, so every
  // colour must hold a chunk (greedy colourings use every colour they count)
  if (L.sweep_mode == SWEEP_PIPE && !every_colour) L.sweep_mode = SWEEP_COLOUR;
  // per-chunk first row and first factor entry, so that a chunk finds its
  // rows and factors with one lookup
  std::vector<int32_t> ck_row0(chunk_blk.size());
  std::vector<int64_t> ck_fac0(chunk_blk.size());
  for (size_t c = 0; c < chunk_blk.size(); ++c) {
    ck_row0[c] = (int32_t)sb_ptr[chunk_blk[c]];
    ck_fac0[c] = fac_off[chunk_blk[c]];
  }
  L.ck_row0 = h->pool.upload(ck_row0, st);
  L.ck_fac0 = h->pool.upload(ck_fac0, st);
  L.chunk_colour = h->pool.upload(chunk_colour.empty() ? std::vector<int32_t>{0} : chunk_colour, st);
  // the smoother's copy of A's rows in star order (pattern here, values at
  // every numeric setup)
  {
    const int64_t nr = sb_ptr[ns];
    std::vector<int64_t> srow_ptr(nr + 1, 0);
    for (int64_t r = 0; r < nr; ++r) {
      const int32_t d = sb_dofs[r];
      srow_ptr[r + 1] = srow_ptr[r] + (L.Apat.ptr[d + 1] - L.Apat.ptr[d]);
    }
    L.srow_nnz = srow_ptr[nr];
    L.srow_ptr = h->pool.upload(srow_ptr, st);

    L.scol = h->pool.get<int32_t>(std::max<int64_t>(L.srow_nnz, 1));   // gathered below
    L.sval = h->pool.get<double>(std::max<int64_t>(L.srow_nnz, 1));
  }
  L.chunk_blk = h->pool.upload(chunk_blk, st);
  L.colour_chunk_dev = h->pool.upload(std::vector<int32_t>(L.colour_chunk.begin(), L.colour_chunk.end()), st);
  L.sweep_sync = h->pool.get<int32_t>((size_t)SYNC_STRIDE * (I.ncolors + 1));
  int grid = h->cu_count;
  if (const char* e = std::getenv("HCURL_AMG_PIPE_GRID")) grid = std::max(1, std::atoi(e));
  L.pipe_grid = std::max(1, std::min(nchunks, grid));
  // the panel form needs all 1 + n/128 of its workgroups resident at once
  // (the chain and the tiles wait on each other): keep it only if the
  // device's CUs can hold them (occupancy query with the launch's LDS
  // padding, for every precision the hierarchy sweeps in); otherwise the
  // pipelined form, which needs no residency, takes the level
  if (L.sweep_mode == SWEEP_PANEL) {
    const int64_t need = 1 + (int64_t)panel_tiles((int)L.n);
    int per_cu = panel_resident_per_cu(64);
    if (h->prec == 32) per_cu = std::min(per_cu, panel_resident_per_cu(32));
    if (per_cu < 1 || need > (int64_t)per_cu * h->cu_count) L.sweep_mode = SWEEP_PIPE;
  }
  if (L.sweep_mode == SWEEP_PANEL) {
    std::vector<int32_t> grp_blk, dgrp, sdup, blk_col(ns), gdof, gsl, gblk, docc, row_slot;
    for (int64_t t = 0; t < ns; ++t) blk_col[t] = I.star_color[order[t]];
    if (build_panel_groups(sb_ptr, sb_dofs, L.n, grp_blk, dgrp, sdup) &&
        build_panel_tables(sb_ptr, sb_dofs, blk_col, grp_blk, L.n, gdof, gsl, gblk, docc, row_slot)) {
      L.ngroups = (int)grp_blk.size() - 1;
      const size_t G = (size_t)L.ngroups;
      L.gdof = h->pool.upload(gdof, st);
      L.gsl = h->pool.upload(gsl, st);
      L.gblk = h->pool.upload(gblk, st);
      L.dgrp = h->pool.upload(dgrp, st);
      L.docc = h->pool.upload(docc, st);
      L.row_slot = h->pool.upload(row_slot, st);
      L.dsl = h->pool.get<double>(G * PANEL_GROUP_SLOTS);
      L.psync = h->pool.get<int>(G * 2 * SYNC_STRIDE);
      L.gslc = h->pool.get<double>(G * PANEL_GROUP_SLOTS * PANEL_GROUP_SLOTS);
      L.gcf = h->pool.get<double>(G * PANEL_GROUP_SLOTS * PANEL_GROUP_SLOTS);
      L.gcb = h->pool.get<double>(G * PANEL_GROUP_SLOTS * PANEL_GROUP_SLOTS);
      L.gbinv = h->pool.get<double>(G * PANEL_GROUP_SLOTS * PANEL_ROW_WIDTH);
    } else {
      L.sweep_mode = SWEEP_PIPE;
    }
  }
  if (L.sweep_mode == SWEEP_DENSE || L.sweep_mode == SWEEP_PANEL)
    L.Acm = h->pool.get<double>((size_t)L.n * L.n);
  L.sb_ptr = h->pool.upload(sb_ptr, st);
  L.sb_dofs = h->pool.upload(sb_dofs, st);
  // the column ids of the star-ordered row copy, gathered on the device
  star_cols(sb_ptr[ns], L.sb_dofs, L.A_ptr, L.A_col, L.srow_ptr, L.scol, st);
  L.ssign = h->pool.upload(ssign, st);
  L.fac_off = h->pool.upload(fac_off, st);
  L.fac_total = fac_off[ns];
  L.fac = h->pool.get<double>(L.fac_total);
  L.binv = h->pool.get<double>(std::max<int64_t>(L.fac_total, 1));
  {
    std::vector<int32_t> row_blk(std::max<int64_t>(sb_ptr[ns], 1), 0);
    for (int64_t b = 0; b < ns; ++b)
      for (int64_t r = sb_ptr[b]; r < sb_ptr[b + 1]; ++r) row_blk[r] = (int32_t)b;
    L.row_blk = h->pool.upload(row_blk, st);
  }
  L.dinv = h->pool.get<double>(L.n);
  // per chunk, padded to rpb row slots: entry ranges and {DoF, block start
  // in the chunk, block size, factor offset in the chunk}, built on the
  // device from the arrays above
  L.ck_q = h->pool.get<int64_t>((size_t)nchunks * (rpb + 1));
  L.ck_row = reinterpret_cast<int4*>(h->pool.get<int32_t>((size_t)nchunks * rpb * 4));
  chunk_tables(nchunks, rpb, L.ck_row0, L.ck_fac0, L.srow_ptr, L.sb_dofs, L.row_blk, L.sb_ptr,
               L.fac_off, L.ck_q, L.ck_row, st);
  HIPC(hipGetLastError());
}

void factor_smoother(amg_hier* h, Level& L, int level, hipStream_t st) {
  if (L.sweep_mode == SWEEP_DENSE || L.sweep_mode == SWEEP_PANEL)
    csr_to_dense_cm(L.n, L.A_ptr, L.A_col, L.A_val, L.Acm, st);
  if (L.sweep_mode == SWEEP_PANEL)
    panel_slices(L.ngroups, L.n, L.gdof, L.Acm, L.gslc, L.gcf, L.gcb, st);
  star_rows((int64_t)L.ints.star_dofs.size(), L.sb_dofs, L.A_ptr, L.A_val, L.srow_ptr, L.sval, st);
  star_chol(L.nstars, L.sb_ptr, L.sb_dofs, L.fac_off, L.A_dev<double>(), L.fac, h->d_flag, st);
  HIPC(hipGetLastError());
  check_flag(h, st, AMG_ERR_NOT_SPD, "smoother block Cholesky: non-positive pivot on level " +
                                         std::to_string(level));
  star_inv((int64_t)L.ints.star_dofs.size(), L.row_blk, L.sb_ptr, L.fac_off, L.fac, L.binv, st);
  if (L.sweep_mode == SWEEP_PANEL) {
    fill<double>((int64_t)L.ngroups * PANEL_GROUP_SLOTS * PANEL_ROW_WIDTH, 0.0, L.gbinv, st);
    pad_inv((int64_t)L.ints.star_dofs.size(), L.row_blk, L.row_slot, L.sb_ptr, L.fac_off, L.binv,
            L.gbinv, st);
  }
  l1inv(L.A_dev<double>(), L.dinv, st);
}

// --- interpolation: pattern upload, exterior signs, stage-by-stage blocks ---
void build_interp_structs(amg_hier* h, Level& L, hipStream_t st) {
  const LevelInts& I = L.ints;
  L.nc = (int64_t)I.r_dof1.size();
  L.p_nnz = I.p.nnz();
  L.P_ptr = h->pool.upload(I.p.ptr, st);
  L.P_col = h->pool.upload(I.p.idx, st);
  L.P_sign = h->pool.upload(I.p_ext_sign, st);
  L.P_val = h->pool.get<double>(L.p_nnz);
  L.lpr_P = lpr_for(L.n, L.p_nnz);
  L.dof_stage = h->pool.upload(I.dof_stage, st);
  L.stages.clear();
  if (I.patch) {
    if (I.patch_max > PATCH_CAP_MAX) fail(AMG_ERR_LIMIT, "patch larger than the kernel's LDS holds");
    L.patch_ptr = h->pool.upload(I.patch_ptr, st);
    L.patch_dofs = h->pool.upload(I.patch_dofs, st);
    L.r_d1 = h->pool.upload(I.r_dof1, st);
    L.r_d2 = h->pool.upload(I.r_dof2, st);
    L.r_sg1 = h->pool.upload(I.r_s1, st);
    L.r_sg2 = h->pool.upload(I.r_s2, st);
  }
  L.blk_ptr = h->pool.upload(I.block_ptr, st);
  L.blk_dofs = h->pool.upload(I.block_dofs, st);
  int64_t nst = I.patch ? 0 : (int64_t)I.stage_ptr.size() - 1;
  for (int64_t s = 0; s < nst; ++s) {
    Stage S{I.stage_ptr[s], I.stage_ptr[s + 1] - I.stage_ptr[s], 0, 0};
    for (int64_t b = I.stage_ptr[s]; b < I.stage_ptr[s + 1]; ++b) {
      int sz = (int)(I.block_ptr[b + 1] - I.block_ptr[b]);
      int32_t d0 = I.block_dofs[I.block_ptr[b]];
      int cc = (int)(I.p.ptr[d0 + 1] - I.p.ptr[d0]);
      S.smax = std::max(S.smax, sz);
      S.cmax = std::max(S.cmax, cc);
    }
    if (S.smax > 64)
      fail(AMG_ERR_LIMIT, "extension block with more than 64 DoFs (" + std::to_string(S.smax) + ")");
    if (ext_block_tile(S.smax) < 1)
      fail(AMG_ERR_LIMIT, "extension block of " + std::to_string(S.smax) + " DoFs does not fit LDS");
    if ((S.cmax + ext_block_tile(S.smax) - 1) / ext_block_tile(S.smax) > 65535)
      fail(AMG_ERR_LIMIT, "extension block with too many P columns (" + std::to_string(S.cmax) + ")");
    L.stages.push_back(S);
  }
  L.p_ptr_h = I.p.ptr;
  L.p_col_h = I.p.idx;
  L.p_row_max = 0;
  for (int64_t i = 0; i < L.n; ++i)
    L.p_row_max = std::max<int>(L.p_row_max, (int)(I.p.ptr[i + 1] - I.p.ptr[i]));
}

// P^T pattern and the permutation P entry -> P^T entry, from the host copy of
// P's (possibly truncated) pattern
void build_transpose(amg_hier* h, Level& L, hipStream_t st) {
  const int64_t n = L.n, nc = L.nc, nnz = L.p_nnz;
  L.PT_val = h->pool.get<double>(std::max<int64_t>(nnz, 1));
  L.lpr_PT = lpr_for(nc, nnz);
  if (nnz < (int64_t)INT32_MAX && nc < (int64_t)INT32_MAX) {
    // on the device from P's uploaded pattern (a stable sort by column)
    L.PT_ptr = h->pool.get<int64_t>(nc + 1);
    L.PT_col = h->pool.get<int32_t>(std::max<int64_t>(nnz, 1));
    L.PT_perm = h->pool.get<int64_t>(std::max<int64_t>(nnz, 1));
    HIPC(transpose_pattern(n, nc, nnz, L.P_ptr, L.P_col, L.PT_ptr, L.PT_col, L.PT_perm, st));
    return;
  }
  // parallel transpose: thread t takes rows [e0(t), e1(t)) of P and counts
  // its entries per column; a column's entries from thread t follow those of
  // threads < t, so P^T's rows come out in ascending P-row order
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 4096));
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::vector<int64_t>> cnt(nt);
  auto run = [&](const std::function<void(int)>& body) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(body, t);
    for (auto& x : th) x.join();
  };
  run([&](int t) {
    cnt[t].assign(nc, 0);
    const int64_t e0 = std::min(n, t * chunk), e1 = std::min(n, e0 + chunk);
    for (int64_t q = L.p_ptr_h[e0]; q < L.p_ptr_h[e1]; ++q) ++cnt[t][L.p_col_h[q]];
  });
  std::vector<int64_t> tptr(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) {
    int64_t acc = tptr[c];
    for (int t = 0; t < nt; ++t) {
      const int64_t k = cnt[t][c];
      cnt[t][c] = acc;
      acc += k;
    }
    tptr[c + 1] = acc;
  }
  std::vector<int64_t> perm(nnz);
  std::vector<int32_t> tcol(nnz);
  run([&](int t) {
    const int64_t e0 = std::min(n, t * chunk), e1 = std::min(n, e0 + chunk);
    for (int64_t e = e0; e < e1; ++e)
      for (int64_t q = L.p_ptr_h[e]; q < L.p_ptr_h[e + 1]; ++q) {
        const int64_t d = cnt[t][L.p_col_h[q]]++;
        tcol[d] = (int32_t)e;
        perm[q] = d;
      }
  });
  L.PT_ptr = h->pool.upload(tptr, st);
  L.PT_col = h->pool.upload(tcol, st);
  L.PT_perm = h->pool.upload(perm, st);
  // the uploads read tcol and perm before they go out of scope
  HIPC(hipStreamSynchronize(st));
}

// Optional sparsification (not in the paper): drop interior-row entries of
// P with |p| < tau * (row max |p|); exterior rows are kept.  Same rule as the
// oracle's truncate_interior.
void truncate_interp(amg_hier* h, Level& L, double tau, hipStream_t st) {
  std::vector<double> val(L.p_nnz);
  HIPC(hipMemcpyAsync(val.data(), L.P_val, L.p_nnz * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  std::vector<int64_t> nptr(L.n + 1, 0);
  std::vector<int32_t> ncol;
  std::vector<double> nval;
  ncol.reserve(L.p_nnz);
  nval.reserve(L.p_nnz);
  for (int64_t e = 0; e < L.n; ++e) {
    const bool interior = L.ints.dof_stage[e] >= 0;
    double mx = 0.0;
    for (int64_t q = L.p_ptr_h[e]; q < L.p_ptr_h[e + 1]; ++q) mx = std::max(mx, std::fabs(val[q]));
    for (int64_t q = L.p_ptr_h[e]; q < L.p_ptr_h[e + 1]; ++q)
      if (!interior || std::fabs(val[q]) >= tau * mx) {
        ncol.push_back(L.p_col_h[q]);
        nval.push_back(val[q]);
      }
    nptr[e + 1] = (int64_t)ncol.size();
  }
  L.p_ptr_h = std::move(nptr);
  L.p_col_h = std::move(ncol);
  L.p_nnz = (int64_t)nval.size();
  L.P_ptr = h->pool.upload(L.p_ptr_h, st);
  L.P_col = h->pool.upload(L.p_col_h, st);
  L.P_val = h->pool.upload(nval, st);
  L.lpr_P = lpr_for(L.n, L.p_nnz);
}

void compute_interp(amg_hier* h, Level& L, int level, hipStream_t st, bool learned = false) {
  sign_to_val(L.p_nnz, L.P_sign, L.P_val, st);   // untruncated pattern (p_trunc = 0 here)
  if (L.ints.patch)
    ext_patches(L.nc, L.patch_ptr, L.patch_dofs, L.P_ptr, L.P_col, L.r_d1, L.r_d2, L.r_sg1,
                L.r_sg2, L.A_dev<double>(), L.P_val, L.ints.patch_max, h->d_flag, st);
  for (size_t s = 0; s < L.stages.size(); ++s) {
    const Stage& S = L.stages[s];
    ext_blocks(S.b0, S.nb, L.blk_ptr, L.blk_dofs, L.dof_stage, (int)s, L.A_dev<double>(), L.P_ptr,
               L.P_col, L.P_val, S.smax, S.cmax, L.p_row_max, h->d_flag, st, learned ? h->fW : nullptr,
               learned ? h->facc : nullptr, learned ? h->fdsq : nullptr);
  }
  HIPC(hipGetLastError());
  check_flag(h, st, AMG_ERR_NOT_SPD,
             "local harmonic extension: non-positive pivot in A_BB on level " + std::to_string(level));
}

// --- caller-given interpolation (AMG_INTERP_USER) ---
void load_user_interp(amg_hier* h, Level& L, const amg_csr& P, int level, hipStream_t st) {
  const std::string lv = "user P on level " + std::to_string(level);
  if (P.nrows != L.n) fail(AMG_ERR_SHAPE, lv + ": rows differ from the level's DoFs");
  if (P.ncols < 1 || P.ncols >= L.n) fail(AMG_ERR_SHAPE, lv + ": needs 1 <= columns < rows");
  if (!P.rowptr || (P.nnz > 0 && (!P.colidx || !P.val))) fail(AMG_ERR_ARG, lv + ": NULL pointer");
  std::vector<double> val;
  host_csr(&P, L.p_ptr_h, L.p_col_h, &val);
  HostError err;
  if (!validate_pattern(P.nrows, P.ncols, L.p_ptr_h.data(), L.p_col_h.data(), err))
    fail((amg_status)err.code, lv + ": " + err.msg);
  L.user_p = true;
  L.nc = P.ncols;
  L.p_nnz = P.nnz;
  L.P_ptr = h->pool.upload(L.p_ptr_h, st);
  L.P_col = h->pool.upload(L.p_col_h, st);
  L.P_val = h->pool.upload(val, st);
  L.lpr_P = lpr_for(L.n, L.p_nnz);
  L.p_row_max = 0;
  for (int64_t i = 0; i < L.n; ++i)
    L.p_row_max = std::max<int>(L.p_row_max, (int)(L.p_ptr_h[i + 1] - L.p_ptr_h[i]));
  HIPC(hipStreamSynchronize(st));
}

Incidence user_gradient(const amg_csr& G, int64_t n, int level) {
  const std::string lv = "user G on level " + std::to_string(level);
  if (!G.rowptr || (G.nnz > 0 && (!G.colidx || !G.val))) fail(AMG_ERR_ARG, lv + ": NULL pointer");
  if (G.nrows != n) fail(AMG_ERR_SHAPE, lv + ": rows differ from the level's DoFs");
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  host_csr(&G, ptr, col, &val);
  Incidence out;
  HostError err;
  if (!incidence_from_csr(G.nrows, G.ncols, ptr.data(), col.data(), val.data(), out, err))
    fail((amg_status)err.code, lv + ": " + err.msg);
  return out;
}

// --- Galerkin product A_c = P^T (A P): symbolic (once) and numeric ---
// C = X Y symbolic: row counts, host scan, sorted columns.  Rows with more
// distinct columns than the LDS hash holds take the bitset passes.  Returns
// the numeric pass's LDS row capacity; rows longer than that are listed in
// `wide` (device) for the numeric pass's wide kernel.
constexpr int64_t MM_LDS_ROW = 65536 / (sizeof(double) + sizeof(int32_t));

int64_t mm_symbolic(amg_hier* h, int64_t nrows, int64_t ncols, const CsrPat& X, const CsrPat& Y,
                    std::vector<int64_t>& cptr, int64_t*& d_cptr, int32_t*& d_ccol,
                    int32_t*& d_wide, int64_t& nwide, const std::string& what, hipStream_t st) {
  StepTimer tm;
  int64_t* d_cnt = h->pool.get<int64_t>(nrows);
  mm_count(nrows, X, Y, d_cnt, h->d_flag, st);
  HIPC(hipGetLastError());
  tm.mark(st, what + ": count");
  std::vector<int64_t> cnt(nrows);
  h->pool.stage.d2h(cnt.data(), d_cnt, nrows * sizeof(int64_t), st);
  std::vector<int32_t> hw;   // rows too wide for the hash passes
  for (int64_t i = 0; i < nrows; ++i)
    if (cnt[i] < 0) hw.push_back((int32_t)i);
  int32_t* d_hw = nullptr;
  if (!hw.empty()) {
    if (mm_wide_lds(ncols) > 65536)
      fail(AMG_ERR_LIMIT, what + ": a row has more than " + std::to_string(mm_hash_cap() / 2) +
                              " columns and the product has too many columns for the wide passes");
    d_hw = h->pool.upload(hw, st);
    HIPC(hipStreamSynchronize(st));
    mm_count_wide((int64_t)hw.size(), d_hw, X, Y, ncols, d_cnt, st);
    HIPC(hipMemcpyAsync(cnt.data(), d_cnt, nrows * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
  }
  cptr.assign(nrows + 1, 0);
  int64_t mmax = 0;
  std::vector<int32_t> nw;   // rows too long for the numeric pass's LDS
  const int64_t lds_row = std::min<int64_t>(MM_LDS_ROW, std::getenv("HCURL_AMG_MM_WIDE") ? mm_wide_at() : MM_LDS_ROW);
  for (int64_t i = 0; i < nrows; ++i) {
    cptr[i + 1] = cptr[i] + cnt[i];
    mmax = std::max(mmax, cnt[i]);
    if (cnt[i] > lds_row) nw.push_back((int32_t)i);
  }
  tm.mark(st, what + ": counts to host, scan");
  d_cptr = h->pool.upload(cptr, st);
  d_ccol = h->pool.get<int32_t>(std::max<int64_t>(cptr[nrows], 1));
  tm.mark(st, what + ": row pointers up, columns allocated");
  mm_fill(nrows, X, Y, d_cptr, d_ccol, h->d_flag, st);
  mm_fill_wide((int64_t)hw.size(), d_hw, X, Y, ncols, d_cptr, d_ccol, st);
  HIPC(hipGetLastError());
  check_flag(h, st, AMG_ERR_LIMIT, what + ": column fill overflow");
  nwide = (int64_t)nw.size();
  d_wide = nw.empty() ? nullptr : h->pool.upload(nw, st);
  HIPC(hipStreamSynchronize(st));
  tm.mark(st, what + ": fill");
  return std::min(mmax, lds_row);
}

void galerkin_symbolic(amg_hier* h, Level& L, Level& C, int level, hipStream_t st) {
  int64_t n = L.n, nc = L.nc;
  std::string lv = " on level " + std::to_string(level);
  CsrPat A{L.A_ptr, L.A_col}, P{L.P_ptr, L.P_col}, PT{L.PT_ptr, L.PT_col};
  std::vector<int64_t> apptr;
  L.ap_mmax = (int)mm_symbolic(h, n, nc, A, P, apptr, L.AP_ptr, L.AP_col, L.ap_wide, L.ap_nwide,
                               "A P" + lv, st);
  L.ap_nnz = apptr[n];
  StepTimer tm;
  L.AP_val = h->pool.get<double>(std::max<int64_t>(L.ap_nnz, 1));
  tm.mark(st, "A P values allocated (" + std::to_string(L.ap_nnz) + " entries)");
  CsrPat AP{L.AP_ptr, L.AP_col};
  std::vector<int64_t> cptr;
  L.rap_mmax = (int)mm_symbolic(h, nc, nc, PT, AP, cptr, C.A_ptr, C.A_col, L.rap_wide,
                                L.rap_nwide, "P^T (A P)" + lv, st);
  C.n = nc;
  C.nnz = cptr[nc];
  C.A_val = h->pool.get<double>(std::max<int64_t>(C.nnz, 1));
  C.lpr_A = lpr_for(C.n, C.nnz);
  C.Apat.n = C.Apat.m = nc;
  C.Apat.ptr = cptr;
  tm.mark(st, "P^T (A P) symbolic");
  C.Apat.idx.resize(C.nnz);
  h->pool.stage.d2h(C.Apat.idx.data(), C.A_col, C.nnz * sizeof(int32_t), st);
  tm.mark(st, "A_c pattern to the host");
}

void galerkin_numeric(amg_hier* h, Level& L, Level& C, hipStream_t st) {
  CsrPat A{L.A_ptr, L.A_col}, P{L.P_ptr, L.P_col}, PT{L.PT_ptr, L.PT_col}, AP{L.AP_ptr, L.AP_col};
  mm_vals(L.n, A, L.A_val, P, L.P_val, L.AP_ptr, L.AP_col, L.AP_val, L.ap_mmax, st);
  mm_vals_wide(L.ap_nwide, L.ap_wide, A, L.A_val, P, L.P_val, L.nc, L.AP_ptr, L.AP_col, L.AP_val, st);
  mm_vals(L.nc, PT, L.PT_val, AP, L.AP_val, C.A_ptr, C.A_col, C.A_val, L.rap_mmax, st);
  mm_vals_wide(L.rap_nwide, L.rap_wide, PT, L.PT_val, AP, L.AP_val, L.nc, C.A_ptr, C.A_col, C.A_val,
               st);
  HIPC(hipGetLastError());
}

void coarsest_factor(amg_hier* h, Level& L, hipStream_t st) {
  if (L.n > 8192) fail(AMG_ERR_COARSEN, "coarsest level has " + std::to_string(L.n) +
                                            " DoFs (more than 8192 for the dense solve)");
  if (!L.Lc) L.Lc = h->pool.get<double>((size_t)L.n * L.n);
  dense_factor(L.n, L.A_ptr, L.A_col, L.A_val, L.Lc, h->d_flag, st);
  check_flag(h, st, AMG_ERR_NOT_SPD, "coarsest Cholesky: non-positive pivot");
}

// Precision of every level of the FP32 form (reading R18): a level runs in
// FP32 unless eps_32 * rho exceeds the tolerance, where rho is the largest
// ratio sum |A_BB| / (s^T A_BB s) over its node stars: the gradient of a hat
// function is the near-kernel (A^s G = 0, only beta A^m sees it), and a
// relative perturbation eps of A's entries, or of a vector on the star,
// perturbs its energy by about eps * rho times itself.  Such a level keeps
// FP64 (matrices, smoother and vectors).  The coarsest level uses its
// parent's vector type (its solve is FP64 in any case).
void choose_precisions(amg_hier* h, hipStream_t st) {
  const size_t nl = h->lv.size();
  const double eps32 = 1.1920928955078125e-07;
  for (size_t l = 0; l < nl; ++l) {
    Level& L = h->lv[l];
    if (L.coarsest) {
      L.prec = l > 0 ? h->lv[l - 1].prec : h->prec;
      continue;
    }
    std::vector<double> rho(std::max<int64_t>(L.nstars, 1), 0.0);
    double* d_rho = h->pool.get<double>(rho.size());
    star_rho(L.nstars, L.sb_ptr, L.sb_dofs, L.ssign, L.srow_ptr, L.scol, L.sval, d_rho, st);
    HIPC(hipMemcpyAsync(rho.data(), d_rho, rho.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    L.grad_ratio = *std::max_element(rho.begin(), rho.end());
    L.prec = (h->prec == 32 && eps32 * L.grad_ratio <= h->opt.fp32_rho_tol) ? 32 : 64;
  }
}

void cast_level(amg_hier* h, Level& L, hipStream_t st) {
  if (L.prec != 32) return;
  if (!L.A_val32) L.A_val32 = h->pool.get<float>(L.nnz);
  cast<double, float>(L.nnz, L.A_val, L.A_val32, st);
  if (L.coarsest) return;
  if (!L.P_val32) {
    L.P_val32 = h->pool.get<float>(L.p_nnz);
    L.PT_val32 = h->pool.get<float>(L.p_nnz);
    L.fac32 = h->pool.get<float>(L.fac_total);
    L.binv32 = h->pool.get<float>(std::max<int64_t>(L.fac_total, 1));
    L.dinv32 = h->pool.get<float>(L.n);
    L.sval32 = h->pool.get<float>(std::max<int64_t>(L.srow_nnz, 1));
  }
  cast<double, float>(L.srow_nnz, L.sval, L.sval32, st);
  cast<double, float>(L.p_nnz, L.P_val, L.P_val32, st);
  cast<double, float>(L.p_nnz, L.PT_val, L.PT_val32, st);
  cast<double, float>(L.fac_total, L.fac, L.fac32, st);
  cast<double, float>(L.fac_total, L.binv, L.binv32, st);
  cast<double, float>(L.n, L.dinv, L.dinv32, st);
  if (L.sweep_mode == SWEEP_PANEL) {
    const int64_t ne = (int64_t)L.ngroups * PANEL_GROUP_SLOTS * PANEL_GROUP_SLOTS;
    const int64_t nf = (int64_t)L.ngroups * PANEL_GROUP_SLOTS * PANEL_ROW_WIDTH;
    if (!L.dsl32) {
      L.dsl32 = h->pool.get<float>((size_t)L.ngroups * PANEL_GROUP_SLOTS);
      L.gslc32 = h->pool.get<float>(ne);
      L.gcf32 = h->pool.get<float>(ne);
      L.gcb32 = h->pool.get<float>(ne);
      L.gbinv32 = h->pool.get<float>(nf);
    }
    cast<double, float>(ne, L.gslc, L.gslc32, st);
    cast<double, float>(ne, L.gcf, L.gcf32, st);
    cast<double, float>(ne, L.gcb, L.gcb32, st);
    cast<double, float>(nf, L.gbinv, L.gbinv32, st);
  }
  if (L.sweep_mode == SWEEP_DENSE || L.sweep_mode == SWEEP_PANEL) {
    if (!L.Acm32) L.Acm32 = h->pool.get<float>((size_t)L.n * L.n);
    cast<double, float>(L.n * L.n, L.Acm, L.Acm32, st);
  }
}

// --- learned setup ---
void ensure_mlp(amg_hier* h, hipStream_t st) {
  if (h->mlp.master) return;
  MlpDev& m = h->mlp;
  m.master = h->pool.get<float>(MLP_NPARAM);
  m.grad = h->pool.get<float>(MLP_NPARAM);
  m.adam_m = h->pool.get<float>(MLP_NPARAM);
  m.adam_v = h->pool.get<float>(MLP_NPARAM);
  m.Wb1 = h->pool.get<uint16_t>((size_t)MLP_IN * MLP_HID);
  m.Wb2 = h->pool.get<uint16_t>((size_t)MLP_HID * MLP_HID);
  m.Wb3 = h->pool.get<uint16_t>((size_t)MLP_HID * MLP_OUT);
  m.b1 = m.master + MLP_OFF_B1;
  m.b2 = m.master + MLP_OFF_B2;
  m.b3 = m.master + MLP_OFF_B3;
  fill<float>(MLP_NPARAM, 0.f, m.adam_m, st);
  fill<float>(MLP_NPARAM, 0.f, m.adam_v, st);
}

void ensure_work(amg_hier* h, int64_t rows) {
  if (h->work.rows >= rows) return;
  MlpWork& w = h->work;
  w.rows = rows;
  w.Z1 = h->pool.get<float>((size_t)rows * MLP_HID);
  w.Z2 = h->pool.get<float>((size_t)rows * MLP_HID);
  w.dH = h->pool.get<float>((size_t)rows * MLP_HID);
  w.H1 = h->pool.get<uint16_t>((size_t)rows * MLP_HID);
  w.H2 = h->pool.get<uint16_t>((size_t)rows * MLP_HID);
  w.dHb = h->pool.get<uint16_t>((size_t)rows * MLP_HID);
  w.dYb = h->pool.get<uint16_t>((size_t)rows * MLP_OUT);
}

// rows per inference pass (a multiple of 16; HCURL_AMG_INFER_ROWS overrides it)
int64_t infer_rows() {
  int64_t r = 16384;
  if (const char* e = std::getenv("HCURL_AMG_INFER_ROWS")) r = std::max<int64_t>(16, std::atoll(e) / 16 * 16);
  return r;
}

// features, exact targets and eligibility of every finest-level extension block
void learned_features(amg_hier* h, double eligible_max, hipStream_t st) {
  Level& L = h->lv[0];
  int64_t nb = L.ints.block_ptr.empty() ? 0 : (int64_t)L.ints.block_ptr.size() - 1;
  if (!h->fX) {
    h->mlp_nb = nb;
    h->mlp_rows = (nb + 15) / 16 * 16;
    int64_t r = std::max<int64_t>(h->mlp_rows, 16);
    h->fX = h->pool.get<uint16_t>((size_t)r * MLP_IN);
    h->fT = h->pool.get<float>((size_t)r * MLP_OUT);
    h->fY = h->pool.get<float>((size_t)r * MLP_OUT);
    h->fAhat = h->pool.get<double>((size_t)std::max<int64_t>(nb, 1) * 36);
    h->fdsq = h->pool.get<double>((size_t)std::max<int64_t>(nb, 1) * 8);
    h->fW = h->pool.get<double>((size_t)std::max<int64_t>(nb, 1) * 36);
    h->fel = h->pool.get<int8_t>(std::max<int64_t>(nb, 1));
    h->facc = h->pool.get<int8_t>(std::max<int64_t>(nb, 1));
    h->fres = h->pool.get<float>(std::max<int64_t>(nb, 1));
    // padding rows stay zero
    HIPC(hipMemsetAsync(h->fX, 0, (size_t)r * MLP_IN * sizeof(uint16_t), st));
  }
  block_features(nb, L.blk_ptr, L.blk_dofs, L.A_ptr, L.A_col, L.A_val, eligible_max, h->fX, h->fT,
                 h->fAhat, h->fdsq, h->fel, st);
}

// network prediction + refinement + check for every finest-level block
void learned_predict(amg_hier* h, hipStream_t st) {
  learned_features(h, 1e300, st);   // eligibility here only needs a valid exact factorisation
  const int64_t chunk = infer_rows();
  ensure_work(h, chunk);
  for (int64_t r0 = 0; r0 < h->mlp_rows; r0 += chunk) {
    int64_t nr = std::min<int64_t>(chunk, h->mlp_rows - r0);
    mlp_forward(h->mlp, h->fX + r0 * MLP_IN, nr, h->work, h->fY + r0 * MLP_OUT, st);
  }
  refine_check(h->mlp_nb, h->lv[0].blk_ptr, h->fel, h->fY, h->fAhat, h->use_cfg.refine_steps,
               h->use_cfg.accept_tol, h->fW, h->facc, h->fres, st);
  std::vector<int8_t> el(h->mlp_nb), acc(h->mlp_nb);
  HIPC(hipMemcpyAsync(el.data(), h->fel, h->mlp_nb, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(acc.data(), h->facc, h->mlp_nb, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  h->mstats.blocks = h->mlp_nb;
  h->mstats.eligible = 0;
  h->mstats.accepted = 0;
  for (int64_t b = 0; b < h->mlp_nb; ++b) {
    h->mstats.eligible += el[b] != 0;
    h->mstats.accepted += acc[b] != 0;
  }
}

void numeric_all(amg_hier* h, hipStream_t st, PhaseClock* clk = nullptr) {
  size_t nl = h->lv.size();
  for (size_t l = 0; l < nl; ++l) {
    Level& L = h->lv[l];
    if (L.coarsest) {
      coarsest_factor(h, L, st);
      if (clk) clk->mark(st, "coarsest dense Cholesky (GPU)", (int)l);
      break;
    }
    factor_smoother(h, L, (int)l, st);
    if (clk) clk->mark(st, "smoother factors + l1 (GPU)", (int)l);
    auto t0 = std::chrono::steady_clock::now();
    const bool use_mlp = l == 0 && h->learned;
    if (use_mlp) learned_predict(h, st);
    if (!L.user_p) compute_interp(h, L, (int)l, st, use_mlp);
    if (l == 0) {
      HIPC(hipStreamSynchronize(st));
      double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (use_mlp) h->mstats.infer_seconds = sec; else h->mstats.exact_seconds = sec;
    }
    permute(L.p_nnz, L.PT_perm, L.P_val, L.PT_val, st);
    if (clk) clk->mark(st, "local extension P (GPU)", (int)l);
    galerkin_numeric(h, L, h->lv[l + 1], st);
    if (clk) clk->mark(st, "Galerkin numeric (GPU)", (int)l);
  }
  if (h->prec == 32)
    for (auto& L : h->lv) cast_level(h, L, st);
  HIPC(hipStreamSynchronize(st));
}

void alloc_vectors(amg_hier* h) {
  for (size_t l = 0; l < h->lv.size(); ++l) {
    Level& L = h->lv[l];
    L.x = h->pool.get<double>(L.n);
    L.t = h->pool.get<double>(L.n);
    L.b = h->pool.get<double>(L.n);
    L.r = h->pool.get<double>(L.n);
    if (h->prec == 32) {
      L.x32 = h->pool.get<float>(L.n);
      L.t32 = h->pool.get<float>(L.n);
      L.b32 = h->pool.get<float>(L.n);
      L.r32 = h->pool.get<float>(L.n);
    }
  }
  int64_t n = h->lv[0].n;
  h->pr = h->pool.get<double>(n);
  h->pz = h->pool.get<double>(n);
  h->pp = h->pool.get<double>(n);
  h->pq = h->pool.get<double>(n);
  h->prold = h->pool.get<double>(n);
  // partial sums: two per workgroup of the fixed-grid dot products, and one
  // per workgroup of the level-0 SpMV-with-dot (n / (256 / lpr) workgroups:
  // the most for the widest lane groups)
  h->partial_cap = std::max<int64_t>(2 * red_grid(), spmv_dot_partials(h->lv[0].lpr_A, n));
  h->d_partial = h->pool.get<double>(h->partial_cap);
  h->d_sc = h->pool.get<double>(SC_COUNT);
  int64_t nL = h->lv.back().n;
  h->dense_work = h->pool.get<double>(std::max<int64_t>(nL, 1));
}

// --- the V(1,1) cycle ---
template <class T>
struct Vec {
  static T* x(Level& L) { if constexpr (std::is_same<T, double>::value) return L.x; else return L.x32; }
  static T* t(Level& L) { if constexpr (std::is_same<T, double>::value) return L.t; else return L.t32; }
  static T* b(Level& L) { if constexpr (std::is_same<T, double>::value) return L.b; else return L.b32; }
  static T* r(Level& L) { if constexpr (std::is_same<T, double>::value) return L.r; else return L.r32; }
  static T* dinv(Level& L) { if constexpr (std::is_same<T, double>::value) return L.dinv; else return L.dinv32; }
};

// One level of the descent: pre-smoothing of A_l x = b from x = 0, the
// residual, and its restriction into the next level's right-hand side (in
// the next level's value type).
template <class T>
void vc_down(amg_hier* h, size_t l, const T* b, T* x, hipStream_t st) {
  Level& L = h->lv[l];
  Level& C = h->lv[l + 1];
  const int mode = h->opt.schwarz_mode;
  CsrDev<T> A = L.A_dev<T>();
  SmootherDev<T> S = L.S_dev<T>(h->d_sweep_err, h->spin_max);
  fill<T>(L.n, (T)0, x, st);
  schwarz_sweep<T>(S, A, 0, b, x, st);
  if (mode != AMG_SCHWARZ_SPLIT) schwarz_sweep<T>(S, A, 1, b, x, st);
  jacobi<T>(A, x, b, Vec<T>::dinv(L), Vec<T>::t(L), st);
  residual<T>(A, Vec<T>::t(L), b, Vec<T>::r(L), st);
  if (C.prec == L.prec) {
    spmv<T>(L.PT_dev<T>(), Vec<T>::r(L), Vec<T>::b(C), st);
  } else if (C.prec == 32) {
    spmv<T>(L.PT_dev<T>(), Vec<T>::r(L), Vec<T>::r(C), st);
    cast<T, float>(C.n, Vec<T>::r(C), C.b32, st);
  } else {
    spmv<T>(L.PT_dev<T>(), Vec<T>::r(L), Vec<T>::r(C), st);
    cast<T, double>(C.n, Vec<T>::r(C), C.b, st);
  }
}

// One level of the ascent: prolongation of the next level's correction (in
// this level's value type), then post-smoothing; x receives the result.
template <class T>
void vc_up(amg_hier* h, size_t l, const T* b, T* x, hipStream_t st) {
  Level& L = h->lv[l];
  Level& C = h->lv[l + 1];
  const int mode = h->opt.schwarz_mode;
  CsrDev<T> A = L.A_dev<T>();
  SmootherDev<T> S = L.S_dev<T>(h->d_sweep_err, h->spin_max);
  const T* xc = Vec<T>::x(C);
  if (C.prec != L.prec) {
    if (C.prec == 32) cast<float, T>(C.n, C.x32, Vec<T>::t(C), st);
    else cast<double, T>(C.n, C.x, Vec<T>::t(C), st);
    xc = Vec<T>::t(C);
  }
  spmv_add<T>(L.P_dev<T>(), xc, Vec<T>::t(L), st);
  if (mode == AMG_SCHWARZ_REPEAT) {
    // post = pre: forward, backward, then l1-Jacobi (t -> x)
    schwarz_sweep<T>(S, A, 0, b, Vec<T>::t(L), st);
    schwarz_sweep<T>(S, A, 1, b, Vec<T>::t(L), st);
    jacobi<T>(A, Vec<T>::t(L), b, Vec<T>::dinv(L), x, st);
    return;
  }
  jacobi<T>(A, Vec<T>::t(L), b, Vec<T>::dinv(L), x, st);
  if (mode != AMG_SCHWARZ_SPLIT) schwarz_sweep<T>(S, A, 0, b, x, st);
  schwarz_sweep<T>(S, A, 1, b, x, st);
}

// The V(1,1) cycle x0 = B b0 on level 0's vectors (of level 0's value
// type); every level works in its own type (all FP64 in the FP64 form).
void vcycle_levels(amg_hier* h, const void* b0, void* x0, hipStream_t st) {
  const size_t nl = h->lv.size();
  auto bptr = [&](size_t l) -> const void* {
    if (l == 0) return b0;
    Level& L = h->lv[l];
    return L.prec == 32 ? (const void*)L.b32 : (const void*)L.b;
  };
  auto xptr = [&](size_t l) -> void* {
    if (l == 0) return x0;
    Level& L = h->lv[l];
    return L.prec == 32 ? (void*)L.x32 : (void*)L.x;
  };
  for (size_t l = 0; l + 1 < nl; ++l) {
    if (h->lv[l].prec == 32) vc_down<float>(h, l, (const float*)bptr(l), (float*)xptr(l), st);
    else vc_down<double>(h, l, (const double*)bptr(l), (double*)xptr(l), st);
  }
  Level& C = h->lv[nl - 1];
  if (C.prec == 32)
    dense_solve<float>((int)C.n, C.Lc, (const float*)bptr(nl - 1), (float*)xptr(nl - 1), h->dense_work, st);
  else
    dense_solve<double>((int)C.n, C.Lc, (const double*)bptr(nl - 1), (double*)xptr(nl - 1), h->dense_work, st);
  for (size_t l = nl - 1; l-- > 0;) {
    if (h->lv[l].prec == 32) vc_up<float>(h, l, (const float*)bptr(l), (float*)xptr(l), st);
    else vc_up<double>(h, l, (const double*)bptr(l), (double*)xptr(l), st);
  }
}

void vcycle_any(amg_hier* h, const double* r, double* z, hipStream_t st) {
  Level& L0 = h->lv[0];
  if (L0.prec == 64) {
    vcycle_levels(h, r, z, st);
  } else {
    cast<double, float>(L0.n, r, L0.b32, st);
    vcycle_levels(h, L0.b32, L0.x32, st);
    cast<float, double>(L0.n, L0.x32, z, st);
  }
}

// V-cycle through a cached HIP graph (captured on first use for this buffer
// pair); the graph runs on the library stream, which waits for the caller's
// stream and is waited for by it, so ordering on `st` is preserved.
void vcycle_graph(amg_hier* h, const double* r, double* z, hipStream_t st) {
  if (!h->use_graphs) {
    vcycle_any(h, r, z, st);
    return;
  }
  if (!h->gstream) {
    HIPC(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    HIPC(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
  }
  hipGraphExec_t exec = nullptr;
  for (auto& g : h->graphs)
    if (g.r == r && g.z == z) exec = g.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    HIPC(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    vcycle_any(h, r, z, h->gstream);
    HIPC(hipStreamEndCapture(h->gstream, &graph));
    HIPC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    if (h->graphs.size() >= 8) {   // bounded cache
      (void)hipGraphExecDestroy(h->graphs.front().exec);
      h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({r, z, exec});
  }
  HIPC(hipEventRecord(h->ev_in, st));
  HIPC(hipStreamWaitEvent(h->gstream, h->ev_in, 0));
  HIPC(hipGraphLaunch(exec, h->gstream));
  HIPC(hipEventRecord(h->ev_out, h->gstream));
  HIPC(hipStreamWaitEvent(st, h->ev_out, 0));
}

double read_scalar(amg_hier* h, int slot, hipStream_t st);

// Asymptotic convergence factor of the stand-alone cycle e <- e - B A e,
// estimated as ||e_k||_A / ||e_{k-1}||_A after `iters` cycles from a fixed
// pseudo-random start (used by the learned setup's global check).
double convergence_factor(amg_hier* h, int iters, hipStream_t st) {
  Level& L0 = h->lv[0];
  int64_t n = L0.n;
  CsrDev<double> A = L0.A_dev<double>();
  double* e = h->prold;
  double* t = h->pq;
  double* z = h->pz;
  hash_fill(n, h->opt.seed, e, st);
  double prev = 0.0, cur = 0.0;
  for (int k = 0; k <= iters; ++k) {
    spmv<double>(A, e, t, st);
    dot2(n, e, t, nullptr, h->d_partial, st);
    reduce(red_grid(), h->d_partial, h->d_sc, SC_RR, -1, st);
    prev = cur;
    cur = std::sqrt(std::max(read_scalar(h, SC_RR, st), 0.0));
    if (k == iters) break;
    vcycle_any(h, t, z, st);
    axpy(n, -1.0, z, e, st);
  }
  return prev > 0.0 ? cur / prev : 0.0;
}

double read_scalar(amg_hier* h, int slot, hipStream_t st) {
  HIPC(hipMemcpyAsync(h->h_sc + slot, h->d_sc + slot, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return h->h_sc[slot];
}

// ||f - A u|| (FP64), with f - A u left in r
double true_residual_norm(amg_hier* h, const double* u, const double* f, double* r, hipStream_t st) {
  Level& L0 = h->lv[0];
  residual<double>(L0.A_dev<double>(), u, f, r, st);
  dot2(L0.n, r, r, nullptr, h->d_partial, st);
  reduce(red_grid(), h->d_partial, h->d_sc, SC_RR, -1, st);
  return std::sqrt(std::max(read_scalar(h, SC_RR, st), 0.0));
}

// 64 eps || |A| |u| ||: the size of the rounding error of f - A u formed in
// FP64, below which no solver can certify a residual (work holds |A||u|)
double fp64_floor_norm(amg_hier* h, const double* u, double* work, hipStream_t st) {
  Level& L0 = h->lv[0];
  spmv_abs(L0.A_dev<double>(), u, work, st);
  dot2(L0.n, work, work, nullptr, h->d_partial, st);
  reduce(red_grid(), h->d_partial, h->d_sc, SC_RR, -1, st);
  return 64.0 * 2.220446049250313e-16 * std::sqrt(std::max(read_scalar(h, SC_RR, st), 0.0));
}

template <class F>
amg_status guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Fail& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return AMG_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return AMG_ERR_ARG;
  }
}

void validate_csr_arg(const amg_csr* M, const char* name) {
  if (!M || !M->rowptr || (M->nnz > 0 && (!M->colidx || !M->val)))
    fail(AMG_ERR_ARG, std::string(name) + ": NULL pointer");
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) fail(AMG_ERR_SHAPE, std::string(name) + ": negative size");
}

// host integer setup of the finest level + everything it needs
struct Level0Host {
  Pattern Apat;
  Incidence G;
  Pattern S;
};

void level0_host(const amg_csr* A, const amg_csr* G, Level0Host& out, std::vector<double>* Aval,
                 Staging* sg = nullptr) {
  validate_csr_arg(A, "A");
  validate_csr_arg(G, "G");
  if (A->nrows != A->ncols) fail(AMG_ERR_SHAPE, "A is not square");
  if (G->nrows != A->nrows) fail(AMG_ERR_SHAPE, "G must have one row per row of A");
  if (A->nrows > INT32_MAX || G->ncols > INT32_MAX) fail(AMG_ERR_SHAPE, "more than 2^31-1 rows or nodes");
  std::vector<int64_t> gptr;
  std::vector<int32_t> gcol;
  std::vector<double> gval;
  const char* ve = std::getenv("HCURL_AMG_VERBOSE");
  const bool steps = ve && std::atoi(ve) >= 2;
  auto t0 = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) {
    if (!steps) return;
    auto t1 = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[amg]   host %-34s %.3f s\n", what, std::chrono::duration<double>(t1 - t0).count());
    t0 = t1;
  };
  host_csr(A, out.Apat.ptr, out.Apat.idx, Aval, sg);
  out.Apat.n = out.Apat.m = A->nrows;
  mark("A to the host");
  HostError err;
  if (!validate_pattern(A->nrows, A->ncols, out.Apat.ptr.data(), out.Apat.idx.data(), err))
    fail((amg_status)err.code, "A: " + err.msg);
  mark("A pattern checked");
  host_csr(G, gptr, gcol, &gval, sg);
  if (!incidence_from_csr(G->nrows, G->ncols, gptr.data(), gcol.data(), gval.data(), out.G, err))
    fail((amg_status)err.code, err.msg);
  mark("G to the host and checked");
  Incidence Gt;
  std::vector<int32_t> B;
  augment_g(out.G, Gt, B);
  out.S = nodal_graph_level0(out.Apat, Gt);
  mark("nodal graph of level 0");
}

void fill_export(const LevelInts& I, amg_int_export* o) {
  std::memset(o, 0, sizeof(*o));
  o->n = I.n;
  o->m_real = I.m_real;
  o->n_art = I.n_art;
  o->cf = I.cf.empty() ? nullptr : I.cf.data();
  o->n_cg = (int64_t)I.cg.size();
  o->cg = I.cg.data();
  o->nc = (int64_t)I.r_dof1.size();
  o->r_dof1 = I.r_dof1.data();
  o->r_dof2 = I.r_dof2.data();
  o->r_i = I.r_i.data();
  o->r_j = I.r_j.data();
  o->r_k = I.r_k.data();
  o->r_s1 = I.r_s1.data();
  o->r_s2 = I.r_s2.data();
  o->n_interior = (int64_t)I.interior.size();
  o->interior = I.interior.data();
  o->nblocks = I.block_ptr.empty() ? 0 : (int64_t)I.block_ptr.size() - 1;
  o->block_ptr = I.block_ptr.data();
  o->block_dofs = I.block_dofs.data();
  o->block_key_depth = I.block_depth.data();
  o->exact_blocks = I.exact_blocks ? 1 : 0;
  o->nstars = I.star_ptr.empty() ? 0 : (int64_t)I.star_ptr.size() - 1;
  o->star_ptr = I.star_ptr.data();
  o->star_dofs = I.star_dofs.data();
  o->star_color = I.star_color.data();
  o->ncolors = I.ncolors;
  o->gc_nrows = I.gc.n;
  o->gc_ncols = I.gc.m;
  o->gc_ptr = I.gc_ptr.data();
  o->gc_col = I.gc_col.data();
  o->gc_val = I.gc_val.data();
  o->gc_cols = I.gc_cols.data();
  o->npatch_entries = I.patch ? (int64_t)I.patch_dofs.size() : 0;
  o->patch_ptr = I.patch ? I.patch_ptr.data() : nullptr;
  o->patch_dofs = I.patch ? I.patch_dofs.data() : nullptr;
}

ExtOptions ext_options(const amg_options& o) {
  ExtOptions e;
  e.ext_block_max = o.ext_block_max;
  e.ext_mode = o.ext_mode;
  e.patch_hops = o.patch_hops;
  e.patch_cap = o.patch_cap;
  return e;
}

void check_ext_options(const amg_options& o) {
  if (o.ext_mode != AMG_EXT_BLOCKS && o.ext_mode != AMG_EXT_PATCH) fail(AMG_ERR_ARG, "unknown ext_mode");
  if (o.ext_mode == AMG_EXT_PATCH) {
    if (o.patch_hops < 1 || o.patch_hops > 8) fail(AMG_ERR_ARG, "patch_hops must be in 1..8");
    if (o.patch_cap < 1 || o.patch_cap > PATCH_CAP_MAX)
      fail(AMG_ERR_ARG, "patch_cap must be in 1.." + std::to_string(PATCH_CAP_MAX));
  }
}

}  // namespace

extern "C" {

void amg_default_options(amg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->interp = AMG_INTERP_ALG;
  opt->max_levels = 20;
  opt->min_coarse = 32;
  opt->vcycle_prec = 64;
  opt->ext_block_max = 64;
  opt->stall_ratio = 0.9;
  opt->p_trunc = 0.0;
  opt->schwarz_mode = AMG_SCHWARZ_ADJOINT;
  opt->seed = 0x5eed1234ull;
  opt->fp32_rho_tol = 1e-3;
  opt->ext_mode = AMG_EXT_BLOCKS;
  opt->patch_hops = 2;
  opt->patch_cap = 128;
}

const char* amg_last_error(void) { return g_err.c_str(); }

amg_status amg_setup(const amg_csr* A, const amg_csr* G, const amg_options* opt, void* stream,
                     amg_hier** out) {
  return guarded([&]() -> amg_status {
    if (!out) fail(AMG_ERR_ARG, "out is NULL");
    *out = nullptr;
    amg_options o;
    if (opt) o = *opt; else amg_default_options(&o);
    if (o.vcycle_prec != 64 && o.vcycle_prec != 32) fail(AMG_ERR_ARG, "vcycle_prec must be 64 or 32");
    if (o.max_levels < 1) fail(AMG_ERR_ARG, "max_levels < 1");
    if (o.interp == AMG_INTERP_REF && o.ref_nlevels > 0 &&
        (!o.ref_coarse_nodes || !o.ref_ncoarse || !o.ref_coarse_bnd || !o.ref_nbnd))
      fail(AMG_ERR_ARG, "refinement mode without coarse node lists");
    if (o.interp != AMG_INTERP_ALG && o.interp != AMG_INTERP_REF && o.interp != AMG_INTERP_USER)
      fail(AMG_ERR_ARG, "unknown interp mode");
    if (o.interp == AMG_INTERP_USER && (o.user_nlevels < 1 || !o.user_P || !o.user_G))
      fail(AMG_ERR_ARG, "user interpolation mode without P and G lists");
    if (o.interp == AMG_INTERP_USER && o.p_trunc > 0.0)
      fail(AMG_ERR_ARG, "p_trunc applies to the paper's interpolation only");
    if (o.schwarz_mode < AMG_SCHWARZ_ADJOINT || o.schwarz_mode > AMG_SCHWARZ_SPLIT)
      fail(AMG_ERR_ARG, "unknown schwarz_mode");
    check_ext_options(o);
    hipStream_t st = (hipStream_t)stream;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(AMG_ERR_HIP, "no HIP device");
    auto h = std::make_unique<amg_hier>();
    h->opt = o;
    if (const char* e = std::getenv("HCURL_AMG_NO_GRAPH"))
      if (e[0] && e[0] != '0') h->use_graphs = false;

    h->prec = o.vcycle_prec;
    h->d_flag = h->pool.get<int>(1);
    HIPC(hipMemsetAsync(h->d_flag, 0, sizeof(int), st));
    h->d_sweep_err = h->pool.get<int>(1);
    HIPC(hipMemsetAsync(h->d_sweep_err, 0, sizeof(int), st));
    {
      int dev = 0, cus = 0;
      HIPC(hipGetDevice(&dev));
      HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      if (cus > 0) h->cu_count = cus;
      if (const char* e = std::getenv("HCURL_AMG_SPIN_MAX")) h->spin_max = std::max(1, std::atoi(e));
    }
    HIPC(hipHostMalloc((void**)&h->h_sc, SC_COUNT * sizeof(double), hipHostMallocDefault));
    PhaseClock clk;
    Level0Host l0;
    std::vector<double> aval;
    level0_host(A, G, l0, A->on_device ? nullptr : &aval, &h->pool.stage);
    clk.mark(st, "input copy + nodal graph", 0);
    h->lv.emplace_back();
    {
      Level& L = h->lv[0];
      L.Apat = std::move(l0.Apat);
      L.G = std::move(l0.G);
      L.S = std::move(l0.S);
      L.n = A->nrows;
      L.nnz = A->nnz;
      h->a_borrowed = o.borrow_a != 0 && A->on_device;
      if (h->a_borrowed) {
        // the caller's arrays, read in place (checked on the host above)
        L.A_ptr = const_cast<int64_t*>(A->rowptr);
        L.A_col = const_cast<int32_t*>(A->colidx);
      } else if (A->on_device) {
        // the pattern checked on the host is the caller's device copy: copy it
        // on the device instead of uploading the host copy again
        L.A_ptr = h->pool.get<int64_t>(L.n + 1);
        L.A_col = h->pool.get<int32_t>(std::max<int64_t>(L.nnz, 1));
        HIPC(hipMemcpyAsync(L.A_ptr, A->rowptr, (L.n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
        if (L.nnz > 0)
          HIPC(hipMemcpyAsync(L.A_col, A->colidx, L.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      } else {
        L.A_ptr = h->pool.upload(L.Apat.ptr, st);
        L.A_col = h->pool.upload(L.Apat.idx, st);
      }
      if (h->a_borrowed) {
        L.A_val = const_cast<double*>(A->val);
      } else if (A->on_device) {
        L.A_val = h->pool.get<double>(L.nnz);
        HIPC(hipMemcpyAsync(L.A_val, A->val, L.nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        L.A_val = h->pool.get<double>(L.nnz);
        HIPC(hipMemcpyAsync(L.A_val, aval.data(), L.nnz * sizeof(double), hipMemcpyHostToDevice, st));
      }
      L.lpr_A = lpr_for(L.n, L.nnz);
    }
    const bool user = o.interp == AMG_INTERP_USER;
    for (int l = 0;; ++l) {
      Level& L = h->lv[l];
      bool stop = user ? (l >= o.user_nlevels || l + 1 >= o.max_levels)
                       : ((l + 1 >= o.max_levels) || (L.n <= o.min_coarse));
      // the smoother's node stars and colouring need only A_l's pattern and
      // G_l: a second host thread builds them while this one does the
      // coarsening (both are sequential passes)
      std::future<LevelInts> stars_f;
      if (!stop)
        stars_f = std::async(std::launch::async, [&L]() {
          LevelInts s;
          stars_and_colours(L.Apat, L.G, s);
          return s;
        });
      if (!stop && user) {
        load_user_interp(h.get(), L, o.user_P[l], l, st);
      } else if (!stop) {
        bool use_ref = o.interp == AMG_INTERP_REF && l < o.ref_nlevels;
        std::vector<int32_t> rc, rb;
        if (use_ref) {
          rc.assign(o.ref_coarse_nodes[l], o.ref_coarse_nodes[l] + o.ref_ncoarse[l]);
          rb.assign(o.ref_coarse_bnd[l], o.ref_coarse_bnd[l] + o.ref_nbnd[l]);
        }
        HostError err;
        if (!setup_level_integers(L.Apat, L.G, L.S, use_ref, rc, rb, ext_options(o), L.ints, err))
          fail((amg_status)err.code, "level " + std::to_string(l) + ": " + err.msg);
        clk.mark(st, "integer setup (Alg. 1-3, P pattern)", l);
        int64_t nc = (int64_t)L.ints.r_dof1.size();
        if (nc == 0 || (double)nc > o.stall_ratio * (double)L.n) stop = true;
      }
      if (stop) {
        L.coarsest = true;
        if (l == 0 && L.n > 8192) fail(AMG_ERR_COARSEN, "no coarse variables on the finest level");
        break;
      }
      {
        LevelInts s = stars_f.get();
        L.ints.star_ptr = std::move(s.star_ptr);
        L.ints.star_dofs = std::move(s.star_dofs);
        L.ints.star_color = std::move(s.star_color);
        L.ints.ncolors = s.ncolors;
      }
      clk.mark(st, "smoother stars + colours (wait)", l);
      build_smoother(h.get(), L, st);
      clk.mark(st, "smoother chunks and row copy", l);
      factor_smoother(h.get(), L, l, st);
      clk.mark(st, "smoother factors + l1 (GPU)", l);
      if (!user) {
        build_interp_structs(h.get(), L, st);
        compute_interp(h.get(), L, l, st);
        if (o.p_trunc > 0.0) truncate_interp(h.get(), L, o.p_trunc, st);
      }
      build_transpose(h.get(), L, st);
      permute(L.p_nnz, L.PT_perm, L.P_val, L.PT_val, st);
      clk.mark(st, "local extension P (GPU)", l);
      h->lv.emplace_back();
      Level& L2 = h->lv[l + 1];
      Level& L1 = h->lv[l];   // re-fetch after emplace_back
      galerkin_symbolic(h.get(), L1, L2, l, st);
      galerkin_numeric(h.get(), L1, L2, st);
      clk.mark(st, "Galerkin A P, P^T (A P) (GPU)", l);
      if (user) {
        L2.G = user_gradient(o.user_G[l + 1], L2.n, l + 1);
      } else {
        L2.G = L1.ints.gc;
        L2.S = nodal_graph_coarse(L1.S, L1.ints.fine_of_next);
      }
      clk.mark(st, "coarse nodal graph", l);
    }
    {
      Level& C = h->lv.back();
      coarsest_factor(h.get(), C, st);
      clk.mark(st, "coarsest dense Cholesky (GPU)", (int)h->lv.size() - 1);
      choose_precisions(h.get(), st);
      if (h->prec == 32)
        for (auto& L : h->lv) cast_level(h.get(), L, st);
    }
    alloc_vectors(h.get());
    HIPC(hipStreamSynchronize(st));
    *out = h.release();
    return AMG_OK;
  });
}

amg_status amg_resetup_numeric(amg_hier* h, const amg_csr* A, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "handle is NULL");
    validate_csr_arg(A, "A");
    Level& L0 = h->lv[0];
    if (A->nrows != L0.n || A->nnz != L0.nnz) fail(AMG_ERR_SHAPE, "A's size differs from the setup's");
    if (h->opt.p_trunc > 0.0)
      fail(AMG_ERR_ARG, "amg_resetup_numeric needs p_trunc = 0 (a truncated P's pattern depends on the values)");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    // the pattern must be the one given to amg_setup; it is checked before
    // any value is copied, so a rejected call leaves the hierarchy as it was
    host_csr(A, ptr, col, nullptr, &h->pool.stage);
    if (ptr != L0.Apat.ptr || col != L0.Apat.idx) fail(AMG_ERR_CSR, "A's pattern differs from the setup's");
    if (h->a_borrowed) {
      if (!A->on_device) fail(AMG_ERR_ARG, "a hierarchy that borrows A needs a device A here too");
      if (A->val != L0.A_val || A->rowptr != L0.A_ptr || A->colidx != L0.A_col) {
        // the captured V-cycles hold the old arrays' addresses
        HIPC(hipStreamSynchronize(st));
        for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
        h->graphs.clear();
      }
      L0.A_ptr = const_cast<int64_t*>(A->rowptr);
      L0.A_col = const_cast<int32_t*>(A->colidx);
      L0.A_val = const_cast<double*>(A->val);
    } else if (A->on_device) {
      HIPC(hipMemcpyAsync(L0.A_val, A->val, L0.nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      HIPC(hipMemcpyAsync(L0.A_val, A->val, L0.nnz * sizeof(double), hipMemcpyHostToDevice, st));
    }
    numeric_all(h, st);
    h->mstats.global_fallback = 0;
    if (h->learned && h->use_cfg.global_iters > 0) {
      double rho = convergence_factor(h, h->use_cfg.global_iters, st);
      h->mstats.rho_learned = rho;
      if (!(rho <= h->mstats.rho_reference + h->use_cfg.global_slack)) {
        // global check failed: redo the numeric setup with exact local solves
        h->learned = false;
        try {
          numeric_all(h, st);
        } catch (...) {
          h->learned = true;
          throw;
        }
        h->learned = true;
        h->mstats.global_fallback = 1;
        h->mstats.accepted = 0;
      }
    }
    return AMG_OK;
  });
}

amg_status amg_vcycle(amg_hier* h, const double* r, double* z, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !r || !z) fail(AMG_ERR_ARG, "NULL argument");
    if (r == z) fail(AMG_ERR_ARG, "r and z alias");
    vcycle_graph(h, r, z, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_pcg_solve(amg_hier* h, const double* f, double* u, double rtol, int maxit,
                         amg_solve_stats* stats, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !f || !u) fail(AMG_ERR_ARG, "NULL argument");
    if (!(rtol >= 0.0) || maxit < 0) fail(AMG_ERR_ARG, "rtol < 0 or maxit < 0");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    Level& L0 = h->lv[0];
    int64_t n = L0.n;
    CsrDev<double> A = L0.A_dev<double>();
    const bool flexible = h->prec != 64;
    double* r = h->pr;
    double* z = h->pz;
    double* p = h->pp;
    double* q = h->pq;
    double* rold = flexible ? h->prold : nullptr;
    const double r0 = true_residual_norm(h, u, f, r, st);
    if (!std::isfinite(r0)) fail(AMG_ERR_NOT_FINITE, "initial residual is not finite");
    int it = 0, replacements = 0;
    double nr = r0, tr_last = 0.0;
    double tr = r0;   // the last true residual norm computed (r0 until CG forms another)
    bool tr_current = true;
    if (stats && stats->history) stats->history[0] = r0;
    if (r0 > 0.0) {
      vcycle_graph(h, r, z, st);
      dot2(n, r, z, nullptr, h->d_partial, st);
      reduce(red_grid(), h->d_partial, h->d_sc, SC_RZ, -1, st);
      cg_dir(n, h->d_sc, z, p, 1, st);
      int64_t np = spmv_dot_partials(A.lpr, n);
      if (np > h->partial_cap) fail(AMG_ERR_LIMIT, "partial-sum buffer smaller than the SpMV grid");
      while (it < maxit) {
        spmv_dot(A, p, q, h->d_partial, st);
        reduce(np, h->d_partial, h->d_sc, SC_PQ, -1, st);
        cg_scalar(h->d_sc, 0, flexible, st);
        cg_update(n, h->d_sc, p, q, u, r, rold, h->d_partial, st);
        reduce(red_grid(), h->d_partial, h->d_sc, SC_RR, -1, st);
        ++it;
        tr_current = false;
        nr = std::sqrt(read_scalar(h, SC_RR, st));
        if (stats && stats->history) stats->history[it] = nr;
        if (!std::isfinite(nr)) fail(AMG_ERR_NOT_FINITE, "residual became non-finite");
        if (verbose() && it % 100 == 0) {
          std::fprintf(stderr, "[amg] pcg iteration %d relres %.3e\n", it, nr / r0);
          std::fflush(stderr);
        }
        if (nr <= rtol * r0) {
          // the recursive residual has drifted from f - A u by rounding:
          // stop once the true residual meets the tolerance, or once a
          // restart no longer halves it (it then sits at the attainable
          // accuracy of FP64 on this system, and the solve reports
          // AMG_NOT_CONVERGED); else continue from it with a fresh direction
          tr = true_residual_norm(h, u, f, r, st);
          tr_current = true;
          if (!std::isfinite(tr)) fail(AMG_ERR_NOT_FINITE, "residual became non-finite");
          if (tr <= rtol * r0 || it >= maxit || (replacements > 0 && tr > 0.5 * tr_last)) break;
          tr_last = tr;
          nr = tr;
          ++replacements;
          vcycle_graph(h, r, z, st);
          dot2(n, r, z, nullptr, h->d_partial, st);
          reduce(red_grid(), h->d_partial, h->d_sc, SC_RZ, -1, st);
          cg_dir(n, h->d_sc, z, p, 1, st);
          continue;
        }
        vcycle_graph(h, r, z, st);
        dot2(n, r, z, rold, h->d_partial, st);
        reduce(red_grid(), h->d_partial, h->d_sc, SC_RZNEW, flexible ? SC_ROLDZ : -1, st);
        cg_scalar(h->d_sc, 1, flexible, st);
        cg_dir(n, h->d_sc, z, p, 0, st);
      }
    }
    HIPC(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    check_sweep_err(h, st);
    if (!tr_current) tr = true_residual_norm(h, u, f, q, st);
    // success means the true residual f - A u meets the tolerance
    const bool converged = tr <= rtol * r0;
    if (stats) {
      stats->iterations = it;
      stats->relres = r0 > 0 ? nr / r0 : 0.0;
      stats->seconds = std::chrono::duration<double>(t1 - t0).count();
      stats->true_relres = r0 > 0 ? tr / r0 : 0.0;
      stats->replacements = replacements;
      stats->floor_relres = r0 > 0 ? fp64_floor_norm(h, u, q, st) / r0 : 0.0;
      stats->conv_factor = (r0 > 0 && it > 0) ? std::pow(nr / r0, 1.0 / it) : 0.0;
    }
    HIPC(hipGetLastError());
    return converged ? AMG_OK : AMG_NOT_CONVERGED;
  });
}

amg_status amg_cycle_solve(amg_hier* h, const double* f, double* u, double rtol, int maxit,
                           amg_solve_stats* stats, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !f || !u) fail(AMG_ERR_ARG, "NULL argument");
    if (!(rtol >= 0.0) || maxit < 0) fail(AMG_ERR_ARG, "rtol < 0 or maxit < 0");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = h->lv[0].n;
    double* r = h->pr;
    double* z = h->pz;
    const double r0 = true_residual_norm(h, u, f, r, st);
    if (!std::isfinite(r0)) fail(AMG_ERR_NOT_FINITE, "initial residual is not finite");
    if (stats && stats->history) stats->history[0] = r0;
    int it = 0;
    double nr = r0, prev = r0;
    while (it < maxit && nr > rtol * r0) {
      vcycle_graph(h, r, z, st);
      axpy(n, 1.0, z, u, st);
      prev = nr;
      nr = true_residual_norm(h, u, f, r, st);
      ++it;
      if (stats && stats->history) stats->history[it] = nr;
      if (!std::isfinite(nr)) fail(AMG_ERR_NOT_FINITE, "residual became non-finite");
    }
    HIPC(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    check_sweep_err(h, st);
    if (stats) {
      stats->iterations = it;
      stats->relres = r0 > 0 ? nr / r0 : 0.0;
      stats->true_relres = stats->relres;
      stats->seconds = std::chrono::duration<double>(t1 - t0).count();
      stats->replacements = 0;
      stats->floor_relres = r0 > 0 ? fp64_floor_norm(h, u, z, st) / r0 : 0.0;
      stats->conv_factor = (it > 0 && prev > 0) ? nr / prev : 0.0;
    }
    HIPC(hipGetLastError());
    return nr <= rtol * r0 ? AMG_OK : AMG_NOT_CONVERGED;
  });
}

amg_status amg_complexity(const amg_hier* h, double* oc, double* gc) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "NULL handle");
    double sn = 0, snnz = 0;
    for (const Level& L : h->lv) {
      sn += (double)L.n;
      snnz += (double)L.nnz;
    }
    if (oc) *oc = snnz / (double)h->lv[0].nnz;
    if (gc) *gc = sn / (double)h->lv[0].n;
    return AMG_OK;
  });
}

amg_status amg_smoother_sweep(amg_hier* h, int level, int prec, const void* b, void* x,
                              int backward, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !b || !x) fail(AMG_ERR_ARG, "NULL argument");
    if (level < 0 || level + 1 >= (int)h->lv.size()) fail(AMG_ERR_ARG, "level has no smoother");
    if (prec != 64 && prec != 32) fail(AMG_ERR_ARG, "prec must be 64 or 32");
    Level& L = h->lv[level];
    if (prec != L.prec) fail(AMG_ERR_ARG, "the level's smoother runs in FP" + std::to_string(L.prec));
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      schwarz_sweep<T>(L.S_dev<T>(h->d_sweep_err, h->spin_max), L.A_dev<T>(), backward, (const T*)b,
                       (T*)x, st);
    };
    if (prec == 64) run(double()); else run(float());
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_check(amg_hier* h, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "NULL handle");
    check_sweep_err(h, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_spmv(const amg_csr* A, const double* x, double* y, void* stream) {
  return guarded([&]() -> amg_status {
    validate_csr_arg(A, "A");
    if (!A->on_device) fail(AMG_ERR_ARG, "amg_spmv needs device CSR arrays");
    if (!x || !y) fail(AMG_ERR_ARG, "NULL vector");
    CsrDev<double> M;
    M.n = A->nrows; M.m = A->ncols; M.nnz = A->nnz;
    M.ptr = A->rowptr; M.col = A->colidx; M.val = A->val;
    M.lpr = lpr_for(M.n, M.nnz);
    spmv<double>(M, x, y, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_spmv_dot(const amg_csr* A, const double* x, double* y, double* dot, void* stream) {
  return guarded([&]() -> amg_status {
    validate_csr_arg(A, "A");
    if (!A->on_device) fail(AMG_ERR_ARG, "amg_spmv_dot needs device CSR arrays");
    if (A->nrows != A->ncols) fail(AMG_ERR_SHAPE, "A is not square");
    if (!x || !y || !dot) fail(AMG_ERR_ARG, "NULL vector");
    CsrDev<double> M;
    M.n = A->nrows; M.m = A->ncols; M.nnz = A->nnz;
    M.ptr = A->rowptr; M.col = A->colidx; M.val = A->val;
    M.lpr = lpr_for(M.n, M.nnz);
    hipStream_t st = (hipStream_t)stream;
    // one partial sum per SpMV workgroup, summed in a fixed order by one
    // workgroup (the same reduction as PCG's q = A p with p^T q)
    const int64_t np = spmv_dot_partials(M.lpr, M.n);
    double* partial = nullptr;
    HIPC(hipMalloc(&partial, (size_t)std::max<int64_t>(np, 1) * sizeof(double)));
    spmv_dot(M, x, y, partial, st);
    reduce(np, partial, dot, 0, -1, st);
    hipError_t e = hipGetLastError();
    hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(partial);
    HIPC(e);
    HIPC(es);
    return AMG_OK;
  });
}

// Scratch of amg_spmv_dot_noalloc: its per-workgroup partial sums (2 MiB).
// Each device holds its own copy until the process ends; host code uses the
// per-device address from hipGetSymbolAddress, never the name itself.
constexpr int64_t NOALLOC_PARTIALS = int64_t(1) << 18;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

double* noalloc_scratch() {
  static std::mutex mu;
  static std::vector<double*> addr;   // by device id
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = (double*)p;
  }
  return addr[dev];
}

amg_status amg_spmv_dot_noalloc(const amg_csr* A, const double* x, double* y, double* dot,
                                void* stream) {
  return guarded([&]() -> amg_status {
    validate_csr_arg(A, "A");
    if (!A->on_device) fail(AMG_ERR_ARG, "amg_spmv_dot_noalloc needs device CSR arrays");
    if (A->nrows != A->ncols) fail(AMG_ERR_SHAPE, "A is not square");
    if (!x || !y || !dot) fail(AMG_ERR_ARG, "NULL vector");
    CsrDev<double> M;
    M.n = A->nrows; M.m = A->ncols; M.nnz = A->nnz;
    M.ptr = A->rowptr; M.col = A->colidx; M.val = A->val;
    M.lpr = lpr_for(M.n, M.nnz);
    const int64_t np = spmv_dot_partials(M.lpr, M.n);
    if (np > NOALLOC_PARTIALS)
      fail(AMG_ERR_LIMIT, "amg_spmv_dot_noalloc: " + std::to_string(np) +
                              " partial sums needed, the static scratch holds " +
                              std::to_string(NOALLOC_PARTIALS) + " (use amg_spmv_dot)");
    double* partial = noalloc_scratch();
    hipStream_t st = (hipStream_t)stream;
    // every workgroup writes its own partial and the reduction reads exactly
    // those: nothing in the scratch has to start at zero
    spmv_dot(M, x, y, partial, st);
    reduce(np, partial, dot, 0, -1, st);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_hier_info(const amg_hier* h, amg_level_info* lv, int cap, int* nlevels) {
  return guarded([&]() -> amg_status {
    if (!h || !nlevels) fail(AMG_ERR_ARG, "NULL argument");
    *nlevels = (int)h->lv.size();
    for (int l = 0; l < cap && l < (int)h->lv.size(); ++l) {
      const Level& L = h->lv[l];
      lv[l].n = L.n;
      lv[l].nnz = L.nnz;
      lv[l].p_nnz = L.coarsest ? 0 : L.p_nnz;
      lv[l].nblocks = L.coarsest ? 0 : L.nstars;
      lv[l].ncolors = L.coarsest ? 0 : L.ncolours;
      lv[l].exact_blocks = L.coarsest ? 0 : (L.ints.exact_blocks ? 1 : 0);
      lv[l].star_rows = L.coarsest ? 0 : L.star_rows;
      lv[l].star_row_nnz = L.coarsest ? 0 : L.star_row_nnz;
      lv[l].fac_entries = L.coarsest ? 0 : L.fac_total;
      lv[l].sweep_form = L.coarsest ? 0 : L.sweep_mode;
      lv[l].sweep_lanes = (L.coarsest || L.sweep_mode == SWEEP_DENSE || L.sweep_mode == SWEEP_PANEL) ? 0 : L.lpr_S;
      lv[l].sweep_pairs = (!L.coarsest && L.sweep_mode == SWEEP_PIPE) ? L.pipe_u : 0;
      lv[l].prec = L.prec;
      lv[l].grad_ratio = L.grad_ratio;
    }
    return AMG_OK;
  });
}

amg_status amg_export_integers(const amg_hier* h, int level, amg_int_export* out) {
  return guarded([&]() -> amg_status {
    if (!h || !out) fail(AMG_ERR_ARG, "NULL argument");
    if (level < 0 || level + 1 >= (int)h->lv.size()) fail(AMG_ERR_ARG, "level out of range");
    fill_export(h->lv[level].ints, out);
    return AMG_OK;
  });
}

amg_status amg_export_level(const amg_hier* h, int level, int64_t* a_ptr, int32_t* a_col,
                            double* a_val, int64_t* p_ptr, int32_t* p_col, double* p_val) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "NULL handle");
    if (level < 0 || level >= (int)h->lv.size()) fail(AMG_ERR_ARG, "level out of range");
    const Level& L = h->lv[level];
    if (a_ptr) HIPC(hipMemcpy(a_ptr, L.A_ptr, (L.n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (a_col) HIPC(hipMemcpy(a_col, L.A_col, L.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (a_val) HIPC(hipMemcpy(a_val, L.A_val, L.nnz * sizeof(double), hipMemcpyDeviceToHost));
    if (!L.coarsest) {
      if (p_ptr) HIPC(hipMemcpy(p_ptr, L.P_ptr, (L.n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
      if (p_col) HIPC(hipMemcpy(p_col, L.P_col, L.p_nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      if (p_val) HIPC(hipMemcpy(p_val, L.P_val, L.p_nnz * sizeof(double), hipMemcpyDeviceToHost));
    }
    return AMG_OK;
  });
}

struct IntsHandle {
  LevelInts ints;
};

amg_status amg_level0_integers(const amg_csr* A, const amg_csr* G, const amg_options* opt,
                               amg_int_export* out, void** handle) {
  return guarded([&]() -> amg_status {
    if (!out || !handle) fail(AMG_ERR_ARG, "NULL argument");
    if (A && A->on_device) fail(AMG_ERR_ARG, "amg_level0_integers takes host arrays");
    if (G && G->on_device) fail(AMG_ERR_ARG, "amg_level0_integers takes host arrays");
    amg_options o;
    if (opt) o = *opt; else amg_default_options(&o);
    Level0Host l0;
    level0_host(A, G, l0, nullptr);
    auto H = std::make_unique<IntsHandle>();
    bool use_ref = o.interp == AMG_INTERP_REF && o.ref_nlevels > 0;
    std::vector<int32_t> rc, rb;
    if (use_ref) {
      rc.assign(o.ref_coarse_nodes[0], o.ref_coarse_nodes[0] + o.ref_ncoarse[0]);
      rb.assign(o.ref_coarse_bnd[0], o.ref_coarse_bnd[0] + o.ref_nbnd[0]);
    }
    HostError err;
    check_ext_options(o);
    if (!setup_level_integers(l0.Apat, l0.G, l0.S, use_ref, rc, rb, ext_options(o), H->ints, err))
      fail((amg_status)err.code, err.msg);
    stars_and_colours(l0.Apat, l0.G, H->ints);
    fill_export(H->ints, out);
    *handle = H.release();
    return AMG_OK;
  });
}

void amg_free_integers(void* handle) { delete (IntsHandle*)handle; }

int64_t amg_mlp_nparams(void) { return MLP_NPARAM; }

amg_status amg_mlp_params(amg_hier* h, float* get, const float* set) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "NULL handle");
    ensure_mlp(h, nullptr);
    if (get) {
      if (!h->mlp.ready) fail(AMG_ERR_ARG, "the network has no parameters yet");
      HIPC(hipMemcpy(get, h->mlp.master, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    }
    if (set) {
      HIPC(hipMemcpy(h->mlp.master, set, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
      fill<float>(MLP_NPARAM, 0.f, h->mlp.adam_m, nullptr);
      fill<float>(MLP_NPARAM, 0.f, h->mlp.adam_v, nullptr);
      h->mlp.step = 0;
      mlp_refresh_bf16(h->mlp, nullptr);
      HIPC(hipDeviceSynchronize());
      h->mlp.ready = true;
    }
    return AMG_OK;
  });
}

amg_status amg_mlp_forward(amg_hier* h, const uint16_t* x, int64_t n, float* y, void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !x || !y) fail(AMG_ERR_ARG, "NULL argument");
    if (n <= 0 || n % 16) fail(AMG_ERR_ARG, "n must be a positive multiple of 16");
    if (!h->mlp.ready) fail(AMG_ERR_ARG, "the network has no parameters yet");
    ensure_work(h, n);
    mlp_forward(h->mlp, x, n, h->work, y, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_mlp_backward(amg_hier* h, const uint16_t* x, int64_t n, const float* dy, float* grad,
                            void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !x || !dy || !grad) fail(AMG_ERR_ARG, "NULL argument");
    if (n <= 0 || n % 16) fail(AMG_ERR_ARG, "n must be a positive multiple of 16");
    if (!h->mlp.ready) fail(AMG_ERR_ARG, "the network has no parameters yet");
    if (h->work.rows < n) fail(AMG_ERR_ARG, "call amg_mlp_forward on the same rows first");
    mlp_backward(h->mlp, x, n, h->work, dy, grad, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_mlp_loss_grad(const float* y, const float* t, const double* ahat, int64_t n,
                             int64_t nvalid, float* dy, float* row_loss, void* stream) {
  return guarded([&]() -> amg_status {
    if (!y || !t || !ahat || !dy || !row_loss) fail(AMG_ERR_ARG, "NULL argument");
    if (n < 0 || nvalid < 0 || nvalid > n) fail(AMG_ERR_ARG, "need 0 <= nvalid <= n");
    mlp_loss(n, y, t, ahat, nullptr, nvalid, dy, row_loss, (hipStream_t)stream);
    HIPC(hipGetLastError());
    return AMG_OK;
  });
}

amg_status amg_mlp_train(amg_hier* h, const amg_mlp_train_cfg* cfg, amg_mlp_stats* stats,
                         void* stream) {
  return guarded([&]() -> amg_status {
    if (!h || !cfg) fail(AMG_ERR_ARG, "NULL argument");
    if (h->lv[0].user_p) fail(AMG_ERR_ARG, "the learned setup needs the paper's interpolation (no user P)");
    if (h->lv[0].ints.patch)
      fail(AMG_ERR_ARG, "the learned setup predicts block solves (ext_mode AMG_EXT_BLOCKS)");
    if (cfg->batch <= 0 || cfg->batch % 16) fail(AMG_ERR_ARG, "batch must be a positive multiple of 16");
    if (cfg->epochs < 0) fail(AMG_ERR_ARG, "epochs < 0");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    ensure_mlp(h, st);
    if (cfg->init) {
      HIPC(hipMemcpyAsync(h->mlp.master, cfg->init, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
      fill<float>(MLP_NPARAM, 0.f, h->mlp.adam_m, st);
      fill<float>(MLP_NPARAM, 0.f, h->mlp.adam_v, st);
      h->mlp.step = 0;
      mlp_refresh_bf16(h->mlp, st);
      h->mlp.ready = true;
    }
    if (!h->mlp.ready) fail(AMG_ERR_ARG, "first training needs initial parameters (cfg->init)");
    learned_features(h, cfg->eligible_max, st);
    std::vector<int8_t> el(h->mlp_nb);
    HIPC(hipMemcpyAsync(el.data(), h->fel, h->mlp_nb, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    std::vector<int32_t> ids;
    for (int64_t b = 0; b < h->mlp_nb; ++b)
      if (el[b]) ids.push_back((int32_t)b);
    const int64_t B = cfg->batch;
    if (h->batch_cap < B) {
      h->bX = h->pool.get<uint16_t>((size_t)B * MLP_IN);
      h->bT = h->pool.get<float>((size_t)B * MLP_OUT);
      h->bY = h->pool.get<float>((size_t)B * MLP_OUT);
      h->bdY = h->pool.get<float>((size_t)B * MLP_OUT);
      h->bloss = h->pool.get<float>(B);
      h->batch_cap = B;
    }
    ensure_work(h, B);
    int32_t* d_ids = h->pool.get<int32_t>(std::max<size_t>(ids.size(), 1));
    uint64_t state = cfg->seed ^ 0x9E3779B97F4A7C15ull;
    auto next = [&]() {   // SplitMix64
      uint64_t z = (state += 0x9E3779B97F4A7C15ull);
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      return z ^ (z >> 31);
    };
    std::vector<float> loss_h(B);
    double first = 0.0, last = 0.0;
    const int64_t nids = (int64_t)ids.size();
    for (int ep = 0; ep < cfg->epochs && nids > 0; ++ep) {
      for (int64_t i = nids - 1; i > 0; --i) std::swap(ids[i], ids[next() % (uint64_t)(i + 1)]);
      HIPC(hipMemcpyAsync(d_ids, ids.data(), nids * sizeof(int32_t), hipMemcpyHostToDevice, st));
      double ep_loss = 0.0;
      const bool track = ep == 0 || ep == cfg->epochs - 1;
      for (int64_t o = 0; o < nids; o += B) {
        const int64_t nb = std::min<int64_t>(B, nids - o);
        const int64_t npad = (nb + 15) / 16 * 16;
        mlp_gather(nb, npad, d_ids + o, h->fX, h->fT, h->bX, h->bT, st);
        mlp_forward(h->mlp, h->bX, npad, h->work, h->bY, st);
        mlp_loss(npad, h->bY, h->bT, h->fAhat, d_ids + o, nb, h->bdY, h->bloss, st);
        mlp_backward(h->mlp, h->bX, npad, h->work, h->bdY, h->mlp.grad, st);
        mlp_adam(h->mlp, (float)cfg->lr, st);
        if (track) {
          HIPC(hipMemcpyAsync(loss_h.data(), h->bloss, nb * sizeof(float), hipMemcpyDeviceToHost, st));
          HIPC(hipStreamSynchronize(st));
          for (int64_t r = 0; r < nb; ++r) ep_loss += loss_h[r];
        }
      }
      if (ep == 0) first = ep_loss / nids;
      if (ep == cfg->epochs - 1) last = ep_loss / nids;
    }
    HIPC(hipStreamSynchronize(st));
    h->mstats.loss_first = first;
    h->mstats.loss_last = last;
    h->mstats.eligible = nids;
    h->mstats.blocks = h->mlp_nb;
    h->mstats.train_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (cfg->global_iters > 0)
      h->mstats.rho_reference = convergence_factor(h, cfg->global_iters, st);
    if (stats) *stats = h->mstats;
    return AMG_OK;
  });
}

amg_status amg_mlp_use(amg_hier* h, const amg_mlp_use_cfg* cfg) {
  return guarded([&]() -> amg_status {
    if (!h) fail(AMG_ERR_ARG, "NULL handle");
    if (!cfg) {
      h->learned = false;
      return AMG_OK;
    }
    if (!h->mlp.ready) fail(AMG_ERR_ARG, "train the network (or set its parameters) first");
    if (cfg->refine_steps < 0 || !(cfg->accept_tol >= 0.0)) fail(AMG_ERR_ARG, "bad use configuration");
    h->use_cfg = *cfg;
    h->learned = true;
    return AMG_OK;
  });
}

amg_status amg_mlp_stats_get(const amg_hier* h, amg_mlp_stats* stats) {
  return guarded([&]() -> amg_status {
    if (!h || !stats) fail(AMG_ERR_ARG, "NULL argument");
    *stats = h->mstats;
    return AMG_OK;
  });
}

void amg_destroy(amg_hier* h) { delete h; }

}  // extern "C"

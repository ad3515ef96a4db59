// Host (CPU) integer phase of the H(curl) AMG setup.
//
// Everything here is graph work on integer patterns: augmentG (Algorithm 1),
// the nodal dual graph and its C/F splitting (Algorithm 2), the matching of
// length-two edge paths (Algorithm 3), the coarse gradient G_c = R G I_C
// (eq. (Gc)), the blocks of A_II used by the local harmonic extension, the
// structural pattern of P and the smoother's node-star blocks and colours.
// The floating-point steps run on the GPU (kernels.hip); these results are
// bit-exact with the reference definitions, which the test suite checks.
#pragma once

#include <cstdint>
#include <string>
#include <functional>
#include <vector>

namespace hamg {

// Host threads of the integer phase (at most 16, or HCURL_AMG_THREADS), and
// body(begin, end) run over [0, n) split across them.
unsigned host_threads();
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);

// CSR pattern (values, where present, live elsewhere).
struct Pattern {
  int64_t n = 0, m = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// A signed incidence matrix with at most two entries per row, stored per
// row as (node a, sign a), (node b, sign b) with a < b; -1 marks "absent".
struct Incidence {
  int64_t n = 0, m = 0;
  std::vector<int32_t> a, b;
  std::vector<int8_t> sa, sb;
  int nnz(int64_t r) const { return (a[r] >= 0) + (b[r] >= 0); }
};

// Integer results of one level (the layout exported through the C ABI).
struct LevelInts {
  int64_t n = 0, m_real = 0, n_art = 0;
  std::vector<int8_t> cf;                 // empty in refinement-based levels
  std::vector<int32_t> cg;
  std::vector<int32_t> r_dof1, r_dof2, r_i, r_j, r_k;
  std::vector<int8_t> r_s1, r_s2;
  std::vector<int32_t> interior;
  std::vector<int64_t> block_ptr;         // extension blocks
  std::vector<int32_t> block_dofs;
  std::vector<int64_t> block_depth;
  bool exact_blocks = true;
  std::vector<int64_t> star_ptr;          // smoother blocks
  std::vector<int32_t> star_dofs;
  std::vector<int32_t> star_color;
  int ncolors = 0;
  Incidence gc;                           // G_{l+1}
  std::vector<int32_t> gc_cols;           // level-l node of each column of G_{l+1}
  std::vector<int64_t> gc_ptr;            // CSR view of G_{l+1} for export
  std::vector<int32_t> gc_col;
  std::vector<int8_t> gc_val;
  std::vector<int32_t> fine_of_next;      // level-l node standing for each node of G~_{l+1}
  // structural pattern of P_l (n x nc); exterior rows hold one entry
  Pattern p;
  std::vector<int8_t> p_ext_sign;         // per P entry: +-1 on exterior rows, 0 on interior rows
  std::vector<int32_t> dof_stage;         // -1 exterior, else depth stage index of the DoF's block
  std::vector<int64_t> stage_ptr;         // blocks of each depth stage: [stage_ptr[s], stage_ptr[s+1])
  // patch extension (ext_mode 1): interior support of every column of P
  // (ascending DoFs)
  bool patch = false;
  std::vector<int64_t> patch_ptr;
  std::vector<int32_t> patch_dofs;
  int patch_max = 0;
};

// How P's interior rows are formed: ext_mode 0 = blocks of A_II (components,
// or depth-ordered owner groups when a component is too large); 1 = per-column
// patches of at most patch_cap interior DoFs grown over patch_hops rounds.
struct ExtOptions {
  int ext_block_max = 64;
  int ext_mode = 0;
  int patch_hops = 2;
  int patch_cap = 128;
};

struct HostError {
  int code;
  std::string msg;
};

// Read G (CSR with values) as an incidence matrix; validates the {+-1},
// {+1,-1} row structure.  Returns false and fills err on failure.
bool incidence_from_csr(int64_t n, int64_t m, const int64_t* ptr, const int32_t* idx,
                        const double* val, Incidence& G, HostError& err);

// Validate a CSR pattern (monotone pointers, sorted unique in-range columns).
bool validate_pattern(int64_t n, int64_t m, const int64_t* ptr, const int32_t* idx,
                      HostError& err);

// Algorithm 1.
void augment_g(const Incidence& G, Incidence& Gt, std::vector<int32_t>& B);

// Nodal dual graph of level 0: off-diagonal pattern of |G~|^T |A| |G~|.
Pattern nodal_graph_level0(const Pattern& A, const Incidence& Gt);

// Nodal graph of a coarser level from the finer one: u ~ v iff
// dist(fine_of[u], fine_of[v]) <= 2 in S_fine.
Pattern nodal_graph_coarse(const Pattern& S_fine, const std::vector<int32_t>& fine_of);

// First-pass C/F splitting (Algorithm 2): returns states 1 = C, 2 = F.
std::vector<int8_t> rs_first_pass(const Pattern& S, const std::vector<int32_t>& c_ini,
                                  const std::vector<int32_t>& f_ini);

// Full integer setup of one level.  `S` is the level's nodal graph (built
// from A on level 0 or from the finer level's graph).  ref_cg / ref_bnd are
// used when `use_ref` is set.  Returns false with err on failure; sets
// `nc_out` = number of coarse DoFs (0 = no coarsening possible).
bool setup_level_integers(const Pattern& A, const Incidence& G, const Pattern& S, bool use_ref,
                          const std::vector<int32_t>& ref_cg, const std::vector<int32_t>& ref_bnd,
                          const ExtOptions& ext, LevelInts& L, HostError& err);

// Node-star blocks of G and their greedy colouring on the conflict graph.
void stars_and_colours(const Pattern& A, const Incidence& G, LevelInts& L);

}  // namespace hamg

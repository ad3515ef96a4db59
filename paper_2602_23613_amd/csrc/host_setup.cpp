// Host integer phase of the H(curl) AMG setup (see host_setup.hpp).
#include "host_setup.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <numeric>
#include <queue>
#include <thread>

namespace hamg {

// Run body(begin, end) over [0, n) split across hardware threads.
// Host threads of the integer phase: hardware threads, at most 16 (or
// HCURL_AMG_THREADS when set).
unsigned host_threads() {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  hw = std::min(hw, 16u);
  if (const char* e = std::getenv("HCURL_AMG_THREADS")) {
    int v = std::atoi(e);
    if (v > 0) hw = (unsigned)v;
  }
  return hw;
}

// HCURL_AMG_VERBOSE=2: wall time of every step of the integer phase on stderr
struct StepClock {
  bool on;
  std::chrono::steady_clock::time_point t;
  StepClock() : t(std::chrono::steady_clock::now()) {
    const char* e = std::getenv("HCURL_AMG_VERBOSE");
    on = e && std::atoi(e) >= 2;
  }
  void mark(const char* what) {
    if (!on) return;
    auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[amg]   host %-30s %8.3f s\n", what,
                 std::chrono::duration<double>(now - t).count());
    t = now;
  }
};

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body) {
  unsigned hw = host_threads();
  int64_t nt = std::min<int64_t>(hw, std::max<int64_t>(1, n / 4096));
  if (nt <= 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back(body, b, e);
  }
  for (auto& x : th) x.join();
}

namespace {

// Build a CSR pattern from per-row lists produced in parallel: count(i)
// returns the row length, fill(i, out) writes the (sorted) row.
template <class Count, class Fill>
Pattern build_rows(int64_t n, int64_t m, Count count, Fill fill) {
  Pattern P;
  P.n = n;
  P.m = m;
  P.ptr.assign(n + 1, 0);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) P.ptr[i + 1] = count(i);
  });
  for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] += P.ptr[i];
  P.idx.resize(P.ptr[n]);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) fill(i, P.idx.data() + P.ptr[i]);
  });
  return P;
}

// Transpose of an incidence matrix: for each node, the rows containing it.
Pattern node_to_rows(const Incidence& G) {
  Pattern T;
  T.n = G.m;
  T.m = G.n;
  T.ptr.assign(G.m + 1, 0);
  for (int64_t r = 0; r < G.n; ++r) {
    if (G.a[r] >= 0) T.ptr[G.a[r] + 1]++;
    if (G.b[r] >= 0) T.ptr[G.b[r] + 1]++;
  }
  for (int64_t i = 0; i < G.m; ++i) T.ptr[i + 1] += T.ptr[i];
  T.idx.resize(T.ptr[G.m]);
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t r = 0; r < G.n; ++r) {   // rows visited ascending: lists come out sorted
    if (G.a[r] >= 0) T.idx[pos[G.a[r]]++] = (int32_t)r;
    if (G.b[r] >= 0) T.idx[pos[G.b[r]]++] = (int32_t)r;
  }
  return T;
}

// Edge graph of G~: nodes joined by a row with two entries; per neighbour
// the joining row (the largest row id if several rows join the same pair).
struct EdgeGraph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> nb;
  std::vector<int32_t> row;
  int32_t row_of(int32_t u, int32_t v) const {
    auto b = nb.begin() + ptr[u], e = nb.begin() + ptr[u + 1];
    auto it = std::lower_bound(b, e, v);
    return row[it - nb.begin()];
  }
};

EdgeGraph edge_graph(const Incidence& Gt) {
  int64_t nn = Gt.m;
  std::vector<int64_t> cnt(nn + 1, 0);
  for (int64_t r = 0; r < Gt.n; ++r)
    if (Gt.a[r] >= 0 && Gt.b[r] >= 0) {
      cnt[Gt.a[r] + 1]++;
      cnt[Gt.b[r] + 1]++;
    }
  for (int64_t i = 0; i < nn; ++i) cnt[i + 1] += cnt[i];
  std::vector<std::pair<int32_t, int32_t>> tmp(cnt[nn]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t r = 0; r < Gt.n; ++r)
    if (Gt.a[r] >= 0 && Gt.b[r] >= 0) {
      tmp[pos[Gt.a[r]]++] = {Gt.b[r], (int32_t)r};
      tmp[pos[Gt.b[r]]++] = {Gt.a[r], (int32_t)r};
    }
  EdgeGraph E;
  E.ptr.assign(nn + 1, 0);
  for (int64_t u = 0; u < nn; ++u) {
    auto b = tmp.begin() + cnt[u], e = tmp.begin() + cnt[u + 1];
    std::sort(b, e);
    // collapse duplicate neighbours keeping the largest row
    int64_t w = cnt[u];
    for (auto it = b; it != e; ++it) {
      if (w > cnt[u] && tmp[w - 1].first == it->first) {
        tmp[w - 1].second = std::max(tmp[w - 1].second, it->second);
      } else {
        tmp[w++] = *it;
      }
    }
    E.ptr[u + 1] = w - cnt[u];
  }
  for (int64_t u = 0; u < nn; ++u) E.ptr[u + 1] += E.ptr[u];
  E.nb.resize(E.ptr[nn]);
  E.row.resize(E.ptr[nn]);
  for (int64_t u = 0; u < nn; ++u)
    for (int64_t t = 0; t < E.ptr[u + 1] - E.ptr[u]; ++t) {
      E.nb[E.ptr[u] + t] = tmp[cnt[u] + t].first;
      E.row[E.ptr[u] + t] = tmp[cnt[u] + t].second;
    }
  return E;
}

int8_t entry(const Incidence& G, int64_t r, int32_t c) {
  if (G.a[r] == c) return G.sa[r];
  if (G.b[r] == c) return G.sb[r];
  return 0;
}

}  // namespace

bool validate_pattern(int64_t n, int64_t m, const int64_t* ptr, const int32_t* idx,
                      HostError& err) {
  if (ptr[0] != 0) {
    err = {-3, "CSR row pointer does not start at 0"};
    return false;
  }
  // rows checked in parallel; the first bad row (and its kind) is reported
  std::atomic<int64_t> bad_row(n);
  std::vector<int8_t> kind(n > 0 ? 1 : 0, 0);
  std::mutex mu;
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi && i < bad_row.load(std::memory_order_relaxed); ++i) {
      int8_t k = 0;
      if (ptr[i + 1] < ptr[i]) {
        k = 1;
      } else {
        for (int64_t t = ptr[i]; t < ptr[i + 1] && !k; ++t) {
          if (idx[t] < 0 || idx[t] >= m) k = 2;
          else if (t > ptr[i] && idx[t] <= idx[t - 1]) k = 3;
        }
      }
      if (k) {
        std::lock_guard<std::mutex> g(mu);
        if (i < bad_row.load()) {
          bad_row.store(i);
          kind[0] = k;
        }
        return;
      }
    }
  });
  const int64_t i = bad_row.load();
  if (i == n) return true;
  const char* what = kind[0] == 1 ? "CSR row pointers decrease at row "
                     : kind[0] == 2 ? "CSR column out of range in row "
                                    : "CSR columns unsorted or duplicated in row ";
  err = {-3, what + std::to_string(i)};
  return false;
}

bool incidence_from_csr(int64_t n, int64_t m, const int64_t* ptr, const int32_t* idx,
                        const double* val, Incidence& G, HostError& err) {
  if (!validate_pattern(n, m, ptr, idx, err)) return false;
  G.n = n;
  G.m = m;
  G.a.assign(n, -1);
  G.b.assign(n, -1);
  G.sa.assign(n, 0);
  G.sb.assign(n, 0);
  for (int64_t r = 0; r < n; ++r) {
    int64_t k = ptr[r + 1] - ptr[r];
    if (k > 2) {
      err = {-4, "G row " + std::to_string(r) + " has more than two entries"};
      return false;
    }
    for (int64_t t = ptr[r]; t < ptr[r + 1]; ++t)
      if (val[t] != 1.0 && val[t] != -1.0) {
        err = {-4, "G row " + std::to_string(r) + " has an entry other than +-1"};
        return false;
      }
    if (k >= 1) {
      G.a[r] = idx[ptr[r]];
      G.sa[r] = (int8_t)val[ptr[r]];
    }
    if (k == 2) {
      G.b[r] = idx[ptr[r] + 1];
      G.sb[r] = (int8_t)val[ptr[r] + 1];
      if (G.sa[r] == G.sb[r]) {
        err = {-4, "G row " + std::to_string(r) + " has two entries of the same sign"};
        return false;
      }
    }
  }
  return true;
}

// Algorithm 1: every row with a single entry delta gets a new column -delta.
void augment_g(const Incidence& G, Incidence& Gt, std::vector<int32_t>& B) {
  Gt = G;
  B.clear();
  int64_t k = 0;
  for (int64_t r = 0; r < G.n; ++r) {
    if (G.nnz(r) == 1) {
      Gt.b[r] = (int32_t)(G.m + k);
      Gt.sb[r] = (int8_t)(-G.sa[r]);
      B.push_back((int32_t)(G.m + k));
      ++k;
    }
  }
  Gt.m = G.m + k;
}

// Off-diagonal pattern of |G~|^T |A| |G~|: u ~ v iff some edge at u is
// coupled in A to some edge at v.
Pattern nodal_graph_level0(const Pattern& A, const Incidence& Gt) {
  Pattern N2R = node_to_rows(Gt);
  const int64_t nn = Gt.m;
  // every thread lists the sorted neighbours of one contiguous range of
  // nodes in a flat vector; the lists are then copied into place
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), nn / 4096));
  const int64_t chunk = (nn + nt - 1) / nt;
  std::vector<std::vector<int32_t>> flat(nt);
  Pattern S;
  S.n = S.m = nn;
  S.ptr.assign(nn + 1, 0);
  auto run_threads = [&](const std::function<void(int)>& body) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(body, t);
    for (auto& x : th) x.join();
  };
  run_threads([&](int t) {
    const int64_t b = std::min(nn, t * chunk), e = std::min(nn, b + chunk);
    std::vector<int32_t> stamp(nn, -1);
    std::vector<int32_t> out;
    auto& dst = flat[t];
    for (int64_t u = b; u < e; ++u) {
      out.clear();
      for (int64_t k = N2R.ptr[u]; k < N2R.ptr[u + 1]; ++k) {
        const int32_t r = N2R.idx[k];
        for (int64_t q = A.ptr[r]; q < A.ptr[r + 1]; ++q) {
          const int32_t j = A.idx[q];
          const int32_t nodes[2] = {Gt.a[j], Gt.b[j]};
          for (int32_t v : nodes) {
            if (v < 0 || v == u || stamp[v] == (int32_t)u) continue;
            stamp[v] = (int32_t)u;
            out.push_back(v);
          }
        }
      }
      std::sort(out.begin(), out.end());
      dst.insert(dst.end(), out.begin(), out.end());
      S.ptr[u + 1] = (int64_t)out.size();
    }
  });
  for (int64_t u = 0; u < nn; ++u) S.ptr[u + 1] += S.ptr[u];
  S.idx.resize(S.ptr[nn]);
  run_threads([&](int t) {
    const int64_t b = std::min(nn, t * chunk);
    std::copy(flat[t].begin(), flat[t].end(), S.idx.begin() + S.ptr[b]);
    std::vector<int32_t>().swap(flat[t]);
  });
  return S;
}

// u ~ v iff the fine counterparts are within distance two in S_fine.
Pattern nodal_graph_coarse(const Pattern& Sf, const std::vector<int32_t>& fine_of) {
  int64_t nc = (int64_t)fine_of.size();
  int64_t nf = Sf.n;
  // fine node -> coarse nodes standing for it
  std::vector<int64_t> iptr(nf + 1, 0);
  for (int64_t u = 0; u < nc; ++u) iptr[fine_of[u] + 1]++;
  for (int64_t i = 0; i < nf; ++i) iptr[i + 1] += iptr[i];
  std::vector<int32_t> inv(nc);
  {
    std::vector<int64_t> pos(iptr.begin(), iptr.end() - 1);
    for (int64_t u = 0; u < nc; ++u) inv[pos[fine_of[u]]++] = (int32_t)u;
  }
  std::vector<std::vector<int32_t>> rows(nc);
  parallel_for(nc, [&](int64_t b, int64_t e) {
    std::vector<int64_t> fstamp(nf, -1), cstamp(nc, -1);
    std::vector<int32_t> reach, out;
    for (int64_t u = b; u < e; ++u) {
      reach.clear();
      out.clear();
      int32_t f = fine_of[u];
      fstamp[f] = u;
      reach.push_back(f);
      for (int64_t t = Sf.ptr[f]; t < Sf.ptr[f + 1]; ++t) {
        int32_t w = Sf.idx[t];
        if (fstamp[w] != u) { fstamp[w] = u; reach.push_back(w); }
      }
      size_t n1 = reach.size();
      for (size_t q = 1; q < n1; ++q) {
        int32_t w1 = reach[q];
        for (int64_t t = Sf.ptr[w1]; t < Sf.ptr[w1 + 1]; ++t) {
          int32_t w = Sf.idx[t];
          if (fstamp[w] != u) { fstamp[w] = u; reach.push_back(w); }
        }
      }
      for (int32_t w : reach)
        for (int64_t t = iptr[w]; t < iptr[w + 1]; ++t) {
          int32_t v = inv[t];
          if (v == u || cstamp[v] == u) continue;
          cstamp[v] = u;
          out.push_back(v);
        }
      std::sort(out.begin(), out.end());
      rows[u] = out;
    }
  });
  Pattern S;
  S.n = S.m = nc;
  S.ptr.assign(nc + 1, 0);
  for (int64_t u = 0; u < nc; ++u) S.ptr[u + 1] = S.ptr[u] + (int64_t)rows[u].size();
  S.idx.resize(S.ptr[nc]);
  for (int64_t u = 0; u < nc; ++u) std::copy(rows[u].begin(), rows[u].end(), S.idx.begin() + S.ptr[u]);
  return S;
}

// Ruge-Stueben first pass: measure |N_U| + 2|N_F|; the undecided node of
// largest measure (smallest id on ties) becomes C, its undecided
// neighbours F; undecided neighbours of new F nodes gain one.  Buckets of
// min-heaps with lazy deletion give exactly that selection order.
namespace {

// Sets of node ids, one per measure value, as two-level bitmaps: insert and
// erase in O(1), the smallest id of a set by scanning the set's summary words
// from a lower bound kept per set.  Replaces a heap per measure with lazy
// deletion (the same selection: largest measure, then smallest id).
struct MeasureSets {
  int64_t words = 0, sums = 0;
  std::vector<uint64_t> bits;     // per set: `words` words over the ids
  std::vector<uint64_t> sum;      // per set: bit w set iff bits word w is nonzero
  std::vector<int64_t> count;     // ids per set
  std::vector<int64_t> hint;      // per set: no nonzero summary word below this one
  MeasureSets(int64_t n, int nsets) {
    words = (n + 63) / 64;
    sums = (words + 63) / 64;
    bits.assign((size_t)nsets * words, 0);
    sum.assign((size_t)nsets * sums, 0);
    count.assign(nsets, 0);
    hint.assign(nsets, sums);
  }
  void insert(int s, int64_t i) {
    const int64_t w = i >> 6;
    uint64_t& b = bits[(size_t)s * words + w];
    if (b == 0) sum[(size_t)s * sums + (w >> 6)] |= uint64_t(1) << (w & 63);
    b |= uint64_t(1) << (i & 63);
    ++count[s];
    hint[s] = std::min(hint[s], w >> 6);
  }
  void erase(int s, int64_t i) {
    const int64_t w = i >> 6;
    uint64_t& b = bits[(size_t)s * words + w];
    b &= ~(uint64_t(1) << (i & 63));
    if (b == 0) sum[(size_t)s * sums + (w >> 6)] &= ~(uint64_t(1) << (w & 63));
    --count[s];
  }
  int64_t smallest(int s) {
    const uint64_t* sm = &sum[(size_t)s * sums];
    int64_t k = hint[s];
    while (sm[k] == 0) ++k;   // count[s] > 0: some summary word is nonzero
    hint[s] = k;
    const int64_t w = (k << 6) + __builtin_ctzll(sm[k]);
    return (w << 6) + __builtin_ctzll(bits[(size_t)s * words + w]);
  }
};

}  // namespace

std::vector<int8_t> rs_first_pass(const Pattern& S, const std::vector<int32_t>& c_ini,
                                  const std::vector<int32_t>& f_ini) {
  const int8_t U = 0, C = 1, F = 2;
  int64_t n = S.n;
  std::vector<int8_t> st(n, U);
  for (int32_t c : c_ini) st[c] = C;
  for (int32_t f : f_ini) st[f] = F;
  std::vector<int32_t> lam(n, 0);
  int64_t maxdeg = 0;
  for (int64_t i = 0; i < n; ++i) maxdeg = std::max<int64_t>(maxdeg, S.ptr[i + 1] - S.ptr[i]);
  // the measure |N_U| + 2 |N_F| of an undecided node never exceeds 2 deg
  MeasureSets sets(n, (int)(2 * maxdeg + 2));
  int64_t top = -1;
  for (int64_t i = 0; i < n; ++i) {
    if (st[i] != U) continue;
    int32_t l = 0;
    for (int64_t t = S.ptr[i]; t < S.ptr[i + 1]; ++t) {
      int8_t s = st[S.idx[t]];
      l += (s == U) ? 1 : (s == F ? 2 : 0);
    }
    lam[i] = l;
    sets.insert(l, i);
    top = std::max<int64_t>(top, l);
  }
  std::vector<int32_t> newf;
  while (top >= 0) {
    if (sets.count[top] == 0) {
      --top;
      continue;
    }
    const int32_t i = (int32_t)sets.smallest((int)top);
    sets.erase((int)top, i);
    st[i] = C;
    newf.clear();
    for (int64_t t = S.ptr[i]; t < S.ptr[i + 1]; ++t) {
      int32_t j = S.idx[t];
      if (st[j] == U) {
        st[j] = F;
        sets.erase(lam[j], j);
        newf.push_back(j);
      }
    }
    for (int32_t j : newf)
      for (int64_t t = S.ptr[j]; t < S.ptr[j + 1]; ++t) {
        int32_t m = S.idx[t];
        if (st[m] == U) {
          sets.erase(lam[m], m);
          ++lam[m];
          sets.insert(lam[m], m);
          if (lam[m] > top) top = lam[m];
        }
      }
  }
  return st;
}

namespace {

// Algorithm 3 over the edge graph of G~.
void form_r(const Incidence& Gt, const EdgeGraph& E, const std::vector<int32_t>& Cp,
            const std::vector<char>& isB, bool skip_bb, LevelInts& L) {
  int64_t nn = Gt.m;
  std::vector<char> inCp(nn, 0), inK(nn, 0), used(Gt.n, 0);
  for (int32_t c : Cp) inCp[c] = 1;
  std::vector<int64_t> stamp(nn, -1);
  std::vector<int32_t> d2;
  for (int32_t i : Cp) {
    // nodes at edge distance exactly two from i
    stamp[i] = i;
    for (int64_t t = E.ptr[i]; t < E.ptr[i + 1]; ++t) stamp[E.nb[t]] = i;
    d2.clear();
    for (int64_t t = E.ptr[i]; t < E.ptr[i + 1]; ++t) {
      int32_t k = E.nb[t];
      for (int64_t q = E.ptr[k]; q < E.ptr[k + 1]; ++q) {
        int32_t j = E.nb[q];
        if (stamp[j] != i) {
          stamp[j] = i;
          d2.push_back(j);
        }
      }
    }
    std::sort(d2.begin(), d2.end());
    for (int32_t j : d2) {
      if (j <= i || !inCp[j]) continue;
      if (skip_bb && isB[i] && isB[j]) continue;
      // smallest mutual neighbour (sorted merge of the two lists)
      int64_t a = E.ptr[i], ae = E.ptr[i + 1], b = E.ptr[j], be = E.ptr[j + 1];
      int32_t k = -1;
      while (a < ae && b < be) {
        if (E.nb[a] == E.nb[b]) { k = E.nb[a]; break; }
        if (E.nb[a] < E.nb[b]) ++a; else ++b;
      }
      if (k < 0 || inK[k]) continue;
      int32_t dof1 = E.row_of(i, k), dof2 = E.row_of(k, j);
      used[dof1] = used[dof2] = 1;
      inK[k] = 1;
      L.r_dof1.push_back(dof1);
      L.r_dof2.push_back(dof2);
      L.r_s1.push_back((int8_t)(-entry(Gt, dof1, i)));
      L.r_s2.push_back(entry(Gt, dof2, j));
      L.r_i.push_back(i);
      L.r_j.push_back(j);
      L.r_k.push_back(k);
    }
  }
  L.interior.clear();
  for (int64_t e = 0; e < Gt.n; ++e)
    if (!used[e]) L.interior.push_back((int32_t)e);
}

// G_c = R G I_C: row r = s1 G(dof1,:) + s2 G(dof2,:), zero sums dropped;
// the kept columns are the nonzero ones, ascending.
void coarse_gradient(const Incidence& G, LevelInts& L) {
  int64_t nc = (int64_t)L.r_dof1.size();
  std::vector<std::vector<std::pair<int32_t, int>>> rows(nc);
  std::vector<char> keep(G.m, 0);
  for (int64_t r = 0; r < nc; ++r) {
    std::pair<int32_t, int> ent[4];
    int ne = 0;
    auto add = [&](int32_t c, int v) {
      if (c < 0) return;
      for (int q = 0; q < ne; ++q)
        if (ent[q].first == c) { ent[q].second += v; return; }
      ent[ne++] = {c, v};
    };
    int64_t d1 = L.r_dof1[r], d2 = L.r_dof2[r];
    add(G.a[d1], L.r_s1[r] * G.sa[d1]);
    add(G.b[d1], L.r_s1[r] * G.sb[d1]);
    add(G.a[d2], L.r_s2[r] * G.sa[d2]);
    add(G.b[d2], L.r_s2[r] * G.sb[d2]);
    for (int q = 0; q < ne; ++q)
      if (ent[q].second != 0) {
        rows[r].push_back(ent[q]);
        keep[ent[q].first] = 1;
      }
    std::sort(rows[r].begin(), rows[r].end());
  }
  std::vector<int32_t> newid(G.m, -1);
  L.gc_cols.clear();
  for (int64_t c = 0; c < G.m; ++c)
    if (keep[c]) {
      newid[c] = (int32_t)L.gc_cols.size();
      L.gc_cols.push_back((int32_t)c);
    }
  Incidence& Gc = L.gc;
  Gc.n = nc;
  Gc.m = (int64_t)L.gc_cols.size();
  Gc.a.assign(nc, -1);
  Gc.b.assign(nc, -1);
  Gc.sa.assign(nc, 0);
  Gc.sb.assign(nc, 0);
  L.gc_ptr.assign(nc + 1, 0);
  L.gc_col.clear();
  L.gc_val.clear();
  for (int64_t r = 0; r < nc; ++r) {
    auto& rw = rows[r];
    if (rw.size() >= 1) { Gc.a[r] = newid[rw[0].first]; Gc.sa[r] = (int8_t)rw[0].second; }
    if (rw.size() >= 2) { Gc.b[r] = newid[rw[1].first]; Gc.sb[r] = (int8_t)rw[1].second; }
    for (auto& pr : rw) {
      L.gc_col.push_back(newid[pr.first]);
      L.gc_val.push_back((int8_t)pr.second);
    }
    L.gc_ptr[r + 1] = (int64_t)L.gc_col.size();
  }
  // fine counterparts of the next level's nodes (real, then artificial in row order)
  L.fine_of_next = L.gc_cols;
  for (int64_t r = 0; r < nc; ++r)
    if (Gc.nnz(r) == 1) {
      int32_t bi = L.r_i[r] >= G.m ? L.r_i[r] : L.r_j[r];
      L.fine_of_next.push_back(bi);
    }
}

// Blocks of A_II (component blocks when all are small, otherwise owner
// groups by BFS depth from the coarse/path nodes), then the structural
// pattern of P.
void extension_and_pattern(const Pattern& A, const Incidence& Gt, const EdgeGraph& E,
                           const std::vector<int32_t>& sources, int ext_block_max, LevelInts& L,
                           bool want_pattern) {
  int64_t n = A.n;
  int64_t nc = (int64_t)L.r_dof1.size();
  std::vector<char> isint(n, 0);
  for (int32_t e : L.interior) isint[e] = 1;
  // --- connected components of graph(A_II) (union-find) ---
  std::vector<int32_t> par(n);
  std::iota(par.begin(), par.end(), 0);
  std::function<int32_t(int32_t)> find = [&](int32_t x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
  };
  for (int32_t e : L.interior)
    for (int64_t t = A.ptr[e]; t < A.ptr[e + 1]; ++t) {
      int32_t j = A.idx[t];
      if (!isint[j]) continue;
      int32_t a = find(e), b = find(j);
      if (a != b) par[std::max(a, b)] = std::min(a, b);
    }
  std::vector<int32_t> csize(n, 0);
  int32_t maxsz = 0;
  for (int32_t e : L.interior) maxsz = std::max(maxsz, ++csize[find(e)]);
  L.block_ptr.assign(1, 0);
  L.block_dofs.clear();
  L.block_depth.clear();
  if (L.interior.empty() || maxsz <= ext_block_max) {
    L.exact_blocks = true;
    // components ordered by their smallest DoF; root = smallest DoF
    std::vector<int64_t> start(n, -1);
    std::vector<int32_t> roots;
    for (int32_t e : L.interior) {
      int32_t r = find(e);
      if (r == e) roots.push_back(e);
    }
    std::vector<int64_t> off(n, 0);
    int64_t acc = 0;
    for (int32_t r : roots) { off[r] = acc; acc += csize[r]; L.block_ptr.push_back(acc); L.block_depth.push_back(0); }
    L.block_dofs.resize(acc);
    std::vector<int64_t> pos(n, 0);
    for (int32_t r : roots) pos[r] = off[r];
    for (int32_t e : L.interior) L.block_dofs[pos[find(e)]++] = e;
  } else {
    L.exact_blocks = false;
    const int64_t INF = std::numeric_limits<int64_t>::max();
    int64_t nn = Gt.m;
    std::vector<int64_t> depth(nn, INF);
    std::vector<int32_t> q;
    q.reserve(nn);
    for (int32_t s : sources) if (depth[s] == INF) { depth[s] = 0; q.push_back(s); }
    for (size_t h = 0; h < q.size(); ++h) {
      int32_t u = q[h];
      for (int64_t t = E.ptr[u]; t < E.ptr[u + 1]; ++t) {
        int32_t v = E.nb[t];
        if (depth[v] == INF) { depth[v] = depth[u] + 1; q.push_back(v); }
      }
    }
    // key = (depth of owner, owner id) or (0, -1-e) for a DoF with no node
    std::vector<std::pair<std::pair<int64_t, int64_t>, int32_t>> keyed;
    keyed.reserve(L.interior.size());
    for (int32_t e : L.interior) {
      std::pair<int64_t, int64_t> key;
      if (Gt.a[e] < 0 && Gt.b[e] < 0) {
        key = {0, -1 - (int64_t)e};
      } else {
        bool first = true;
        int32_t nodes[2] = {Gt.a[e], Gt.b[e]};
        for (int32_t v : nodes) {
          if (v < 0) continue;
          std::pair<int64_t, int64_t> c = {depth[v], v};
          if (first || c > key) key = c;
          first = false;
        }
      }
      keyed.push_back({key, e});
    }
    std::sort(keyed.begin(), keyed.end());
    for (size_t t = 0; t < keyed.size(); ++t) {
      if (t > 0 && keyed[t].first != keyed[t - 1].first) {
        L.block_ptr.push_back((int64_t)L.block_dofs.size());
        L.block_depth.push_back(keyed[t - 1].first.first);
      }
      L.block_dofs.push_back(keyed[t].second);
    }
    if (!keyed.empty()) {
      L.block_ptr.push_back((int64_t)L.block_dofs.size());
      L.block_depth.push_back(keyed.back().first.first);
    }
  }
  // --- depth stages (blocks are sorted by depth) ---
  int64_t nb = (int64_t)L.block_depth.size();
  L.stage_ptr.assign(1, 0);
  L.dof_stage.assign(n, -1);
  for (int64_t b = 0; b < nb; ++b) {
    if (b > 0 && L.block_depth[b] != L.block_depth[b - 1]) L.stage_ptr.push_back(b);
  }
  L.stage_ptr.push_back(nb);
  int64_t nst = (int64_t)L.stage_ptr.size() - 1;
  for (int64_t s = 0; s < nst; ++s)
    for (int64_t b = L.stage_ptr[s]; b < L.stage_ptr[s + 1]; ++b)
      for (int64_t t = L.block_ptr[b]; t < L.block_ptr[b + 1]; ++t) L.dof_stage[L.block_dofs[t]] = (int32_t)s;
  if (!want_pattern) return;   // the patch extension builds its own pattern
  // --- structural pattern of P: exterior rows from R^T; a block's rows share
  //     the union of the done-row patterns reached through A ---
  std::vector<std::vector<int32_t>> rowcols(n);
  std::vector<int8_t> extsign(n, 0);
  for (int64_t r = 0; r < nc; ++r) {
    rowcols[L.r_dof1[r]] = {(int32_t)r};
    rowcols[L.r_dof2[r]] = {(int32_t)r};
    extsign[L.r_dof1[r]] = L.r_s1[r];
    extsign[L.r_dof2[r]] = L.r_s2[r];
  }
  std::vector<int64_t> block_cols_ptr(nb + 1, 0);
  for (int64_t s = 0; s < nst; ++s) {
    int64_t b0 = L.stage_ptr[s], b1 = L.stage_ptr[s + 1];
    std::vector<std::vector<int32_t>> bcols(b1 - b0);
    parallel_for(b1 - b0, [&](int64_t lo, int64_t hi) {
      std::vector<int64_t> stamp(nc, -1);
      for (int64_t bb = lo; bb < hi; ++bb) {
        int64_t b = b0 + bb;
        auto& out = bcols[bb];
        for (int64_t t = L.block_ptr[b]; t < L.block_ptr[b + 1]; ++t) {
          int32_t e = L.block_dofs[t];
          for (int64_t q2 = A.ptr[e]; q2 < A.ptr[e + 1]; ++q2) {
            int32_t j = A.idx[q2];
            int32_t sj = L.dof_stage[j];
            if (sj >= 0 && sj >= s) continue;     // not done yet
            for (int32_t c : rowcols[j])
              if (stamp[c] != b) { stamp[c] = b; out.push_back(c); }
          }
        }
        std::sort(out.begin(), out.end());
      }
    });
    for (int64_t bb = 0; bb < b1 - b0; ++bb) {
      int64_t b = b0 + bb;
      for (int64_t t = L.block_ptr[b]; t < L.block_ptr[b + 1]; ++t) rowcols[L.block_dofs[t]] = bcols[bb];
    }
  }
  Pattern& P = L.p;
  P.n = n;
  P.m = nc;
  P.ptr.assign(n + 1, 0);
  for (int64_t e = 0; e < n; ++e) P.ptr[e + 1] = P.ptr[e] + (int64_t)rowcols[e].size();
  P.idx.resize(P.ptr[n]);
  L.p_ext_sign.assign(P.ptr[n], 0);
  for (int64_t e = 0; e < n; ++e) {
    std::copy(rowcols[e].begin(), rowcols[e].end(), P.idx.begin() + P.ptr[e]);
    if (extsign[e] != 0) L.p_ext_sign[P.ptr[e]] = extsign[e];
  }
}

// Patch extension: column c of P is R^T e_c plus its least-energy extension
// into the interior DoFs S_c.  S_c grows from {} over `hops` rounds: every
// interior DoF outside S_c coupled in A to the column's two exterior DoFs or
// to S_c (as it was at the start of the round) counts those couplings, and
// the coupled DoFs join in order of count (largest first, ties to the smaller
// id) until S_c holds `cap` DoFs.  Replaces the block pattern of P: interior
// row i holds the columns c with i in S_c (ascending), exterior rows keep
// their R^T entry.

// Open-addressing map from DoF ids to small counts for the candidates of one
// round; a generation number clears it in O(1).
struct CandMap {
  std::vector<int32_t> key, val;
  std::vector<uint32_t> gen;
  uint32_t g = 0, mask = 0;
  void reset(int64_t most) {
    size_t cap = 64;
    while ((int64_t)cap < 2 * most) cap <<= 1;
    if (cap > key.size()) {
      key.assign(cap, 0);
      val.assign(cap, 0);
      gen.assign(cap, 0);
      g = 0;
    }
    mask = (uint32_t)(key.size() - 1);
    if (++g == 0) {
      std::fill(gen.begin(), gen.end(), 0u);
      g = 1;
    }
  }
  uint32_t slot(int32_t k) const {
    uint32_t h = ((uint32_t)k * 2654435761u) & mask;
    while (gen[h] == g && key[h] != k) h = (h + 1) & mask;
    return h;
  }
  bool has(int32_t k) const { return gen[slot(k)] == g; }
  // count one more coupling of k; true if k is new this round
  bool bump(int32_t k) {
    const uint32_t h = slot(k);
    if (gen[h] != g) {
      gen[h] = g;
      key[h] = k;
      val[h] = 1;
      return true;
    }
    ++val[h];
    return false;
  }
  int32_t count(int32_t k) const { return val[slot(k)]; }
};

void patch_extension_pattern(const Pattern& A, int hops, int cap, LevelInts& L) {
  StepClock clk;
  const int64_t n = A.n;
  const int64_t nc = (int64_t)L.r_dof1.size();
  std::vector<char> isint(n, 0);
  for (int32_t e : L.interior) isint[e] = 1;
  // every thread takes one contiguous range of columns and lists their
  // supports in one flat vector; the ranges are then copied into place
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), nc / 4096));
  const int64_t chunk = (nc + nt - 1) / std::max(nt, 1);
  auto run_threads = [&](const std::function<void(int)>& body) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(body, t);
    for (auto& x : th) x.join();
  };
  std::vector<std::vector<int32_t>> flat(nt);
  L.patch_ptr.assign(nc + 1, 0);
  run_threads([&](int t) {
    const int64_t c0 = std::min(nc, t * chunk), c1 = std::min(nc, c0 + chunk);
    CandMap cand_map, in_s;
    std::vector<int32_t> S, snap, cand, tie;
    std::vector<int32_t> hist;
    auto& out = flat[t];
    for (int64_t c = c0; c < c1; ++c) {
      S.clear();
      in_s.reset(cap);
      const int32_t ext[2] = {L.r_dof1[c], L.r_dof2[c]};
      for (int h = 0; h < hops && (int64_t)S.size() < (int64_t)cap; ++h) {
        snap.assign(ext, ext + 2);
        snap.insert(snap.end(), S.begin(), S.end());
        int64_t most = 0;
        for (int32_t e : snap) most += A.ptr[e + 1] - A.ptr[e];
        cand_map.reset(std::min<int64_t>(most, n));
        cand.clear();
        for (int32_t e : snap)
          for (int64_t q = A.ptr[e]; q < A.ptr[e + 1]; ++q) {
            const int32_t j = A.idx[q];
            if (!isint[j] || in_s.has(j)) continue;
            if (cand_map.bump(j)) cand.push_back(j);
          }
        const int64_t room = std::max<int64_t>(0, (int64_t)cap - (int64_t)S.size());
        auto take = [&](int32_t j) {
          S.push_back(j);
          in_s.bump(j);
        };
        if ((int64_t)cand.size() <= room) {
          for (int32_t j : cand) take(j);
          continue;
        }
        // the first `room` candidates in (count descending, id ascending)
        // order: every candidate above the threshold count, then the
        // smallest ids of the threshold count
        int32_t cmax = 0;
        for (int32_t j : cand) cmax = std::max(cmax, cand_map.count(j));
        hist.assign(cmax + 2, 0);
        for (int32_t j : cand) ++hist[cand_map.count(j)];
        int32_t thr = cmax;
        int64_t above = 0;
        while (above + hist[thr] < room) above += hist[thr--];
        tie.clear();
        for (int32_t j : cand) {
          const int32_t k = cand_map.count(j);
          if (k > thr) take(j);
          else if (k == thr) tie.push_back(j);
        }
        const int64_t rest = room - above;
        std::nth_element(tie.begin(), tie.begin() + (rest - 1), tie.end());
        for (int64_t q = 0; q < rest; ++q) take(tie[q]);
      }
      std::sort(S.begin(), S.end());
      out.insert(out.end(), S.begin(), S.end());
      L.patch_ptr[c + 1] = (int64_t)S.size();
    }
  });
  clk.mark("patch supports");
  L.patch = true;
  L.patch_max = 0;
  for (int64_t c = 0; c < nc; ++c) {
    L.patch_max = std::max<int>(L.patch_max, (int)L.patch_ptr[c + 1]);
    L.patch_ptr[c + 1] += L.patch_ptr[c];
  }
  L.patch_dofs.resize(L.patch_ptr[nc]);
  run_threads([&](int t) {
    const int64_t c0 = std::min(nc, t * chunk);
    std::copy(flat[t].begin(), flat[t].end(), L.patch_dofs.begin() + L.patch_ptr[c0]);
    std::vector<int32_t>().swap(flat[t]);
  });
  // P's pattern: exterior rows one entry, interior rows one per patch holding
  // them, in ascending column order.  A parallel transpose of the patch lists:
  // thread t takes columns [c0(t), c1(t)) and counts its entries per row; a
  // row's entries from thread t follow those of threads < t, so every row
  // comes out sorted without a sort.
  Pattern& P = L.p;
  P.n = n;
  P.m = nc;
  std::vector<std::vector<int32_t>> cnt(nt);
  run_threads([&](int t) {
    cnt[t].assign(n, 0);
    const int64_t c0 = std::min(nc, t * chunk), c1 = std::min(nc, c0 + chunk);
    for (int64_t q = L.patch_ptr[c0]; q < L.patch_ptr[c1]; ++q) ++cnt[t][L.patch_dofs[q]];
  });
  std::vector<char> ext(n, 0);
  for (int64_t c = 0; c < nc; ++c) ext[L.r_dof1[c]] = ext[L.r_dof2[c]] = 1;
  // per-thread start of each row's run (relative to the row) in place of the
  // counts, and the row lengths; then the row pointers
  P.ptr.assign(n + 1, 0);
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t e = lo; e < hi; ++e) {
      int32_t acc = ext[e];
      for (int t = 0; t < nt; ++t) {
        const int32_t c = cnt[t][e];
        cnt[t][e] = acc;
        acc += c;
      }
      P.ptr[e + 1] = acc;
    }
  });
  for (int64_t e = 0; e < n; ++e) P.ptr[e + 1] += P.ptr[e];
  P.idx.resize(P.ptr[n]);
  L.p_ext_sign.assign(P.ptr[n], 0);
  for (int64_t c = 0; c < nc; ++c) {
    P.idx[P.ptr[L.r_dof1[c]]] = (int32_t)c;
    L.p_ext_sign[P.ptr[L.r_dof1[c]]] = L.r_s1[c];
    P.idx[P.ptr[L.r_dof2[c]]] = (int32_t)c;
    L.p_ext_sign[P.ptr[L.r_dof2[c]]] = L.r_s2[c];
  }
  run_threads([&](int t) {
    const int64_t c0 = std::min(nc, t * chunk), c1 = std::min(nc, c0 + chunk);
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t q = L.patch_ptr[c]; q < L.patch_ptr[c + 1]; ++q) {
        const int32_t j = L.patch_dofs[q];
        P.idx[P.ptr[j] + cnt[t][j]++] = (int32_t)c;
      }
  });
  clk.mark("P pattern from the patches");
  // no depth stages: every interior DoF is extended in one pass
  L.stage_ptr.assign(1, 0);
  for (int32_t e : L.interior) L.dof_stage[e] = 0;
}

}  // namespace

void stars_and_colours(const Pattern& A, const Incidence& G, LevelInts& L) {
  Pattern N2R = node_to_rows(G);
  L.star_ptr.assign(1, 0);
  L.star_dofs.clear();
  std::vector<int32_t> star_of_node(G.m, -1);
  for (int64_t v = 0; v < G.m; ++v) {
    if (N2R.ptr[v + 1] == N2R.ptr[v]) continue;
    star_of_node[v] = (int32_t)(L.star_ptr.size() - 1);
    for (int64_t t = N2R.ptr[v]; t < N2R.ptr[v + 1]; ++t) L.star_dofs.push_back(N2R.idx[t]);
    L.star_ptr.push_back((int64_t)L.star_dofs.size());
  }
  int64_t ns = (int64_t)L.star_ptr.size() - 1;
  L.star_color.assign(ns, -1);
  // the (at most two) stars holding each DoF, -1 for none
  std::vector<int32_t> dstar(2 * A.n, -1);
  parallel_for(A.n, [&](int64_t lo, int64_t hi) {
    for (int64_t d = lo; d < hi; ++d) {
      if (G.a[d] >= 0) dstar[2 * d] = star_of_node[G.a[d]];
      if (G.b[d] >= 0) dstar[2 * d + 1] = star_of_node[G.b[d]];
    }
  });
  // the earlier stars (smaller index) that share a DoF with, or are
  // A-coupled to, each star: listed in parallel, one contiguous range of
  // stars per thread
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), ns / 4096));
  const int64_t chunk = (ns + nt - 1) / std::max(nt, 1);
  std::vector<std::vector<int32_t>> flat(nt);
  std::vector<int64_t> nb_ptr(ns + 1, 0);
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t]() {
        const int64_t b0 = std::min(ns, t * chunk), b1 = std::min(ns, b0 + chunk);
        std::vector<int32_t> sstamp(ns, -1);
        auto& out = flat[t];
        for (int64_t b = b0; b < b1; ++b) {
          const size_t before = out.size();
          for (int64_t t2 = L.star_ptr[b]; t2 < L.star_ptr[b + 1]; ++t2) {
            const int32_t e = L.star_dofs[t2];
            for (int64_t q = A.ptr[e]; q <= A.ptr[e + 1]; ++q) {
              const int32_t d = (q == A.ptr[e + 1]) ? e : A.idx[q];
              for (int k = 0; k < 2; ++k) {
                const int32_t c = dstar[2 * (int64_t)d + k];
                if (c >= 0 && c < b && sstamp[c] != (int32_t)b) {
                  sstamp[c] = (int32_t)b;
                  out.push_back(c);
                }
              }
            }
          }
          nb_ptr[b + 1] = (int64_t)(out.size() - before);
        }
      });
    for (auto& x : th) x.join();
  }
  for (int64_t b = 0; b < ns; ++b) nb_ptr[b + 1] += nb_ptr[b];
  // greedy colouring in star order: the smallest colour no earlier
  // neighbour has
  std::vector<int64_t> cstamp(64, -1);
  int ncol = 0;
  for (int t = 0; t < nt; ++t) {
    const int64_t b0 = std::min(ns, t * chunk), b1 = std::min(ns, b0 + chunk);
    const std::vector<int32_t>& nb = flat[t];
    for (int64_t b = b0; b < b1; ++b) {
      for (int64_t q = nb_ptr[b]; q < nb_ptr[b + 1]; ++q) {
        const int col = L.star_color[nb[q - nb_ptr[b0]]];
        if (col >= (int)cstamp.size()) cstamp.resize(col + 1, -1);
        cstamp[col] = b;
      }
      int col = 0;
      while (col < (int)cstamp.size() && cstamp[col] == b) ++col;
      L.star_color[b] = col;
      ncol = std::max(ncol, col + 1);
    }
    std::vector<int32_t>().swap(flat[t]);
  }
  L.ncolors = ncol;
}

bool setup_level_integers(const Pattern& A, const Incidence& G, const Pattern& S, bool use_ref,
                          const std::vector<int32_t>& ref_cg, const std::vector<int32_t>& ref_bnd,
                          const ExtOptions& ext, LevelInts& L, HostError& err) {
  StepClock clk;
  L.n = A.n;
  L.m_real = G.m;
  Incidence Gt;
  std::vector<int32_t> B;
  augment_g(G, Gt, B);
  clk.mark("augmentG");
  L.n_art = (int64_t)B.size();
  if (S.n != Gt.m) {
    err = {-2, "nodal graph size does not match G~"};
    return false;
  }
  std::vector<char> isB(Gt.m, 0);
  for (int32_t b : B) isB[b] = 1;
  std::vector<int32_t> Cp;
  bool skip_bb = true;
  if (use_ref) {
    L.cg = ref_cg;
    std::sort(L.cg.begin(), L.cg.end());
    L.cg.erase(std::unique(L.cg.begin(), L.cg.end()), L.cg.end());
    for (int32_t c : L.cg)
      if (c < 0 || c >= G.m) { err = {-1, "refinement coarse node out of range"}; return false; }
    Cp = L.cg;
    for (int32_t b : ref_bnd) {
      if (b < G.m || b >= Gt.m) { err = {-1, "refinement boundary node out of range"}; return false; }
      Cp.push_back(b);
    }
    skip_bb = false;
    L.cf.clear();
  } else {
    std::vector<char> mark(Gt.m, 0);
    std::vector<int32_t> f_ini;
    for (int32_t b : B)
      for (int64_t t = S.ptr[b]; t < S.ptr[b + 1]; ++t) {
        int32_t v = S.idx[t];
        if (!isB[v] && !mark[v]) { mark[v] = 1; f_ini.push_back(v); }
      }
    std::sort(f_ini.begin(), f_ini.end());
    L.cf = rs_first_pass(S, B, f_ini);
    L.cg.clear();
    for (int64_t u = 0; u < G.m; ++u)
      if (L.cf[u] == 1) L.cg.push_back((int32_t)u);
    Cp = L.cg;
    Cp.insert(Cp.end(), B.begin(), B.end());
  }
  clk.mark("C/F splitting");
  std::sort(Cp.begin(), Cp.end());
  Cp.erase(std::unique(Cp.begin(), Cp.end()), Cp.end());
  EdgeGraph E = edge_graph(Gt);
  clk.mark("edge graph");
  L.r_dof1.clear(); L.r_dof2.clear(); L.r_s1.clear(); L.r_s2.clear();
  L.r_i.clear(); L.r_j.clear(); L.r_k.clear();
  form_r(Gt, E, Cp, isB, skip_bb, L);
  clk.mark("matching (Alg. 3)");
  if (L.r_dof1.empty()) return true;
  std::vector<int32_t> sources = Cp;
  sources.insert(sources.end(), L.r_k.begin(), L.r_k.end());
  std::sort(sources.begin(), sources.end());
  sources.erase(std::unique(sources.begin(), sources.end()), sources.end());
  L.patch = false;
  L.patch_ptr.clear();
  L.patch_dofs.clear();
  L.patch_max = 0;
  if (ext.ext_mode == 1) {
    // no blocks of A_II: every interior DoF is extended through the patches
    L.exact_blocks = false;
    L.block_ptr.assign(1, 0);
    L.block_dofs.clear();
    L.block_depth.clear();
    L.dof_stage.assign(A.n, -1);
    patch_extension_pattern(A, ext.patch_hops, ext.patch_cap, L);
    clk.mark("patches + P pattern");
  } else {
    extension_and_pattern(A, Gt, E, sources, ext.ext_block_max, L, true);
    clk.mark("extension blocks + P pattern");
  }
  coarse_gradient(G, L);
  clk.mark("coarse gradient");
  return true;
}

}  // namespace hamg

// Host symbolic analysis (Sect. 3.2.1 of Bouchet et al.: ordering, symbolic
// factorisation, elimination/assembly tree).
//
// The ordering is chosen for the structure the coded-mask model gives.  An
// unknown whose measurement rows contain no other selected unknown can be
// eliminated first: such "leaf" unknowns are pairwise uncoupled in
// A = H^T W H (they share no row), so each is a leaf of the elimination tree
// whose row structure is the set of remaining unknowns seen in its rows.
// Leaves are picked greedily by increasing work (the total length of their
// rows, a bound on their degree in A), which selects the per-detector,
// per-time-bin background unknowns before any sky pixel.  Consecutive
// leaves with overlapping structure are amalgamated into one front
// (supernode) while the dense panel stays dense enough; every other unknown
// goes into one dense root front, numbered for locality (below).  The result is a
// two-level assembly tree: independent leaf fronts, all children of the root.
// It is exact for any SPD matrix (with no leaves it is a dense Cholesky).
//
// The root front is assembled output-stationary: its original entries
// (sum over rows of w h h^T, grouped into dense "row panels") and the leaf
// contribution blocks (-L_Ug L_Ug^T) are all weighted panel products
// Q diag(w) Q^T on an index set U.  For every 64 x 64 lower tile of the root
// the analysis lists the panels that touch it ("incidences", with the
// positions of U inside the tile's row and column ranges), so one workgroup
// per tile sums its contributions and writes the tile once.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <sstream>
#include <chrono>
#include <cstdio>
#include <functional>
#include <cstdlib>
#include <thread>

#include "spi_internal.h"

namespace spi {

namespace {

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// With SPI_VERBOSE set in the environment the analysis reports the time of
// each phase on stderr (large patterns take minutes on the host).
struct PhaseLog {
  bool on = std::getenv("SPI_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void operator()(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[spi analysis] %-30s %8.2f s\n", what,
                 std::chrono::duration<double>(now - t).count());
    std::fflush(stderr);
    t = now;
  }
};

// Host threads of the analysis: up to 16, or SPI_ANALYSIS_THREADS (1..64;
// the results do not depend on it, which a test checks).
unsigned n_threads() {
  if (const char* e = std::getenv("SPI_ANALYSIS_THREADS")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 64) return (unsigned)v;
  }
  return std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

// Run f(t) for t in [0, T) on T threads.
template <class F>
void parallel(unsigned T, F f) {
  if (T <= 1) {
    f(0u);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  for (unsigned t = 0; t < T; ++t) th.emplace_back([&f, t]() { f(t); });
  for (auto& x : th) x.join();
}

// Split [0, n) into T ranges of about equal weight, weight(i) = w[i+1]-w[i]
// for a prefix array w (e.g. rowptr).
std::vector<int64_t> balanced_ranges(const int64_t* w, int64_t n, unsigned T) {
  std::vector<int64_t> b(T + 1, n);
  b[0] = 0;
  const int64_t total = w[n] - w[0];
  for (unsigned t = 1; t < T; ++t) {
    const int64_t target = w[0] + total * (int64_t)t / (int64_t)T;
    b[t] = std::lower_bound(w, w + n + 1, target) - w;
    b[t] = std::min(std::max(b[t], b[t - 1]), n);
  }
  return b;
}

// Runs of a sorted index list by tile of edge `tile`: (tile, first position,
// end position).
void tile_runs(const int32_t* U, int64_t nU, int tile,
               std::vector<std::array<int32_t, 3>>& runs) {
  runs.clear();
  int64_t a = 0;
  while (a < nU) {
    const int32_t t = U[a] / tile;
    int64_t b = a + 1;
    while (b < nU && U[b] / tile == t) ++b;
    runs.push_back({t, (int32_t)a, (int32_t)b});
    a = b;
  }
}
// Locality numbering of the root unknowns (the dense root front's order is
// free: any symmetric permutation is factored in the same flops).  Two root
// columns are neighbours when they appear together in many rows: each
// column keeps its kNbr most frequent partners, counted over up to
// kSampleRows of its rows (evenly spaced, so the result is deterministic;
// ties go to the lower index).  The numbering recursively bisects that
// graph: a part is ordered by breadth-first distance from a far node (the
// last one reached by a first search) and split in two, at a multiple of 64
// when it is larger than 128, down to parts of at most 64 that become
// consecutive root indices.  A row's root columns then fall in few 64-column
// tiles, and the tile-by-tile assembly reads each row panel fewer times.
constexpr int kNbr = 8;
constexpr int kSampleRows = 128;

std::vector<int32_t> root_locality_order(const Analysis& a, const int64_t* rowptr,
                                         const int32_t* col,
                                         const std::vector<int32_t>& roots,
                                         const std::vector<int32_t>& rof,
                                         unsigned NT) {
  const int64_t nr = (int64_t)roots.size();
  std::vector<int32_t> perm(nr);
  std::iota(perm.begin(), perm.end(), 0);
  if (nr <= 64) return perm;
  // neighbours
  std::vector<int32_t> nbr((size_t)nr * kNbr, -1);
  parallel(NT, [&](unsigned t) {
    std::vector<int32_t> cnt(nr, 0), touched;
    std::vector<std::pair<int32_t, int32_t>> cand;
    for (int64_t j = t; j < nr; j += NT) {
      const int32_t c0 = roots[j];
      const int64_t r0 = a.colptr[c0], len = a.colptr[c0 + 1] - r0;
      const int64_t ns = std::min<int64_t>(len, kSampleRows);
      touched.clear();
      for (int64_t i = 0; i < ns; ++i) {
        const int32_t r = a.csc_row[r0 + (i * len) / ns];
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int32_t c = rof[col[e]];
          if (c < 0 || c == j) continue;
          if (cnt[c]++ == 0) touched.push_back(c);
        }
      }
      cand.clear();
      for (int32_t c : touched) {
        cand.emplace_back(-cnt[c], c);
        cnt[c] = 0;
      }
      const size_t k = std::min<size_t>(kNbr, cand.size());
      std::partial_sort(cand.begin(), cand.begin() + k, cand.end());
      for (size_t q = 0; q < k; ++q) nbr[(size_t)j * kNbr + q] = cand[q].second;
    }
  });
  // symmetric adjacency (CSR)
  std::vector<int64_t> ap(nr + 1, 0);
  for (int64_t j = 0; j < nr; ++j)
    for (int q = 0; q < kNbr; ++q) {
      const int32_t c = nbr[(size_t)j * kNbr + q];
      if (c >= 0) {
        ++ap[j + 1];
        ++ap[c + 1];
      }
    }
  for (int64_t j = 0; j < nr; ++j) ap[j + 1] += ap[j];
  std::vector<int32_t> adj(ap[nr]);
  {
    std::vector<int64_t> fill(ap.begin(), ap.end() - 1);
    for (int64_t j = 0; j < nr; ++j)
      for (int q = 0; q < kNbr; ++q) {
        const int32_t c = nbr[(size_t)j * kNbr + q];
        if (c >= 0) {
          adj[fill[j]++] = c;
          adj[fill[c]++] = (int32_t)j;
        }
      }
  }
  // recursive bisection; label[v] = the part v is in, seen[v] = last search
  std::vector<int32_t> label(nr, 0), seen(nr, -1);
  int32_t next_label = 1, search = 0;
  std::vector<int32_t> out;
  out.reserve(nr);
  std::vector<int32_t> queue;
  // breadth-first order of `part` from `src` within label L; unreached
  // vertices follow in their given order
  auto bfs = [&](const std::vector<int32_t>& part, int32_t src, int32_t L,
                 std::vector<int32_t>& order) {
    const int32_t sid = search++;
    order.clear();
    order.push_back(src);
    seen[src] = sid;
    for (size_t h = 0; h < order.size(); ++h) {
      const int32_t v = order[h];
      for (int64_t e = ap[v]; e < ap[v + 1]; ++e) {
        const int32_t u = adj[e];
        if (label[u] == L && seen[u] != sid) {
          seen[u] = sid;
          order.push_back(u);
        }
      }
    }
    for (int32_t v : part)
      if (seen[v] != sid) order.push_back(v);
  };
  std::function<void(std::vector<int32_t>&, int32_t)> bisect =
      [&](std::vector<int32_t>& part, int32_t L) {
        if (part.size() <= 64) {
          out.insert(out.end(), part.begin(), part.end());
          return;
        }
        std::vector<int32_t> o1, o2;
        bfs(part, part[0], L, o1);
        bfs(part, o1.back(), L, o2);
        size_t h = part.size() / 2;
        if (part.size() > 128) h = std::max<size_t>(64, h / 64 * 64);
        std::vector<int32_t> left(o2.begin(), o2.begin() + h),
            right(o2.begin() + h, o2.end());
        const int32_t La = next_label++, Lb = next_label++;
        for (int32_t v : left) label[v] = La;
        for (int32_t v : right) label[v] = Lb;
        part.clear();
        part.shrink_to_fit();
        bisect(left, La);
        bisect(right, Lb);
      };
  std::vector<int32_t> all(nr);
  std::iota(all.begin(), all.end(), 0);
  bisect(all, 0);
  return out;
}

}  // namespace

std::string analyze(int64_t m, int64_t n, const int64_t* rowptr,
                    const int32_t* col, const spi_opts& o, Analysis& a) {
  std::ostringstream err;
  PhaseLog phase;
  if (m < 1 || n < 1) return "m and n must be >= 1";
  if (n > INT32_MAX - 1 || m > INT32_MAX - 1) return "m and n must fit int32";
  if (!rowptr || !col) return "rowptr and col must be non-null host pointers";
  if (rowptr[0] != 0) return "rowptr[0] must be 0";
  for (int64_t r = 0; r < m; ++r) {
    if (rowptr[r + 1] < rowptr[r]) {
      err << "rowptr decreases at row " << r;
      return err.str();
    }
  }
  const int64_t nnz = rowptr[m];
  {
    // every thread checks a range of rows; the first bad row is reported
    const unsigned NT = n_threads();
    const std::vector<int64_t> rb = balanced_ranges(rowptr, m, NT);
    std::vector<int64_t> bad(NT, m);
    std::vector<int> kind(NT, 0);
    parallel(NT, [&](unsigned t) {
      for (int64_t r = rb[t]; r < rb[t + 1] && bad[t] == m; ++r)
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int32_t c = col[e];
          if (c < 0 || c >= n) {
            bad[t] = r;
            kind[t] = 1;
            break;
          }
          if (e > rowptr[r] && col[e - 1] >= c) {
            bad[t] = r;
            kind[t] = 2;
            break;
          }
        }
    });
    for (unsigned t = 0; t < NT; ++t)
      if (bad[t] < m) {
        const int64_t r = bad[t];
        if (kind[t] == 1) {
          for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
            if (col[e] < 0 || col[e] >= n) {
              err << "column index " << col[e] << " out of range in row " << r;
              return err.str();
            }
        }
        err << "columns not strictly increasing in row " << r;
        return err.str();
      }
  }
  a = Analysis();
  a.m = m;
  a.n = n;
  a.nnz = nnz;
  a.rowptr.assign(rowptr, rowptr + m + 1);
  a.col.assign(col, col + nnz);

  // ---- transpose of the pattern (parallel counting sort over row ranges;
  // rows stay in increasing order within each column)
  const unsigned NT = n_threads();
  {
    const std::vector<int64_t> rb = balanced_ranges(rowptr, m, NT);
    std::vector<std::vector<int64_t>> off(NT, std::vector<int64_t>(n, 0));
    parallel(NT, [&](unsigned t) {
      int64_t* c = off[t].data();
      for (int64_t e = rowptr[rb[t]]; e < rowptr[rb[t + 1]]; ++e) c[col[e]]++;
    });
    a.colptr.assign(n + 1, 0);
    for (int64_t j = 0; j < n; ++j) {
      int64_t s = a.colptr[j];
      for (unsigned t = 0; t < NT; ++t) {
        const int64_t c = off[t][j];
        off[t][j] = s;
        s += c;
      }
      if (s == a.colptr[j]) {
        err << "unknown " << j << " appears in no row (A would be singular)";
        return err.str();
      }
      a.colptr[j + 1] = s;
    }
    a.csc_pos.resize(nnz);
    a.csc_row.resize(nnz);
    parallel(NT, [&](unsigned t) {
      int64_t* o = off[t].data();
      for (int64_t r = rb[t]; r < rb[t + 1]; ++r)
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int64_t k = o[col[e]]++;
          a.csc_pos[k] = e;
          a.csc_row[k] = (int32_t)r;
        }
    });
  }

  phase("transpose");
  // ---- leaf selection: greedy independent set by increasing work
  std::vector<int64_t> work(n, 0);
  parallel(NT, [&](unsigned t) {
    for (int64_t j = t; j < n; j += NT)
      for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k) {
        int32_t r = a.csc_row[k];
        work[j] += rowptr[r + 1] - rowptr[r];
      }
  });
  std::vector<int32_t> cand;
  for (int64_t j = 0; j < n; ++j)
    if ((double)work[j] <= o.leaf_max_work) cand.push_back((int32_t)j);
  std::stable_sort(cand.begin(), cand.end(), [&](int32_t x, int32_t y) {
    return work[x] < work[y];
  });
  std::vector<char> claimed(m, 0), is_leaf(n, 0);
  for (int32_t j : cand) {
    bool free_rows = true;
    for (int64_t k = a.colptr[j]; k < a.colptr[j + 1] && free_rows; ++k)
      if (claimed[a.csc_row[k]]) free_rows = false;
    if (!free_rows) continue;
    is_leaf[j] = 1;
    for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k)
      claimed[a.csc_row[k]] = 1;
  }

  phase("leaf selection");
  // ---- root numbering: locality order (or the original order)
  a.root_of_col.assign(n, -1);
  for (int64_t j = 0; j < n; ++j)
    if (!is_leaf[j]) {
      a.root_of_col[j] = (int32_t)a.root_cols.size();
      a.root_cols.push_back((int32_t)j);
    }
  if (!o.keep_root_order) {
    const std::vector<int32_t> perm =
        root_locality_order(a, rowptr, col, a.root_cols, a.root_of_col, NT);
    std::vector<int32_t> orig = a.root_cols;
    for (size_t i = 0; i < perm.size(); ++i) {
      a.root_cols[i] = orig[perm[i]];
      a.root_of_col[orig[perm[i]]] = (int32_t)i;
    }
  }
  a.n_root = (int64_t)a.root_cols.size();
  a.n_pad = a.n_root ? round_up(a.n_root, kRootPad) : 0;

  phase("root numbering");
  // ---- amalgamate consecutive leaves into fronts.  The leaves are taken in
  // fixed chunks of kAmalgChunk (a front never spans two chunks), the chunks
  // in parallel and concatenated in order: the fronts do not depend on the
  // number of threads.
  constexpr int64_t kAmalgChunk = 4096;
  std::vector<int32_t> leaves;
  for (int64_t j = 0; j < n; ++j)
    if (is_leaf[j]) leaves.push_back((int32_t)j);
  const int64_t nr = std::max<int64_t>(a.n_root, 1);
  struct FrontPart {
    std::vector<int32_t> cols, U;
    std::vector<int64_t> col_end, U_end, panel;  // per front
    double work = 0.0, update = 0.0;
  };
  const int64_t n_lv = (int64_t)leaves.size();
  const int64_t n_ch = (n_lv + kAmalgChunk - 1) / kAmalgChunk;
  std::vector<FrontPart> fparts(n_ch);
  parallel(NT, [&](unsigned t) {
    std::vector<int64_t> mark(nr, -1), seen(nr, -1);
    std::vector<int32_t> curU, curCols, rj;
    for (int64_t ch = t; ch < n_ch; ch += NT) {
      FrontPart& P = fparts[ch];
      int64_t front = ch * kAmalgChunk;  // unique mark ids across chunks
      int64_t cur_sum = 0;
      curU.clear();
      curCols.clear();
      auto close_front = [&]() {
        std::sort(curU.begin(), curU.end());
        P.cols.insert(P.cols.end(), curCols.begin(), curCols.end());
        P.U.insert(P.U.end(), curU.begin(), curU.end());
        P.col_end.push_back((int64_t)P.cols.size());
        P.U_end.push_back((int64_t)P.U.size());
        P.panel.push_back((int64_t)curU.size() * (int64_t)curCols.size());
        ++front;
        curU.clear();
        curCols.clear();
        cur_sum = 0;
      };
      const int64_t l1 = std::min(n_lv, (ch + 1) * kAmalgChunk);
      for (int64_t li = ch * kAmalgChunk; li < l1; ++li) {
        const int32_t j = leaves[li];
        rj.clear();
        for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k) {
          int32_t r = a.csc_row[k];
          for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            int32_t ri = a.root_of_col[col[e]];
            if (ri >= 0 && seen[ri] != j) {
              seen[ri] = j;
              rj.push_back(ri);
            }
          }
        }
        if (!curCols.empty()) {
          int64_t add = 0;
          for (int32_t u : rj)
            if (mark[u] != front) ++add;
          int64_t newU = (int64_t)curU.size() + add;
          int64_t newp = (int64_t)curCols.size() + 1;
          bool ok = newp <= o.max_group;
          if (ok && newU > 0) {
            double dens = (double)(cur_sum + (int64_t)rj.size()) /
                          ((double)newU * (double)newp);
            ok = dens >= o.amalg_density;
          }
          if (!ok) close_front();
        }
        for (int32_t u : rj)
          if (mark[u] != front) {
            mark[u] = front;
            curU.push_back(u);
          }
        curCols.push_back(j);
        cur_sum += (int64_t)rj.size();
        // algorithmic work of leaf j as its own front (p = 1, c = the root
        // unknowns of its rows, its exact column count in L)
        const double c = (double)rj.size();
        P.work += 1.0 / 3.0 + c + c * c;
        P.update += c * (c + 1.0);
      }
      if (!curCols.empty()) close_front();
    }
  });
  a.grp_col_ptr.push_back(0);
  a.grp_U_ptr.push_back(0);
  a.grp_panel_off.push_back(0);
  double leaf_work = 0.0, leaf_update = 0.0;
  int64_t front = 0;
  for (const FrontPart& P : fparts) {
    const int64_t c0 = (int64_t)a.leaf_cols.size(), u0 = (int64_t)a.U.size();
    int64_t cb = 0;
    for (size_t f = 0; f < P.col_end.size(); ++f) {
      for (int64_t q = cb; q < P.col_end[f]; ++q) {
        a.leaf_cols.push_back(P.cols[q]);
        a.leaf_grp.push_back((int32_t)front);
      }
      cb = P.col_end[f];
      a.grp_col_ptr.push_back(c0 + P.col_end[f]);
      a.grp_U_ptr.push_back(u0 + P.U_end[f]);
      a.grp_panel_off.push_back(a.grp_panel_off.back() + P.panel[f]);
      ++front;
    }
    a.U.insert(a.U.end(), P.U.begin(), P.U.end());
    leaf_work += P.work;
    leaf_update += P.update;
  }
  a.n_groups = front;
  fparts.clear();
  fparts.shrink_to_fit();

  a.leaf_of_col.assign(n, -1);
  for (size_t l = 0; l < a.leaf_cols.size(); ++l) a.leaf_of_col[a.leaf_cols[l]] = (int32_t)l;

  phase("amalgamation");
  // ---- slots (rows of the leaf fronts, by leaf unknown) and their compact
  // root entries with U-local positions.  Sizes first, then every front
  // fills its own ranges (in parallel).
  const int64_t n_leaf = (int64_t)a.leaf_cols.size();
  std::vector<int32_t> root_cnt(m, 0);  // root entries per row
  parallel(NT, [&](unsigned t) {
    for (int64_t r = t; r < m; r += NT) {
      int32_t c = 0;
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) c += a.root_of_col[col[e]] >= 0;
      root_cnt[r] = c;
    }
  });
  a.leaf_slot_ptr.assign(n_leaf + 1, 0);
  for (int64_t l = 0; l < n_leaf; ++l) {
    const int32_t j = a.leaf_cols[l];
    a.leaf_slot_ptr[l + 1] = a.leaf_slot_ptr[l] + (a.colptr[j + 1] - a.colptr[j]);
  }
  a.n_slots = a.leaf_slot_ptr[n_leaf];
  a.grp_slot_ptr.resize(a.n_groups + 1);
  for (int64_t g = 0; g <= a.n_groups; ++g) a.grp_slot_ptr[g] = a.leaf_slot_ptr[a.grp_col_ptr[g]];
  a.slot_row.resize(a.n_slots);
  a.slot_leaf_src.resize(a.n_slots);
  a.slot_rr_ptr.assign(a.n_slots + 1, 0);
  for (int64_t l = 0; l < n_leaf; ++l) {
    const int32_t j = a.leaf_cols[l];
    int64_t sl = a.leaf_slot_ptr[l];
    for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k, ++sl) {
      a.slot_row[sl] = a.csc_row[k];
      a.slot_leaf_src[sl] = a.csc_pos[k];
      a.slot_rr_ptr[sl + 1] = a.slot_rr_ptr[sl] + root_cnt[a.csc_row[k]];
    }
  }
  a.rr_lpos.resize(a.slot_rr_ptr[a.n_slots]);
  a.rr_src.resize(a.slot_rr_ptr[a.n_slots]);
  parallel(NT, [&](unsigned t) {
    std::vector<int64_t> pm(nr, -1);
    for (int64_t g = t; g < a.n_groups; g += NT) {
      for (int64_t u = a.grp_U_ptr[g]; u < a.grp_U_ptr[g + 1]; ++u)
        pm[a.U[u]] = u - a.grp_U_ptr[g];
      for (int64_t sl = a.grp_slot_ptr[g]; sl < a.grp_slot_ptr[g + 1]; ++sl) {
        const int32_t r = a.slot_row[sl];
        int64_t q = a.slot_rr_ptr[sl];
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int32_t ri = a.root_of_col[col[e]];
          if (ri < 0) continue;
          a.rr_lpos[q] = (int32_t)pm[ri];
          a.rr_src[q] = e;
          ++q;
        }
      }
    }
  });

  phase("slots");
  // ---- row panels: consecutive rows (original order) with overlapping
  // root structure; rows without root entries contribute nothing to A_RR.
  // Each decision depends on the open panel, so the rows are grouped in
  // fixed chunks of kRowChunk (a panel never spans two chunks), the chunks
  // in parallel and concatenated in order (independent of the number of
  // threads); the per-entry maps are then filled panel by panel in parallel.
  constexpr int64_t kRowChunk = 65536;
  a.rp_U_base = (int64_t)a.U.size();
  a.rp_row_ptr.assign(1, 0);
  a.rp_U_ptr.assign(1, 0);
  a.rp_val_off.assign(1, 0);
  {
    struct PanelPart {
      std::vector<int32_t> rows, U;
      std::vector<int64_t> row_end, U_end, val;  // per panel
    };
    const int64_t n_rc = (m + kRowChunk - 1) / kRowChunk;
    std::vector<PanelPart> rparts(n_rc);
    parallel(NT, [&](unsigned t) {
      std::vector<int64_t> mark(nr, -1);
      for (int64_t ch = t; ch < n_rc; ch += NT) {
        PanelPart& P = rparts[ch];
        int64_t panel = ch * kRowChunk;  // unique mark ids across chunks
        int64_t rows_in = 0, sum = 0, pU0 = 0;
        auto close_panel = [&]() {
          std::sort(P.U.begin() + pU0, P.U.end());
          const int64_t nU = (int64_t)P.U.size() - pU0;
          P.row_end.push_back((int64_t)P.rows.size());
          P.U_end.push_back((int64_t)P.U.size());
          P.val.push_back(nU * rows_in);
          ++panel;
          pU0 = (int64_t)P.U.size();
          rows_in = 0;
          sum = 0;
        };
        const int64_t r1 = std::min(m, (ch + 1) * kRowChunk);
        for (int64_t r = ch * kRowChunk; r < r1; ++r) {
          const int64_t len = root_cnt[r];
          if (len == 0) continue;
          if (rows_in > 0) {
            int64_t add = 0;
            for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
              const int32_t ri = a.root_of_col[col[e]];
              if (ri >= 0 && mark[ri] != panel) ++add;
            }
            const int64_t newU = (int64_t)P.U.size() - pU0 + add;
            const double dens =
                (double)(sum + len) / ((double)newU * (double)(rows_in + 1));
            if (rows_in + 1 > o.max_group || dens < o.amalg_density) close_panel();
          }
          for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            const int32_t ri = a.root_of_col[col[e]];
            if (ri >= 0 && mark[ri] != panel) {
              mark[ri] = panel;
              P.U.push_back(ri);
            }
          }
          P.rows.push_back((int32_t)r);
          ++rows_in;
          sum += len;
        }
        if (rows_in > 0) close_panel();
      }
    });
    int64_t panel = 0;
    for (const PanelPart& P : rparts) {
      const int64_t r0 = (int64_t)a.rp_rows.size();
      const int64_t u0 = (int64_t)a.U.size() - a.rp_U_base;
      for (size_t q = 0; q < P.row_end.size(); ++q) {
        a.rp_row_ptr.push_back(r0 + P.row_end[q]);
        a.rp_U_ptr.push_back(u0 + P.U_end[q]);
        a.rp_val_off.push_back(a.rp_val_off.back() + P.val[q]);
        ++panel;
      }
      a.rp_rows.insert(a.rp_rows.end(), P.rows.begin(), P.rows.end());
      a.U.insert(a.U.end(), P.U.begin(), P.U.end());
    }
    a.n_rp = panel;
  }
  {
    const int64_t nrows = (int64_t)a.rp_rows.size();
    a.rp_rowbase.resize(nrows);
    a.rpe_ptr.assign(nrows + 1, 0);
    for (int64_t q = 0; q < nrows; ++q) a.rpe_ptr[q + 1] = a.rpe_ptr[q] + root_cnt[a.rp_rows[q]];
    a.rpe_pos.resize(a.rpe_ptr[nrows]);
    a.rpe_src.resize(a.rpe_ptr[nrows]);
    parallel(NT, [&](unsigned t) {
      std::vector<int64_t> pm(nr, -1);
      for (int64_t p = t; p < a.n_rp; p += NT) {
        const int32_t* Up = a.U.data() + a.rp_U_base + a.rp_U_ptr[p];
        const int64_t nU = a.rp_U_ptr[p + 1] - a.rp_U_ptr[p];
        for (int64_t x = 0; x < nU; ++x) pm[Up[x]] = x;
        for (int64_t q = a.rp_row_ptr[p]; q < a.rp_row_ptr[p + 1]; ++q) {
          const int32_t r = a.rp_rows[q];
          a.rp_rowbase[q] = a.rp_val_off[p] + (q - a.rp_row_ptr[p]) * nU;
          int64_t z = a.rpe_ptr[q];
          for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            const int32_t ri = a.root_of_col[col[e]];
            if (ri < 0) continue;
            a.rpe_pos[z] = (int32_t)pm[ri];
            a.rpe_src[z] = e;
            ++z;
          }
        }
      }
    });
  }

  phase("row panels");
  // ---- update-panel descriptors: leaf fronts (weight -1), row panels
  const int64_t leaf_panel_total = a.grp_panel_off[a.n_groups];
  for (int64_t g = 0; g < a.n_groups; ++g) {
    a.up_U_off.push_back(a.grp_U_ptr[g]);
    a.up_Q_off.push_back(a.grp_panel_off[g]);
    a.up_nU.push_back((int32_t)(a.grp_U_ptr[g + 1] - a.grp_U_ptr[g]));
    a.up_k.push_back((int32_t)(a.grp_col_ptr[g + 1] - a.grp_col_ptr[g]));
    a.up_w_off.push_back(-1);
  }
  for (int64_t p = 0; p < a.n_rp; ++p) {
    a.up_U_off.push_back(a.rp_U_base + a.rp_U_ptr[p]);
    a.up_Q_off.push_back(leaf_panel_total + a.rp_val_off[p]);
    a.up_nU.push_back((int32_t)(a.rp_U_ptr[p + 1] - a.rp_U_ptr[p]));
    a.up_k.push_back((int32_t)(a.rp_row_ptr[p + 1] - a.rp_row_ptr[p]));
    a.up_w_off.push_back((int32_t)a.rp_row_ptr[p]);
  }
  a.n_up = a.n_groups + a.n_rp;
  // the root assembly addresses an update panel with 32-bit byte offsets,
  // up to 24 columns (a batch of loads and one MFMA step) and 32 rows past
  // its end
  for (int64_t u = 0; u < a.n_up; ++u)
    if ((int64_t)(a.up_k[u] + 24) * (a.up_nU[u] + 32) * 8 >= ((int64_t)1 << 31))
      return "an update panel exceeds 2^31 bytes (reduce max_group)";

  // ---- incidences on the 64 x 64 lower tiles of the root
  if (a.n_pad) {
    a.asm_tile = o.asm_tile ? o.asm_tile
                            : (a.n_pad >= kAsmTile128From ? kAsmTileLarge : kAsmTileSmall);
    const int64_t T = a.n_pad / a.asm_tile;
    a.n_tiles = T * (T + 1) / 2;
    // Two passes over the updates, split into NT contiguous ranges (balanced
    // by |U|^2): counts per range and tile, then every range fills its own
    // stretch of each tile's list, so the lists hold their incidences in
    // increasing u whatever the number of threads.
    std::vector<int64_t> wpre(a.n_up + 1, 0);
    for (int64_t u = 0; u < a.n_up; ++u)
      wpre[u + 1] = wpre[u] + (int64_t)a.up_nU[u] * a.up_nU[u];
    const std::vector<int64_t> ub = balanced_ranges(wpre.data(), a.n_up, NT);
    std::vector<std::vector<int64_t>> cnt(NT, std::vector<int64_t>(a.n_tiles, 0));
    auto each = [&](unsigned t, auto&& f) {
      std::vector<std::array<int32_t, 3>> runs;
      for (int64_t u = ub[t]; u < ub[t + 1]; ++u) {
        if (a.up_k[u] == 0) continue;
        tile_runs(a.U.data() + a.up_U_off[u], a.up_nU[u], a.asm_tile, runs);
        for (size_t x = 0; x < runs.size(); ++x)
          for (size_t y = 0; y <= x; ++y) {
            const int64_t I = runs[x][0], J = runs[y][0];
            f(u, I * (I + 1) / 2 + J, runs[x], runs[y]);
          }
      }
    };
    parallel(NT, [&](unsigned t) {
      int64_t* c = cnt[t].data();
      each(t, [&](int64_t, int64_t tt, const std::array<int32_t, 3>&,
                  const std::array<int32_t, 3>&) { c[tt]++; });
    });
    a.inc_ptr.assign(a.n_tiles + 1, 0);
    for (int64_t tt = 0; tt < a.n_tiles; ++tt) {
      int64_t sum = a.inc_ptr[tt];
      for (unsigned t = 0; t < NT; ++t) {
        const int64_t c = cnt[t][tt];
        cnt[t][tt] = sum;  // this range's first slot in the tile's list
        sum += c;
      }
      a.inc_ptr[tt + 1] = sum;
    }
    a.inc.resize(4 * a.inc_ptr[a.n_tiles]);
    parallel(NT, [&](unsigned t) {
      int64_t* fillp = cnt[t].data();
      each(t, [&](int64_t u, int64_t tt, const std::array<int32_t, 3>& rx,
                  const std::array<int32_t, 3>& ry) {
        int32_t* p = a.inc.data() + 4 * fillp[tt]++;
        p[0] = (int32_t)u;
        p[1] = rx[1];
        p[2] = ry[1];
        p[3] = (rx[2] - rx[1]) | ((ry[2] - ry[1]) << 16);
      });
    });
    // the first row-panel incidence of each tile (leaf fronts, u < n_groups,
    // come first: incidences are listed by increasing u)
    a.inc_split.assign(a.n_tiles, 0);
    for (int64_t t = 0; t < a.n_tiles; ++t) {
      int64_t q = a.inc_ptr[t];
      while (q < a.inc_ptr[t + 1] && a.inc[4 * q] < a.n_groups) ++q;
      a.inc_split[t] = q;
    }
    // launch order: column by column (J), down each column (I >= J).  With
    // the XCD remap, consecutive tiles of a column run together on one XCD
    // and share the column tile's panel rows in its L2.  Measured against
    // groups of 8, 16, 32, 64 and 128 tile rows taken column by column
    // (root assembly, medium / large, ms): 4.50 / 482, 4.28 / 474,
    // 3.69 / 467, 3.71 / 459, 3.63 / 456; whole columns 3.62 / 448.
    a.tile_order.clear();
    a.tile_order.reserve(a.n_tiles);
    for (int64_t J = 0; J < T; ++J)
      for (int64_t I = J; I < T; ++I)
        a.tile_order.push_back((int32_t)(I * (I + 1) / 2 + J));
  }

  phase("incidences");
  // ---- selected-inversion tasks of the leaf fronts: (front, I, J) for the
  // kET-blocks I >= J of the front's U, front by front; the partial sums of
  // a task take one entry per pivot of its front.  Filled by ranges of fronts
  // in parallel.
  a.grp_task_ptr.assign(a.n_groups + 1, 0);
  std::vector<int64_t> part_base(a.n_groups + 1, 0);
  for (int64_t f = 0; f < a.n_groups; ++f) {
    const int64_t nb = (a.grp_U_ptr[f + 1] - a.grp_U_ptr[f] + kET - 1) / kET;
    const int64_t p = a.grp_col_ptr[f + 1] - a.grp_col_ptr[f];
    a.grp_task_ptr[f + 1] = a.grp_task_ptr[f] + nb * (nb + 1) / 2;
    part_base[f + 1] = part_base[f] + nb * (nb + 1) / 2 * p;
  }
  const int64_t nt_all = a.grp_task_ptr[a.n_groups];
  a.tasks.resize(3 * nt_all);
  a.task_part_off.resize(nt_all + 1);
  a.task_part_off[nt_all] = part_base[a.n_groups];
  const std::vector<int64_t> fb = balanced_ranges(a.grp_task_ptr.data(), a.n_groups, NT);
  parallel(NT, [&](unsigned th) {
    for (int64_t f = fb[th]; f < fb[th + 1]; ++f) {
      const int64_t nb = (a.grp_U_ptr[f + 1] - a.grp_U_ptr[f] + kET - 1) / kET;
      const int64_t p = a.grp_col_ptr[f + 1] - a.grp_col_ptr[f];
      int64_t t = a.grp_task_ptr[f];
      for (int64_t I = 0; I < nb; ++I)
        for (int64_t J = 0; J <= I; ++J, ++t) {
          a.tasks[3 * t] = (int32_t)f;
          a.tasks[3 * t + 1] = (int32_t)I;
          a.tasks[3 * t + 2] = (int32_t)J;
          a.task_part_off[t] = part_base[f] + (t - a.grp_task_ptr[f]) * p;
        }
    }
  });
  // launch order: by 512 x 512 block of the root front at the task's first
  // row / column (a block's Z entries fit an XCD's L2), then by task index.
  // Large workload's leaf selected inversion: 309 ms with 2048-blocks, 292
  // with 512, 294 with 256, 297 with 1024.  A stable counting sort over
  // contiguous ranges of tasks (each range fills its own stretch of every
  // key's list, so the order does not depend on the number of threads).
  {
    constexpr int kOrderBlock = 512;
    const int64_t nt = nt_all;
    const int64_t nb = std::max<int64_t>(1, (a.n_pad + kOrderBlock - 1) / kOrderBlock);
    const int64_t nk = nb * nb;
    bigvec<int32_t> key(nt);
    std::vector<int64_t> tb(NT + 1);
    for (unsigned th = 0; th <= NT; ++th) tb[th] = nt * (int64_t)th / (int64_t)NT;
    std::vector<std::vector<int64_t>> kc(NT, std::vector<int64_t>(nk, 0));
    parallel(NT, [&](unsigned th) {
      int64_t* c = kc[th].data();
      for (int64_t t = tb[th]; t < tb[th + 1]; ++t) {
        const int64_t f = a.tasks[3 * t], I = a.tasks[3 * t + 1], J = a.tasks[3 * t + 2];
        const int32_t* Uf = a.U.data() + a.grp_U_ptr[f];
        const int64_t bi = Uf[I * kET] / kOrderBlock, bj = Uf[J * kET] / kOrderBlock;
        key[t] = (int32_t)(bj * nb + bi);
        c[key[t]]++;
      }
    });
    int64_t sum = 0;
    for (int64_t k = 0; k < nk; ++k)
      for (unsigned th = 0; th < NT; ++th) {
        const int64_t c = kc[th][k];
        kc[th][k] = sum;
        sum += c;
      }
    a.sel_order.resize(nt);
    parallel(NT, [&](unsigned th) {
      int64_t* fill = kc[th].data();
      for (int64_t t = tb[th]; t < tb[th + 1]; ++t) a.sel_order[fill[key[t]]++] = (int32_t)t;
    });
  }

  phase("selected-inversion tasks");
  // ---- root incidences of the leaf panels (forward solve)
  // (a counting sort over contiguous ranges of fronts, each range filling
  // its own stretch of every root index's list: in increasing front order
  // whatever the number of threads)
  a.rinc_ptr.assign(a.n_root + 1, 0);
  {
    const std::vector<int64_t> gb = balanced_ranges(a.grp_U_ptr.data(), a.n_groups, NT);
    std::vector<std::vector<int64_t>> rc(NT, std::vector<int64_t>(a.n_root, 0));
    parallel(NT, [&](unsigned t) {
      int64_t* c = rc[t].data();
      for (int64_t u = a.grp_U_ptr[gb[t]]; u < a.grp_U_ptr[gb[t + 1]]; ++u) c[a.U[u]]++;
    });
    for (int64_t i = 0; i < a.n_root; ++i) {
      int64_t sum = a.rinc_ptr[i];
      for (unsigned t = 0; t < NT; ++t) {
        const int64_t c = rc[t][i];
        rc[t][i] = sum;
        sum += c;
      }
      a.rinc_ptr[i + 1] = sum;
    }
    a.rinc_grp.resize(a.rinc_ptr[a.n_root]);
    a.rinc_u.resize(a.rinc_ptr[a.n_root]);
    parallel(NT, [&](unsigned t) {
      int64_t* fill = rc[t].data();
      for (int64_t g = gb[t]; g < gb[t + 1]; ++g)
        for (int64_t u = a.grp_U_ptr[g]; u < a.grp_U_ptr[g + 1]; ++u) {
          const int64_t k = fill[a.U[u]]++;
          a.rinc_grp[k] = (int32_t)g;
          a.rinc_u[k] = (int32_t)(u - a.grp_U_ptr[g]);
        }
    });
  }

  phase("root incidences");
  // ---- counters: nnz(A) (both triangles), nnz(L) as stored, flops.
  // The exact structural count of A costs sum over rows of len^2 scattered
  // visits; above kNnzACountCap of them it is not taken (nnz_a = -1).
  constexpr double kNnzACountCap = 2e10;
  double visits = 0.0;
  for (int64_t r = 0; r < m; ++r) {
    const double len = (double)(rowptr[r + 1] - rowptr[r]);
    visits += len * len;
  }
  a.nnz_a = -1;
  if (visits <= kNnzACountCap) {
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<int64_t> c(nth, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        std::vector<int64_t> st(n, -1);
        int64_t s = 0;
        for (int64_t j = t; j < n; j += nth)
          for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k) {
            int32_t r = a.csc_row[k];
            for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
              if (st[col[e]] != j) {
                st[col[e]] = j;
                ++s;
              }
          }
        c[t] = s;
      });
    for (auto& x : th) x.join();
    a.nnz_a = std::accumulate(c.begin(), c.end(), (int64_t)0);
  }
  // Algorithmic flops: per front p^3/3 + c p^2 + c^2 p for the factor and
  // twice that for the selected inversion, with the exact structure of L:
  // every leaf is a front of its own (leaves share no row, so the pivot
  // block of an amalgamated front is diagonal) and c is the number of root
  // unknowns in its rows; the root is a dense front of its unpadded order.
  double nR = (double)a.n_root;
  a.nnz_l = n_leaf + a.grp_panel_off[a.n_groups] + a.n_root * (a.n_root + 1) / 2;
  a.flops_factor = nR * nR * nR / 3.0 + leaf_work;
  a.flops_selinv = 2.0 * (nR * nR * nR / 3.0 + leaf_work);
  // Executed flops, zeros of the dense panels included: the root
  // assembly's matrix-core products per incidence, and the leaf selected
  // inversion's per task.
  // Root front assembly, algorithmic: the lower triangles of the row
  // products w_r h_rR h_rR^T and of the leaf updates l_U l_U^T, each a
  // multiply-add per entry on the exact structure.
  a.flops_root_asm = leaf_update;
  for (int64_t r = 0; r < m; ++r) {
    const double len = (double)root_cnt[r];
    a.flops_root_asm += len * (len + 1.0);
  }
  a.flops_exec_asm = 0.0;
  for (int64_t q = 0; q < (int64_t)a.inc.size() / 4; ++q) {
    const int32_t* p = a.inc.data() + 4 * q;
    const double nI = p[3] & 0xffff, nJ = p[3] >> 16;
    a.flops_exec_asm += 2.0 * nI * nJ * (double)a.up_k[p[0]];
  }
  a.flops_exec_selinv = 0.0;
  for (int64_t t = 0; t < (int64_t)a.tasks.size() / 3; ++t) {
    const int64_t f = a.tasks[3 * t], I = a.tasks[3 * t + 1], J = a.tasks[3 * t + 2];
    const int64_t nU = a.grp_U_ptr[f + 1] - a.grp_U_ptr[f];
    const double na = (double)std::min<int64_t>(kET, nU - I * kET);
    const double nb = (double)std::min<int64_t>(kET, nU - J * kET);
    a.flops_exec_selinv +=
        2.0 * na * nb * (double)(a.grp_col_ptr[f + 1] - a.grp_col_ptr[f]);
  }
  a.flops_solve = 4.0 * (double)a.nnz_l;
  a.flops_asm = 0;
  for (int64_t r = 0; r < m; ++r) {
    double len = (double)(rowptr[r + 1] - rowptr[r]);
    a.flops_asm += 2.0 * len * len;
  }
  phase("counters");
  return std::string();
}

}  // namespace spi

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
// goes into one dense root front, in its original order.  The result is a
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
#include <thread>

#include "spi_internal.h"

namespace spi {

namespace {
constexpr int kTile = 64;  // root assembly tile

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Runs of a sorted index list by tile: (tile, first position, end position).
void tile_runs(const int32_t* U, int64_t nU,
               std::vector<std::array<int32_t, 3>>& runs) {
  runs.clear();
  int64_t a = 0;
  while (a < nU) {
    const int32_t t = U[a] / kTile;
    int64_t b = a + 1;
    while (b < nU && U[b] / kTile == t) ++b;
    runs.push_back({t, (int32_t)a, (int32_t)b});
    a = b;
  }
}
}  // namespace

std::string analyze(int64_t m, int64_t n, const int64_t* rowptr,
                    const int32_t* col, const spi_opts& o, Analysis& a) {
  std::ostringstream err;
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
  for (int64_t r = 0; r < m; ++r) {
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      int32_t c = col[e];
      if (c < 0 || c >= n) {
        err << "column index " << c << " out of range in row " << r;
        return err.str();
      }
      if (e > rowptr[r] && col[e - 1] >= c) {
        err << "columns not strictly increasing in row " << r;
        return err.str();
      }
    }
  }
  a = Analysis();
  a.m = m;
  a.n = n;
  a.nnz = nnz;
  a.rowptr.assign(rowptr, rowptr + m + 1);
  a.col.assign(col, col + nnz);

  // ---- transpose of the pattern
  a.colptr.assign(n + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) a.colptr[col[e] + 1]++;
  for (int64_t j = 0; j < n; ++j) {
    if (a.colptr[j + 1] == 0) {
      err << "unknown " << j << " appears in no row (A would be singular)";
      return err.str();
    }
    a.colptr[j + 1] += a.colptr[j];
  }
  a.csc_pos.resize(nnz);
  a.csc_row.resize(nnz);
  {
    std::vector<int64_t> fill(a.colptr.begin(), a.colptr.end() - 1);
    for (int64_t r = 0; r < m; ++r)
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int64_t k = fill[col[e]]++;
        a.csc_pos[k] = e;
        a.csc_row[k] = (int32_t)r;
      }
  }

  // ---- leaf selection: greedy independent set by increasing work
  std::vector<int64_t> work(n, 0);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k) {
      int32_t r = a.csc_row[k];
      work[j] += rowptr[r + 1] - rowptr[r];
    }
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

  // ---- root numbering (original order)
  a.root_of_col.assign(n, -1);
  for (int64_t j = 0; j < n; ++j)
    if (!is_leaf[j]) {
      a.root_of_col[j] = (int32_t)a.root_cols.size();
      a.root_cols.push_back((int32_t)j);
    }
  a.n_root = (int64_t)a.root_cols.size();
  a.n_pad = a.n_root ? round_up(a.n_root, kRootPad) : 0;

  // ---- amalgamate consecutive leaves into fronts
  std::vector<int32_t> leaves;
  for (int64_t j = 0; j < n; ++j)
    if (is_leaf[j]) leaves.push_back((int32_t)j);
  const int64_t nr = std::max<int64_t>(a.n_root, 1);
  std::vector<int64_t> mark(nr, -1), seen(nr, -1), posmap(nr, -1);
  a.grp_col_ptr.push_back(0);
  a.grp_U_ptr.push_back(0);
  a.grp_panel_off.push_back(0);
  int64_t front = 0;
  std::vector<int32_t> curU, curCols;
  int64_t cur_sum = 0;
  auto close_front = [&]() {
    std::sort(curU.begin(), curU.end());
    for (int32_t j : curCols) {
      a.leaf_cols.push_back(j);
      a.leaf_grp.push_back((int32_t)front);
    }
    a.U.insert(a.U.end(), curU.begin(), curU.end());
    a.grp_col_ptr.push_back((int64_t)a.leaf_cols.size());
    a.grp_U_ptr.push_back((int64_t)a.U.size());
    a.grp_panel_off.push_back(a.grp_panel_off.back() +
                              (int64_t)curU.size() * (int64_t)curCols.size());
    ++front;
    curU.clear();
    curCols.clear();
    cur_sum = 0;
  };
  std::vector<int32_t> rj;
  for (int32_t j : leaves) {
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
  }
  if (!curCols.empty()) close_front();
  a.n_groups = front;

  // ---- slots (rows of the leaf fronts, by leaf unknown) and their compact
  // root entries with U-local positions
  const int64_t n_leaf = (int64_t)a.leaf_cols.size();
  a.leaf_slot_ptr.assign(n_leaf + 1, 0);
  a.grp_slot_ptr.push_back(0);
  a.slot_rr_ptr.push_back(0);
  std::fill(posmap.begin(), posmap.end(), -1);
  for (int64_t g = 0; g < a.n_groups; ++g) {
    for (int64_t u = a.grp_U_ptr[g]; u < a.grp_U_ptr[g + 1]; ++u)
      posmap[a.U[u]] = u - a.grp_U_ptr[g];
    for (int64_t l = a.grp_col_ptr[g]; l < a.grp_col_ptr[g + 1]; ++l) {
      int32_t j = a.leaf_cols[l];
      for (int64_t k = a.colptr[j]; k < a.colptr[j + 1]; ++k) {
        const int32_t r = a.csc_row[k];
        a.slot_row.push_back(r);
        a.slot_leaf_src.push_back(a.csc_pos[k]);
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          int32_t ri = a.root_of_col[col[e]];
          if (ri < 0) continue;
          a.rr_lpos.push_back((int32_t)posmap[ri]);
          a.rr_src.push_back(e);
        }
        a.slot_rr_ptr.push_back((int64_t)a.rr_src.size());
      }
      a.leaf_slot_ptr[l + 1] = (int64_t)a.slot_row.size();
    }
    a.grp_slot_ptr.push_back((int64_t)a.slot_row.size());
  }
  a.n_slots = (int64_t)a.slot_row.size();

  // ---- row panels: consecutive rows (original order) with overlapping
  // root structure; rows without root entries contribute nothing to A_RR
  a.rp_U_base = (int64_t)a.U.size();
  a.rp_row_ptr.push_back(0);
  a.rp_U_ptr.push_back(0);
  a.rp_val_off.push_back(0);
  a.rpe_ptr.push_back(0);
  std::fill(mark.begin(), mark.end(), -1);
  {
    int64_t panel = 0, rows_in = 0, sum = 0;
    std::vector<int32_t> pU, pRows;
    auto close_panel = [&]() {
      std::sort(pU.begin(), pU.end());
      for (size_t x = 0; x < pU.size(); ++x) posmap[pU[x]] = (int64_t)x;
      const int64_t nU = (int64_t)pU.size();
      for (size_t q = 0; q < pRows.size(); ++q) {
        const int32_t r = pRows[q];
        a.rp_rows.push_back(r);
        a.rp_rowbase.push_back(a.rp_val_off.back() + (int64_t)q * nU);
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          int32_t ri = a.root_of_col[col[e]];
          if (ri < 0) continue;
          a.rpe_pos.push_back((int32_t)posmap[ri]);
          a.rpe_src.push_back(e);
        }
        a.rpe_ptr.push_back((int64_t)a.rpe_src.size());
      }
      a.U.insert(a.U.end(), pU.begin(), pU.end());
      a.rp_row_ptr.push_back((int64_t)a.rp_rows.size());
      a.rp_U_ptr.push_back((int64_t)a.U.size() - a.rp_U_base);
      a.rp_val_off.push_back(a.rp_val_off.back() + nU * (int64_t)pRows.size());
      ++panel;
      pU.clear();
      pRows.clear();
      rows_in = 0;
      sum = 0;
    };
    for (int64_t r = 0; r < m; ++r) {
      int64_t len = 0, add = 0;
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int32_t ri = a.root_of_col[col[e]];
        if (ri < 0) continue;
        ++len;
        if (mark[ri] != panel) ++add;
      }
      if (len == 0) continue;
      if (rows_in > 0) {
        const int64_t newU = (int64_t)pU.size() + add;
        const double dens = (double)(sum + len) / ((double)newU * (double)(rows_in + 1));
        if (rows_in + 1 > o.max_group || dens < o.amalg_density) close_panel();
      }
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int32_t ri = a.root_of_col[col[e]];
        if (ri >= 0 && mark[ri] != panel) {
          mark[ri] = panel;
          pU.push_back(ri);
        }
      }
      pRows.push_back((int32_t)r);
      ++rows_in;
      sum += len;
    }
    if (rows_in > 0) close_panel();
    a.n_rp = panel;
  }

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

  // ---- incidences on the 64 x 64 lower tiles of the root
  if (a.n_pad) {
    const int64_t T = a.n_pad / kTile;
    a.n_tiles = T * (T + 1) / 2;
    std::vector<int64_t> cnt(a.n_tiles + 1, 0);
    std::vector<std::array<int32_t, 3>> runs;
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int64_t> fillp;
      if (pass == 1) {
        a.inc_ptr.assign(a.n_tiles + 1, 0);
        for (int64_t t = 0; t < a.n_tiles; ++t) a.inc_ptr[t + 1] = a.inc_ptr[t] + cnt[t];
        a.inc.resize(4 * a.inc_ptr[a.n_tiles]);
        fillp.assign(a.inc_ptr.begin(), a.inc_ptr.end() - 1);
      }
      for (int64_t u = 0; u < a.n_up; ++u) {
        if (a.up_k[u] == 0) continue;
        tile_runs(a.U.data() + a.up_U_off[u], a.up_nU[u], runs);
        for (size_t x = 0; x < runs.size(); ++x)
          for (size_t y = 0; y <= x; ++y) {
            const int64_t I = runs[x][0], J = runs[y][0];
            const int64_t t = I * (I + 1) / 2 + J;
            if (pass == 0) {
              cnt[t]++;
            } else {
              int32_t* p = a.inc.data() + 4 * fillp[t]++;
              p[0] = (int32_t)u;
              p[1] = runs[x][1];
              p[2] = runs[y][1];
              p[3] = (runs[x][2] - runs[x][1]) | ((runs[y][2] - runs[y][1]) << 16);
            }
          }
      }
    }
    // tiles with the most work first
    std::vector<double> tw(a.n_tiles, 0.0);
    for (int64_t t = 0; t < a.n_tiles; ++t)
      for (int64_t q = a.inc_ptr[t]; q < a.inc_ptr[t + 1]; ++q) {
        const int32_t* p = a.inc.data() + 4 * q;
        const int nI = p[3] & 0xffff, nJ = p[3] >> 16;
        tw[t] += (double)((nI + 15) / 16) * ((nJ + 15) / 16) * (a.up_k[p[0]] + 3) / 4 + 1.0;
      }
    a.tile_order.resize(a.n_tiles);
    std::iota(a.tile_order.begin(), a.tile_order.end(), 0);
    std::stable_sort(a.tile_order.begin(), a.tile_order.end(),
                     [&](int32_t x, int32_t y) { return tw[x] > tw[y]; });
  }

  // ---- selected-inversion tasks of the leaf fronts
  a.grp_task_ptr.push_back(0);
  a.task_part_off.push_back(0);
  for (int64_t f = 0; f < a.n_groups; ++f) {
    int64_t nU = a.grp_U_ptr[f + 1] - a.grp_U_ptr[f];
    int64_t p = a.grp_col_ptr[f + 1] - a.grp_col_ptr[f];
    int64_t nt = (nU + kET - 1) / kET;
    for (int64_t I = 0; I < nt; ++I)
      for (int64_t J = 0; J <= I; ++J) {
        a.tasks.push_back((int32_t)f);
        a.tasks.push_back((int32_t)I);
        a.tasks.push_back((int32_t)J);
        a.task_part_off.push_back(a.task_part_off.back() + p);
      }
    a.grp_task_ptr.push_back((int64_t)a.tasks.size() / 3);
  }
  // launch order: by 2-D block of the root front at the task's first row /
  // column, then by task index
  {
    constexpr int kOrderBlock = 2048;
    const int64_t nt = (int64_t)a.tasks.size() / 3;
    std::vector<int64_t> key(nt);
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t f = a.tasks[3 * t], I = a.tasks[3 * t + 1],
                    J = a.tasks[3 * t + 2];
      const int32_t* Uf = a.U.data() + a.grp_U_ptr[f];
      const int64_t bi = Uf[I * kET] / kOrderBlock, bj = Uf[J * kET] / kOrderBlock;
      key[t] = (bj << 20) | bi;
    }
    a.sel_order.resize(nt);
    std::iota(a.sel_order.begin(), a.sel_order.end(), 0);
    std::stable_sort(a.sel_order.begin(), a.sel_order.end(),
                     [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  }

  // ---- root incidences of the leaf panels (forward solve)
  a.rinc_ptr.assign(a.n_root + 1, 0);
  for (int64_t g = 0; g < a.n_groups; ++g)
    for (int64_t u = a.grp_U_ptr[g]; u < a.grp_U_ptr[g + 1]; ++u)
      a.rinc_ptr[a.U[u] + 1]++;
  for (int64_t i = 0; i < a.n_root; ++i) a.rinc_ptr[i + 1] += a.rinc_ptr[i];
  a.rinc_grp.resize(a.rinc_ptr[a.n_root]);
  a.rinc_u.resize(a.rinc_ptr[a.n_root]);
  {
    std::vector<int64_t> fill(a.rinc_ptr.begin(), a.rinc_ptr.end() - 1);
    for (int64_t g = 0; g < a.n_groups; ++g)
      for (int64_t u = a.grp_U_ptr[g]; u < a.grp_U_ptr[g + 1]; ++u) {
        int64_t k = fill[a.U[u]]++;
        a.rinc_grp[k] = (int32_t)g;
        a.rinc_u[k] = (int32_t)(u - a.grp_U_ptr[g]);
      }
  }

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
  double nR = (double)a.n_root;
  a.nnz_l = n_leaf + a.grp_panel_off[a.n_groups] + a.n_root * (a.n_root + 1) / 2;
  a.flops_factor = nR * nR * nR / 3.0;
  a.flops_selinv = 2.0 * nR * nR * nR / 3.0;
  for (int64_t g = 0; g < a.n_groups; ++g) {
    double p = (double)(a.grp_col_ptr[g + 1] - a.grp_col_ptr[g]);
    double c = (double)(a.grp_U_ptr[g + 1] - a.grp_U_ptr[g]);
    a.flops_factor += p * p * p / 3.0 + c * p * p + c * c * p;
    a.flops_selinv += 2.0 * (p * p * p / 3.0 + c * p * p + c * c * p);
  }
  a.flops_solve = 4.0 * (double)a.nnz_l;
  a.flops_asm = 0;
  for (int64_t r = 0; r < m; ++r) {
    double len = (double)(rowptr[r + 1] - rowptr[r]);
    a.flops_asm += 2.0 * len * len;
  }
  return std::string();
}

}  // namespace spi

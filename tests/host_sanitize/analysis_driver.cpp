// Host analysis under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Test support (built and run by tests/test_host_sanitizers.py with g++;
// no GPU code): runs spi::analyze on generated patterns (coded-mask shaped
// systems, random sparse systems, a dense root, empty rows, one unknown)
// with 1, 3 and 7 analysis threads, checks the invariants of the result,
// and feeds it invalid patterns that must be refused with an error text.
// Any out-of-bounds access, use after free, leak or undefined operation in
// the analysis stops the run with the sanitizer's report.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1305_5683_amd/csrc/spi_internal.h"

namespace {

struct Csr {
  int64_t m = 0, n = 0;
  std::vector<int64_t> rowptr{0};
  std::vector<int32_t> col;
  void add_row(const std::vector<int32_t>& c) {
    col.insert(col.end(), c.begin(), c.end());
    rowptr.push_back((int64_t)col.size());
    ++m;
  }
};

spi_opts default_opts() {
  spi_opts o;
  std::memset(&o, 0, sizeof(o));
  o.precision = SPI_FP64;
  o.max_group = 32;
  o.leaf_max_work = 65536.0;
  o.amalg_density = 0.35;
  o.refine_steps = 1;
  o.root_inverse = 1;
  o.equilibrate = 1;
  return o;
}

// A coded-mask shaped system: S x S sky, P pointings with random centres,
// F x F field of view, nd detectors each seeing about half the field, one
// background unknown per detector per time bin of 1..L pointings.
Csr coded_mask(int S, int P, int F, int nd, int L, unsigned seed) {
  std::mt19937 g(seed);
  std::vector<int> bin_of(P);
  int nb = 0;
  for (int p = 0; p < P;) {
    const int len = 1 + (int)(g() % L);
    for (int q = 0; q < len && p < P; ++q) bin_of[p++] = nb;
    ++nb;
  }
  Csr h;
  const int n_bg = nb * nd;
  h.n = n_bg + S * S;
  const int r = F / 2;
  for (int p = 0; p < P; ++p) {
    const int cx = (int)(g() % S), cy = (int)(g() % S);
    for (int d = 0; d < nd; ++d) {
      std::vector<int32_t> c{bin_of[p] * nd + d};
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          const int y = cy + dy, x = cx + dx;
          if (y < 0 || y >= S || x < 0 || x >= S || (g() & 1)) continue;
          c.push_back(n_bg + y * S + x);
        }
      h.add_row(c);
    }
  }
  return h;
}

// Random rows of 1..k distinct sorted columns out of n.
Csr random_rows(int64_t m, int64_t n, int k, unsigned seed) {
  std::mt19937 g(seed);
  Csr h;
  h.n = n;
  std::vector<char> seen(n, 0);
  for (int64_t r = 0; r < m; ++r) {
    const int len = 1 + (int)(g() % k);
    std::vector<int32_t> c;
    for (int t = 0; t < len; ++t) {
      const int32_t j = (int32_t)(g() % n);
      if (!seen[j]) {
        seen[j] = 1;
        c.push_back(j);
      }
    }
    for (int32_t j : c) seen[j] = 0;
    std::sort(c.begin(), c.end());
    h.add_row(c);
  }
  return h;
}

int failures = 0;

void expect(bool ok, const char* what, const char* name) {
  if (!ok) {
    std::printf("FAIL %s: %s\n", name, what);
    ++failures;
  }
}

// Invariants of a successful analysis (of the pattern h when with_pattern).
void check(const spi::Analysis& a, const Csr& h, const char* name,
           bool with_pattern = true) {
  const int64_t nl = (int64_t)a.leaf_cols.size();
  const int64_t n = with_pattern ? h.n : a.n;
  expect(nl + a.n_root == n, "leaves + root != n", name);
  std::vector<int> hit(n, 0);
  for (int32_t j : a.leaf_cols) ++hit[j];
  for (int32_t j : a.root_cols) ++hit[j];
  for (int64_t j = 0; j < n; ++j) expect(hit[j] == 1, "column not placed once", name);
  expect(a.n_pad % 128 == 0 && a.n_pad >= a.n_root, "root padding", name);
  expect((int64_t)a.grp_col_ptr.size() == a.n_groups + 1 &&
             a.grp_col_ptr.back() == nl, "front column pointers", name);
  for (int64_t g = 0; g < a.n_groups; ++g) {
    expect(a.grp_col_ptr[g] <= a.grp_col_ptr[g + 1], "front columns decrease", name);
    for (int64_t u = a.grp_U_ptr[g] + 1; u < a.grp_U_ptr[g + 1]; ++u)
      expect(a.U[u - 1] < a.U[u], "front structure not sorted", name);
  }
  for (int64_t u = 0; u < (int64_t)a.U.size(); ++u)
    expect(a.U[u] >= 0 && a.U[u] < a.n_root, "root index out of range", name);
  for (int64_t q = 0; q < (int64_t)a.inc.size() / 4; ++q) {
    const int32_t* p = a.inc.data() + 4 * q;
    expect(p[0] >= 0 && p[0] < a.n_up, "incidence update out of range", name);
    const int nI = p[3] & 0xffff, nJ = p[3] >> 16;
    expect(nI > 0 && nJ > 0 && p[1] + nI <= a.up_nU[p[0]] && p[2] + nJ <= a.up_nU[p[0]],
           "incidence run out of range", name);
  }
  std::vector<int> perm(a.sel_order.size(), 0);
  for (int32_t t : a.sel_order)
    if (t >= 0 && t < (int32_t)perm.size()) ++perm[t];
  for (int v : perm) expect(v == 1, "task order not a permutation", name);
}

// Analysis files: write, read back, write again: the same bytes.
void round_trip(const spi::Analysis& a, const spi_opts& o, const char* name) {
  const char* p1 = "analysis_driver_1.spia";
  const char* p2 = "analysis_driver_2.spia";
  std::string e = spi::save_analysis(a, o, p1);
  expect(e.empty(), e.c_str(), name);
  spi::Analysis b;
  spi_opts q = default_opts();
  e = spi::load_analysis(p1, b, q);
  expect(e.empty(), e.c_str(), name);
  if (!e.empty()) return;
  check(b, Csr(), name, false);
  e = spi::save_analysis(b, q, p2);
  expect(e.empty(), e.c_str(), name);
  std::FILE* f1 = std::fopen(p1, "rb");
  std::FILE* f2 = std::fopen(p2, "rb");
  bool same = f1 && f2;
  while (same) {
    const int c1 = std::fgetc(f1), c2 = std::fgetc(f2);
    same = c1 == c2;
    if (c1 == EOF || c2 == EOF) break;
  }
  if (f1) std::fclose(f1);
  if (f2) std::fclose(f2);
  expect(same, "analysis file differs after a round trip", name);
  std::remove(p1);
  std::remove(p2);
}

// Damaged analysis files: every byte of the header and of the first field
// descriptors changed in turn, then random single-byte changes and
// truncations over the whole file.  Each must be refused; under the
// sanitizers the reader must also touch no memory it does not own while it
// finds out.
void damaged_files(const spi::Analysis& a, const spi_opts& o, const char* name) {
  const char* p = "analysis_driver_d.spia";
  std::string e = spi::save_analysis(a, o, p);
  expect(e.empty(), e.c_str(), name);
  std::string buf;
  {
    std::FILE* f = std::fopen(p, "rb");
    int c;
    while (f && (c = std::fgetc(f)) != EOF) buf.push_back((char)c);
    if (f) std::fclose(f);
  }
  expect(buf.size() > 64, "analysis file too short", name);
  std::mt19937_64 rng(12345);
  int refused = 0, tried = 0;
  auto attempt = [&](const std::string& b) {
    std::FILE* f = std::fopen(p, "wb");
    if (!f) return;
    std::fwrite(b.data(), 1, b.size(), f);
    std::fclose(f);
    spi::Analysis c;
    spi_opts q = default_opts();
    const std::string err = spi::load_analysis(p, c, q);
    ++tried;
    refused += !err.empty();
  };
  for (size_t i = 0; i < std::min<size_t>(buf.size(), 320); ++i) {
    std::string b = buf;
    b[i] = (char)(b[i] ^ 0x5a);
    attempt(b);
  }
  for (int k = 0; k < 200; ++k) {
    std::string b = buf;
    if (k % 4 == 3) {
      b.resize(rng() % b.size());
    } else {
      const size_t i = rng() % b.size();
      b[i] = (char)(b[i] ^ (char)(1 + rng() % 255));
    }
    attempt(b);
  }
  expect(refused == tried, "a damaged analysis file was accepted", name);
  std::remove(p);
  std::printf("refused %d of %d damaged files (%s)\n", refused, tried, name);
}

void run_valid(const Csr& h, const spi_opts& o, const char* name, bool damage = false) {
  std::string first;
  for (const char* nt : {"1", "3", "7"}) {
    setenv("SPI_ANALYSIS_THREADS", nt, 1);
    spi::Analysis a;
    const std::string e = spi::analyze(h.m, h.n, h.rowptr.data(), h.col.data(), o, a);
    expect(e.empty(), e.c_str(), name);
    if (!e.empty()) return;
    check(a, h, name);
    if (nt[0] == '3') round_trip(a, o, name);
    if (nt[0] == '3' && damage) damaged_files(a, o, name);
    std::string sig = std::to_string(a.n_groups) + "/" + std::to_string(a.n_root) + "/" +
                      std::to_string(a.inc.size()) + "/" + std::to_string(a.tasks.size());
    if (first.empty()) first = sig;
    expect(sig == first, "result depends on the thread count", name);
  }
  std::printf("ok %s (m=%lld n=%lld)\n", name, (long long)h.m, (long long)h.n);
}

void run_invalid(const Csr& h, const char* name) {
  spi::Analysis a;
  const std::string e =
      spi::analyze(h.m, h.n, h.rowptr.data(), h.col.data(), default_opts(), a);
  expect(!e.empty(), "invalid pattern accepted", name);
  std::printf("refused %s: %s\n", name, e.c_str());
}

}  // namespace

// argv[1] == "threads": the multithreaded analyses only (the damaged-file
// reads are single-threaded and slow under ThreadSanitizer)
int main(int argc, char** argv) {
  const bool threads_only = argc > 1 && std::strcmp(argv[1], "threads") == 0;
  const spi_opts o = default_opts();
  run_valid(coded_mask(24, 300, 9, 19, 10, 1), o, "coded-mask 24x24", !threads_only);
  run_valid(coded_mask(40, 700, 15, 19, 6, 2), o, "coded-mask 40x40");
  spi_opts o64 = o;
  o64.asm_tile = 128;
  run_valid(coded_mask(30, 500, 11, 7, 4, 3), o64, "coded-mask, 128 tiles");
  spi_opts o1 = o;
  o1.max_group = 1;
  run_valid(coded_mask(20, 200, 7, 5, 3, 4), o1, "one pivot per front");
  spi_opts ok = o;
  ok.keep_root_order = 1;
  run_valid(coded_mask(20, 200, 7, 5, 3, 5), ok, "original root order");
  run_valid(random_rows(3000, 900, 12, 6), o, "random rows");
  spi_opts od = o;
  od.leaf_max_work = 0.0;
  run_valid(random_rows(600, 200, 10, 7), od, "dense root");
  {
    Csr h = random_rows(400, 150, 8, 8);
    Csr e;
    e.n = h.n;
    for (int64_t r = 0; r < h.m; ++r) {
      if (r % 5 == 0) e.add_row({});
      e.add_row(std::vector<int32_t>(h.col.begin() + h.rowptr[r],
                                     h.col.begin() + h.rowptr[r + 1]));
    }
    run_valid(e, o, "empty rows");
  }
  {
    Csr h;
    h.n = 1;
    h.add_row({0});
    h.add_row({0});
    run_valid(h, o, "one unknown");
  }
  {
    Csr h = random_rows(50, 30, 5, 9);
    h.col[3] = 30;
    run_invalid(h, "column out of range");
  }
  {
    Csr h = random_rows(50, 30, 5, 10);
    h.col[h.rowptr[7]] = -1;
    run_invalid(h, "negative column");
  }
  {
    Csr h;
    h.n = 10;
    h.add_row({1, 4, 3});
    run_invalid(h, "unsorted row");
  }
  {
    Csr h;
    h.n = 10;
    h.add_row({2, 2, 5});
    run_invalid(h, "duplicate column");
  }
  {
    Csr h = random_rows(20, 10, 3, 11);
    h.rowptr[5] = h.rowptr[6] + 1;
    run_invalid(h, "decreasing rowptr");
  }
  if (failures) {
    std::printf("FAILED %d checks\n", failures);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}

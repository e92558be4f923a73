// Checkpoint of the host analysis (Sect. 3.2.1: the ordering and symbolic
// factorisation are done once per pattern; bands of one pattern, and later
// runs, reuse them).  A binary file of this library's own format:
//
//   magic "SPIANL01", format version, sizeof(Analysis) on the writing side
//   the analysis options that shaped it (max_group, leaf_max_work,
//     amalg_density, keep_root_order, asm_tile)
//   every scalar and vector of the Analysis, each as (tag, element size,
//     element count, bytes)
//   a 64-bit FNV-1a hash (over words) of everything before it
//
// Reading checks the magic, the version, every tag, element size and the
// counts the structure implies (vector lengths against m, n, the number of
// fronts, tiles, tasks ...), and the hash, so a truncated, corrupted or
// foreign file is refused instead of reaching the device.
#include <cstdio>
#include <cstring>
#include <fstream>

#include "spi_internal.h"

namespace spi {

namespace {

constexpr char kMagic[8] = {'S', 'P', 'I', 'A', 'N', 'L', '0', '1'};
constexpr uint32_t kVersion = 1;
// the field list below covers every member: a new member changes the size
// and must be added to it (and the version raised)
static_assert(sizeof(Analysis) == 1248, "Analysis changed: update its file format");

// FNV-1a over 64-bit words (the bytes of a final partial word one by one):
// a checksum against truncation and corruption, not a cryptographic hash.
struct Hash {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
      uint64_t w;
      std::memcpy(&w, c + i, 8);
      h ^= w;
      h *= 1099511628211ull;
    }
    for (; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  }
};

// Every member of an Analysis, in a fixed order, with a 4-character tag.
template <class A, class F>
void visit(A& a, F&& f) {
  f("m   ", a.m); f("n   ", a.n); f("nnz ", a.nnz);
  f("rptr", a.rowptr); f("col ", a.col);
  f("cptr", a.colptr); f("cpos", a.csc_pos); f("crow", a.csc_row);
  f("lcol", a.leaf_cols); f("lgrp", a.leaf_grp); f("lslp", a.leaf_slot_ptr);
  f("ngrp", a.n_groups);
  f("gcol", a.grp_col_ptr); f("gU  ", a.grp_U_ptr); f("U   ", a.U);
  f("gpan", a.grp_panel_off); f("gslp", a.grp_slot_ptr);
  f("nslt", a.n_slots);
  f("srow", a.slot_row); f("srrp", a.slot_rr_ptr); f("slsr", a.slot_leaf_src);
  f("rrlp", a.rr_lpos); f("rrsr", a.rr_src);
  f("nrp ", a.n_rp); f("rpUb", a.rp_U_base);
  f("rprp", a.rp_row_ptr); f("rprw", a.rp_rows); f("rpUp", a.rp_U_ptr);
  f("rpvo", a.rp_val_off); f("rprb", a.rp_rowbase);
  f("rpep", a.rpe_ptr); f("rpeq", a.rpe_pos); f("rpes", a.rpe_src);
  f("nup ", a.n_up);
  f("upUo", a.up_U_off); f("upQo", a.up_Q_off); f("upnU", a.up_nU);
  f("upk ", a.up_k); f("upwo", a.up_w_off);
  f("asmt", a.asm_tile); f("ntil", a.n_tiles);
  f("tord", a.tile_order); f("iptr", a.inc_ptr); f("ispl", a.inc_split);
  f("inc ", a.inc);
  f("nrt ", a.n_root); f("npad", a.n_pad);
  f("rcol", a.root_cols); f("rofc", a.root_of_col); f("lofc", a.leaf_of_col);
  f("rinp", a.rinc_ptr); f("ring", a.rinc_grp); f("rinu", a.rinc_u);
  f("task", a.tasks); f("gtsk", a.grp_task_ptr); f("tpof", a.task_part_off);
  f("sord", a.sel_order);
  f("nnzA", a.nnz_a); f("nnzL", a.nnz_l);
  f("flfa", a.flops_factor); f("flsi", a.flops_selinv); f("flso", a.flops_solve);
  f("flas", a.flops_asm); f("flea", a.flops_exec_asm); f("fles", a.flops_exec_selinv);
  f("flra", a.flops_root_asm);
}

// Streams to the file (no copy of the whole analysis in memory).
struct Writer {
  std::ofstream& out;
  Hash hash;
  explicit Writer(std::ofstream& o) : out(o) {}
  void raw(const void* p, size_t n) {
    out.write(static_cast<const char*>(p), (std::streamsize)n);
    hash.add(p, n);
  }
  void item(const char* tag, uint32_t esize, uint64_t count, const void* p) {
    raw(tag, 4);
    raw(&esize, sizeof(esize));
    raw(&count, sizeof(count));
    if (count) raw(p, esize * count);
  }
  template <class T>
  void operator()(const char* tag, const T& v) { item(tag, sizeof(T), 1, &v); }
  template <class T, class Al>
  void operator()(const char* tag, const std::vector<T, Al>& v) {
    item(tag, sizeof(T), v.size(), v.data());
  }
};

// Streams from the file; `left` (the bytes not yet read) bounds every
// length before anything is allocated for it.
struct Reader {
  std::ifstream& in;
  uint64_t left;
  Hash hash;
  std::string err;
  Reader(std::ifstream& i, uint64_t size) : in(i), left(size) {}
  bool raw(void* p, size_t n) {
    if (!err.empty()) return false;
    if (n > left) {
      err = "the analysis file is truncated";
      return false;
    }
    in.read(static_cast<char*>(p), (std::streamsize)n);
    if (!in) {
      err = "cannot read the analysis file";
      return false;
    }
    hash.add(p, n);
    left -= n;
    return true;
  }
  bool head(const char* tag, uint32_t esize, uint64_t& count) {
    char t[4];
    uint32_t es = 0;
    if (!raw(t, 4) || !raw(&es, sizeof(es)) || !raw(&count, sizeof(count))) return false;
    if (std::memcmp(t, tag, 4) != 0 || es != esize) {
      err = std::string("the analysis file does not match this format at field '") +
            std::string(tag, 4) + "'";
      return false;
    }
    if (count > left / esize) {
      err = "the analysis file is truncated";
      return false;
    }
    return true;
  }
  template <class T>
  void operator()(const char* tag, T& v) {
    uint64_t c = 0;
    if (!head(tag, sizeof(T), c)) return;
    if (c != 1) {
      err = "the analysis file does not match this format";
      return;
    }
    raw(&v, sizeof(T));
  }
  template <class T, class Al>
  void operator()(const char* tag, std::vector<T, Al>& v) {
    uint64_t c = 0;
    if (!head(tag, sizeof(T), c)) return;
    v.resize(c);
    if (c) raw(v.data(), sizeof(T) * c);
  }
};

// The lengths the structure implies; the device code indexes by them.
std::string check_shape(const Analysis& a) {
  const int64_t nl = (int64_t)a.leaf_cols.size();
  const int64_t nt = (int64_t)a.tasks.size() / 3;
  auto sz = [](const auto& v) { return (int64_t)v.size(); };
  const bool ok =
      a.m >= 1 && a.n >= 1 && sz(a.rowptr) == a.m + 1 && a.rowptr.back() == a.nnz &&
      sz(a.col) == a.nnz && sz(a.colptr) == a.n + 1 && sz(a.csc_pos) == a.nnz &&
      sz(a.csc_row) == a.nnz && sz(a.leaf_grp) == nl && sz(a.leaf_slot_ptr) == nl + 1 &&
      nl + a.n_root == a.n && sz(a.grp_col_ptr) == a.n_groups + 1 &&
      sz(a.grp_U_ptr) == a.n_groups + 1 && sz(a.grp_panel_off) == a.n_groups + 1 &&
      sz(a.grp_slot_ptr) == a.n_groups + 1 && sz(a.grp_task_ptr) == a.n_groups + 1 &&
      sz(a.slot_row) == a.n_slots && sz(a.slot_rr_ptr) == a.n_slots + 1 &&
      sz(a.slot_leaf_src) == a.n_slots && sz(a.rr_lpos) == sz(a.rr_src) &&
      sz(a.rp_row_ptr) == a.n_rp + 1 && sz(a.rp_U_ptr) == a.n_rp + 1 &&
      sz(a.rp_val_off) == a.n_rp + 1 && sz(a.rpe_pos) == sz(a.rpe_src) &&
      a.n_up == a.n_groups + a.n_rp && sz(a.up_U_off) == a.n_up &&
      sz(a.up_Q_off) == a.n_up && sz(a.up_nU) == a.n_up && sz(a.up_k) == a.n_up &&
      sz(a.up_w_off) == a.n_up && sz(a.tile_order) == a.n_tiles &&
      sz(a.inc_split) == a.n_tiles &&
      (a.n_tiles == 0 ? sz(a.inc_ptr) <= 1 && a.inc.empty()
                      : sz(a.inc_ptr) == a.n_tiles + 1 &&
                            sz(a.inc) == 4 * a.inc_ptr.back()) &&
      sz(a.root_cols) == a.n_root && sz(a.root_of_col) == a.n &&
      sz(a.leaf_of_col) == a.n && sz(a.rinc_ptr) == a.n_root + 1 &&
      sz(a.rinc_grp) == sz(a.rinc_u) &&
      sz(a.tasks) == 3 * nt && sz(a.task_part_off) == nt + 1 && sz(a.sel_order) == nt &&
      a.n_pad >= a.n_root && a.n_pad % 128 == 0 &&
      (a.asm_tile == kAsmTileSmall || a.asm_tile == kAsmTileLarge);
  return ok ? std::string() : "the analysis file's arrays do not fit together";
}

}  // namespace

std::string save_analysis(const Analysis& a, const spi_opts& o, const char* path) {
  if (!path) return "null path";
  std::ofstream f(path, std::ios::binary | std::ios::trunc);
  if (!f) return std::string("cannot write the analysis file ") + path;
  Writer w(f);
  w.raw(kMagic, sizeof(kMagic));
  const uint32_t ver = kVersion, asz = (uint32_t)sizeof(Analysis);
  w.raw(&ver, sizeof(ver));
  w.raw(&asz, sizeof(asz));
  w("omgr", o.max_group);
  w("olmw", o.leaf_max_work);
  w("oamd", o.amalg_density);
  w("okro", o.keep_root_order);
  w("oast", o.asm_tile);
  visit(a, w);
  const uint64_t h = w.hash.h;
  f.write(reinterpret_cast<const char*>(&h), sizeof(h));
  f.close();
  if (!f) return std::string("cannot write the analysis file ") + path;
  return std::string();
}

std::string load_analysis(const char* path, Analysis& a, spi_opts& o) {
  if (!path) return "null path";
  std::ifstream f(path, std::ios::binary | std::ios::ate);
  if (!f) return std::string("cannot open the analysis file ") + path;
  const std::streamoff size = f.tellg();
  f.seekg(0);
  if (size < 0 || !f) return std::string("cannot read the analysis file ") + path;
  Reader r(f, (uint64_t)size);
  char magic[8];
  uint32_t ver = 0, asz = 0;
  if (!r.raw(magic, 8) || std::memcmp(magic, kMagic, 8) != 0)
    return "not an analysis file of this library";
  if (!r.raw(&ver, sizeof(ver)) || !r.raw(&asz, sizeof(asz)) || ver != kVersion ||
      asz != (uint32_t)sizeof(Analysis))
    return "the analysis file is of another format version";
  Analysis b;
  spi_opts q = o;
  r("omgr", q.max_group);
  r("olmw", q.leaf_max_work);
  r("oamd", q.amalg_density);
  r("okro", q.keep_root_order);
  r("oast", q.asm_tile);
  visit(b, r);
  if (!r.err.empty()) return r.err;
  uint64_t h = 0;
  const uint64_t want = r.hash.h;
  if (r.left != sizeof(h)) return "the analysis file is truncated or too long";
  f.read(reinterpret_cast<char*>(&h), sizeof(h));
  if (!f) return "the analysis file is truncated";
  if (h != want) return "the analysis file is corrupted (hash mismatch)";
  const std::string e = check_shape(b);
  if (!e.empty()) return e;
  a = std::move(b);
  o = q;
  return std::string();
}

}  // namespace spi

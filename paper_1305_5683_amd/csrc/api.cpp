// C ABI entry points of libspi (declared in include/spi.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <limits>
#include <new>
#include <sstream>
#include <vector>

#include "spi_internal.h"

using namespace spi;

namespace {

thread_local std::string g_analyze_err;

template <class T, class Al>
hipError_t dev_copy(T*& dst, const std::vector<T, Al>& src, hipStream_t s) {
  dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)&dst, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T),
                        hipMemcpyHostToDevice, s);
}

template <class T>
hipError_t dev_alloc(T*& dst, int64_t count) {
  dst = nullptr;
  if (count <= 0) return hipSuccess;
  return hipMalloc((void**)&dst, (size_t)count * sizeof(T));
}


// ---- phase timers: event pairs on the handle's stream
hipEvent_t take_event(PhaseTimer& t) {
  if (!t.free_ev.empty()) {
    hipEvent_t e = t.free_ev.back();
    t.free_ev.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void collect(PhaseTimer& t) {
  for (auto& pr : t.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess &&
        hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      t.total_ms += ms;
      t.count += 1;
    }
    t.free_ev.push_back(pr.first);
    t.free_ev.push_back(pr.second);
  }
  t.pending.clear();
}

}  // namespace

namespace spi {
void phase_begin(Handle& h, Phase p) {
  if (!h.opts.timing) return;
  PhaseTimer& t = h.timer[p];
  if (t.pending.size() > 4096) collect(t);
  t.open = take_event(t);
  if (t.open) (void)hipEventRecord(t.open, h.stream);
}

void phase_end(Handle& h, Phase p) {
  if (!h.opts.timing) return;
  PhaseTimer& t = h.timer[p];
  if (!t.open) return;
  hipEvent_t e = take_event(t);
  if (!e) return;
  (void)hipEventRecord(e, h.stream);
  t.pending.emplace_back(t.open, e);
  t.open = nullptr;
}

}  // namespace spi

namespace {

void free_timers(Handle& h) {
  for (auto& t : h.timer) {
    collect(t);
    for (hipEvent_t e : t.free_ev) (void)hipEventDestroy(e);
    t.free_ev.clear();
  }
}

void free_all(Handle& h) {
  free_timers(h);
  if (h.ev_next) (void)hipEventDestroy(h.ev_next);
  if (h.ev_panel) (void)hipEventDestroy(h.ev_panel);
  if (h.side) (void)hipStreamDestroy(h.side);
  DevAnalysis& d = h.d;
  void* ptrs[] = {d.rowptr, d.col, d.colptr, d.csc_pos, d.csc_row, d.leaf_cols,
                  d.leaf_grp, d.leaf_slot_ptr, d.grp_col_ptr, d.grp_U_ptr, d.U,
                  d.grp_panel_off, d.grp_slot_ptr, d.slot_row, d.slot_rr_ptr,
                  d.slot_leaf_src, d.rr_lpos, d.rr_src, d.root_cols, d.rinc_ptr,
                  d.rinc_grp, d.rinc_u, d.tasks, d.grp_task_ptr, d.task_part_off,
                  d.sel_order, d.rp_rows, d.rp_rowbase, d.rpe_ptr, d.rpe_pos,
                  d.rpe_src, d.up_U_off, d.up_Q_off, d.up_nU, d.up_k,
                  d.up_w_off, d.tile_order, d.inc_ptr, d.inc, d.inc_split,
                  h.val, h.w, h.sw, h.sleaf, h.rrval, h.panel, h.ldiag, h.S,
                  h.invd, h.W, h.Z, h.part, h.flag, h.vleaf, h.vroot, h.vres,
                  h.vx, h.vdd, h.vnorm, h.vroot2, h.vpart, h.invd2,
                  h.colscale, h.vbh, h.vxh, h.diagA, d.root_of_col, d.leaf_of_col,
                  h.vfront,
                  h.band, h.valc, h.Akeep, h.vrow, h.vsum, h.vb2, h.vm1, h.vm2,
                  h.vw, h.vr, h.panelS};
  free_lp_work(h);
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}


bool check_opts(spi_opts& o) {
  if (o.precision != SPI_FP64 && o.precision != SPI_MIXED) {
    g_analyze_err = "unknown precision";
    return false;
  }
  if (o.max_group < 1 || o.refine_steps < 0 || !(o.amalg_density >= 0.0) ||
      !(o.refine_tol >= 0.0) || (o.keep_root_order != 0 && o.keep_root_order != 1) ||
      o.leaf_lds_cap < 0 || o.leaf_lds_cap > kLeafLdsCapMax || o.selinv_chunk < 0 ||
      (o.keep_root_sum != 0 && o.keep_root_sum != 1) ||
      (o.indefinite != 0 && o.indefinite != 1) ||
      (o.asm_tile != 0 && o.asm_tile != kAsmTileSmall && o.asm_tile != kAsmTileLarge)) {
    g_analyze_err = "invalid options";
    return false;
  }
  if (o.device_mem_cap < 0 || (o.fp64_fallback != 0 && o.fp64_fallback != 1)) {
    g_analyze_err = "invalid options";
    return false;
  }
  if (o.indefinite && !o.root_inverse) {
    g_analyze_err = "indefinite = 1 needs root_inverse = 1";
    return false;
  }
  if (o.precision == SPI_MIXED && o.refine_tol == 0.0) {
    // the FP32 root factor needs refinement to reach FP64 accuracy in x
    o.refine_tol = 1e-14;
    o.refine_steps = std::max(o.refine_steps, 10);
  }
  return true;
}

// Upload the analysis and size every buffer of a handle whose h.an is set;
// deletes H on failure.
int setup_device(spi_handle* H) {
  Handle& h = H->h;
  const Analysis& a = h.an;
  DevAnalysis& d = h.d;
  hipError_t he = hipSuccess;
  // opts.device_mem_cap: every allocation is counted first and refused
  // (hipErrorOutOfMemory, reported as SPI_E_OOM) once the total would pass it
  bool capped = false;
  h.dev_bytes = 0;
  auto admit = [&](int64_t bytes) {
    if (he != hipSuccess) return false;
    if (h.opts.device_mem_cap > 0 && h.dev_bytes + bytes > h.opts.device_mem_cap) {
      he = hipErrorOutOfMemory;
      capped = true;
      return false;
    }
    h.dev_bytes += bytes;
    return true;
  };
#define UP(field)                                                           \
  if (admit((int64_t)(a.field.size() * sizeof(a.field[0]))))                \
  he = dev_copy(d.field, a.field, h.stream)
  UP(rowptr); UP(col); UP(colptr); UP(csc_pos); UP(csc_row); UP(leaf_cols);
  UP(leaf_grp); UP(leaf_slot_ptr); UP(grp_col_ptr); UP(grp_U_ptr); UP(U);
  UP(grp_panel_off); UP(grp_slot_ptr); UP(slot_row); UP(slot_rr_ptr);
  UP(slot_leaf_src); UP(rr_lpos); UP(rr_src); UP(root_cols); UP(rinc_ptr);
  UP(rinc_grp); UP(rinc_u); UP(tasks); UP(grp_task_ptr); UP(task_part_off);
  UP(sel_order); UP(rp_rows); UP(rp_rowbase); UP(rpe_ptr); UP(rpe_pos);
  UP(rpe_src); UP(up_U_off); UP(up_Q_off); UP(up_nU); UP(up_k); UP(up_w_off);
  UP(tile_order); UP(inc_ptr); UP(inc); UP(inc_split); UP(root_of_col);
  UP(leaf_of_col);
#undef UP
  const int64_t nl = (int64_t)a.leaf_cols.size();
  const int64_t np = a.n_pad;
#define AL(ptr, cnt)                                                   \
  if (admit(std::max<int64_t>(0, (int64_t)(cnt)) * (int64_t)sizeof(*ptr))) { \
    he = dev_alloc(ptr, cnt);                                          \
    if (ptr) h.bufs.emplace_back((void*)ptr, (size_t)(cnt) * sizeof(*ptr)); \
  }
  AL(h.val, a.nnz); AL(h.valc, a.nnz); AL(h.w, a.m); AL(h.sw, a.n_slots);
  AL(h.sleaf, a.n_slots);
  AL(h.rrval, (int64_t)a.rr_src.size());
  AL(h.panel, a.grp_panel_off.back() + a.rp_val_off.back());
  if (h.opts.indefinite) AL(h.panelS, a.rp_val_off.back());
  AL(h.ldiag, nl);
  AL(h.S, np * np);
  if (h.opts.keep_root_sum) AL(h.Akeep, np * np);
  // the Cholesky route's buffers: the inverse factor, the root block of A^-1
  // and the inverses of the diagonal blocks (the sweeps need none of them)
  if (!h.opts.root_inverse) {
    AL(h.W, np * np); AL(h.Z, np * np);
    AL(h.invd, np * kNB); AL(h.invd2, ((np + 255) / 256) * 256 * 256);
  }
  // widest band of the root sweeps: 1024 columns in binary64 (a band's
  // bulk update reads and writes the root once per band), 512 with binary32
  // products (two binary32 sums of at most 256 terms per launch)
  h.band_nb = (int)std::min<int64_t>(
      h.opts.root_inverse && h.opts.precision == SPI_FP64 ? 1024 : 512, np);
  AL(h.band, 4 * (int64_t)h.band_nb * np + 2 * (int64_t)h.band_nb * h.band_nb);
  AL(h.part, a.task_part_off.back());
  AL(h.flag, 4); AL(h.vleaf, nl); AL(h.vfront, a.grp_U_ptr.back()); AL(h.vroot, np); AL(h.vres, a.n);
  AL(h.vx, a.n); AL(h.vdd, 2 * a.m); AL(h.vnorm, 4);
  AL(h.vroot2, np); AL(h.vpart, root_inv_part_size(np));
  AL(h.colscale, a.n); AL(h.vbh, a.n); AL(h.vxh, a.n); AL(h.diagA, a.n);
  AL(h.vrow, a.m); AL(h.vsum, sum_scratch_size()); AL(h.vb2, a.n);
  AL(h.vm1, a.n); AL(h.vm2, a.n); AL(h.vw, a.m); AL(h.vr, a.m);
#undef AL
  if (he == hipSuccess) he = hipStreamSynchronize(h.stream);
  if (he != hipSuccess) {
    g_analyze_err = capped ? std::string("device memory cap exceeded: the handle needs "
                                         "more than opts.device_mem_cap bytes")
                           : std::string("device setup failed: ") + hipGetErrorString(he);
    free_all(h);
    delete H;
    return he == hipErrorOutOfMemory ? SPI_E_OOM : SPI_E_HIP;
  }
  return SPI_OK;
}

}  // namespace

// ---- stream-ordered pieces of the entry points (also used by batches)
namespace spi {

// Converged once the last correction (relative max-norm `cur`) is below
// tol, or once two corrections contract (by at least half) at a rate that
// puts the next one, i.e. the error left in x, below tol.  prev <= 0: no
// earlier correction.
bool refine_converged(double cur, double prev, double tol) {
  if (cur <= tol) return true;
  return prev > 0.0 && cur <= 0.5 * prev && cur * (cur / prev) <= tol;
}


int factor_enqueue(Handle& h, bool may_sync) {
  h.have_factor = false;
  h.have_inv = false;
  h.z_valid = false;
  h.failed_col = -1;
  // root assembly: everything (mode 0), everything keeping A_RR (1), or the
  // kept A_RR plus the leaf fronts (2) after a leaf-only value change whose
  // root entries were found unchanged
  int mode = 0;
  if (h.Akeep) {
    mode = 1;
    if (may_sync && h.akeep_valid && h.leaf_update) {
      uint64_t changed = 1;
      SPI_CK(hipMemcpyAsync(&changed, h.flag + 2, sizeof(changed),
                            hipMemcpyDeviceToHost, h.stream), "update flag");
      SPI_CK(hipStreamSynchronize(h.stream), "update flag");
      if (!changed) mode = 2;
    }
  }
  SPI_CK(fill_i64(h.stream, h.flag, -1, 1), "flag");
  phase_begin(h, kPhLeaf);
  SPI_CK(launch_leaf_assemble(h), "leaf assembly");
  phase_end(h, kPhLeaf);
  if (h.an.n_pad) {
    phase_begin(h, kPhExtend);
    SPI_CK(launch_assemble_root(h, mode), "root assembly");
    phase_end(h, kPhExtend);
    if (mode == 1) h.akeep_valid = true;
    h.leaf_update = false;
    h.last_asm_mode = mode;
    // root inverse wanted: sweeps turn S into A_RR^-1; otherwise Cholesky
    h.swept = h.opts.root_inverse != 0;
    phase_begin(h, kPhPotrf);
    SPI_CK(h.swept ? root_sweep(h) : root_potrf(h), "root factorisation");
    phase_end(h, kPhPotrf);
    if (h.opts.root_inverse && !h.swept) {
      phase_begin(h, kPhTrtri);
      SPI_CK(root_trtri(h), "root factor inversion");
      phase_end(h, kPhTrtri);
    }
  }
  // work enqueued after this point may use the inverse (stream order);
  // factor_finish withdraws it if a pivot failed
  h.have_inv = h.an.n_pad > 0 && h.opts.root_inverse;
  return SPI_OK;
}

// Interpret the pivot flag read back after factor_enqueue's work completed.
int factor_finish(Handle& h, const uint64_t* f) {
  if (f[1] != 0) {
    h.have_inv = false;
    return fail(h, SPI_E_ARG, hipSuccess,
                "a value or weight given to spi_set_values is NaN or infinite");
  }
  if (f[0] != std::numeric_limits<uint64_t>::max()) {
    const int64_t nl = (int64_t)h.an.leaf_cols.size();
    int64_t k = (int64_t)f[0];
    if (k < nl) h.failed_col = h.an.leaf_cols[k];
    else if (k - nl < h.an.n_root) h.failed_col = h.an.root_cols[k - nl];
    std::ostringstream os;
    os << "matrix not positive definite: non-positive pivot at column "
       << h.failed_col;
    h.err = os.str();
    h.have_inv = false;
    return SPI_E_NOT_SPD;
  }
  h.have_factor = true;
  return SPI_OK;
}

// One right-hand side with exactly `steps` refinement steps (no readback).
int solve_enqueue(Handle& h, const double* bc, double* xc, int steps) {
  const bool eq = h.opts.equilibrate != 0;
  const double* src = bc;
  double* dst = xc;
  if (eq) {
    SPI_CK(launch_scale_vec(h, bc, h.vbh, 0), "scale rhs");
    src = h.vbh;
    dst = h.vxh;
  }
  SPI_CK(launch_solve_pass(h, src, dst), "solve");
  // step s leaves (max |dx|, max |x|) in vnorm[2 (s & 1) ..], so the sizes
  // of the last two corrections can be read back after the work completes
  for (int s = 0; s < steps; ++s) {
    SPI_CK(launch_residual_dd(h, src, dst, h.vres), "residual");
    SPI_CK(launch_solve_pass(h, h.vres, h.vx), "correction");
    double* nv = h.vnorm + 2 * (s & 1);
    SPI_CK(fill_f64(h.stream, nv, 0.0, 2), "norms");
    SPI_CK(launch_axpy_norms(h, dst, h.vx, nv), "update");
  }
  if (eq) SPI_CK(launch_scale_vec(h, h.vxh, xc, 0), "scale solution");
  return SPI_OK;
}

int diag_enqueue(Handle& h, double* d, double* part) {
  h.Zr = h.swept ? h.S : h.Z;
  if (h.an.n_pad && !h.swept) {
    if (!h.have_inv) {
      phase_begin(h, kPhTrtri);
      SPI_CK(root_trtri(h), "root factor inversion");
      phase_end(h, kPhTrtri);
      h.have_inv = true;
    }
    phase_begin(h, kPhLauum);
    SPI_CK(root_lauum(h), "root inverse product");
    phase_end(h, kPhLauum);
    h.z_valid = true;
  }
  phase_begin(h, kPhSelinv);
  if (h.an.n_pad) SPI_CK(launch_diag_root(h, d), "root diagonal");
  SPI_CK(launch_selinv_leaves(h, d, part ? part : h.part), "leaf selected inversion");
  // (S A S)^-1 = S^-1 A^-1 S^-1: undo the scaling, d_i = s_i^2 d'_i
  if (h.opts.equilibrate) SPI_CK(launch_scale_vec(h, d, d, 2), "scale variances");
  phase_end(h, kPhSelinv);
  return SPI_OK;
}

}  // namespace spi

extern "C" {

void spi_default_opts(spi_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SPI_FP64;
  o->max_group = 32;
  o->leaf_max_work = 65536.0;
  o->amalg_density = 0.35;
  o->refine_steps = 1;
  o->root_inverse = 1;
  o->equilibrate = 1;
  o->refine_tol = 0.0;
}

int spi_analyze(spi_handle** out, int64_t m, int64_t n, const int64_t* rowptr,
                const int32_t* col, const spi_opts* opts, void* stream) {
  g_analyze_err.clear();
  if (!out) {
    g_analyze_err = "null handle pointer";
    return SPI_E_ARG;
  }
  *out = nullptr;
  spi_opts o;
  spi_default_opts(&o);
  if (opts) o = *opts;
  if (!check_opts(o)) return SPI_E_ARG;
  spi_handle* H = new (std::nothrow) spi_handle();
  if (!H) {
    g_analyze_err = "host allocation failed";
    return SPI_E_OOM;
  }
  Handle& h = H->h;
  h.opts = o;
  h.req_precision = o.precision;
  h.stream = (hipStream_t)stream;
  (void)hipGetDevice(&h.device);
  auto t0 = std::chrono::steady_clock::now();
  std::string e = analyze(m, n, rowptr, col, o, h.an);
  if (!e.empty()) {
    g_analyze_err = e;
    delete H;
    return SPI_E_ARG;
  }
  const int st = setup_device(H);
  if (st != SPI_OK) return st;
  h.t_analyze_ms = std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return SPI_OK;
}

int spi_analyze_like(spi_handle** out, const spi_handle* src, const spi_opts* opts,
                     void* stream) {
  g_analyze_err.clear();
  if (!out || !src) {
    g_analyze_err = "null handle pointer";
    return SPI_E_ARG;
  }
  *out = nullptr;
  spi_opts o = src->h.opts;
  o.precision = src->h.req_precision;  // not a binary64 fallback of src's
  if (opts) o = *opts;
  if (!check_opts(o)) return SPI_E_ARG;
  if (o.max_group != src->h.opts.max_group ||
      o.leaf_max_work != src->h.opts.leaf_max_work ||
      o.amalg_density != src->h.opts.amalg_density ||
      o.keep_root_order != src->h.opts.keep_root_order ||
      o.asm_tile != src->h.opts.asm_tile) {
    g_analyze_err = "analysis options must match the source handle";
    return SPI_E_ARG;
  }
  spi_handle* H = new (std::nothrow) spi_handle();
  if (!H) {
    g_analyze_err = "host allocation failed";
    return SPI_E_OOM;
  }
  Handle& h = H->h;
  h.opts = o;
  h.req_precision = o.precision;
  h.stream = (hipStream_t)stream;
  (void)hipGetDevice(&h.device);
  auto t0 = std::chrono::steady_clock::now();
  h.an = src->h.an;  // host copy of the analysis: no re-analysis
  const int st = setup_device(H);
  if (st != SPI_OK) return st;
  h.t_analyze_ms = std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return SPI_OK;
}

int spi_set_values(spi_handle* H, const double* val, const double* w) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!val || !w) return fail(h, SPI_E_ARG, hipSuccess, "null value pointer");
  SPI_CK(hipMemcpyAsync(h.val, val, h.an.nnz * sizeof(double),
                        hipMemcpyDeviceToDevice, h.stream), "copy values");
  SPI_CK(hipMemcpyAsync(h.w, w, h.an.m * sizeof(double),
                        hipMemcpyDeviceToDevice, h.stream), "copy weights");
  // flag[1] collects non-finite inputs (values: while gathered into column
  // order; weights: here); spi_factor reports it
  SPI_CK(fill_i64(h.stream, h.flag + 1, 0, 1), "input flag");
  SPI_CK(launch_check_finite(h, h.w, h.an.m), "weights");
  SPI_CK(launch_equilibrate(h), "diagonal / equilibration");
  h.val32_ok = false;
  SPI_CK(launch_gather_values(h), "gather values");
  SPI_CK(launch_fill_rowpanels(h), "row panels");
  h.opts.precision = h.req_precision;  // new values: the precision asked for
  h.have_values = true;
  h.have_factor = false;
  h.have_inv = false;
  h.akeep_valid = false;
  h.leaf_update = false;
  return SPI_OK;
}

int spi_debug_poison(spi_handle* H) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  for (const auto& b : h.bufs)
    SPI_CK(hipMemsetAsync(b.first, 0xff, b.second, h.stream), "poison");
  h.have_values = false;
  h.have_factor = false;
  h.have_inv = false;
  h.akeep_valid = false;
  h.z_valid = false;
  return SPI_OK;
}

int spi_set_leaf_values(spi_handle* H, const double* val) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!val) return fail(h, SPI_E_ARG, hipSuccess, "null value pointer");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_set_leaf_values before spi_set_values");
  SPI_CK(hipMemcpyAsync(h.val, val, h.an.nnz * sizeof(double),
                        hipMemcpyDeviceToDevice, h.stream), "copy values");
  // the weights are those of the last spi_set_values (already checked)
  SPI_CK(fill_i64(h.stream, h.flag + 1, 0, 2), "input flags");
  SPI_CK(launch_equilibrate(h), "diagonal / equilibration");
  h.val32_ok = false;
  SPI_CK(launch_gather_values(h), "gather values");
  // rewrite the row panels comparing with the root entries in use
  SPI_CK(launch_fill_rowpanels(h, true), "row panels");
  h.opts.precision = h.req_precision;
  h.have_factor = false;
  h.have_inv = false;
  h.leaf_update = true;
  return SPI_OK;
}

namespace {

// The factorisation, its pivot flag read back and interpreted.
int factor_sync(Handle& h) {
  int st = factor_enqueue(h, true);
  if (st != SPI_OK) return st;
  uint64_t f[2] = {0, 0};
  SPI_CK(hipMemcpyAsync(f, h.flag, sizeof(f), hipMemcpyDeviceToHost, h.stream),
         "flag readback");
  SPI_CK(hipStreamSynchronize(h.stream), "factor");
  return factor_finish(h, f);
}

// opts.fp64_fallback: a SPI_MIXED handle whose binary32 stages failed is
// switched to binary64 (until new values arrive) and refactored.
bool can_fall_back(const Handle& h) {
  return h.opts.fp64_fallback && h.opts.precision == SPI_MIXED;
}

int refactor_fp64(Handle& h) {
  h.opts.precision = SPI_FP64;
  ++h.fp64_fallbacks;
  return factor_sync(h);
}

}  // namespace

int spi_factor(spi_handle* H) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_factor before spi_set_values");
  const int st = factor_sync(h);
  if (st == SPI_E_NOT_SPD && can_fall_back(h)) return refactor_fp64(h);
  return st;
}

int spi_rhs(spi_handle* H, const double* y, double* b) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!y || !b) return fail(h, SPI_E_ARG, hipSuccess, "null pointer");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_rhs before spi_set_values");
  SPI_CK(launch_rhs(h, y, b), "rhs");
  return SPI_OK;
}

int spi_solve(spi_handle* H, const double* b, double* x, int32_t nrhs,
              int64_t ldb) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!b || !x || nrhs < 1 || ldb < h.an.n)
    return fail(h, SPI_E_ARG, hipSuccess, "invalid solve arguments");
  if (!h.have_factor)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_solve without a valid factor");
  // With equilibration the factor is that of S A S: solve (S A S) x' = S b
  // and return x = S x'.  The refinement residual S b - (H S)^T W (H S) x'
  // is S (b - A x) exactly (powers of two).
  const bool eq = h.opts.equilibrate != 0;
  const double tol = h.opts.refine_tol;
  int status = SPI_OK, done_max = 0;
  phase_begin(h, kPhSolve);
  for (int32_t c = 0; c < nrhs; ++c) {
    const double* bc = b + (int64_t)c * ldb;
    double* xc = x + (int64_t)c * ldb;
    const double* src = bc;
    double* dst = xc;
    if (eq) {
      SPI_CK(launch_scale_vec(h, bc, h.vbh, 0), "scale rhs");
      src = h.vbh;
      dst = h.vxh;
    }
    SPI_CK(launch_solve_pass(h, src, dst), "solve");
    bool converged = tol <= 0.0;
    int done = 0;
    double prev = 0.0;  // relative size of the previous correction
    for (int s = 0; s < h.opts.refine_steps; ++s) {
      SPI_CK(launch_residual_dd(h, src, dst, h.vres), "residual");
      SPI_CK(launch_solve_pass(h, h.vres, h.vx), "correction");
      SPI_CK(fill_f64(h.stream, h.vnorm, 0.0, 2), "norms");
      SPI_CK(launch_axpy_norms(h, dst, h.vx, h.vnorm), "update");
      ++done;
      if (tol > 0.0) {
        double nv[2];
        SPI_CK(hipMemcpyAsync(nv, h.vnorm, sizeof(nv), hipMemcpyDeviceToHost,
                              h.stream), "norm readback");
        SPI_CK(hipStreamSynchronize(h.stream), "refinement");
        const double cur = nv[1] > 0.0 ? nv[0] / nv[1] : 0.0;
        if (refine_converged(cur, prev, tol)) {
          converged = true;
          break;
        }
        prev = cur;
      }
    }
    if (eq) SPI_CK(launch_scale_vec(h, h.vxh, xc, 0), "scale solution");
    done_max = std::max(done_max, done);
    if (!converged) status = SPI_E_NOCONV;
  }
  phase_end(h, kPhSolve);
  h.refine_done = done_max;
  h.last_norm_pair = 0;
  if (status == SPI_E_NOCONV && can_fall_back(h)) {
    // the binary32 factor does not refine to refine_tol: binary64 throughout
    const int fs = refactor_fp64(h);
    if (fs != SPI_OK) return fs;
    return spi_solve(H, b, x, nrhs, ldb);
  }
  if (status != SPI_OK)
    return fail(h, status, hipSuccess,
                "iterative refinement did not reach refine_tol");
  return SPI_OK;
}

int spi_diag_inv(spi_handle* H, double* d) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!d) return fail(h, SPI_E_ARG, hipSuccess, "null output");
  if (!h.have_factor)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_diag_inv without a valid factor");
  return diag_enqueue(h, d);
}

int spi_inv_entries(spi_handle* H, int64_t k, const int32_t* rows,
                    const int32_t* cols, double* out) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (k < 0 || (k > 0 && (!rows || !cols || !out)))
    return fail(h, SPI_E_ARG, hipSuccess, "invalid inverse-entry arguments");
  if (!h.have_factor)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_inv_entries without a valid factor");
  if (k == 0) return SPI_OK;
  // the requested columns, checked on the host
  std::vector<int32_t> rc(2 * (size_t)k);
  SPI_CK(hipMemcpyAsync(rc.data(), rows, k * sizeof(int32_t), hipMemcpyDeviceToHost,
                        h.stream), "index readback");
  SPI_CK(hipMemcpyAsync(rc.data() + k, cols, k * sizeof(int32_t),
                        hipMemcpyDeviceToHost, h.stream), "index readback");
  SPI_CK(hipStreamSynchronize(h.stream), "index readback");
  for (int32_t v : rc)
    if (v < 0 || v >= h.an.n)
      return fail(h, SPI_E_ARG, hipSuccess, "inverse-entry index out of range");
  // the root block of A^-1: from the sweeps, or formed from the factor
  h.Zr = h.swept ? h.S : h.Z;
  if (h.an.n_pad && !h.swept && !h.z_valid) {
    if (!h.have_inv) {
      SPI_CK(root_trtri(h), "root factor inversion");
      h.have_inv = true;
    }
    SPI_CK(root_lauum(h), "root inverse product");
    h.z_valid = true;
  }
  SPI_CK(launch_inv_entries(h, rows, cols, out, k), "inverse entries");
  return SPI_OK;
}

static void fill_analysis_info(const Analysis& a, spi_info_t* info) {
  info->m = a.m;
  info->n = a.n;
  info->nnz_h = a.nnz;
  info->nnz_a = a.nnz_a;
  info->nnz_l = a.nnz_l;
  info->n_leaf = (int64_t)a.leaf_cols.size();
  info->n_groups = a.n_groups;
  info->n_root = a.n_root;
  info->n_root_padded = a.n_pad;
  info->asm_tile = a.asm_tile;
  info->flops_factor = a.flops_factor;
  info->flops_selinv = a.flops_selinv;
  info->flops_solve = a.flops_solve;
  info->flops_assembly = a.flops_asm;
  info->flops_exec_assembly = a.flops_exec_asm;
  info->flops_exec_selinv = a.flops_exec_selinv;
  info->flops_root_assembly = a.flops_root_asm;
}

int spi_symbolic(int64_t m, int64_t n, const int64_t* rowptr,
                 const int32_t* col, const spi_opts* opts, spi_info_t* info,
                 int32_t* elim_order, int32_t* col_parent, int32_t* front_of) {
  g_analyze_err.clear();
  spi_opts o;
  spi_default_opts(&o);
  if (opts) o = *opts;
  if (!check_opts(o)) return SPI_E_ARG;
  Analysis a;
  auto t0 = std::chrono::steady_clock::now();
  std::string e = analyze(m, n, rowptr, col, o, a);
  if (!e.empty()) {
    g_analyze_err = e;
    return SPI_E_ARG;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    fill_analysis_info(a, info);
    info->failed_col = -1;
    info->precision = o.precision;
    info->t_analyze_ms = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - t0).count();
  }
  const int64_t nl = (int64_t)a.leaf_cols.size();
  if (elim_order) {
    for (int64_t l = 0; l < nl; ++l) elim_order[l] = a.leaf_cols[l];
    for (int64_t i = 0; i < a.n_root; ++i) elim_order[nl + i] = a.root_cols[i];
  }
  if (col_parent) {
    for (int64_t g = 0; g < a.n_groups; ++g) {
      int64_t u0 = a.grp_U_ptr[g], u1 = a.grp_U_ptr[g + 1];
      for (int64_t l = a.grp_col_ptr[g]; l < a.grp_col_ptr[g + 1]; ++l) {
        // the panel column of a leaf is stored over the whole front structure,
        // but its own non-zeros are the root unknowns of its own rows
        int32_t j = a.leaf_cols[l];
        int32_t best = -1;
        for (int64_t s = a.leaf_slot_ptr[l]; s < a.leaf_slot_ptr[l + 1]; ++s)
          for (int64_t k = a.slot_rr_ptr[s]; k < a.slot_rr_ptr[s + 1]; ++k) {
            int32_t ri = a.U[u0 + a.rr_lpos[k]];
            if (best < 0 || ri < best) best = ri;
          }
        (void)u1;
        col_parent[j] = best < 0 ? -1 : a.root_cols[best];
      }
    }
    for (int64_t i = 0; i < a.n_root; ++i)
      col_parent[a.root_cols[i]] = (i + 1 < a.n_root) ? a.root_cols[i + 1] : -1;
  }
  if (front_of) {
    for (int64_t j = 0; j < a.n; ++j) front_of[j] = -1;
    for (int64_t l = 0; l < nl; ++l) front_of[a.leaf_cols[l]] = a.leaf_grp[l];
  }
  return SPI_OK;
}

int spi_save_analysis(const spi_handle* H, const char* path) {
  if (!H) return SPI_E_ARG;
  Handle& h = const_cast<spi_handle*>(H)->h;  // only its error text changes
  const std::string e = save_analysis(h.an, h.opts, path);
  if (!e.empty()) return fail(h, SPI_E_ARG, hipSuccess, e.c_str());
  return SPI_OK;
}

int spi_symbolic_save(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                      const spi_opts* opts, const char* path) {
  g_analyze_err.clear();
  spi_opts o;
  spi_default_opts(&o);
  if (opts) o = *opts;
  if (!check_opts(o)) return SPI_E_ARG;
  Analysis a;
  std::string e = analyze(m, n, rowptr, col, o, a);
  if (e.empty()) e = save_analysis(a, o, path);
  if (!e.empty()) {
    g_analyze_err = e;
    return SPI_E_ARG;
  }
  return SPI_OK;
}

int spi_analysis_file_info(const char* path, spi_info_t* info) {
  g_analyze_err.clear();
  if (!info) {
    g_analyze_err = "null info pointer";
    return SPI_E_ARG;
  }
  spi_opts o;
  spi_default_opts(&o);
  Analysis a;
  const std::string e = load_analysis(path, a, o);
  if (!e.empty()) {
    g_analyze_err = e;
    return SPI_E_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  fill_analysis_info(a, info);
  info->failed_col = -1;
  return SPI_OK;
}

int spi_analyze_load(spi_handle** out, const char* path, const spi_opts* opts,
                     void* stream) {
  g_analyze_err.clear();
  if (!out) {
    g_analyze_err = "null handle pointer";
    return SPI_E_ARG;
  }
  *out = nullptr;
  spi_opts o;
  spi_default_opts(&o);
  if (opts) o = *opts;
  auto t0 = std::chrono::steady_clock::now();
  Analysis a;
  const std::string e = load_analysis(path, a, o);  // the file's analysis options
  if (!e.empty()) {
    g_analyze_err = e;
    return SPI_E_ARG;
  }
  if (!check_opts(o)) return SPI_E_ARG;
  spi_handle* H = new (std::nothrow) spi_handle();
  if (!H) {
    g_analyze_err = "host allocation failed";
    return SPI_E_OOM;
  }
  Handle& h = H->h;
  h.opts = o;
  h.req_precision = o.precision;
  h.stream = (hipStream_t)stream;
  (void)hipGetDevice(&h.device);
  h.an = std::move(a);
  const int st = setup_device(H);
  if (st != SPI_OK) return st;
  h.t_analyze_ms = std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return SPI_OK;
}

int spi_info(const spi_handle* Hc, spi_info_t* info) {
  if (!Hc || !info) return SPI_E_ARG;
  // collecting timers mutates the handle's event pools, not its results
  Handle& h = const_cast<spi_handle*>(Hc)->h;
  for (auto& t : h.timer) collect(t);
  const Analysis& a = h.an;
  std::memset(info, 0, sizeof(*info));
  fill_analysis_info(a, info);
  info->failed_col = h.failed_col;
  info->device_bytes = h.dev_bytes;
  info->fp64_fallbacks = h.fp64_fallbacks;
  info->t_analyze_ms = h.t_analyze_ms;
  info->precision = h.opts.precision;
  info->refine_steps_done = h.refine_done;
  if (h.refine_done > 0 && h.vnorm) {
    double nv[2] = {0, 0};
    if (hipMemcpyAsync(nv, h.vnorm + 2 * h.last_norm_pair, sizeof(nv),
                       hipMemcpyDeviceToHost,
                       h.stream) == hipSuccess &&
        hipStreamSynchronize(h.stream) == hipSuccess && nv[1] > 0)
      info->last_refine_norm = nv[0] / nv[1];
  }
  info->t_leaf_ms = h.timer[kPhLeaf].total_ms;
  info->t_extend_ms = h.timer[kPhExtend].total_ms;
  info->t_potrf_ms = h.timer[kPhPotrf].total_ms;
  info->t_solve_ms = h.timer[kPhSolve].total_ms;
  info->t_trtri_ms = h.timer[kPhTrtri].total_ms;
  info->t_lauum_ms = h.timer[kPhLauum].total_ms;
  info->t_selinv_ms = h.timer[kPhSelinv].total_ms;
  info->t_sweep_bulk_ms = h.timer[kPhBulk].total_ms;
  info->flops_sweep_bulk = h.bulk_flops;
  info->root_assembly_mode = h.last_asm_mode;
  return SPI_OK;
}

const char* spi_last_error(const spi_handle* H) {
  if (!H) return g_analyze_err.c_str();
  return H->h.err.c_str();
}

void spi_destroy(spi_handle* H) {
  if (!H) return;
  (void)hipStreamSynchronize(H->h.stream);
  free_all(H->h);
  delete H;
}

}  // extern "C"

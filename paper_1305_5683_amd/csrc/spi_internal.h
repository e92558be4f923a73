// Internal declarations of libspi: handle layout, host analysis, kernel
// launchers.  Not part of the public ABI (that is include/spi.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spi.h"

namespace spi {

// Root front is padded to a multiple of this (identity on the padding), so
// every dense kernel works on whole tiles.
constexpr int kRootPad = 128;
// Block size of the root POTRF / TRTRI sweeps and of the stored inverse
// diagonal blocks.
constexpr int kNB = 64;
// Tile edge of the extend-add and leaf selected-inversion tasks, in
// positions of a front's row structure U.
constexpr int kET = 64;
// Rows of the dense root triangular-solve chunks.
constexpr int kTrsvChunk = 512;
// Edges of the root tiles the output-stationary assembly sums in LDS.
// Every panel row is read once per tile pair it meets, so larger tiles read
// less: 128 x 128 (one workgroup of 16 waves per CU, 140 KB of LDS) against
// 64 x 64 (two of 8 waves): medium root assembly 4.50 against 4.61 ms,
// large 481 against 551 ms.  Roots below order kAsmTile128From keep 64 x 64
// tiles, four times as many workgroups for a small front.
constexpr int kAsmTileSmall = 64, kAsmTileLarge = 128;
constexpr int64_t kAsmTile128From = 8192;
// Widest leaf front (root positions) accumulated in LDS by the leaf
// assembly: 4 waves x 2048 x 8 B = 64 KB per workgroup.
constexpr int kLeafLdsCapMax = 2048;
// Default tasks per launch of the leaf selected inversion (a launch stays
// below 2^24 workgroups of 256 threads).
constexpr int64_t kSelinvChunk = int64_t(1) << 22;

// ---------------------------------------------------------------- analysis
// Host result of the symbolic analysis.  "slot" = a measurement row in
// front order: rows of front 0, rows of front 1, ...; within a leaf front
// the rows of its first leaf column, then its second, and so on.
// Allocator whose new elements are left uninitialised: the analysis sizes
// its largest index arrays (one entry per non-zero of H) and fills every
// element in parallel right away, and value-initialising them first would
// be a serial pass over gigabytes.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U*) noexcept {}
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new ((void*)p) U(std::forward<Args>(args)...);
  }
};
template <class T>
using bigvec = std::vector<T, NoInitAlloc<T>>;

struct Analysis {
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int64_t> rowptr;
  bigvec<int32_t> col;
  // transpose of the pattern
  std::vector<int64_t> colptr;    // n + 1
  bigvec<int64_t> csc_pos;        // CSR position of each CSC entry
  bigvec<int32_t> csc_row;        // row of each CSC entry
  // leaves (eliminated first), in front order
  std::vector<int32_t> leaf_cols;       // original column of leaf l
  std::vector<int32_t> leaf_grp;        // front of leaf l
  std::vector<int64_t> leaf_slot_ptr;   // n_leaf + 1, slots of leaf l
  // leaf fronts (supernodes of leaf unknowns)
  int64_t n_groups = 0;
  std::vector<int64_t> grp_col_ptr;    // n_groups + 1 into leaf_cols
  std::vector<int64_t> grp_U_ptr;      // n_groups + 1 into U
  std::vector<int32_t> U;              // root indices, sorted per front; the
                                       // row panels' lists follow (rp_U_base)
  std::vector<int64_t> grp_panel_off;  // n_groups + 1, dense |U| x p panels
  std::vector<int64_t> grp_slot_ptr;   // n_groups + 1 into slots
  // slots: the rows of the leaf fronts, by leaf unknown
  int64_t n_slots = 0;
  std::vector<int32_t> slot_row;       // original row
  std::vector<int64_t> slot_rr_ptr;    // n_slots + 1 into the compact root entries
  std::vector<int64_t> slot_leaf_src;  // CSR position of the leaf entry
  bigvec<int32_t> rr_lpos;             // U-local position of each root entry
  bigvec<int64_t> rr_src;              // CSR position of each root entry
  // row panels: consecutive rows with overlapping root structure, stored
  // dense |U| x rows (values h, weights w kept per row) for the assembly of
  // A_RR = sum_r w_r h_rR h_rR^T
  int64_t n_rp = 0;
  int64_t rp_U_base = 0;               // offset of the row panels' U lists
  std::vector<int64_t> rp_row_ptr;     // n_rp + 1 into rp_rows
  std::vector<int32_t> rp_rows;        // original rows, panel order
  std::vector<int64_t> rp_U_ptr;       // n_rp + 1 (relative to rp_U_base)
  std::vector<int64_t> rp_val_off;     // n_rp + 1, offsets of the dense panels
  std::vector<int64_t> rp_rowbase;     // per panel row: offset of its column
  std::vector<int64_t> rpe_ptr;        // per panel row + 1: its root entries
  bigvec<int32_t> rpe_pos;             // U-local position
  bigvec<int64_t> rpe_src;             // CSR position
  // update panels (leaf fronts, then row panels): descriptors
  int64_t n_up = 0;
  std::vector<int64_t> up_U_off;       // into U
  std::vector<int64_t> up_Q_off;       // into the panel buffer (leaf | rows)
  std::vector<int32_t> up_nU;
  std::vector<int32_t> up_k;
  std::vector<int32_t> up_w_off;       // -1: leaf panel (sign -1); else row panel
  // incidences of the update panels on the asm_tile x asm_tile lower tiles
  // of the root; within a tile the leaf fronts' incidences come first
  int asm_tile = kAsmTileSmall;        // root assembly tile edge (64 or 128)
  int64_t n_tiles = 0;                 // T (T + 1) / 2, T = n_pad / asm_tile
  std::vector<int32_t> tile_order;     // launch order of the tiles
  std::vector<int64_t> inc_ptr;        // n_tiles + 1
  std::vector<int64_t> inc_split;      // n_tiles: first row-panel incidence
  bigvec<int32_t> inc;                 // 4 per incidence: up, aI0, aJ0, nI|nJ<<16
  // root
  int64_t n_root = 0, n_pad = 0;
  std::vector<int32_t> root_cols;      // original column of root index i
  std::vector<int32_t> root_of_col;    // n, root index or -1
  std::vector<int32_t> leaf_of_col;    // n, leaf index or -1
  // root incidences (transpose of the U lists): for root index i the
  // (front, U-local position) pairs, as global panel row offsets
  std::vector<int64_t> rinc_ptr;       // n_root + 1
  bigvec<int32_t> rinc_grp;
  bigvec<int32_t> rinc_u;
  // selected-inversion tasks of the leaf fronts: (front, I, J), I >= J,
  // tiles of kET positions of the front's U
  bigvec<int32_t> tasks;               // 3 per task
  std::vector<int64_t> grp_task_ptr;   // n_groups + 1
  bigvec<int64_t> task_part_off;       // n_tasks + 1 (partial sums)
  // launch order of the tasks: grouped by the 2-D block of the root front
  // they read, so that tasks running together share a region of it
  bigvec<int32_t> sel_order;
  // counters
  int64_t nnz_a = 0, nnz_l = 0;
  double flops_factor = 0, flops_selinv = 0, flops_solve = 0, flops_asm = 0;
  double flops_exec_asm = 0, flops_exec_selinv = 0, flops_root_asm = 0;
};

// Returns an empty string on success, else the error text.
std::string analyze(int64_t m, int64_t n, const int64_t* rowptr,
                    const int32_t* col, const spi_opts& opts, Analysis& out);
// Analysis files (analysis_io.cpp): write `a` and the analysis options of
// `o`; read them back into `a` and the analysis options of `o`, refusing a
// truncated, corrupted or foreign file.  Empty string on success.
std::string save_analysis(const Analysis& a, const spi_opts& o, const char* path);
std::string load_analysis(const char* path, Analysis& a, spi_opts& o);

// ------------------------------------------------------------ device side
struct DevAnalysis {
  // pattern
  int64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  int64_t* colptr = nullptr;
  int64_t* csc_pos = nullptr;
  int32_t* csc_row = nullptr;
  // fronts
  int32_t* leaf_cols = nullptr;
  int32_t* leaf_grp = nullptr;
  int64_t* leaf_slot_ptr = nullptr;
  int64_t* grp_col_ptr = nullptr;
  int64_t* grp_U_ptr = nullptr;
  int32_t* U = nullptr;
  int64_t* grp_panel_off = nullptr;
  int64_t* grp_slot_ptr = nullptr;
  int32_t* slot_row = nullptr;
  int64_t* slot_rr_ptr = nullptr;
  int64_t* slot_leaf_src = nullptr;
  int32_t* rr_lpos = nullptr;
  int64_t* rr_src = nullptr;
  int32_t* root_cols = nullptr;
  int64_t* rinc_ptr = nullptr;
  int32_t* rinc_grp = nullptr;
  int32_t* rinc_u = nullptr;
  int32_t* tasks = nullptr;
  int64_t* grp_task_ptr = nullptr;
  int64_t* task_part_off = nullptr;
  int32_t* sel_order = nullptr;
  // row panels and root assembly
  int32_t* rp_rows = nullptr;
  int64_t* rp_rowbase = nullptr;
  int64_t* rpe_ptr = nullptr;
  int32_t* rpe_pos = nullptr;
  int64_t* rpe_src = nullptr;
  int64_t* up_U_off = nullptr;
  int64_t* up_Q_off = nullptr;
  int32_t* up_nU = nullptr;
  int32_t* up_k = nullptr;
  int32_t* up_w_off = nullptr;
  int32_t* tile_order = nullptr;
  int64_t* inc_ptr = nullptr;
  int64_t* inc_split = nullptr;
  int32_t* inc = nullptr;
  int32_t* root_of_col = nullptr;  // n: root index of a column, -1 for leaves
  int32_t* leaf_of_col = nullptr;  // n: leaf index of a column, -1 for the root
};

enum Phase { kPhLeaf = 0, kPhExtend, kPhPotrf, kPhSolve, kPhTrtri, kPhLauum,
             kPhSelinv, kPhBulk, kNumPhases };

struct PhaseTimer {
  std::vector<hipEvent_t> free_ev;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  hipEvent_t open = nullptr;
  double total_ms = 0;
  int64_t count = 0;
};

struct Handle {
  spi_opts opts{};
  int64_t dev_bytes = 0;     // device memory sized by the analysis (held)
  int req_precision = 0;     // the precision asked for (opts.precision is the
                             // one in use: binary64 after a fallback)
  int fp64_fallbacks = 0;    // opts.fp64_fallback: switches so far
  hipStream_t stream = nullptr;
  int device = 0;
  Analysis an;
  DevAnalysis d;
  // values in front (slot) order
  double* val = nullptr;     // H values, CSR order (copy)
  double* valc = nullptr;    // H values, CSC order (same scaling)
  double* w = nullptr;       // weights, original row order (copy)
  double* sw = nullptr;      // weight per slot
  double* sleaf = nullptr;   // leaf coefficient per slot
  double* rrval = nullptr;   // root entries in compact slot order
  // factor
  double* panel = nullptr;   // leaf panels L_UG, dense column-major per front,
                             // followed by the dense row panels
  double* panelS = nullptr;  // opts.indefinite: the row panels with their rows'
                             // weight signs (sign(w_r) sqrt|w_r| h_r)
  double* ldiag = nullptr;   // leaf pivots L_ll
  double* S = nullptr;       // root front n_pad x n_pad, column-major; L after factor
  double* Akeep = nullptr;   // opts.keep_root_sum: A_RR (row panels only), lower tiles
  bool akeep_valid = false;  // Akeep holds A_RR of the current root values
  bool leaf_update = false;  // values last set by spi_set_leaf_values
  int last_asm_mode = 0;     // root assembly mode of the last factorisation
  double* invd = nullptr;    // inverses of the kNB diagonal blocks of L_RR
  double* W = nullptr;       // L_RR^-1 (selected inversion scratch)
  double* invd2 = nullptr;   // inverses of the 256 x 256 diagonal blocks
  hipStream_t side = nullptr;       // lookahead stream of the root POTRF
  hipEvent_t ev_next = nullptr, ev_panel = nullptr;
  double* Z = nullptr;       // A^-1 restricted to the root (lower triangle)
  double* band = nullptr;    // root sweeps: 2 x (band, copy) np x band_nb,
                             // 2 pivot blocks band_nb x band_nb
  int band_nb = 0;           // widest band: min(512, n_pad)
  bool swept = false;        // S holds A_RR^-1 (sweeps) instead of L_RR
  bool z_valid = false;      // Cholesky route: Z holds A_RR^-1 of the factor
  double* Zr = nullptr;      // where the root block of A^-1 is: S or Z
  double* part = nullptr;    // selected-inversion partial sums
  int64_t* flag = nullptr;   // [0] first failing pivot in elimination
                             // order, [1] non-finite input seen, [2] root
                             // entries changed by spi_set_leaf_values,
                             // [3] a non-positive model value (likelihood)
  // solve scratch
  double* vleaf = nullptr;   // n_leaf
  double* vfront = nullptr;  // sum of |U| over leaf fronts: L_Ug y_g
  double* vroot = nullptr;   // n_pad
  double* vres = nullptr;    // n (residual / correction)
  double* vx = nullptr;      // n (iterate)
  double* vdd = nullptr;     // 2 m (double-double row values)
  double* vnorm = nullptr;   // 4: (max |dx|, max |x|) of the last two
                             // refinement steps (step s at 2 (s & 1))
  double* vroot2 = nullptr;  // n_pad
  double* vpart = nullptr;   // partial products of the root GEMV
  double* colscale = nullptr;  // equilibration: power-of-two column scales s
  double* vbh = nullptr;     // n: scaled right-hand side S b
  double* vxh = nullptr;     // n: solution of the scaled system
  double* diagA = nullptr;   // n: diagonal of A = H^T W H (unscaled)
  double* vrow = nullptr;    // m: per-row terms of the model loops
  double* vsum = nullptr;    // fixed-order sum partials (sum_scratch_size())
  double* vb2 = nullptr;     // n: right-hand side inside the model loops
  double* vm1 = nullptr;     // n: Newton step
  double* vm2 = nullptr;     // n: trial point
  double* vw = nullptr;      // m: Newton weights
  double* vr = nullptr;      // m: d/e - 1
  // scratch of the learned preconditioner and of PCG, allocated on first use
  struct LpWork {
    float* v32 = nullptr;                   // nnz: H in binary32
    float *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr,
          *e = nullptr, *t = nullptr;       // n (t: m)
    double *d = nullptr, *x = nullptr, *r64 = nullptr, *u = nullptr,
           *v = nullptr, *w = nullptr, *g = nullptr, *part = nullptr;
    float* phi = nullptr;                   // 3 n features
    double* fpart = nullptr;                // feature partial sums
  } lp;
  bool val32_ok = false;
  int potrf_block = 256;     // outer block of the root POTRF (autotuned)
  int bulk_tile = 128;       // tile edge of the sweeps' bulk update (autotuned)
  double bulk_flops = 0;     // algorithmic flops of the timed sweep bulk updates
  bool have_inv = false;     // W = L_RR^-1 is valid
  // phase timing (opts.timing): HIP event pairs recorded on the stream,
  // accumulated lazily (spi_info synchronises and sums them)
  PhaseTimer timer[kNumPhases];
  std::vector<std::pair<void*, size_t>> bufs;  // device work buffers (bytes)
  bool have_values = false, have_factor = false;
  int64_t failed_col = -1;
  double t_analyze_ms = 0;
  int refine_done = 0;
  int last_norm_pair = 0;    // vnorm pair of the last refinement step
  double last_refine_norm = 0;
  std::string err;
};

// Failure helper of the entry points: records the text, maps OOM.
inline int fail(Handle& h, int code, hipError_t e, const char* what) {
  h.err = what;
  if (e != hipSuccess) h.err += std::string(": ") + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory) return SPI_E_OOM;
  return code;
}

#define SPI_CK(expr, what)                                               \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) return ::spi::fail(h, SPI_E_HIP, e_, what);    \
  } while (0)

void free_lp_work(Handle& h);

// Stream-ordered pieces of the entry points (api.cpp): enqueue the work
// with no host synchronisation; factor_finish interprets the pivot flag
// once the factorisation has completed.
// may_sync: the root assembly may read a flag back to decide whether the
// kept A_RR still holds (not under graph capture)
int factor_enqueue(Handle& h, bool may_sync = false);
int factor_finish(Handle& h, const uint64_t* flag);
bool refine_converged(double cur, double prev, double tol);
int solve_enqueue(Handle& h, const double* b, double* x, int steps);
// part: the selected inversion's partial sums (nullptr: the handle's own
// buffer, h.part; task_part_off.back() doubles)
int diag_enqueue(Handle& h, double* d, double* part = nullptr);
hipError_t ensure_side_stream(Handle& h);

// Workgroup index -> logical work item, XCD-aware.  Workgroups are
// dispatched round-robin over the 8 XCDs (w % 8).  xcd_remap<B>: logical
// items come in chunks of 8 B; chunk item block x (B consecutive items) goes
// to XCD x, so the items running together on an XCD are consecutive ones,
// which share data in that XCD's L2.  The last partial chunk maps to itself.
//   B = 8:  the dense GEMM (8 tiles of one column of a group of 8 rows);
//   B = 64: the root assembly (64 consecutive tiles of a tile column) and
//           the selected inversion (tasks of one 512 x 512 block of the root).
template <int B>
__device__ inline int xcd_remap(int w, int n) {
  constexpr int C = 8 * B;
  if (w >= (n / C) * C) return w;
  const int x = w & 7, j = w >> 3;
  return (j / B) * C + x * B + (j % B);
}

// kernel launchers (stream-ordered); return hipError_t of the launch
hipError_t launch_gather_values(Handle& h);
hipError_t launch_leaf_assemble(Handle& h);
// compare: the panels already hold the root entries in use; flag[2] is set
// if a new value differs (no zeroing first)
hipError_t launch_fill_rowpanels(Handle& h, bool compare = false);
// mode 0: S from all panels; 1: also keep A_RR in h.Akeep; 2: S from the
// kept A_RR and the leaf fronts only
hipError_t launch_assemble_root(Handle& h, int mode);
hipError_t launch_rhs(Handle& h, const double* y, double* b);
hipError_t root_potrf(Handle& h);
hipError_t root_trsv_fwd(Handle& h, double* z);
hipError_t root_trsv_bwd(Handle& h, double* z);
hipError_t root_inv_apply(Handle& h, double* z, double* tmp);
int64_t root_inv_part_size(int64_t np);
hipError_t root_trtri(Handle& h);
hipError_t root_sweep(Handle& h);
// phase timing (opts.timing): event pairs on the handle's stream
void phase_begin(Handle& h, Phase p);
void phase_end(Handle& h, Phase p);
hipError_t root_sym_apply(Handle& h, double* z);
hipError_t root_lauum(Handle& h);
hipError_t launch_solve_pass(Handle& h, const double* b, double* x);
hipError_t launch_residual_dd(Handle& h, const double* b, const double* x,
                              double* r);
hipError_t launch_axpy_norms(Handle& h, double* x, const double* dx,
                             double* norms);
hipError_t launch_check_finite(Handle& h, const double* v, int64_t n);
hipError_t launch_selinv_leaves(Handle& h, double* d, double* part);
hipError_t launch_diag_root(Handle& h, double* d);
// out[k] = (A^-1)_{rows[k], cols[k]} from the root block of A^-1 (h.Zr) and
// the leaf panels (columns validated by the caller)
hipError_t launch_inv_entries(Handle& h, const int32_t* rows, const int32_t* cols,
                              double* out, int64_t k);
hipError_t launch_equilibrate(Handle& h);
// y = s x (mode 0), x / s (mode 1), s^2 x (mode 2) with the column scales
hipError_t launch_scale_vec(Handle& h, const double* x, double* y, int mode);
hipError_t fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t n);
hipError_t fill_f64(hipStream_t s, double* p, double v, int64_t n);

// dense kernels, exposed for tests of the root-front building blocks
enum GemmOp { kXC = 0, kKC = 1 };  // operand access, see k_gemm.hip
enum GemmKMask { kGemmKStartCol = 1, kGemmKEndRow = 2 };
// Tiles of C whose rows meet [r0, r1) or whose columns meet [c0, c1) are
// left alone (empty ranges: none).
struct GemmSkip {
  int r0 = 0, r1 = 0, c0 = 0, c1 = 0;  // rows [r0, r1), columns [c0, c1)
  int s0 = 0, s1 = 0;                  // the square [s0, s1) x [s0, s1)
};
hipError_t gemm(hipStream_t s, int bm, int bn, int opA, int opB,
                const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc, int M, int N, int K, double alpha,
                double beta, bool lower, bool kstart_diag,
                bool diag_mask = false, bool f32 = false,
                int kmask = 0, GemmSkip skip = GemmSkip(), int ksplit = 0);

// model-level loops (k_model.hip): empty-field pattern, fixed-order sums
int64_t sum_scratch_size();
hipError_t launch_sum(hipStream_t s, const double* v, int64_t n, double* part);
hipError_t launch_ef_rows(Handle& h, const double* val, const double* y,
                          const double* x, const int64_t* bg_pos, const double* t,
                          int stat);
hipError_t launch_ef_units(Handle& h, const int64_t* grp_ptr, const int32_t* grp_rows,
                           int n_u, const int64_t* bg_pos, const double* t, double* U,
                           double* val, bool update);

// Poisson likelihood (k_model.hip): per-row terms into h.vrow (c), w, r;
// flag[3] set if some e_i <= 0
hipError_t launch_cash_rows(Handle& h, const double* val, const double* x,
                            const double* y, double* w, double* r);
hipError_t launch_htr(Handle& h, const double* r, double* g);
// sum of a_i b_i into h.vsum[sum_scratch_size() - 1] (tmp: n doubles)
hipError_t launch_dot(Handle& h, const double* a, const double* b, double* tmp,
                      int64_t n);
hipError_t launch_axpy_to(Handle& h, const double* x, double a, const double* dx,
                          double* xt);
hipError_t launch_maxabs2(Handle& h, const double* dx, double a, const double* x,
                          double* nm);

// learned preconditioner and PCG (k_learned.hip)
int64_t lp_param_count(int hidden);
hipError_t lp_features(hipStream_t s, const double* diag_b, const double* diag_r,
                       const int32_t* root_of_col, float* phi, double* part,
                       int64_t n);
int lp_backward_blocks(int64_t n);
hipError_t lp_forward(hipStream_t s, int hidden, const float* params,
                      const float* phi, double* d, int64_t n);
hipError_t lp_backward(hipStream_t s, int hidden, const float* params,
                       const float* phi, const double* dLdd, const double* d,
                       double* part, double* grad, int64_t n);
hipError_t lp_adam(hipStream_t s, float* params, const double* grad, float* m,
                   float* v, int P, float lr, int step);
hipError_t vec_mul(hipStream_t s, const double* a, const double* b, double* out,
                   int64_t n);
hipError_t lp_err(hipStream_t s, const double* d, const double* v, const double* x,
                  double* e, int64_t n);
hipError_t lp_u(hipStream_t s, const double* d, const double* q, double sc,
                double* u, int64_t n);
hipError_t lp_dldd(hipStream_t s, const double* q, double sc, const double* v,
                   const double* rhs, const double* w, double* out, int64_t n);
hipError_t vec_neg(hipStream_t s, const double* x, double* y, int64_t n);
hipError_t vec_ones(hipStream_t s, double* x, int64_t n);
hipError_t dot_partials64(hipStream_t s, const double* a, const double* b,
                          double* part, int64_t n);
hipError_t dot_partials32(hipStream_t s, const float* a, const float* b,
                          double* part, int64_t n);
int dot_blocks();
hipError_t pcg_val32(Handle& h, float* v32);
hipError_t pcg_spmv32(Handle& h, const float* v32, const float* p, float* t,
                      float* q);
hipError_t vec_to64(hipStream_t s, const float* in, const double* d, double* out,
                    int64_t n);
hipError_t vec_to32(hipStream_t s, const double* in, const double* d, float* out,
                    int64_t n);
hipError_t vec_axpy32(hipStream_t s, float a, const float* x, float* y, int64_t n);
hipError_t vec_xpby32(hipStream_t s, const float* x, float b, float* y, int64_t n);
hipError_t vec_acc64(hipStream_t s, const float* e, double* x, int64_t n);
hipError_t vec_zero32(hipStream_t s, float* e, int64_t n);

}  // namespace spi

struct spi_handle {
  spi::Handle h;
};

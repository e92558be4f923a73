// Sparse-side kernels (gfx950): assembly of A = H^T W H into the fronts,
// extend-add of the leaf contribution blocks into the root, right-hand side,
// the leaf parts of the triangular solves and of the selected inversion,
// and the double-double residual of the refinement.
//
// Notation: a leaf front g holds p = |G| pivots (unknowns that share no
// measurement row with any other pivot, so its pivot block is diagonal) and
// the row structure U_g (root unknowns seen in its rows).  Its panel
// L_Ug = A_Ug,G L_GG^-T is stored dense, column-major, |U_g| x p.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "spi_internal.h"

namespace spi {

typedef double v4d __attribute__((ext_vector_type(4)));

// panel columns staged in LDS at a time by the selected-inversion tasks
constexpr int kQC = 16;

// Grid of a grid-stride kernel (capped: the kernel loops).
static int grid_for(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

// Grid of a one-wave-per-item kernel (4 waves per 256-thread block, no
// loop): exact.  Items are rows or columns of H (< 2^31), so it fits.
static unsigned wave_grid(int64_t items) {
  return (unsigned)std::max<int64_t>(1, (items + 3) / 4);
}

// ------------------------------------------------------------ value layout
// Gather H values and weights into front (slot) order.
__global__ void k_gather_slots(const double* __restrict__ val,
                               const double* __restrict__ w,
                               const int32_t* __restrict__ slot_row,
                               const int64_t* __restrict__ slot_leaf_src,
                               double* __restrict__ sw,
                               double* __restrict__ sleaf, int64_t m) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m;
       s += (int64_t)gridDim.x * blockDim.x) {
    sw[s] = w[slot_row[s]];
    int64_t e = slot_leaf_src[s];
    sleaf[s] = e >= 0 ? val[e] : 0.0;
  }
}

__global__ void k_gather_rr(const double* __restrict__ val,
                            const int64_t* __restrict__ rr_src,
                            double* __restrict__ rrval, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    rrval[k] = val[rr_src[k]];
}

hipError_t launch_gather_values(Handle& h) {
  const Analysis& a = h.an;
  if (a.n_slots)
    hipLaunchKernelGGL(k_gather_slots, dim3(grid_for(a.n_slots, 256)), dim3(256),
                       0, h.stream, h.val, h.w, h.d.slot_row, h.d.slot_leaf_src,
                       h.sw, h.sleaf, a.n_slots);
  int64_t nrr = (int64_t)a.rr_src.size();
  if (nrr)
    hipLaunchKernelGGL(k_gather_rr, dim3(grid_for(nrr, 256)), dim3(256), 0,
                       h.stream, h.val, h.d.rr_src, h.rrval, nrr);
  return hipGetLastError();
}

// ---------------------------------------------------------- leaf assembly
// One wave per leaf unknown l (front g, position q): accumulate
// A_ll = sum_r w_r h_rl^2 and the panel column A_Ug,l = sum_r w_r h_rl h_rU
// over the rows of l (sequentially, lanes over a row's entries, which have
// distinct positions), then L_ll = sqrt(A_ll) and the column / L_ll.  With
// kLds the column is accumulated in a wave-private LDS buffer of `cap`
// entries (dynamic LDS, cap >= |U| of every front) and written once;
// otherwise in place in the panel.
template <bool kLds>
__global__ __launch_bounds__(256) void k_leaf_assemble(
    const int32_t* __restrict__ leaf_grp, const int64_t* __restrict__ leaf_slot_ptr,
    const int64_t* __restrict__ grp_col_ptr, const int64_t* __restrict__ grp_U_ptr,
    const int64_t* __restrict__ grp_panel_off, const int64_t* __restrict__ slot_rr_ptr,
    const int32_t* __restrict__ rr_lpos, const double* __restrict__ rrval,
    const double* __restrict__ sw, const double* __restrict__ sleaf,
    double* panel, double* __restrict__ ldiag, int64_t* fail, int64_t n_leaf, int cap) {
  extern __shared__ double lbuf[];
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= n_leaf) return;
  const int g = leaf_grp[l];
  const int64_t q = l - grp_col_ptr[g];
  const int64_t nU = grp_U_ptr[g + 1] - grp_U_ptr[g];
  double* P = panel + grp_panel_off[g] + q * nU;
  double* acc = kLds ? lbuf + (int64_t)(threadIdx.x >> 6) * cap : P;
  for (int64_t u = lane; u < nU; u += 64) acc[u] = 0.0;
  __threadfence_block();
  double d = 0.0;
  for (int64_t s = leaf_slot_ptr[l]; s < leaf_slot_ptr[l + 1]; ++s) {
    const double t = sw[s] * sleaf[s];
    d += t * sleaf[s];
    for (int64_t k = slot_rr_ptr[s] + lane; k < slot_rr_ptr[s + 1]; k += 64)
      acc[rr_lpos[k]] += t * rrval[k];
    __threadfence_block();
  }
  bool bad = !(d > 0.0) || !isfinite(d);
  const double lll = bad ? 1.0 : sqrt(d);
  if (lane == 0) {
    ldiag[l] = lll;
    if (bad) atomicMin((unsigned long long*)fail, (unsigned long long)l);
  }
  const double inv = 1.0 / lll;
  for (int64_t u = lane; u < nU; u += 64) P[u] = acc[u] * inv;
}

hipError_t launch_leaf_assemble(Handle& h) {
  const Analysis& a = h.an;
  const int64_t nl = (int64_t)a.leaf_cols.size();
  if (!nl) return hipSuccess;
  int64_t max_u = 1;
  for (int64_t g = 0; g < a.n_groups; ++g)
    max_u = std::max<int64_t>(max_u, a.grp_U_ptr[g + 1] - a.grp_U_ptr[g]);
  // LDS per wave of the accumulating variant, at most (4 waves per workgroup)
  const int64_t lds_cap = h.opts.leaf_lds_cap > 0 ? h.opts.leaf_lds_cap : kLeafLdsCapMax;
  if (max_u <= lds_cap) {
    const int cap = (int)max_u;
    hipLaunchKernelGGL(k_leaf_assemble<true>, dim3(wave_grid(nl)), dim3(256),
                       4 * (size_t)cap * sizeof(double), h.stream, h.d.leaf_grp,
                       h.d.leaf_slot_ptr, h.d.grp_col_ptr, h.d.grp_U_ptr,
                       h.d.grp_panel_off, h.d.slot_rr_ptr, h.d.rr_lpos, h.rrval, h.sw,
                       h.sleaf, h.panel, h.ldiag, h.flag, nl, cap);
  } else {
    hipLaunchKernelGGL(k_leaf_assemble<false>, dim3(wave_grid(nl)), dim3(256), 0,
                       h.stream, h.d.leaf_grp, h.d.leaf_slot_ptr, h.d.grp_col_ptr,
                       h.d.grp_U_ptr, h.d.grp_panel_off, h.d.slot_rr_ptr,
                       h.d.rr_lpos, h.rrval, h.sw, h.sleaf, h.panel, h.ldiag,
                       h.flag, nl, 0);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ row panels
// Dense row panels for the assembly of A_RR: column q of a panel holds the
// root entries of its q-th row (zeros elsewhere); the row weights are kept
// apart.  Filled once per set of values.
__global__ void k_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// With `changed`, the panel already holds the values in use: any new value
// that differs sets *changed (one atomic per wave that saw one).  With
// `sbuf` (symmetric indefinite matrices, weights of either sign) rows are
// stored scaled by sqrt|w_r| in rpbuf and by sign(w_r) sqrt|w_r| in sbuf
// (same layout), so that Q S^T = sum_r w_r h_r h_r^T.
__global__ __launch_bounds__(256) void k_fill_rowpanels(
    const double* __restrict__ val, const double* __restrict__ w,
    const int32_t* __restrict__ rp_rows, const int64_t* __restrict__ rp_rowbase,
    const int64_t* __restrict__ rpe_ptr, const int32_t* __restrict__ rpe_pos,
    const int64_t* __restrict__ rpe_src, double* __restrict__ rpbuf,
    double* __restrict__ sbuf, int64_t nrows, int64_t* changed) {
  const int lane = threadIdx.x & 63;
  const int64_t pr = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pr >= nrows) return;
  double* col = rpbuf + rp_rowbase[pr];
  // rows are stored scaled by sqrt(w_r): the panel product is then
  // Q Q^T = sum_r w_r h_r h_r^T with no weights to load in the assembly
  const double wr = w[rp_rows[pr]];
  const double sw = sqrt(sbuf ? fabs(wr) : wr);
  const double sg = wr < 0.0 ? -1.0 : 1.0;
  bool diff = false;
  for (int64_t e = rpe_ptr[pr] + lane; e < rpe_ptr[pr + 1]; e += 64) {
    const double v = sw * val[rpe_src[e]];
    if (changed) diff |= col[rpe_pos[e]] != v;
    col[rpe_pos[e]] = v;
    if (sbuf) sbuf[rp_rowbase[pr] + rpe_pos[e]] = sg * v;
  }
  if (changed && __any(diff) && lane == 0) atomicOr((unsigned long long*)changed, 1ull);
}

hipError_t launch_fill_rowpanels(Handle& h, bool compare) {
  const Analysis& a = h.an;
  const int64_t nrows = (int64_t)a.rp_rows.size();
  if (!nrows) return hipSuccess;
  double* rpbuf = h.panel + a.grp_panel_off[a.n_groups];
  const int64_t total = a.rp_val_off[a.n_rp];
  // (the positions of a panel that no row entry fills stay zero)
  if (!compare)
    hipLaunchKernelGGL(k_zero, dim3(grid_for(total, 256 * 8)), dim3(256), 0,
                       h.stream, rpbuf, total);
  // (the signed copy's positions that no row entry fills stay zero too)
  if (!compare && h.panelS)
    hipLaunchKernelGGL(k_zero, dim3(grid_for(total, 256 * 8)), dim3(256), 0, h.stream,
                       h.panelS, total);
  hipLaunchKernelGGL(k_fill_rowpanels, dim3(wave_grid(nrows)), dim3(256), 0,
                     h.stream, h.val, h.w, h.d.rp_rows, h.d.rp_rowbase,
                     h.d.rpe_ptr, h.d.rpe_pos, h.d.rpe_src, rpbuf, h.panelS, nrows,
                     compare ? h.flag + 2 : nullptr);
  return hipGetLastError();
}

// --------------------------------------------------------- root assembly
// One workgroup per TS x TS lower tile (I, J) of the root front (TS = 64 or
// 128, chosen by the analysis: 8 or 16 waves).
// The tile is the sum of its incidences: update panel u (a leaf front's
// panel L_Ug with sign -1, or a row panel, stored as sqrt(w_r) h_r with sign
// +1) restricted to the positions of U that fall in the tile's rows
// (aI0 .. aI0 + nI) and columns (aJ0 .. aJ0 + nJ):
//   C[U[a] - TS I][U[b] - TS J] += sign sum_q Q[a][q] Q[b][q].
// The tile's incidences are staged in LDS in chunks, with their panel and
// index offsets resolved, so a wave's work on an incidence starts with no
// dependent descriptor loads.  Each wave takes one incidence at a time and
// computes it in 32 x 32 super-blocks of up to 2 x 2 blocks of 16 x 16 on
// the FP64 matrix cores; all loads of a super-block (indices, kAsmKC panel
// columns of both row blocks and both column blocks) are issued together
// before its MFMAs, and each loaded panel row serves two products.  Results
// are added into the LDS tile (LDS atomics, since waves work on different
// incidences); the tile is then written once.
//
// The work per super-block is mostly instruction issue, so it is kept to a
// few vector instructions per load and per result:
//  - panel and index loads are buffer loads on a per-update resource whose
//    range is the update's panel (or index list): a lane's offset is one
//    32-bit add per load, and every load past the range returns zero, so the
//    panel columns past k (the last MFMA step's padding) read as zeros on
//    both sides and rows past the incidence read finite values of the same
//    panel (their products land in output rows or columns that are dropped);
//  - a dropped output row or column is sent to spare LDS cells (rows
//    TS .. TS + 7, column TS) instead of being masked, so the LDS adds are
//    unconditional; entries above the diagonal of a diagonal tile are added
//    too and never written out;
//  - the sign of the leaf fronts' products is the MFMA's operand negation.
//
// Within a tile the leaf fronts' incidences come first ([beg, split)), the
// row panels' after ([split, end)).  Modes:
//   0  S = row panels + leaf fronts;
//   1  the same, and the row panels' sum alone (A_RR, the root block of
//      H^T W H) is also written to Akeep;
//   2  S = Akeep + leaf fronts (only the leaf fronts' values changed).
// incidences staged per pass (fewer passes, fewer barriers and less waiting
// on a tile's slowest wave: root assembly medium / large 3.96 / 488 ms with
// 64, 3.62 / 448 with 128, 3.43 / 425 with 256, 3.32 / 417 with 512; the
// 128 x 128 kernel's LDS then holds 159 KB of its 160)
constexpr int kAsmChunk = 512;
constexpr int kAsmKC = 20;      // panel columns per batch of loads
template <int TS>
constexpr int asm_threads() { return TS >= 128 ? 1024 : 512; }
constexpr int kAsmSpare = 8;    // spare LDS rows for dropped output rows
// word 3 of a raw buffer resource on gfx9 (32-bit data, no swizzle)
constexpr int kBufWord3 = 0x00020000;

// A wave-uniform 64-bit value moved to scalar registers.
__device__ inline int64_t uniform64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
__device__ inline int buf_load_i32(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}

// MFMA 16x16x4 FP64 step, the A operand negated when NEG (the leaf fronts).
template <bool NEG>
__device__ inline v4d mfma_step(double b, double a, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, NEG ? 1 : 0);
}

// One incidence, wave-uniform: the update's panel and index list (element
// offsets), the run starts in U and the run lengths.  The values are passed
// through readfirstlane where they are used, so the buffer resources and
// branch conditions built from them stay in scalar registers.
struct AsmInc {
  int64_t qo, uo;
  int pa, pb, nI, nJ, k, nU;
};

// One side of a super-block for kAsmKC panel columns: lane (lx, lk) holds
// rows s0 + 16 x + lx (x = 0, 1) of column kc + 4 s + lk; and the lane's
// root index of row s0 + (lane & 31).
struct AsmSide {
  double v[2][kAsmKC / 4];
  int u;
};

__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The update's panel (nU x k, column-major) and index list as buffer
// resources whose range is the panel (the analysis keeps nU k 8 and the
// offsets computed here below 2^31).
__device__ inline __amdgpu_buffer_rsrc_t asm_panel_rsrc(const AsmInc& d,
                                                        const double* panel) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(panel + uniform64(d.qo)), (short)0,
                                           uni(d.nU) * uni(d.k) * 8, kBufWord3);
}
__device__ inline __amdgpu_buffer_rsrc_t asm_index_rsrc(const AsmInc& d,
                                                        const int32_t* U) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(U + uniform64(d.uo)), (short)0,
                                           uni(d.nU) * 4, kBufWord3);
}

// Panel columns kc .. kc + kAsmKC - 1 of the run rows p0 + s0 + 16 x + lx,
// the second block only when `two` (the run reaches it).  Columns past k
// lie past the panel's range and read as zeros.
__device__ inline void asm_load_vals(const AsmInc& d, const double* panel, int p0, int s0,
                                     bool two, int kc, int lane, AsmSide& o) {
  const __amdgpu_buffer_rsrc_t rq = asm_panel_rsrc(d, panel);
  const int lx = lane & 15, lk = lane >> 4;
  const int cbytes = uni(d.nU) * 8;
  const int c0 = (p0 + s0 + lx) * 8 + (kc + lk) * cbytes;
#pragma unroll
  for (int s = 0; s < kAsmKC / 4; ++s) {
    o.v[0][s] = buf_load_f64(rq, c0 + 4 * s * cbytes);
    if (two) o.v[1][s] = buf_load_f64(rq, c0 + 128 + 4 * s * cbytes);
  }
}

__device__ inline void asm_load_side(const AsmInc& d, const double* panel, const int32_t* U,
                                     int p0, int s0, bool two, int lane, AsmSide& o) {
  o.u = buf_load_i32(asm_index_rsrc(d, U), (p0 + s0 + (lane & 31)) * 4);
  asm_load_vals(d, panel, p0, s0, two, 0, lane, o);
}

// The products of one super-block (run rows sa .. of A, sb .. of B) from
// the loaded sides; for k > kAsmKC the further column batches are loaded
// here into the same registers (the sides are then spent).  The results are
// added into the LDS tile Cf (row stride TS + 1).
template <bool NEG, int TS>
__device__ inline void asm_compute(const AsmInc& d, const double* panel,
                                   const double* panelB, int sa, int sb, AsmSide& A,
                                   AsmSide& B, double* Cf, int i0, int j0, int lane) {
  const int lx = lane & 15, lk = lane >> 4;
  const int nI = uni(d.nI), nJ = uni(d.nJ), k = uni(d.k);
  const bool a2 = sa + 16 < nI, b2 = sb + 16 < nJ;  // wave-uniform
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
  auto products = [&]() {
    // lane (lx, lk) item v of block (x, y): row sa + 16 x + lx, column
    // sb + 16 y + 4 v + lk (operand order as in the root GEMM)
#pragma unroll
    for (int s = 0; s < kAsmKC / 4; ++s) {
      acc[0][0] = mfma_step<NEG>(B.v[0][s], A.v[0][s], acc[0][0]);
      if (b2) acc[0][1] = mfma_step<NEG>(B.v[1][s], A.v[0][s], acc[0][1]);
      if (a2) {
        acc[1][0] = mfma_step<NEG>(B.v[0][s], A.v[1][s], acc[1][0]);
        if (b2) acc[1][1] = mfma_step<NEG>(B.v[1][s], A.v[1][s], acc[1][1]);
      }
    }
  };
  products();
  for (int kc = kAsmKC; kc < k; kc += kAsmKC) {
    asm_load_vals(d, panel, uni(d.pa), sa, a2, kc, lane, A);
    asm_load_vals(d, panelB, uni(d.pb), sb, b2, kc, lane, B);
    products();
  }
  // output rows and columns in the tile; dropped ones go to the spare cells
  int ra[2], rb[2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int r = __shfl(A.u, 16 * x + lx, 64);
    ra[x] = (sa + 16 * x + lx < nI ? r - i0 : TS + (lx & (kAsmSpare - 1))) * (TS + 1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = __shfl(B.u, 16 * x + 4 * v + lk, 64);
      rb[x][v] = sb + 16 * x + 4 * v + lk < nJ ? c - j0 : TS;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) atomicAdd(Cf + ra[0] + rb[0][v], acc[0][0][v]);
  if (b2) {
#pragma unroll
    for (int v = 0; v < 4; ++v) atomicAdd(Cf + ra[0] + rb[1][v], acc[0][1][v]);
  }
  if (a2) {
#pragma unroll
    for (int v = 0; v < 4; ++v) atomicAdd(Cf + ra[1] + rb[0][v], acc[1][0][v]);
    if (b2) {
#pragma unroll
      for (int v = 0; v < 4; ++v) atomicAdd(Cf + ra[1] + rb[1][v], acc[1][1][v]);
    }
  }
}

template <int TS>
__global__ __launch_bounds__(asm_threads<TS>()) void k_assemble_root(
    const int32_t* __restrict__ tile_order, const int64_t* __restrict__ inc_ptr,
    const int64_t* __restrict__ inc_split,
    const int32_t* __restrict__ inc, const int64_t* __restrict__ up_U_off,
    const int64_t* __restrict__ up_Q_off, const int32_t* __restrict__ up_nU,
    const int32_t* __restrict__ up_k, const int32_t* __restrict__ U,
    const double* __restrict__ panel, const double* __restrict__ panelB,
    double* __restrict__ S, double* __restrict__ Akeep, int64_t ld, int64_t n_root,
    int mode) {
  __shared__ double C[TS + kAsmSpare][TS + 1];
  __shared__ int64_t s_q[kAsmChunk], s_u[kAsmChunk];
  __shared__ int32_t s_next;  // next incidence of the chunk to hand out
  __shared__ int32_t s_ab[kAsmChunk][2], s_nU[kAsmChunk], s_k[kAsmChunk],
      s_n[kAsmChunk];
  const int t = tile_order[xcd_remap<64>(blockIdx.x, gridDim.x)];
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int64_t i0 = (int64_t)I * TS, j0 = (int64_t)J * TS;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // (uniform)
  constexpr int kThreads = asm_threads<TS>(), NW = kThreads / 64;
  if (mode == 2) {  // start from the kept A_RR tile
    for (int e = tid; e < TS * TS; e += kThreads) {
      const int a = e % TS, b = e / TS;
      C[a][b] = (I == J && a < b) ? 0.0 : Akeep[(i0 + a) + (j0 + b) * ld];
    }
  } else {
    for (int e = tid; e < TS * TS; e += kThreads) {
      const int a = e % TS, b = e / TS;
      C[a][b] = (I == J && a == b && i0 + a >= n_root) ? 1.0 : 0.0;
    }
  }
  double* Cf = &C[0][0];
  // Sum the incidences [q_beg, q_end) into C, negated when NEG.
  auto accumulate = [&](auto neg_tag, int64_t q_beg, int64_t q_end) {
    constexpr bool NEG = decltype(neg_tag)::value;
    for (int64_t c0 = q_beg; c0 < q_end; c0 += kAsmChunk) {
      const int nc = (int)min((int64_t)kAsmChunk, q_end - c0);
      __syncthreads();  // previous chunk consumed (and C initialised)
      for (int e = tid; e < nc; e += kThreads) {
        const int32_t* p = inc + 4 * (c0 + e);
        const int u = p[0];
        s_q[e] = up_Q_off[u];
        s_u[e] = up_U_off[u];
        s_ab[e][0] = p[1];
        s_ab[e][1] = p[2];
        s_nU[e] = up_nU[u];
        s_k[e] = up_k[u];
        s_n[e] = p[3];
      }
      if (tid == 0) s_next = NW;  // waves start on incidences 0 .. NW - 1
      __syncthreads();
      // A wave takes incidence `wave` first, then whichever is next when it
      // is done (an LDS counter), so the waves of a tile finish together;
      // each incidence by row strips of
      // 32: with k <= kAsmKC the strip's A side is loaded once for all its
      // column super-blocks.  In a diagonal tile an incidence pairs a run
      // with itself: super-blocks above the diagonal are skipped and those
      // on it take their B side from the A side (unless it is the signed
      // copy).
      const bool diag = I == J;
      // B side: the leaf fronts' panels, or the row panels' (signed) copy
      const double* pB = NEG ? panel : panelB;
      for (int q = wave; q < nc;) {
        AsmInc d;
        d.qo = uniform64(s_q[q]);
        d.uo = uniform64(s_u[q]);
        d.pa = uni(s_ab[q][0]);
        d.pb = uni(s_ab[q][1]);
        d.nU = uni(s_nU[q]);
        d.k = uni(s_k[q]);
        const int nn = uni(s_n[q]);
        d.nI = nn & 0xffff;
        d.nJ = nn >> 16;
        const bool multi = d.k > kAsmKC;  // further column batches
        for (int sa = 0; sa < d.nI; sa += 32) {
          const bool a2 = sa + 16 < d.nI;
          AsmSide A, B;
          asm_load_side(d, panel, U, d.pa, sa, a2, lane, A);
          const int sb_end = diag ? sa + 1 : d.nJ;
          for (int sb = 0; sb < sb_end; sb += 32) {
            if (multi && sb > 0) asm_load_side(d, panel, U, d.pa, sa, a2, lane, A);
            if (diag && sb == sa && !multi && pB == panel) B = A;
            else asm_load_side(d, pB, U, d.pb, sb, sb + 16 < d.nJ, lane, B);
            asm_compute<NEG, TS>(d, panel, pB, sa, sb, A, B, Cf, (int)i0, (int)j0, lane);
          }
        }
        int nq = 0;
        if (lane == 0) nq = atomicAdd(&s_next, 1);
        q = __builtin_amdgcn_readfirstlane(nq);
      }
    }
  };
  auto write_tile = [&](double* out) {
    __syncthreads();
    for (int e = tid; e < TS * TS; e += kThreads) {
      const int a = e % TS, b = e / TS;
      if (I == J && a < b) continue;
      out[(i0 + a) + (j0 + b) * ld] = C[a][b];
    }
  };
  using neg_t = std::integral_constant<bool, true>;
  using pos_t = std::integral_constant<bool, false>;
  const int64_t q_beg = inc_ptr[t], q_split = inc_split[t], q_end = inc_ptr[t + 1];
  if (mode == 1) {
    accumulate(pos_t(), q_split, q_end);  // row panels: A_RR
    write_tile(Akeep);
    accumulate(neg_t(), q_beg, q_split);  // leaf fronts
  } else if (mode == 2) {
    accumulate(neg_t(), q_beg, q_split);
  } else {
    accumulate(neg_t(), q_beg, q_split);
    accumulate(pos_t(), q_split, q_end);
  }
  write_tile(S);
}

hipError_t launch_assemble_root(Handle& h, int mode) {
  const Analysis& a = h.an;
  if (!a.n_tiles) return hipSuccess;
  // the row panels' B side: the signed copy for indefinite matrices (its
  // offsets are the row panels' offsets in the panel buffer less the leaf
  // panels' total)
  const double* panelB =
      h.panelS ? h.panelS - a.grp_panel_off[a.n_groups] : h.panel;
  if (a.asm_tile == kAsmTileLarge)
    hipLaunchKernelGGL(k_assemble_root<kAsmTileLarge>, dim3((unsigned)a.n_tiles),
                       dim3(asm_threads<kAsmTileLarge>()), 0, h.stream, h.d.tile_order,
                       h.d.inc_ptr, h.d.inc_split, h.d.inc, h.d.up_U_off, h.d.up_Q_off,
                       h.d.up_nU, h.d.up_k, h.d.U, h.panel, panelB, h.S, h.Akeep, a.n_pad,
                       a.n_root, mode);
  else
    hipLaunchKernelGGL(k_assemble_root<kAsmTileSmall>, dim3((unsigned)a.n_tiles),
                       dim3(asm_threads<kAsmTileSmall>()), 0, h.stream, h.d.tile_order,
                       h.d.inc_ptr, h.d.inc_split, h.d.inc, h.d.up_U_off, h.d.up_Q_off,
                       h.d.up_nU, h.d.up_k, h.d.U, h.panel, panelB, h.S, h.Akeep, a.n_pad,
                       a.n_root, mode);
  return hipGetLastError();
}

// ------------------------------------------------------------ equilibration
// Symmetric diagonal scaling A -> S A S with S = diag(s), applied as a column
// scaling of H (H -> H S).  s_c is the power of two 2^-floor(log2|A_cc| / 2),
// A_cc = sum_r w_r h_rc^2, so the scaled |diagonal| lies in [1, 4).  Powers of
// two make the scaling exact: every product, sum, square root and quotient
// of the factorisation of S A S is the scaled image of the same operation
// on A, so it changes no rounding; what it buys is range (the FP32
// intermediates of the mixed-precision path stay finite whatever the
// column scales of H).  Columns with a zero or non-finite diagonal keep
// s_c = 1 and fail at their pivot as before.
// valc[k] = val[csc_pos[k]]: H's values in column order, so that the
// column-wise kernels (diagonal, right-hand side, residual) read them
// contiguously instead of gathering them from the row-ordered copy.
// A NaN or infinity among the values sets *bad (one atomic per wave that
// saw one): the factorisation reports it.
__global__ void k_gather_csc(const double* __restrict__ val,
                             const int64_t* __restrict__ csc_pos,
                             double* __restrict__ valc, int64_t nnz,
                             int64_t* bad) {
  bool nonfinite = false;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double v = val[csc_pos[k]];
    nonfinite |= !isfinite(v);
    valc[k] = v;
  }
  if (__any(nonfinite) && (threadIdx.x & 63) == 0)
    atomicOr((unsigned long long*)bad, 1ull);
}

__global__ void k_check_finite(const double* __restrict__ v, int64_t n, int64_t* bad) {
  bool nonfinite = false;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    nonfinite |= !isfinite(v[k]);
  if (__any(nonfinite) && (threadIdx.x & 63) == 0)
    atomicOr((unsigned long long*)bad, 1ull);
}

hipError_t launch_check_finite(Handle& h, const double* v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, 256 * 8)), dim3(256), 0,
                     h.stream, v, n, h.flag + 1);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_col_scale(
    const int64_t* __restrict__ colptr, const int32_t* __restrict__ csc_row,
    double* __restrict__ valc, const double* __restrict__ w,
    double* __restrict__ diag, double* __restrict__ scale, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  double d = 0.0;
  for (int64_t k = colptr[c] + lane; k < colptr[c + 1]; k += 64) {
    const double v = valc[k];
    d += w[csc_row[k]] * v * v;
  }
  for (int off = 32; off > 0; off >>= 1) d += __shfl_down(d, off, 64);
  d = __shfl(d, 0, 64);
  double s = 1.0;
  const double ad = fabs(d);  // (a negative diagonal: indefinite matrices)
  if (ad > 0.0 && ad <= 1.7976931348623157e308) {
    const int e = ilogb(ad);    // |d| = m 2^e, 1 <= m < 2
    s = ldexp(1.0, -(e >> 1));  // arithmetic shift: floor(e / 2)
  }
  if (lane == 0) {
    diag[c] = d;
    if (scale) scale[c] = s;
  }
  if (scale)  // the column-ordered copy takes the scale here (exact)
    for (int64_t k = colptr[c] + lane; k < colptr[c + 1]; k += 64) valc[k] *= s;
}

__global__ void k_scale_vals(double* __restrict__ val, const int32_t* __restrict__ col,
                             const double* __restrict__ scale, int64_t nnz) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    val[e] *= scale[col[e]];
}

// y = s x (mode 0), x / s (mode 1), s^2 x (mode 2); exact for powers of two.
__global__ void k_scale_vec(const double* x, const double* __restrict__ s, double* y,
                            int64_t n, int mode) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double si = s[i];
    y[i] = mode == 0 ? x[i] * si : (mode == 1 ? x[i] / si : x[i] * si * si);
  }
}

// diag(A) into h.diagA, the column-ordered copy of H's values, and with
// opts.equilibrate the column scales and the scaled values of H (both
// copies).
hipError_t launch_equilibrate(Handle& h) {
  const Analysis& a = h.an;
  const bool eq = h.opts.equilibrate != 0;
  if (a.nnz)
    hipLaunchKernelGGL(k_gather_csc, dim3((unsigned)std::min<int64_t>(
                                         (a.nnz + 255) / 256, 16384)),
                       dim3(256), 0, h.stream, h.val, h.d.csc_pos, h.valc, a.nnz,
                       h.flag + 1);
  hipLaunchKernelGGL(k_col_scale, dim3(wave_grid(a.n)), dim3(256), 0, h.stream,
                     h.d.colptr, h.d.csc_row, h.valc, h.w, h.diagA,
                     eq ? h.colscale : nullptr, a.n);
  if (eq && a.nnz)
    hipLaunchKernelGGL(k_scale_vals, dim3((unsigned)std::min<int64_t>(
                                         (a.nnz + 255) / 256, 16384)),
                       dim3(256), 0, h.stream, h.val, h.d.col, h.colscale, a.nnz);
  return hipGetLastError();
}

hipError_t launch_scale_vec(Handle& h, const double* x, double* y, int mode) {
  const int64_t n = h.an.n;
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_scale_vec, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, h.stream, x, h.colscale, y, n, mode);
  return hipGetLastError();
}

// Fill kernels (used instead of hipMemsetAsync so that a captured graph
// holds only kernel nodes).
__global__ void k_fill_i64(int64_t* p, int64_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t fill_i64(hipStream_t s, int64_t* p, int64_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_f64(hipStream_t s, double* p, double v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rhs
// b_c = sum_{r} h_rc w_r y_r over the column's entries (one wave per column).
__global__ __launch_bounds__(256) void k_rhs(const int64_t* __restrict__ colptr,
                                             const int32_t* __restrict__ csc_row,
                                             const double* __restrict__ valc,
                                             const double* __restrict__ w,
                                             const double* __restrict__ y,
                                             const double* __restrict__ scale,
                                             double* __restrict__ b, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  double s = 0.0;
  for (int64_t k = colptr[c] + lane; k < colptr[c + 1]; k += 64) {
    int32_t r = csc_row[k];
    s += valc[k] * (w[r] * y[r]);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  // val holds H S: undo the (power-of-two, exact) column scale
  if (lane == 0) b[c] = scale ? s / scale[c] : s;
}

hipError_t launch_rhs(Handle& h, const double* y, double* b) {
  hipLaunchKernelGGL(k_rhs, dim3(wave_grid(h.an.n)), dim3(256), 0, h.stream,
                     h.d.colptr, h.d.csc_row, h.valc, h.w, y,
                     h.opts.equilibrate ? h.colscale : nullptr, b, h.an.n);
  return hipGetLastError();
}

// ------------------------------------------------ double-double residual
// r = b - H^T W H x with every product and sum in double-double
// (error-free transformations: two_sum, two_prod by fma), rounded once.
struct dd {
  double hi, lo;
};
__device__ inline dd two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  double lo = s.lo + a.lo + b.lo;
  return two_sum(s.hi, lo);
}
__device__ inline dd dd_mul_d(dd a, double b) {
  double p = a.hi * b;
  double e = fma(a.hi, b, -p);
  return two_sum(p, e + a.lo * b);
}
__device__ inline dd prod_dd(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ inline dd shfl_down_dd(dd v, int off) {
  return {__shfl_down(v.hi, off, 64), __shfl_down(v.lo, off, 64)};
}

// t_r = w_r * (H x)_r in double-double (one wave per row).
__global__ __launch_bounds__(256) void k_hx_dd(const int64_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ val,
                                               const double* __restrict__ w,
                                               const double* __restrict__ x,
                                               double* __restrict__ t, int64_t m) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  dd s{0.0, 0.0};
  for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64)
    s = dd_add(s, prod_dd(val[e], x[col[e]]));
  for (int off = 32; off > 0; off >>= 1) s = dd_add(s, shfl_down_dd(s, off));
  if (lane == 0) {
    dd v = dd_mul_d(s, w[r]);
    t[2 * r] = v.hi;
    t[2 * r + 1] = v.lo;
  }
}

// r_c = b_c - sum_r h_rc t_r in double-double (one wave per column).
__global__ __launch_bounds__(256) void k_htt_dd(const int64_t* __restrict__ colptr,
                                                const int32_t* __restrict__ csc_row,
                                                const double* __restrict__ valc,
                                                const double* __restrict__ t,
                                                const double* __restrict__ b,
                                                double* __restrict__ r, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  dd s{0.0, 0.0};
  for (int64_t k = colptr[c] + lane; k < colptr[c + 1]; k += 64) {
    const int32_t row = csc_row[k];
    const double h = valc[k];
    dd tr{t[2 * row], t[2 * row + 1]};
    s = dd_add(s, dd_mul_d(tr, h));
  }
  for (int off = 32; off > 0; off >>= 1) s = dd_add(s, shfl_down_dd(s, off));
  if (lane == 0) {
    dd v = dd_add(dd{b ? b[c] : 0.0, 0.0}, dd{-s.hi, -s.lo});
    r[c] = v.hi + v.lo;
  }
}

hipError_t launch_residual_dd(Handle& h, const double* b, const double* x,
                              double* r) {
  const Analysis& a = h.an;
  hipLaunchKernelGGL(k_hx_dd, dim3(wave_grid(a.m)), dim3(256), 0, h.stream,
                     h.d.rowptr, h.d.col, h.val, h.w, x, h.vdd, a.m);
  hipLaunchKernelGGL(k_htt_dd, dim3(wave_grid(a.n)), dim3(256), 0, h.stream,
                     h.d.colptr, h.d.csc_row, h.valc, h.vdd, b, r, a.n);
  return hipGetLastError();
}

// x += dx; norms[0] = max |dx|, norms[1] = max |x| (as ordered bit patterns
// of non-negative doubles, reduced with atomicMax).
__global__ void k_axpy_norms(double* __restrict__ x, const double* __restrict__ dx,
                             unsigned long long* norms, int64_t n) {
  double mdx = 0.0, mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = x[i] + dx[i];
    x[i] = v;
    mdx = fmax(mdx, fabs(dx[i]));
    mx = fmax(mx, fabs(v));
  }
  for (int off = 32; off > 0; off >>= 1) {
    mdx = fmax(mdx, __shfl_down(mdx, off, 64));
    mx = fmax(mx, __shfl_down(mx, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&norms[0], (unsigned long long)__double_as_longlong(mdx));
    atomicMax(&norms[1], (unsigned long long)__double_as_longlong(mx));
  }
}

hipError_t launch_axpy_norms(Handle& h, double* x, const double* dx,
                             double* norms) {
  hipLaunchKernelGGL(k_axpy_norms, dim3(grid_for(h.an.n, 256)), dim3(256), 0,
                     h.stream, x, dx, (unsigned long long*)norms, h.an.n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- solves
// Permute into the elimination order: leaf values y_l = b[leaf_col] / L_ll
// (forward substitution at the leaves), root values z_i = b[root_col].
__global__ void k_fwd_leaf(const double* __restrict__ b,
                           const int32_t* __restrict__ leaf_cols,
                           const double* __restrict__ ldiag,
                           double* __restrict__ vleaf, int64_t n_leaf) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_leaf;
       l += (int64_t)gridDim.x * blockDim.x)
    vleaf[l] = b[leaf_cols[l]] / ldiag[l];
}

// Forward substitution's update of the root, z_R = b_R - sum_g L_Ug y_g, in
// two deterministic passes.  (1) One workgroup per leaf front: t_g = L_Ug y_g,
// reading the column-major panel along U (coalesced).  (2) One wave per root
// unknown i: z_i = b_i - sum of t_g[u] over the (front, position) pairs
// that contain i, in a fixed order.
__global__ __launch_bounds__(256) void k_fwd_front(
    const int64_t* __restrict__ grp_U_ptr, const int64_t* __restrict__ grp_col_ptr,
    const int64_t* __restrict__ grp_panel_off, const double* __restrict__ panel,
    const double* __restrict__ vleaf, double* __restrict__ t, int64_t n_groups) {
  const int64_t g = blockIdx.x;  // one workgroup per front
  if (g >= n_groups) return;
  const int64_t u0 = grp_U_ptr[g], nU = grp_U_ptr[g + 1] - u0;
  const int64_t c0 = grp_col_ptr[g];
  const int p = (int)(grp_col_ptr[g + 1] - c0);
  const double* P = panel + grp_panel_off[g];
  for (int64_t u = threadIdx.x; u < nU; u += 256) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};  // independent chains, loads in flight
    int q = 0;
    for (; q + 4 <= p; q += 4)
#pragma unroll
      for (int e = 0; e < 4; ++e) s[e] += P[u + (q + e) * nU] * vleaf[c0 + q + e];
    for (; q < p; ++q) s[0] += P[u + q * nU] * vleaf[c0 + q];
    t[u0 + u] = (s[0] + s[1]) + (s[2] + s[3]);
  }
}

__global__ __launch_bounds__(256) void k_fwd_root_gather(
    const double* __restrict__ b, const int32_t* __restrict__ root_cols,
    const int64_t* __restrict__ rinc_ptr, const int32_t* __restrict__ rinc_grp,
    const int32_t* __restrict__ rinc_u, const int64_t* __restrict__ grp_U_ptr,
    const double* __restrict__ t, double* __restrict__ z, int64_t n_root,
    int64_t n_pad) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n_pad) return;
  if (i >= n_root) {
    if (lane == 0) z[i] = 0.0;
    return;
  }
  double s = 0.0;
  for (int64_t k = rinc_ptr[i] + lane; k < rinc_ptr[i + 1]; k += 64)
    s += t[grp_U_ptr[rinc_grp[k]] + rinc_u[k]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) z[i] = b[root_cols[i]] - s;
}

// Backward at the leaves: x_l = (y_l - L_Ul^T x_U) / L_ll (one wave per
// leaf), then scatter root and leaf values to the original order.
__global__ __launch_bounds__(256) void k_bwd_leaf(
    const int32_t* __restrict__ leaf_grp, const int64_t* __restrict__ grp_col_ptr,
    const int64_t* __restrict__ grp_U_ptr, const int32_t* __restrict__ U,
    const int64_t* __restrict__ grp_panel_off, const double* __restrict__ panel,
    const double* __restrict__ ldiag, const int32_t* __restrict__ leaf_cols,
    const double* __restrict__ vleaf, const double* __restrict__ z,
    double* __restrict__ x, int64_t n_leaf) {
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= n_leaf) return;
  const int g = leaf_grp[l];
  const int64_t q = l - grp_col_ptr[g];
  const int64_t u0 = grp_U_ptr[g], nU = grp_U_ptr[g + 1] - u0;
  const double* P = panel + grp_panel_off[g] + q * nU;
  double s = 0.0;
  for (int64_t u = lane; u < nU; u += 64) s += P[u] * z[U[u0 + u]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[leaf_cols[l]] = (vleaf[l] - s) / ldiag[l];
}

__global__ void k_scatter_root(const double* __restrict__ z,
                               const int32_t* __restrict__ root_cols,
                               double* __restrict__ x, int64_t n_root) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_root;
       i += (int64_t)gridDim.x * blockDim.x)
    x[root_cols[i]] = z[i];
}

hipError_t launch_solve_pass(Handle& h, const double* b, double* x) {
  const Analysis& a = h.an;
  const int64_t nl = (int64_t)a.leaf_cols.size();
  hipError_t e;
  if (nl)
    hipLaunchKernelGGL(k_fwd_leaf, dim3(grid_for(nl, 256)), dim3(256), 0,
                       h.stream, b, h.d.leaf_cols, h.ldiag, h.vleaf, nl);
  if (a.n_pad) {
    if (a.n_groups)
      hipLaunchKernelGGL(k_fwd_front, dim3((unsigned)a.n_groups), dim3(256), 0,
                         h.stream, h.d.grp_U_ptr, h.d.grp_col_ptr, h.d.grp_panel_off,
                         h.panel, h.vleaf, h.vfront, a.n_groups);
    hipLaunchKernelGGL(k_fwd_root_gather, dim3(wave_grid(a.n_pad)), dim3(256),
                       0, h.stream, b, h.d.root_cols, h.d.rinc_ptr, h.d.rinc_grp,
                       h.d.rinc_u, h.d.grp_U_ptr, h.vfront, h.vroot, a.n_root,
                       a.n_pad);
    if (h.swept) {
      if ((e = root_sym_apply(h, h.vroot)) != hipSuccess) return e;
    } else if (h.have_inv) {
      if ((e = root_inv_apply(h, h.vroot, h.vroot2)) != hipSuccess) return e;
    } else {
      if ((e = root_trsv_fwd(h, h.vroot)) != hipSuccess) return e;
      if ((e = root_trsv_bwd(h, h.vroot)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scatter_root, dim3(grid_for(a.n_root, 256)), dim3(256),
                       0, h.stream, h.vroot, h.d.root_cols, x, a.n_root);
  }
  if (nl)
    hipLaunchKernelGGL(k_bwd_leaf, dim3(wave_grid(nl)), dim3(256), 0,
                       h.stream, h.d.leaf_grp, h.d.grp_col_ptr, h.d.grp_U_ptr,
                       h.d.U, h.d.grp_panel_off, h.panel, h.ldiag, h.d.leaf_cols,
                       h.vleaf, h.vroot, x, nl);
  return hipGetLastError();
}

// ------------------------------------------------- selected inversion
// Root: d[root_col_i] = Z_ii.
__global__ void k_diag_root(const double* __restrict__ Z, int64_t ld,
                            const int32_t* __restrict__ root_cols,
                            double* __restrict__ d, int64_t n_root) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_root;
       i += (int64_t)gridDim.x * blockDim.x)
    d[root_cols[i]] = Z[i + i * ld];
}

hipError_t launch_diag_root(Handle& h, double* d) {
  if (!h.an.n_root) return hipSuccess;
  hipLaunchKernelGGL(k_diag_root, dim3(grid_for(h.an.n_root, 256)), dim3(256),
                     0, h.stream, h.Zr, h.an.n_pad, h.d.root_cols, d,
                     h.an.n_root);
  return hipGetLastError();
}

// General entries of A^-1 (covariances), one workgroup per requested entry
// (i, j), from the root block Z' = (S A S)^-1 restricted to the root and
// the leaf panels (the same relations as the leaf selected inversion: for a
// leaf l of front g with panel column c_l over U_g and pivot L_ll,
//   Z'_{r,l} = -(Z'_{r,U_g} c_l) / L_ll              (r a root unknown),
//   Z'_{l,k} = [l = k] / L_ll^2 + c_l^T Z'_{U_g,U_h} c_k / (L_ll L_kk)
// for leaves l, k of fronts g, h), then (A^-1)_ij = s_i s_j Z'_ij with the
// equilibration scales.  Z' is read from its lower storage.
__device__ inline double zlow(const double* Z, int64_t ld, int64_t a, int64_t b) {
  return a >= b ? Z[a + b * ld] : Z[b + a * ld];
}

__global__ __launch_bounds__(256) void k_inv_entries(
    const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
    const int32_t* __restrict__ root_of_col, const int32_t* __restrict__ leaf_of_col,
    const int32_t* __restrict__ leaf_grp, const int64_t* __restrict__ grp_col_ptr,
    const int64_t* __restrict__ grp_U_ptr, const int32_t* __restrict__ U,
    const int64_t* __restrict__ grp_panel_off, const double* __restrict__ panel,
    const double* __restrict__ ldiag, const double* __restrict__ Z, int64_t ld,
    const double* __restrict__ scale, double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x;
  int32_t i = rows[k], j = cols[k];
  int32_t ri = root_of_col[i], rj = root_of_col[j];
  if (ri >= 0 && rj < 0) {  // leaf first
    const int32_t x = i; i = j; j = x;
    ri = root_of_col[i];
    rj = root_of_col[j];
  }
  const double sij = scale ? scale[i] * scale[j] : 1.0;
  double v = 0.0;
  if (ri >= 0) {  // both root
    if (tid == 0) out[k] = sij * zlow(Z, ld, ri, rj);
    return;
  }
  // i is a leaf: front g, panel column c_l over U_g
  const int32_t l = leaf_of_col[i];
  const int32_t g = leaf_grp[l];
  const int64_t ug = grp_U_ptr[g], nUg = grp_U_ptr[g + 1] - ug;
  const double* cl = panel + grp_panel_off[g] + (l - grp_col_ptr[g]) * nUg;
  const double Lll = ldiag[l];
  if (rj >= 0) {  // leaf-root
    for (int64_t a = tid; a < nUg; a += 256) v += zlow(Z, ld, U[ug + a], rj) * cl[a];
  } else {        // leaf-leaf
    const int32_t q = leaf_of_col[j];
    const int32_t gh = leaf_grp[q];
    const int64_t uh = grp_U_ptr[gh], nUh = grp_U_ptr[gh + 1] - uh;
    const double* ck = panel + grp_panel_off[gh] + (q - grp_col_ptr[gh]) * nUh;
    for (int64_t b = tid; b < nUh; b += 256) {
      const int64_t rb = U[uh + b];
      const double cb = ck[b];
      double t = 0.0;
      for (int64_t a = 0; a < nUg; ++a) t += cl[a] * zlow(Z, ld, U[ug + a], rb);
      v += t * cb;
    }
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    double r;
    if (rj >= 0) {
      r = -s / Lll;
    } else {
      const int32_t q = leaf_of_col[j];
      const double Lkk = ldiag[q];
      r = s / (Lll * Lkk) + (q == l ? 1.0 / (Lll * Lll) : 0.0);
    }
    out[k] = sij * r;
  }
}

hipError_t launch_inv_entries(Handle& h, const int32_t* rows, const int32_t* cols,
                              double* out, int64_t k) {
  if (k <= 0) return hipSuccess;
  const int64_t chunk = int64_t(1) << 24;
  for (int64_t k0 = 0; k0 < k; k0 += chunk) {
    const int64_t c = std::min(chunk, k - k0);
    hipLaunchKernelGGL(k_inv_entries, dim3((unsigned)c), dim3(256), 0, h.stream,
                       rows + k0, cols + k0, h.d.root_of_col, h.d.leaf_of_col,
                       h.d.leaf_grp, h.d.grp_col_ptr, h.d.grp_U_ptr, h.d.U,
                       h.d.grp_panel_off, h.panel, h.ldiag, h.Zr, h.an.n_pad,
                       h.opts.equilibrate ? h.colscale : nullptr, out + k0);
  }
  return hipGetLastError();
}

// Leaves (Takahashi: Z L = L^-T): for pivot l of front g with panel column
// c = L_Ul, Z_Ul = -Z_UU c / L_ll and Z_ll = (1 + c^T Z_UU c) / L_ll^2.
// Task (g, I, J) adds its block of the quadratic forms c^T Z_UU c for all
// pivots of g: the full square block for I == J, twice the block for I > J.
__global__ __launch_bounds__(256, 6) void k_selinv_leaf(
    const int32_t* __restrict__ tasks, const int32_t* __restrict__ order,
    const int64_t* __restrict__ grp_U_ptr,
    const int32_t* __restrict__ U, const int64_t* __restrict__ grp_col_ptr,
    const int64_t* __restrict__ grp_panel_off, const double* __restrict__ panel,
    const double* __restrict__ Z, int64_t ld, const int64_t* __restrict__ grp_task_ptr,
    const int64_t* __restrict__ task_part_off, double* __restrict__ part) {
  __shared__ double PI[kQC][kET + 1];  // padded rows: the MFMA operand reads
  __shared__ double PJ[kQC][kET + 1];  // of 16 different q are conflict-free
  __shared__ double red[4][kQC];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tk = order[xcd_remap<64>(blockIdx.x, gridDim.x)];
  const int g = tasks[3 * tk], I = tasks[3 * tk + 1], J = tasks[3 * tk + 2];
  const int p = (int)(grp_col_ptr[g + 1] - grp_col_ptr[g]);
  if (p == 0) return;
  const int64_t nU = grp_U_ptr[g + 1] - grp_U_ptr[g];
  const int32_t* Ug = U + grp_U_ptr[g];
  const int I0 = I * kET, J0 = J * kET;
  const int na = (int)min<int64_t>(kET, nU - I0), nb = (int)min<int64_t>(kET, nU - J0);
  const double* Pg = panel + grp_panel_off[g];
  // Three round trips to memory per task at most: (1) the panel values of
  // the first pivot chunk and the root indices of the two U ranges, (2)
  // every gather of the Z_UU block at once (clamped, always valid
  // addresses), (3) the panel values of a second chunk (fronts of more than
  // kQC pivots).  No value waits for a load until it is used: the Z entries
  // of rows or columns past the ranges are not zeroed, the zero padding of
  // the panel blocks in LDS cancels them (a finite Z entry times zero).
  constexpr int kPP = kQC * kET / 256;
  double pi[kPP], pj[kPP];
  auto load_panel = [&](int q0, int pc) {
#pragma unroll
    for (int i = 0; i < kPP; ++i) {  // all panel loads in flight together
      const int e = t + 256 * i, r = e % kET, q = e / kET;
      const int64_t col = (int64_t)(q0 + min(q, pc - 1)) * nU;
      pi[i] = Pg[col + I0 + min(r, na - 1)];
      pj[i] = Pg[col + J0 + min(r, nb - 1)];
    }
  };
  load_panel(0, min(kQC, p));
  __shared__ int32_t sU[2][kET];
  if (t < 2 * kET) {
    const int side = t / kET, a = t % kET;
    const int len = side ? nb : na, base = side ? J0 : I0;
    sU[side][a] = Ug[base + min(a, len - 1)];
  }
  __syncthreads();
  // The block Z_IJ stays in registers as the first operand of the FP64
  // matrix-core products: wave w holds rows a = 16 w + lx, lane (lx, lk)
  // the columns b = 4 s + lk for the 16 steps s over b.
  const int lx = lane & 15, lk = lane >> 4;
  const int64_t ua = sU[0][16 * wave + lx];
  double zf[kET / 4];
#pragma unroll
  for (int st = 0; st < kET / 4; ++st) {
    const int64_t ub = sU[1][4 * st + lk];
    zf[st] = ua >= ub ? Z[ua + ub * ld] : Z[ub + ua * ld];  // lower storage
  }
  const double fac = (I == J) ? 1.0 : 2.0;
  // the front's partial sums, pivot-major: [q][task of the front]
  const int64_t t0g = grp_task_ptr[g], ntg = grp_task_ptr[g + 1] - t0g;
  double* pg = part + task_part_off[t0g] + (tk - t0g);
  for (int q0 = 0; q0 < p; q0 += kQC) {
    const int pc = min(kQC, p - q0);
    if (q0 > 0) {
      __syncthreads();  // the previous chunk's PI, PJ and red are consumed
      load_panel(q0, pc);
    }
#pragma unroll
    for (int i = 0; i < kPP; ++i) {
      const int e = t + 256 * i, r = e % kET, q = e / kET;
      PI[q][r] = (q < pc && r < na) ? pi[i] : 0.0;
      PJ[q][r] = (q < pc && r < nb) ? pj[i] : 0.0;
    }
    __syncthreads();
    // Y = Z_IJ PJ^T (rows a of the wave, 16 q), K = 64 over b.  Result
    // layout: Y[a][q] in lane q + 16 (a % 4), item a / 4 (a local to the
    // wave).  Then s_q += sum_a PI[q][a] Y[a][q]: over the items, then over
    // the four lane groups, then over the waves.
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < kET / 4; ++st)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(zf[st], PJ[lx][4 * st + lk], acc, 0, 0,
                                                 0);
    double y = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) y += acc[v] * PI[lx][16 * wave + 4 * v + lk];
    y += __shfl_xor(y, 16, 64);
    y += __shfl_xor(y, 32, 64);
    if (lk == 0) red[wave][lx] = y;
    __syncthreads();
    if (t < pc)
      pg[(q0 + t) * ntg] = fac * ((red[0][t] + red[1][t]) + (red[2][t] + red[3][t]));
  }
}

// d[leaf_col_l] = (1 + sum over the front's tasks of the partial sums) / L_ll^2:
// one wave per pivot, lanes over the front's tasks (contiguous in the
// pivot-major layout), then a fixed reduction tree.
__global__ __launch_bounds__(256) void k_selinv_reduce(
    const int32_t* __restrict__ leaf_grp, const int64_t* __restrict__ grp_col_ptr,
    const int64_t* __restrict__ grp_task_ptr, const int64_t* __restrict__ task_part_off,
    const double* __restrict__ part, const double* __restrict__ ldiag,
    const int32_t* __restrict__ leaf_cols, double* __restrict__ d, int64_t n_leaf) {
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= n_leaf) return;
  const int g = leaf_grp[l];
  const int64_t q = l - grp_col_ptr[g];
  const int64_t t0g = grp_task_ptr[g], ntg = grp_task_ptr[g + 1] - t0g;
  const double* pq = part + task_part_off[t0g] + q * ntg;
  double s = 0.0;
  for (int64_t t = lane; t < ntg; t += 64) s += pq[t];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    const double L = ldiag[l];
    d[leaf_cols[l]] = (1.0 + s) / (L * L);
  }
}

hipError_t launch_selinv_leaves(Handle& h, double* d, double* part) {
  const Analysis& a = h.an;
  const int64_t nl = (int64_t)a.leaf_cols.size();
  if (!nl) return hipSuccess;
  const int64_t n_lt = a.grp_task_ptr[a.n_groups];  // tasks of leaf fronts
  if (n_lt && a.n_pad) {
    const int64_t chunk = h.opts.selinv_chunk > 0 ? h.opts.selinv_chunk : kSelinvChunk;
    for (int64_t t0 = 0; t0 < n_lt; t0 += chunk) {
      int64_t c = std::min(chunk, n_lt - t0);
      hipLaunchKernelGGL(k_selinv_leaf, dim3((unsigned)c), dim3(256), 0,
                         h.stream, h.d.tasks, h.d.sel_order + t0, h.d.grp_U_ptr,
                         h.d.U,
                         h.d.grp_col_ptr, h.d.grp_panel_off, h.panel, h.Zr,
                         a.n_pad, h.d.grp_task_ptr, h.d.task_part_off, part);
    }
  }
  hipLaunchKernelGGL(k_selinv_reduce, dim3(wave_grid(nl)), dim3(256), 0,
                     h.stream, h.d.leaf_grp, h.d.grp_col_ptr, h.d.grp_task_ptr,
                     h.d.task_part_off, part, h.ldiag, h.d.leaf_cols, d, nl);
  return hipGetLastError();
}

}  // namespace spi

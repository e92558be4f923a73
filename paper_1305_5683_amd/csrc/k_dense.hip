// Dense kernels of the root front (gfx950, FP64 MFMA).
//
// The root front of the multifrontal factorisation (Sect. 3.2.2 of Bouchet
// et al.: a partial factorisation of a dense matrix at every node, here the
// complete factorisation at the root) is a dense SPD matrix stored
// column-major (lower triangle), n_pad x n_pad, padded with identity.  By
// default it is inverted in place by symmetric block sweeps (the root block
// of A^-1 is what the variances need); otherwise its Cholesky factor, the
// inverse of that factor and the product W^T W are formed.  Either way the
// bulk is one tiled GEMM kernel on the 16x16x4 FP64 (or 16x16x4 FP32)
// matrix cores; 64 x 64 diagonal blocks are factored, inverted or swept by
// small kernels in registers and LDS.  Also here: the dense root solves.
#include <hip/hip_runtime.h>

#include <vector>

#include <algorithm>
#include <cmath>

#include "spi_internal.h"

namespace spi {

typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------ diagonal block kernels
// 1 / sqrt(d) for d > 0: hardware estimate refined by two Newton steps
// (quadratic convergence from the estimate to full binary64 accuracy), a
// much shorter dependent chain than a rounded square root and division.
__device__ inline double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

// Cholesky of the kNB x kNB diagonal block at (k0, k0) and its inverse, in
// one right-looking sweep over column blocks of 4, by 1024 threads.
// Thread (ti, tg) keeps row ti, columns j = tg + 16q (q < 4), of the factor
// (r) and of the inverse (x) in registers; the block loop is fully unrolled
// so every register index is a compile-time constant.  Per block the four
// column values of every row and the block's four rows of the (partially
// eliminated) inverse are published through LDS (double-buffered by parity:
// one barrier per block); every thread then factors the 4x4 diagonal block
// redundantly, scales its row, applies the rank-4 update to its remaining
// columns and eliminates the block from its row of the inverse (the same
// operations applied to the identity).  A pivot that is not positive and
// finite records its elimination index (base + k0 + k) with atomicMin in
// `fail` and continues with pivot 1.  Writes L (lower triangle incl.
// diagonal) back to S and L_kk^-1, column-major with zeros above the
// diagonal, to `inv`.
__global__ __launch_bounds__(1024) void k_potrf_diag(double* S, int64_t ld,
                                                     int k0, double* inv,
                                                     int64_t* fail,
                                                     int64_t base) {
  constexpr int G = 16, Q = kNB / G;
  __shared__ double blk[2][kNB][4];   // block columns of every row
  __shared__ double xb[2][4][kNB];    // block rows of the inverse
  const int t = threadIdx.x, ti = t % kNB, tg = t / kNB;
  double r[Q], x[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = tg + G * q;
    r[q] = (ti >= j) ? S[(int64_t)(k0 + ti) + (int64_t)(k0 + j) * ld] : 0.0;
    x[q] = (ti == j) ? 1.0 : 0.0;
  }
#pragma clang loop unroll(full)
  for (int kb = 0; kb < kNB / 4; ++kb) {
    const int k = 4 * kb, par = kb & 1, qk = kb / 4;
    const bool owner = (tg >> 2) == (kb & 3);   // owns column k + (tg & 3)
    if (owner) blk[par][ti][tg & 3] = r[qk];
    if (ti >= k && ti < k + 4) {
#pragma unroll
      for (int q = 0; q < Q; ++q) xb[par][ti - k][tg + G * q] = x[q];
    }
    __syncthreads();
    // 4x4 diagonal block: D = Lb Lb^T (Li = Lb^-1), redundantly per thread
    double Lb[4][4] = {}, Li[4][4] = {};
    bool badany = false;
    int badc = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double d = blk[par][k + c][c];
#pragma unroll
      for (int e = 0; e < c; ++e) d -= Lb[c][e] * Lb[c][e];
      const bool bad = !(d > 0.0) || !isfinite(d);
      if (bad && !badany) { badany = true; badc = c; }
      const double dd = bad ? 1.0 : d;
      const double rc = rsqrt_nr(dd);
      Lb[c][c] = dd * rc;
      Li[c][c] = rc;
#pragma unroll
      for (int a = c + 1; a < 4; ++a) {
        double v = blk[par][k + a][c];
#pragma unroll
        for (int e = 0; e < c; ++e) v -= Lb[a][e] * Lb[c][e];
        Lb[a][c] = v * rc;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int a = c + 1; a < 4; ++a) {
        double v = 0.0;
#pragma unroll
        for (int e = c; e < a; ++e) v -= Lb[a][e] * Li[e][c];
        Li[a][c] = v * Li[a][a];
      }
    if (t == 0 && badany)
      atomicMin((unsigned long long*)fail, (unsigned long long)(base + k0 + k + badc));
    // this row's block entries: l = Li v (rows below the block)
    double l[4] = {0.0, 0.0, 0.0, 0.0};
    if (ti >= k + 4) {
      double v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = blk[par][ti][c];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int e = 0; e <= c; ++e) sacc += Li[c][e] * v[e];
        l[c] = sacc;
      }
    }
    // rank-4 update of this row's later columns (lower part only)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = tg + G * q;
      if (ti >= k + 4 && j > k + 3 && j <= ti) {
        double w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) w[c] = blk[par][j][c];
        double sacc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double ljc = 0.0;
#pragma unroll
          for (int e = 0; e <= c; ++e) ljc += Li[c][e] * w[e];
          sacc += l[c] * ljc;
        }
        r[q] -= sacc;
      }
    }
    // the block column of the factor is final
    if (owner) {
      const int c = tg & 3;
      double v = r[qk];
      if (ti >= k + 4) {
        v = (c == 0) ? l[0] : (c == 1) ? l[1] : (c == 2) ? l[2] : l[3];
      } else if (ti >= k) {
        v = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int cc = 0; cc <= a; ++cc)
            if (a == ti - k && cc == c) v = Lb[a][cc];
      }
      r[qk] = v;
    }
    // inverse: X_b = Li Xtilde_b; rows of the block take it, rows below
    // eliminate it (only columns j <= k + 3 are non-zero)
    if (ti >= k) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int j = tg + G * q;
        if (j <= k + 3) {
          double xt[4], xf[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) xt[c] = xb[par][c][j];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double sacc = 0.0;
#pragma unroll
            for (int e = 0; e <= c; ++e) sacc += Li[c][e] * xt[e];
            xf[c] = sacc;
          }
          if (ti >= k + 4) {
            x[q] -= l[0] * xf[0] + l[1] * xf[1] + l[2] * xf[2] + l[3] * xf[3];
          } else {
            const int a = ti - k;
            x[q] = (a == 0) ? xf[0] : (a == 1) ? xf[1] : (a == 2) ? xf[2] : xf[3];
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = tg + G * q;
    if (ti >= j) S[(int64_t)(k0 + ti) + (int64_t)(k0 + j) * ld] = r[q];
    inv[ti + j * kNB] = (ti >= j) ? x[q] : 0.0;
  }
}

// Inverses of the kNBO x kNBO diagonal blocks of the factor (the last one
// may be narrower), one block per workgroup, from the inverses of their
// kNB x kNB diagonal sub-blocks:  X_ii = L_ii^-1 and, column by column,
// X_ij = -X_ii sum_{j<=k<i} L_ik X_kj  for i > j.  Output column-major with
// leading dimension kNBO and zeros above the diagonal.
__global__ __launch_bounds__(256) void k_invert_outer_blocks(const double* S,
                                                             int64_t ld,
                                                             const double* invd,
                                                             double* out,
                                                             int np) {
  constexpr int NBO = 256, NS = NBO / kNB;
  __shared__ double La[kNB][kNB + 1];
  __shared__ double Xb[kNB][kNB + 1];
  const int K0 = blockIdx.x * NBO;
  const int ns = min(NS, (np - K0) / kNB);
  double* X = out + (int64_t)blockIdx.x * NBO * NBO;
  const int t = threadIdx.x;
  const int ri = (t % 16) * 4, cj = (t / 16) * 4;  // this thread's 4 x 4 block
  // diagonal sub-blocks and zeros above
  for (int bj = 0; bj < NS; ++bj)
    for (int bi = 0; bi < NS; ++bi)
      for (int e = t; e < kNB * kNB; e += 256) {
        const int i = e % kNB, j = e / kNB;
        double v = 0.0;
        if (bi == bj && bi < ns)
          v = invd[(int64_t)(K0 / kNB + bi) * kNB * kNB + i + j * kNB];
        if (bi <= bj || bi >= ns || bj >= ns)
          X[(bi * kNB + i) + (int64_t)(bj * kNB + j) * NBO] = v;
      }
  __syncthreads();
  for (int bj = 0; bj < ns; ++bj)
    for (int bi = bj + 1; bi < ns; ++bi) {
      double acc[4][4] = {};
      for (int bk = bj; bk < bi; ++bk) {  // acc += L_ik X_kj
        for (int e = t; e < kNB * kNB; e += 256) {
          const int i = e % kNB, j = e / kNB;
          La[i][j] = S[(int64_t)(K0 + bi * kNB + i) + (int64_t)(K0 + bk * kNB + j) * ld];
          Xb[i][j] = X[(bk * kNB + i) + (int64_t)(bj * kNB + j) * NBO];
        }
        __syncthreads();
        for (int q = 0; q < kNB; ++q) {
          double a[4], b[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            a[x] = La[ri + x][q];
            b[x] = Xb[q][cj + x];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
      }
      // X_ij = -X_ii acc
      for (int e = t; e < kNB * kNB; e += 256) {
        const int i = e % kNB, j = e / kNB;
        La[i][j] = X[(bi * kNB + i) + (int64_t)(bi * kNB + j) * NBO];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) Xb[ri + x][cj + y] = acc[x][y];
      __syncthreads();
      double r[4][4] = {};
      for (int q = 0; q < kNB; ++q) {
        double a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          a[x] = La[ri + x][q];
          b[x] = Xb[q][cj + x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) r[x][y] += a[x] * b[y];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          X[(bi * kNB + ri + x) + (int64_t)(bj * kNB + cj + y) * NBO] = -r[x][y];
      __syncthreads();
    }
}

// Copy the lower triangle (and zeros above) of S into W.
__global__ void k_copy_lower(const double* __restrict__ S, double* __restrict__ W,
                             int64_t n_pad) {
  int64_t total = n_pad * n_pad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e % n_pad, j = e / n_pad;
    W[e] = (i >= j) ? S[e] : 0.0;
  }
}

static int fill_grid(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (int)std::min<int64_t>(g, 65536);
}

static int pick_bm(int M) { return (M % 128 == 0) ? 128 : 64; }

// Outer block of the root POTRF / TRTRI sweeps: the bulk updates run with
// K = kNBO (a quarter of the C traffic of kNB steps); the panels inside an
// outer block are factored in kNB steps.
constexpr int kNBO = 256;

// Factor the outer panel [K0, K0 + KB) of the root (all rows below K0):
// kNB diagonal blocks, their panel solves, and the updates of the panel's
// remaining columns.
static hipError_t factor_panel(Handle& h, hipStream_t s, int K0, int KB) {
  const bool f32 = h.opts.precision == SPI_MIXED;
  const int np = (int)h.an.n_pad;
  const int64_t ld = np;
  const int64_t base = (int64_t)h.an.leaf_cols.size();
  hipError_t e;
  for (int k0 = K0; k0 < K0 + KB; k0 += kNB) {
    double* inv = h.invd + (int64_t)(k0 / kNB) * kNB * kNB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(1024), 0, s, h.S, ld, k0,
                       inv, h.flag, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int rest = np - k0 - kNB;
    if (rest <= 0) break;
    // panel solve P := P L_kk^-T as a product with the inverse (each tile
    // owns whole rows of the 64-wide panel, so it is safe in place)
    double* Pp = h.S + (int64_t)(k0 + kNB) + (int64_t)k0 * ld;
    // (64-row tiles: these products are on the critical path and short,
    // so more, smaller workgroups finish sooner)
    e = gemm(s, 64, 64, kXC, kXC, Pp, ld, inv, kNB, Pp, ld, rest, kNB, kNB, 1.0,
             0.0, false, false, false, f32);
    if (e != hipSuccess) return e;
    const int ncols = K0 + KB - k0 - kNB;  // panel columns still to update
    if (ncols > 0) {
      double* P = h.S + (int64_t)(k0 + kNB) + (int64_t)k0 * ld;
      double* C = h.S + (int64_t)(k0 + kNB) * (ld + 1);
      e = gemm(s, 64, 64, kXC, kXC, P, ld, P, ld, C, ld, rest, ncols, kNB, -1.0,
               1.0, false, false, true, f32);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t ensure_side_stream(Handle& h) {
  hipError_t e;
  if (!h.side) {
    if ((e = hipStreamCreateWithFlags(&h.side, hipStreamNonBlocking)) != hipSuccess)
      return e;
  }
  hipEvent_t* evs[] = {&h.ev_next, &h.ev_panel};
  for (hipEvent_t* ev : evs)
    if (!*ev && (e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess)
      return e;
  return hipSuccess;
}

// Right-looking blocked Cholesky of the root front with a one-panel
// lookahead: after outer step K0 has updated the next panel's columns (T1),
// the side stream factors that panel while the main stream applies the rest
// of the trailing update (T2); the two touch disjoint columns.  Then the
// inverses of all kNB diagonal blocks (used by the factor inversion).
hipError_t root_potrf(Handle& h) {
  const bool f32 = h.opts.precision == SPI_MIXED;
  const int np = (int)h.an.n_pad;
  const int64_t ld = np;
  hipError_t e;
  if ((e = ensure_side_stream(h)) != hipSuccess) return e;
  // outer block: 128, 256 or 512; binary32 accumulation (mixed precision)
  // runs over at most kNBO terms, so its trailing updates use K <= kNBO
  const int NBO = f32 ? std::min(h.potrf_block, kNBO) : h.potrf_block;
  if ((e = factor_panel(h, h.stream, 0, std::min(NBO, np))) != hipSuccess)
    return e;
  for (int K0 = 0; K0 < np; K0 += NBO) {
    const int KB = std::min(NBO, np - K0), K1 = K0 + KB;
    const int rest = np - K1;
    if (rest <= 0) break;
    const int KB2 = std::min(NBO, rest);
    double* P = h.S + (int64_t)K1 + (int64_t)K0 * ld;  // rows >= K1 of the panel
    // T1: next panel's columns [K1, K1 + KB2), all rows >= K1
    e = gemm(h.stream, pick_bm(rest), (KB2 % 128 == 0) ? 128 : 64, kXC, kXC, P,
             ld, P, ld, h.S + (int64_t)K1 * (ld + 1), ld, rest, KB2, KB, -1.0,
             1.0, false, false, true, f32);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(h.ev_next, h.stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(h.side, h.ev_next, 0)) != hipSuccess) return e;
    if ((e = factor_panel(h, h.side, K1, KB2)) != hipSuccess) return e;
    if ((e = hipEventRecord(h.ev_panel, h.side)) != hipSuccess) return e;
    // T2: trailing square beyond the next panel, lower triangle
    const int r2 = rest - KB2;
    if (r2 > 0) {
      const int t = (r2 % 128 == 0) ? 128 : 64;
      e = gemm(h.stream, t, t, kXC, kXC, P + KB2, ld, P + KB2, ld,
               h.S + (int64_t)(K1 + KB2) * (ld + 1), ld, r2, r2, KB, -1.0, 1.0,
               true, false, false, f32);
      if (e != hipSuccess) return e;
    }
    if ((e = hipStreamWaitEvent(h.stream, h.ev_panel, 0)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_invert_outer_blocks, dim3((np + kNBO - 1) / kNBO),
                     dim3(256), 0, h.stream, h.S, ld, h.invd, h.invd2, np);
  return hipGetLastError();
}

// 2-D copy of a rows x cols column-major block.
__global__ void k_copy2d(const double* __restrict__ src, int64_t lds,
                         double* __restrict__ dst, int64_t ldd, int rows,
                         int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    dst[i + j * ldd] = src[i + j * lds];
  }
}

static hipError_t copy2d(hipStream_t s, const double* src, int64_t lds,
                         double* dst, int64_t ldd, int rows, int cols) {
  const int64_t total = (int64_t)rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy2d, dim3(fill_grid(total)), dim3(256), 0, s, src,
                     lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

// Right-looking inversion of the diagonal block [off, off + size) of the
// factor, in place on W (which holds that block of L on entry).  With the
// first block columns of the block already inverted, row block k to the left
// holds L_k,<k X_<k and the block rows below hold L_>k,<k X_<k.  Step k, with
// X_kk = L_kk^-1 (the stored kNBO-block inverses):
//   T       = L_>k,k X_kk             (becomes the state of block column k)
//   S_>k,<k -= T * S_k,<k
//   S_k,<k   = -X_kk * S_k,<k         (final row block k of L^-1)
//   S_kk     = X_kk
// The two in-place products read their input from a staged copy in rows
// [off, off + size) of Z (which holds nothing until the root block of A^-1
// is formed), so inversions of disjoint blocks may run concurrently.  Each
// product sums kNBO terms (binary32 in mixed precision, then binary64).
static hipError_t trtri_sweep(Handle& h, hipStream_t st, int off, int size,
                              bool f32) {
  const int64_t ld = h.an.n_pad;
  double* Wb = h.W + off + (int64_t)off * ld;
  double* scr = h.Z + off;  // staging, leading dimension ld
  hipError_t e;
  for (int K0 = 0; K0 < size; K0 += kNBO) {
    const int KB = std::min(kNBO, size - K0), K1 = K0 + KB;
    const int rest = size - K1;
    const double* X11 = h.invd2 + (int64_t)((off + K0) / kNBO) * kNBO * kNBO;
    double* W21 = Wb + (int64_t)K1 + (int64_t)K0 * ld;
    double* W10 = Wb + (int64_t)K0;
    double* W20 = Wb + (int64_t)K1;
    const int bk = (KB % 128 == 0) ? 128 : 64;
    if (rest > 0) {
      if ((e = copy2d(st, W21, ld, scr, ld, rest, KB)) != hipSuccess) return e;
      e = gemm(st, pick_bm(rest), bk, kXC, kKC, scr, ld, X11, kNBO, W21, ld, rest,
               KB, KB, 1.0, 0.0, false, false, false, f32);
      if (e != hipSuccess) return e;
      if (K0 > 0) {
        e = gemm(st, pick_bm(rest), 128, kXC, kKC, W21, ld, W10, ld, W20, ld, rest,
                 K0, KB, -1.0, 1.0, false, false, false, f32);
        if (e != hipSuccess) return e;
      }
    }
    if (K0 > 0) {
      if ((e = copy2d(st, W10, ld, scr, ld, KB, K0)) != hipSuccess) return e;
      e = gemm(st, bk, 128, kXC, kKC, X11, kNBO, scr, ld, W10, ld, KB, K0, KB, -1.0,
               0.0, false, false, false, f32);
      if (e != hipSuccess) return e;
    }
    if ((e = copy2d(st, X11, kNBO, Wb + (int64_t)K0 * (ld + 1), ld, KB, KB)) !=
        hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Below this order a diagonal block is inverted by the sweep: its GEMMs
// span all rows below the step and keep the GPU busy, where further halving
// would launch products of a few tiles each.
constexpr int kTrtriRecMin = 2048;

// Inversion by halving (FP64): split at hh (a multiple of kNBO), invert both
// diagonal halves, then
//   W21 = -X22 (L21 X11)
// as two GEMMs with a triangular operand each (the K range of a tile is
// trimmed to where that operand is non-zero).  These GEMMs have K up to
// size / 2 and carry most of the flops; the sweep's products have K = kNBO.
// T = L21 X11 is staged in rows [off + hh, off + size) of Z.
static hipError_t trtri_join(Handle& h, hipStream_t st, int off, int size, int hh);

static hipError_t trtri_rec(Handle& h, hipStream_t st, int off, int size) {
  if (size <= kTrtriRecMin) return trtri_sweep(h, st, off, size, false);
  const int hh = ((size / 2 + kNBO - 1) / kNBO) * kNBO;
  hipError_t e;
  if ((e = trtri_rec(h, st, off, hh)) != hipSuccess) return e;
  if ((e = trtri_rec(h, st, off + hh, size - hh)) != hipSuccess) return e;
  return trtri_join(h, st, off, size, hh);
}

// The products that join two inverted halves (see trtri_rec).
static hipError_t trtri_join(Handle& h, hipStream_t st, int off, int size, int hh) {
  const int64_t ld = h.an.n_pad;
  const int r = size - hh;
  const double* L21 = h.S + (off + hh) + (int64_t)off * ld;
  const double* X11 = h.W + off + (int64_t)off * ld;
  const double* X22 = h.W + (off + hh) + (int64_t)(off + hh) * ld;
  double* W21 = h.W + (off + hh) + (int64_t)off * ld;
  double* T = h.Z + (off + hh);
  hipError_t e = gemm(st, pick_bm(r), 128, kXC, kKC, L21, ld, X11, ld, T, ld, r, hh,
                      hh, 1.0, 0.0, false, false, false, false, kGemmKStartCol);
  if (e != hipSuccess) return e;
  return gemm(st, pick_bm(r), 128, kXC, kKC, X22, ld, T, ld, W21, ld, r, hh, r, -1.0,
              0.0, false, false, false, false, kGemmKEndRow);
}

// Inverse of the root factor, W = L^-1.  W starts as a copy of L's lower
// triangle with zeros above (the zeros matter: later products read whole
// diagonal tiles).  FP64: the two halves of the top split are inverted
// concurrently (main and side streams), then joined.  Mixed precision uses
// the sweep alone, whose products sum at most kNBO terms in binary32 before
// the binary64 accumulation.
hipError_t root_trtri(Handle& h) {
  const bool f32 = h.opts.precision == SPI_MIXED;
  const int np = (int)h.an.n_pad;
  hipLaunchKernelGGL(k_copy_lower, dim3(fill_grid((int64_t)np * np)), dim3(256), 0,
                     h.stream, h.S, h.W, (int64_t)np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (f32) return trtri_sweep(h, h.stream, 0, np, true);
  if (np <= kTrtriRecMin) return trtri_sweep(h, h.stream, 0, np, false);
  if ((e = ensure_side_stream(h)) != hipSuccess) return e;
  const int hh = ((np / 2 + kNBO - 1) / kNBO) * kNBO;
  if ((e = hipEventRecord(h.ev_next, h.stream)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(h.side, h.ev_next, 0)) != hipSuccess) return e;
  if ((e = trtri_rec(h, h.side, hh, np - hh)) != hipSuccess) return e;
  if ((e = hipEventRecord(h.ev_panel, h.side)) != hipSuccess) return e;
  if ((e = trtri_rec(h, h.stream, 0, hh)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(h.stream, h.ev_panel, 0)) != hipSuccess) return e;
  return trtri_join(h, h.stream, 0, np, hh);
}

// Z = W^T W (lower tiles); tile (I, J) sums over K >= I since W is lower
// triangular with stored zeros above the diagonal.  Always FP64: these sums
// are the diagonal accumulation of the selected inversion, and an FP32
// accumulation over n_R terms would cost about sqrt(n_R / 4) binary32
// roundings of relative error in the variances.
hipError_t root_lauum(Handle& h) {
  const int np = (int)h.an.n_pad;
  return gemm(h.stream, 128, 128, kKC, kKC, h.W, np, h.W, np, h.Z, np, np, np,
              np, 1.0, 0.0, true, true);
}

// ------------------------------------- root inverse by symmetric sweeps
// The root block of A^-1 is the inverse of the dense root front, and the
// factorisation, the inversion of the factor and the product W^T W of the
// Takahashi route (Sect. 3.3 asks for the diagonal of A^-1) can be traded
// for one sweep per column block: with M the root front and K a block of
// kb columns whose pivot block D = M_KK (the Schur complement of the blocks
// swept before, the same matrix the Cholesky factorisation pivots on):
//   M_ij -= M_iK D^-1 M_Kj     for i, j outside K
//   M_iK  = M_iK D^-1          for i outside K
//   M_KK  = -D^-1
// After every block has been swept, M = -A_RR^-1 (Schur complement form of
// the root).  Each step's bulk is one symmetric rank-kb update of the whole
// lower triangle, n^3 flops in total as for factor + inversion + product,
// but in uniform launches that fill the GPU instead of shrinking trailing
// matrices.  The pivot blocks are the ones Cholesky sees, so a pivot that is
// not positive is reported at the same elimination index.
//
// A step gathers the band of K (all np rows of columns K, the rows above K
// taken from row block K of the lower storage) into a column-major buffer V,
// sweeps its pivot block D alone in kNB steps (one launch each; the first
// reads D from the lower storage, then they ping-pong between two kb x kb
// buffers) to get -D^-1, forms B = V D^-1 outside K in one product, and
// writes B (and -D^-1 on K) back.  The bulk is then M_ij -= B_i V_j^T over
// rows and columns outside K.  With a one-band lookahead only the next
// band's pivot block is brought up to date first (a small launch); its
// sweep steps then run on the side stream while the main stream's bulk
// updates everything else, the rest of the next band included, and the
// next band's columns are gathered after the bulk.  The last bulk and the
// last band are written negated, so S ends holding +A_RR^-1.

// Band [k0, k0 + kb) of the symmetric matrix in lower storage S (leading
// dimension ld) <-> column-major np x kb buffers; 64 x 64 tiles through LDS,
// over the rows from row0 (one tile row per blockIdx.x).
// to_band: V (if given) receives the full symmetric columns and D (if
// given; leading dimension kb) its rows in K; otherwise the lower-storage
// positions of S receive sgn times B, or D on the rows in K.
__global__ __launch_bounds__(256) void k_band_move(double* __restrict__ S, int64_t ld,
                                                   const double* __restrict__ B,
                                                   double* __restrict__ V,
                                                   double* __restrict__ D,
                                                   int64_t np, int k0, int kb,
                                                   int to_band, double sgn, int row0) {
  __shared__ double T[64][65];
  const int i0 = row0 + blockIdx.x * 64, c0 = blockIdx.y * 64, g0 = k0 + c0;
  const int t = threadIdx.x, a = t & 63, q = t >> 6;
  // kind: 1 direct (all rows below the columns), -1 transposed (all rows
  // above), 0 diagonal tile (rows of the tile are the tile's columns)
  const int kind = (i0 > g0) ? 1 : (i0 < g0 ? -1 : 0);
  const bool inK = i0 >= k0 && i0 < k0 + kb;
  if (to_band) {
    for (int b = q; b < 64; b += 4) {
      // T[a][b]: element (i0 + a, g0 + b) of the symmetric matrix
      if (kind >= 0)
        T[a][b] = S[(int64_t)(i0 + a) + (int64_t)(g0 + b) * ld];
      else  // S row g0 + a, column i0 + b holds element (i0 + b, g0 + a)
        T[b][a] = S[(int64_t)(g0 + a) + (int64_t)(i0 + b) * ld];
    }
    __syncthreads();
    for (int b = q; b < 64; b += 4) {
      const double v = (kind == 0 && a < b) ? T[b][a] : T[a][b];
      if (V) V[i0 + a + (int64_t)(c0 + b) * np] = v;
      if (inK && D) D[(i0 - k0 + a) + (int64_t)(c0 + b) * kb] = v;
    }
  } else {
    for (int b = q; b < 64; b += 4)
      T[a][b] = sgn * (inK ? D[(i0 - k0 + a) + (int64_t)(c0 + b) * kb]
                           : B[i0 + a + (int64_t)(c0 + b) * np]);
    __syncthreads();
    for (int b = q; b < 64; b += 4) {
      if (kind > 0 || (kind == 0 && a >= b))
        S[(int64_t)(i0 + a) + (int64_t)(g0 + b) * ld] = T[a][b];
      else if (kind < 0)
        S[(int64_t)(g0 + a) + (int64_t)(i0 + b) * ld] = T[b][a];
    }
  }
}

// 1 / d for d > 0: hardware estimate refined by two Newton steps (a
// shorter dependent chain than a rounded division).
__device__ inline double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = y * fma(-d, y, 2.0);
  y = y * fma(-d, y, 2.0);
  return y;
}

// One kNB-column step s of the sweep of a kb x kb symmetric block held in
// full (both triangles, leading dimension kb): Din -> Dout, so the step
// reads only values from before it.  A workgroup per lower 64 x 64 tile
// (I, C), I >= C, writing the tile and its transpose.  Every workgroup
// sweeps the pivot block Ds = Din_ss itself (64 rank-1 steps on 16 entries
// per thread in registers, one column broadcast through LDS per step) to
// get M = -Ds^-1, then
//   (s, s):          M
//   (I, s), I != s:  Din_Is Ds^-1 = -Din_Is M
//   (s, C), C != s:  Ds^-1 Din_sC = -M Din_sC
//   otherwise:       Din_IC + (Din_Is M) Din_sC
// The workgroup of tile (s, s) records a pivot that is not positive and
// finite (index base + s * kNB + k) with atomicMin in `fail` and continues
// with pivot 1.  Two 64 x 64 LDS buffers, so the workgroup fits beside a
// GEMM workgroup on one CU.
//
// INDEF (symmetric indefinite matrices): the pivot block is swept with
// Bunch-Kaufman pivots chosen inside it instead of in index order with
// positive pivots.  The sweep operator's result does not depend on the
// order in which indices are swept, nor on sweeping two at once, so M is
// -Ds^-1 either way; the order only decides the rounding.  Each step looks
// at the lowest unswept index k: with lambda the largest |M_ik| over the
// other unswept i (at r), it sweeps k alone if |M_kk| >= alpha lambda; else,
// with sigma the largest |M_jr| over the unswept j != r, k alone if
// |M_kk| sigma >= alpha lambda^2, r alone if |M_rr| >= alpha sigma, and the
// pair {k, r} as one 2 x 2 pivot otherwise (alpha = (1 + sqrt 17) / 8).
// Pivots of either sign are taken; a block with no usable pivot (k's
// column all zero, a zero or non-finite pivot or 2 x 2 determinant) is
// reported at k and swept with pivot 1.
template <bool INDEF>
__global__ __launch_bounds__(256, 2) void k_dsweep_step(const double* __restrict__ Din,
                                                        int64_t ldin, int sym_lower,
                                                        double* __restrict__ Dout,
                                                        int kb, int sb, int64_t* fail,
                                                        int64_t base) {
  __shared__ double Mv[kNB][kNB + 1];
  __shared__ double Xa[kNB][kNB + 1];
  __shared__ double colk[2][kNB];
  __shared__ double colb[2][kNB];
  // these steps are the critical path while bulk updates share the CUs:
  // issue ahead of their waves
  __builtin_amdgcn_s_setprio(3);
  int I = 0, C = blockIdx.x;
  while (C > I) C -= ++I;  // lower tiles in row order: (0,0), (1,0), (1,1), ...
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)sb * kNB;
  // Din: the full kb x kb block (leading dimension ldin), or with sym_lower
  // its lower triangle only (element (r, c), r < c, read at (c, r))
  auto at = [&](int bi, int bc, int r, int c) -> double {
    int64_t gr = (int64_t)bi * kNB + r, gc = (int64_t)bc * kNB + c;
    if (sym_lower && gr < gc) {
      const int64_t x = gr;
      gr = gc;
      gc = x;
    }
    return Din[gr + gc * ldin];
  };
  // Pivot block in registers: wave w holds rows [16 w, 16 w + 16) and lane l
  // column l (read through the symmetric twin, so the loads are contiguous
  // over lanes).
  const int lane = t & 63, wave = t >> 6;
  double m[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) m[q] = at(sb, sb, lane, 16 * wave + q);
  const bool reporter = (I == sb && C == sb && t == 0);
  // Step k: the wave holding row k publishes it (= column k) in LDS; then
  // element (i, l) becomes M_il - M_ik M_kl / d, column k (lane k) M_ik / d,
  // row k M_kl / d and the pivot -1 / d.  Column k is written as
  // fma(M_ik, r, 0 * m) and the others as fma(-M_ik, M_kl r, 1 * m), so all
  // lanes run the same instructions.
  if constexpr (!INDEF) {
  for (int kw = 0; kw < 4; ++kw) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 16 * kw + q, par = q & 1;
      if (wave == kw) colk[par][lane] = m[q];
      __syncthreads();
      double d = colk[par][k];
      if (!(d > 0.0) || !isfinite(d)) {
        if (reporter)
          atomicMin((unsigned long long*)fail, (unsigned long long)(base + s0 + k));
        d = 1.0;
      }
      const double r = rcp_nr(d);
      const bool piv = lane == k;
      const double tl = colk[par][lane] * r;  // M_kl / d
      const double a = piv ? r : -tl;
      const double keep = piv ? 0.0 : 1.0;
#pragma unroll
      for (int q2 = 0; q2 < 16; ++q2)
        m[q2] = fma(colk[par][16 * wave + q2], a, keep * m[q2]);
      if (wave == kw) m[q] = piv ? -r : tl;
    }
  }
  } else {
    const double alpha = 0.6403882032022076;  // (1 + sqrt(17)) / 8
    // the largest |v| over the lanes not in `skip`, and the lowest such lane
    auto lane_max = [&](double v, uint64_t skip, int& at) {
      double x = ((skip >> lane) & 1) ? -1.0 : fabs(v);
      int i = lane;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double xo = __shfl_xor(x, off, 64);
        const int io = __shfl_xor(i, off, 64);
        if (xo > x || (xo == x && io < i)) {
          x = xo;
          i = io;
        }
      }
      at = i;
      return x;
    };
    // column c of the block (= row c) into buf: lane c of every wave holds
    // its 16 rows of it
    auto publish = [&](double* buf, int c) {
      if (lane == c) {
#pragma unroll
        for (int q = 0; q < 16; ++q) buf[16 * wave + q] = m[q];
      }
    };
    uint64_t done = 0;  // swept indices (wave-uniform)
    int par = 0;
    while (done != ~0ull) {
      const int k = __builtin_ctzll(~done);
      double* ca = colk[par];
      double* cb = colb[par];
      publish(ca, k);
      __syncthreads();
      int r;
      const double lam = lane_max(ca[lane], done | (1ull << k), r);
      const double akk = fabs(ca[k]);
      int p = k, s2 = -1;      // 1 x 1 at p, or 2 x 2 at {k, s2}
      const double* cp = ca;   // column of p
      bool bad = false;
      if (!(lam > 0.0)) {
        bad = !(akk > 0.0) || !isfinite(akk);
      } else if (!(akk >= alpha * lam)) {
        publish(cb, r);
        __syncthreads();
        int rr;
        const double sig = lane_max(cb[lane], done | (1ull << r), rr);
        if (akk * sig >= alpha * lam * lam) {
          // k alone
        } else if (fabs(cb[r]) >= alpha * sig) {
          p = r;
          cp = cb;
        } else {
          s2 = r;
        }
      }
      if (s2 < 0) {
        double d = cp[p];
        if (bad || d == 0.0 || !isfinite(d)) {
          if (reporter)
            atomicMin((unsigned long long*)fail, (unsigned long long)(base + s0 + k));
          d = 1.0;
        }
        const double rc = 1.0 / d;
        const bool piv = lane == p;
        const double tl = cp[lane] * rc;  // M_pl / d
        const double a = piv ? rc : -tl;
        const double keep = piv ? 0.0 : 1.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          m[q] = fma(cp[16 * wave + q], a, keep * m[q]);
          if (16 * wave + q == p) m[q] = piv ? -rc : tl;
        }
        done |= 1ull << p;
      } else {
        // 2 x 2 pivot P = [[a, b], [b, c]] on {k, s2}: E = P^-1
        const int sI = s2;
        const double pa = ca[k], pb = ca[sI], pc = cb[sI];
        double det = pa * pc - pb * pb;
        double e00, e01, e11;
        if (!(det != 0.0) || !isfinite(det)) {
          if (reporter)
            atomicMin((unsigned long long*)fail, (unsigned long long)(base + s0 + k));
          e00 = 1.0, e01 = 0.0, e11 = 1.0;
        } else {
          const double ri = 1.0 / det;
          e00 = pc * ri;
          e01 = -pb * ri;
          e11 = pa * ri;
        }
        const bool lk_ = lane == k, ls_ = lane == sI;
        // t = E [M_kl; M_sl] for the other columns
        const double t0 = e00 * ca[lane] + e01 * cb[lane];
        const double t1 = e01 * ca[lane] + e11 * cb[lane];
        const double a0 = lk_ ? e00 : (ls_ ? e01 : -t0);
        const double a1 = lk_ ? e01 : (ls_ ? e11 : -t1);
        const double keep = (lk_ || ls_) ? 0.0 : 1.0;
        const double rowk = lk_ ? -e00 : (ls_ ? -e01 : t0);
        const double rows = lk_ ? -e01 : (ls_ ? -e11 : t1);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int i = 16 * wave + q;
          m[q] = fma(ca[i], a0, fma(cb[i], a1, keep * m[q]));
          if (i == k) m[q] = rowk;
          if (i == sI) m[q] = rows;
        }
        done |= (1ull << k) | (1ull << sI);
      }
      par ^= 1;
    }
  }
  auto load = [&](double (*X)[kNB + 1], int bi, int bc) {
    constexpr int kPer = kNB * kNB / 256;
    double v[kPer];  // every load in flight before the LDS stores
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = t + 256 * q;
      v[q] = at(bi, bc, e % kNB, e / kNB);
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = t + 256 * q;
      X[e % kNB][e / kNB] = v[q];
    }
  };
  // 64 x 64 products on the FP64 matrix cores: wave w owns the 32 x 32
  // quadrant (32 (w & 1), 32 (w >> 1)) as 2 x 2 blocks of 16 x 16; element
  // (bi, bj, v) of a lane is row 32 wr + 16 bi + lx, column 32 wc + 16 bj +
  // 4 v + lk (the 16x16x4 FP64 result layout with the B fragment first)
  const int lx = lane & 15, lk = lane >> 4;
  const int r0 = 32 * (wave & 1), c0 = 32 * (wave >> 1);
  auto mul = [&](double (*X)[kNB + 1], double (*Y)[kNB + 1], v4d (&acc)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < kNB; k += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        fa[q] = X[r0 + 16 * q + lx][k + lk];
        fb[q] = Y[k + lk][c0 + 16 * q + lx];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[bj], fa[bi], acc[bi][bj],
                                                            0, 0, 0);
    }
  };
  auto row_of = [&](int bi) { return r0 + 16 * bi + lx; };
  auto col_of = [&](int bj, int v) { return c0 + 16 * bj + 4 * v + lk; };
  auto store = [&](const v4d (&o)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = (int64_t)I * kNB + row_of(bi);
          const int64_t c = (int64_t)C * kNB + col_of(bj, v);
          Dout[r + c * kb] = o[bi][bj][v];
          if (I != C) Dout[c + r * kb] = o[bi][bj][v];
        }
  };
  if (I == sb && C == sb) {  // M itself (written through the symmetric twin)
#pragma unroll
    for (int q = 0; q < 16; ++q) Dout[(s0 + lane) + (s0 + 16 * wave + q) * kb] = m[q];
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) Mv[16 * wave + q][lane] = m[q];
  v4d acc[2][2];
  if (C == sb || I == sb) {
    // (I, s) below the pivot block: -Din_Is M; (s, C) left of it: -M Din_sC
    load(Xa, C == sb ? I : sb, C == sb ? sb : C);
    __syncthreads();
    if (C == sb) mul(Xa, Mv, acc); else mul(Mv, Xa, acc);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = -acc[bi][bj];
  } else {
    load(Xa, I, sb);
    __syncthreads();
    mul(Xa, Mv, acc);   // T = Din_Is M
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xa[row_of(bi)][col_of(bj, v)] = acc[bi][bj][v];
    load(Mv, sb, C);    // Din_sC
    __syncthreads();
    double cin[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) cin[bi][bj][v] = at(I, C, row_of(bi), col_of(bj, v));
    mul(Xa, Mv, acc);   // T Din_sC
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[bi][bj][v] += cin[bi][bj][v];
  }
  store(acc);
}

static hipError_t band_move(hipStream_t st, Handle& h, const double* B, double* V,
                            double* D, int k0, int kb, bool to_band, double sgn,
                            int row0 = 0, int rows = -1) {
  const int64_t np = h.an.n_pad;
  if (rows < 0) rows = (int)np;
  hipLaunchKernelGGL(k_band_move, dim3((unsigned)(rows / 64), (unsigned)(kb / 64)),
                     dim3(256), 0, st, h.S, np, B, V, D, np, k0, kb,
                     to_band ? 1 : 0, sgn, row0);
  return hipGetLastError();
}

// The band of [k0, k0 + kb) in three parts: gather its columns into V;
// sweep the pivot block to -D^-1 (kb / kNB launches, the first reading S,
// ending in Dw[0] since kb / kNB is even); B = V D^-1 outside K and scatter
// back (negated for the last band).
static hipError_t band_gather(Handle& h, hipStream_t st, int k0, int kb, double* V) {
  return band_move(st, h, nullptr, V, nullptr, k0, kb, true, 1.0);
}

// The first step reads the pivot block from the lower storage of S.
static hipError_t band_pivot_sweep(Handle& h, hipStream_t st, int k0, int kb) {
  const int64_t np = h.an.n_pad;
  const int64_t base = (int64_t)h.an.leaf_cols.size() + k0;
  double* Dw[2] = {h.band + 4 * np * h.band_nb,
                   h.band + 4 * np * h.band_nb + (int64_t)h.band_nb * h.band_nb};
  const int nsb = kb / kNB, nt = nsb * (nsb + 1) / 2;
  for (int sb = 0; sb < nsb; ++sb) {
    const bool first = sb == 0;
    if (h.opts.indefinite)
      hipLaunchKernelGGL(k_dsweep_step<true>, dim3(nt), dim3(256), 0, st,
                         first ? h.S + (int64_t)k0 * (np + 1) : Dw[sb & 1],
                         first ? np : (int64_t)kb, first ? 1 : 0,
                         Dw[(sb + 1) & 1], kb, sb, h.flag, base);
    else
      hipLaunchKernelGGL(k_dsweep_step<false>, dim3(nt), dim3(256), 0, st,
                         first ? h.S + (int64_t)k0 * (np + 1) : Dw[sb & 1],
                         first ? np : (int64_t)kb, first ? 1 : 0,
                         Dw[(sb + 1) & 1], kb, sb, h.flag, base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Tile edges of the band product and of the next pivot block's update (a
// 512 x 512 lower triangle: small tiles give it more workgroups; the bulk
// uses 128).
constexpr int kBandTile = 64;
constexpr int kPivotTile = 32;

static hipError_t band_product(Handle& h, hipStream_t st, int k0, int kb, double* B,
                               const double* V) {
  const int64_t np = h.an.n_pad;
  const double* Dm = h.band + 4 * np * h.band_nb;  // -D^-1, full
  GemmSkip rows;
  rows.r0 = k0;
  rows.r1 = k0 + kb;
  return gemm(st, kBandTile, kBandTile, kXC, kXC, V, np, Dm, kb, B, np, (int)np, kb,
              kb, -1.0, 0.0, false, false, false, false, 0, rows);
}

static hipError_t band_scatter(Handle& h, hipStream_t st, int k0, int kb,
                               const double* B, bool last) {
  double* Dm = h.band + 4 * (int64_t)h.an.n_pad * h.band_nb;
  return band_move(st, h, B, nullptr, Dm, k0, kb, false, last ? -1.0 : 1.0);
}

// C = beta C + alpha A B^T for the sweep updates (A, B: kXC, column-major
// band buffers).  Mixed precision: binary32 matrix-core products in sums of
// at most kNBO terms that add up in binary64: a band of up to 2 kNBO in one
// launch (two binary32 sums per tile, added in the epilogue), wider ones in
// launches of kNBO.
static hipError_t sweep_update(Handle& h, hipStream_t st, int bm, const double* A,
                               int64_t lda, const double* B, int64_t ldb, double* C,
                               int64_t ldc, int M, int N, int K, double alpha,
                               double beta, bool lower, bool diag_mask,
                               GemmSkip skip = GemmSkip()) {
  const bool f32 = h.opts.precision == SPI_MIXED;
  if (f32 && K <= 2 * kNBO)
    return gemm(st, bm, bm, kXC, kXC, A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, lower,
                false, diag_mask, true, 0, skip, K > kNBO ? kNBO : 0);
  const int kc = f32 ? kNBO : K;
  for (int k0 = 0; k0 < K; k0 += kc) {
    const int kk = std::min(kc, K - k0);
    hipError_t e = gemm(st, bm, bm, kXC, kXC, A + (int64_t)k0 * lda, lda,
                        B + (int64_t)k0 * ldb, ldb, C, ldc, M, N, kk, alpha,
                        k0 == 0 ? beta : 1.0, lower, false, diag_mask, f32, 0, skip);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t root_sweep(Handle& h) {
  const int np = (int)h.an.n_pad;
  const int64_t ld = np;
  hipError_t e;
  if ((e = ensure_side_stream(h)) != hipSuccess) return e;
  const int NB = std::min(h.potrf_block, h.band_nb);
  const int nblk = (np + NB - 1) / NB;
  double* Bb[2] = {h.band, h.band + 2 * (int64_t)np * h.band_nb};
  double* Vb[2] = {h.band + (int64_t)np * h.band_nb, h.band + 3 * (int64_t)np * h.band_nb};
  auto width = [&](int k) { return std::min(NB, np - k * NB); };
  // band 0: gathered, swept, multiplied and scattered on the main stream
  if ((e = band_gather(h, h.stream, 0, width(0), Vb[0])) != hipSuccess) return e;
  if ((e = band_pivot_sweep(h, h.stream, 0, width(0))) != hipSuccess) return e;
  if ((e = band_product(h, h.stream, 0, width(0), Bb[0], Vb[0])) != hipSuccess) return e;
  if ((e = band_scatter(h, h.stream, 0, width(0), Bb[0], nblk == 1)) != hipSuccess)
    return e;
  for (int k = 0; k < nblk; ++k) {
    const int k0 = k * NB, kb = width(k), k1 = k0 + kb;
    const double* Bk = Bb[k & 1];
    const double* Vk = Vb[k & 1];
    const bool next = k + 1 < nblk;
    const int kbn = next ? width(k + 1) : 0, k2 = k1 + kbn;
    if (next) {
      // Lookahead: band k's update of the next pivot block alone (lower
      // storage, a small launch ahead of the bulk), then its sweeps on the
      // side stream during the bulk.  Band k is already scattered, so the
      // pivot buffers are free.
      e = sweep_update(h, h.stream, kPivotTile, Bk + k1, np, Vk + k1, np,
                       h.S + (int64_t)k1 * (ld + 1), ld, kbn, kbn, kb, -1.0, 1.0,
                       false, true);
      if (e != hipSuccess) return e;
      if ((e = hipEventRecord(h.ev_next, h.stream)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(h.side, h.ev_next, 0)) != hipSuccess) return e;
      if ((e = band_pivot_sweep(h, h.side, k1, kbn)) != hipSuccess) return e;
      if ((e = hipEventRecord(h.ev_panel, h.side)) != hipSuccess) return e;
    }
    // bulk: the lower triangle outside band k's rows and columns and outside
    // the next pivot block (negated at the end for the last band); it also
    // brings the rest of the next band up to date
    const double R = (double)(np - kb);
    const double cells = R * (R + 1) / 2 - (double)kbn * (kbn + 1) / 2;
    if (cells > 0) {
      GemmSkip band;
      band.r0 = band.c0 = k0;
      band.r1 = band.c1 = k1;
      band.s0 = k1;
      band.s1 = k2;
      phase_begin(h, kPhBulk);
      e = sweep_update(h, h.stream, h.bulk_tile, Bk, np, Vk, np, h.S, ld, np, np, kb,
                       next ? -1.0 : 1.0, next ? 1.0 : -1.0, true, false, band);
      if (e != hipSuccess) return e;
      phase_end(h, kPhBulk);
      if (h.opts.timing) h.bulk_flops += 2.0 * kb * cells;
    }
    if (next) {
      // the next band's columns (after the bulk and band k's scatter), its
      // product once the sweeps are done, and its scatter before the next
      // lookahead
      if ((e = band_gather(h, h.stream, k1, kbn, Vb[(k + 1) & 1])) != hipSuccess)
        return e;
      if ((e = hipStreamWaitEvent(h.stream, h.ev_panel, 0)) != hipSuccess) return e;
      e = band_product(h, h.stream, k1, kbn, Bb[(k + 1) & 1], Vb[(k + 1) & 1]);
      if (e != hipSuccess) return e;
      e = band_scatter(h, h.stream, k1, kbn, Bb[(k + 1) & 1], k + 2 == nblk);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// ------------------------------------------------ dense triangular solves
// Forward L z = b on the root, in chunks of kTrsvChunk rows: a single
// workgroup solves the chunk block by block with the stored inverse
// diagonal blocks, then a GEMV subtracts the chunk's contribution from all
// later rows.
__global__ __launch_bounds__(256) void k_trsv_fwd_chunk(const double* L,
                                                        int64_t ld,
                                                        const double* invd,
                                                        double* z, int c0,
                                                        int c1) {
  __shared__ double part[4][kNB];
  __shared__ double acc[kNB];
  const int t = threadIdx.x, i = t % kNB, q = t / kNB;
  for (int r0 = c0; r0 < c1; r0 += kNB) {
    double s = 0.0;
    for (int j = c0 + q; j < r0; j += 4) s += L[(int64_t)(r0 + i) + (int64_t)j * ld] * z[j];
    part[q][i] = s;
    __syncthreads();
    if (t < kNB) acc[t] = z[r0 + t] - (part[0][t] + part[1][t] + part[2][t] + part[3][t]);
    __syncthreads();
    const double* X = invd + (int64_t)(r0 / kNB) * kNB * kNB;
    double v = 0.0;
    for (int p = q; p < kNB; p += 4) v += X[i + p * kNB] * acc[p];
    part[q][i] = v;
    __syncthreads();
    if (t < kNB) z[r0 + t] = part[0][t] + part[1][t] + part[2][t] + part[3][t];
    __syncthreads();
  }
}

// z[r] -= sum_{j in [c0, c1)} L[r, j] z[j] for r in [c1, n): 64 rows per block.
__global__ __launch_bounds__(256) void k_gemv_n(const double* L, int64_t ld,
                                                double* z, int c0, int c1) {
  __shared__ double part[4][kNB];
  const int t = threadIdx.x, i = t % kNB, q = t / kNB;
  const int r = c1 + blockIdx.x * kNB + i;
  double s = 0.0;
  for (int j = c0 + q; j < c1; j += 4) s += L[(int64_t)r + (int64_t)j * ld] * z[j];
  part[q][i] = s;
  __syncthreads();
  if (t < kNB) z[c1 + blockIdx.x * kNB + t] -= part[0][t] + part[1][t] + part[2][t] + part[3][t];
}

// Backward L^T x = z on chunk [c0, c1), blocks in reverse order.
__global__ __launch_bounds__(256) void k_trsv_bwd_chunk(const double* L,
                                                        int64_t ld,
                                                        const double* invd,
                                                        double* z, int c0,
                                                        int c1) {
  __shared__ double acc[kNB];
  __shared__ double part[4][kNB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int r0 = c1 - kNB; r0 >= c0; r0 -= kNB) {
    // acc[i] = z[r0+i] - sum_{j in [r0+kNB, c1)} L[j, r0+i] x[j]
    for (int ii = wave; ii < kNB; ii += 4) {
      double s = 0.0;
      for (int j = r0 + kNB + lane; j < c1; j += 64)
        s += L[(int64_t)j + (int64_t)(r0 + ii) * ld] * z[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) acc[ii] = z[r0 + ii] - s;
    }
    __syncthreads();
    // x_blk = X^T acc
    const double* X = invd + (int64_t)(r0 / kNB) * kNB * kNB;
    const int i = t % kNB, q = t / kNB;
    double v = 0.0;
    for (int p = q; p < kNB; p += 4) v += X[p + i * kNB] * acc[p];
    part[q][i] = v;
    __syncthreads();
    if (t < kNB) z[r0 + t] = part[0][t] + part[1][t] + part[2][t] + part[3][t];
    __syncthreads();
  }
}

// z[i] -= sum_{j in [c0, c1)} L[j, i] x[j] for i in [0, c0): 4 outputs per block.
__global__ __launch_bounds__(256) void k_gemv_t(const double* L, int64_t ld,
                                                double* z, int c0, int c1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + wave;
  if (i >= c0) return;
  double s = 0.0;
  for (int j = c0 + lane; j < c1; j += 64) s += L[(int64_t)j + (int64_t)i * ld] * z[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) z[i] -= s;
}

// ------------------------------------- solves with the inverse root factor
// With W = L^-1 available (lower triangular, zeros stored above the
// diagonal) the two root substitutions are the products z = W v and
// x = W^T z, read once from HBM at full width instead of a serial sweep.
constexpr int kMvChunk = 512;

// part[C][r] = sum_{j in chunk C} W[r, j] v[j] for the 64 rows of block I
__global__ __launch_bounds__(256) void k_trmv_lower_part(const double* __restrict__ W,
                                                         int64_t ld,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ part,
                                                         int np) {
  __shared__ double red[4][kNB];
  const int I = blockIdx.x, C = blockIdx.y;
  const int c0 = C * kMvChunk;
  if (c0 > I * kNB + kNB - 1) return;  // chunk entirely above the diagonal
  const int t = threadIdx.x, i = t % kNB, g = t / kNB;
  const int r = I * kNB + i;
  const int c1 = min(np, c0 + kMvChunk);
  double s = 0.0;
  for (int j = c0 + g; j < c1; j += 4) s += W[(int64_t)r + (int64_t)j * ld] * v[j];
  red[g][i] = s;
  __syncthreads();
  if (t < kNB)
    part[(int64_t)C * np + I * kNB + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

__global__ void k_trmv_lower_reduce(const double* __restrict__ part,
                                    double* __restrict__ z, int np) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np;
       r += gridDim.x * blockDim.x) {
    const int last = (r / kNB * kNB + kNB - 1) / kMvChunk;
    double s = 0.0;
    for (int C = 0; C <= last; ++C) s += part[(int64_t)C * np + r];
    z[r] = s;
  }
}

// x[j] = sum_{i >= j} W[i, j] z[i]: one wave per column.
__global__ __launch_bounds__(256) void k_trmv_upper_t(const double* __restrict__ W,
                                                      int64_t ld,
                                                      const double* __restrict__ z,
                                                      double* __restrict__ x, int np) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= np) return;
  const double* col = W + (int64_t)j * ld;
  double s = 0.0;
  for (int i = j + lane; i < np; i += 64) s += col[i] * z[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[j] = s;
}

// z (in/out, length n_pad): z := W^T (W z), using tmp (n_pad) and part.
hipError_t root_inv_apply(Handle& h, double* z, double* tmp) {
  const int np = (int)h.an.n_pad;
  const int nch = (np + kMvChunk - 1) / kMvChunk;
  hipLaunchKernelGGL(k_trmv_lower_part, dim3(np / kNB, nch), dim3(256), 0,
                     h.stream, h.W, (int64_t)np, z, h.vpart, np);
  hipLaunchKernelGGL(k_trmv_lower_reduce, dim3((np + 255) / 256), dim3(256), 0,
                     h.stream, h.vpart, tmp, np);
  hipLaunchKernelGGL(k_trmv_upper_t, dim3((np + 3) / 4), dim3(256), 0, h.stream,
                     h.W, (int64_t)np, tmp, z, np);
  return hipGetLastError();
}

// y = Z v with Z symmetric in lower storage, in one pass over the lower
// triangle.  Workgroup (I, C) stages the 64 x 64 tiles (I, J), J <= I, of
// column chunk C through LDS one after the other (the next tile's loads in
// flight during the current one's sums) and forms both products of each
// tile: the row sums Z_IJ v_J, added up over the chunk into rowpart[C][r],
// and the column sums Z_IJ^T v_I (strictly below the diagonal) into
// colpart[I][c].  k_symv_reduce adds the partial sums of each entry in a
// fixed order.
constexpr int kSymChunk = 128;  // columns per workgroup of the symmetric product

__global__ __launch_bounds__(256) void k_symv_part(const double* __restrict__ Z,
                                                   int64_t ld,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ rowpart,
                                                   double* __restrict__ colpart,
                                                   int np) {
  __shared__ double T[kNB][kNB + 1];
  __shared__ double vI[kNB], vJ[kNB];
  __shared__ double red[4][kNB];
  const int I = blockIdx.x, C = blockIdx.y;
  const int J0 = C * (kSymChunk / kNB), J1 = min(I + 1, J0 + kSymChunk / kNB);
  if (J0 > I) return;  // chunk entirely above the diagonal
  const int t = threadIdx.x, i = t % kNB, g = t / kNB;
  const int64_t r0 = (int64_t)I * kNB;
  if (t < kNB) vI[t] = v[r0 + t];
  constexpr int kPer = kNB * kNB / 256;
  double zr[kPer];
  auto load = [&](int J) {
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      zr[q] = Z[(r0 + i) + ((int64_t)J * kNB + g + 4 * q) * ld];
  };
  load(J0);
  double rs = 0.0;
  for (int J = J0; J < J1; ++J) {
    __syncthreads();  // the previous tile's sums are done
#pragma unroll
    for (int q = 0; q < kPer; ++q) T[i][g + 4 * q] = zr[q];
    if (t < kNB) vJ[t] = v[(int64_t)J * kNB + t];
    __syncthreads();
    if (J + 1 < J1) load(J + 1);
    const bool diag = J == I;
    // row i: columns b = g, g + 4, ... (b <= i on the diagonal tile)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int b = g + 4 * q;
      if (!diag || b <= i) rs += T[i][b] * vJ[b];
    }
    // column j = i: rows a = g, g + 4, ... (a > j on the diagonal tile)
    double cs = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int a = g + 4 * q;
      if (!diag || a > i) cs += T[a][i] * vI[a];
    }
    red[g][i] = cs;
    __syncthreads();
    if (t < kNB)
      colpart[(int64_t)I * np + (int64_t)J * kNB + t] =
          (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
  }
  __syncthreads();
  red[g][i] = rs;
  __syncthreads();
  if (t < kNB)
    rowpart[(int64_t)C * np + r0 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// y[r] = sum of the row partial sums of r's chunks, then of the column
// partial sums of the tile rows at or below r's.
__global__ void k_symv_reduce(const double* __restrict__ rowpart,
                              const double* __restrict__ colpart,
                              double* __restrict__ y, int np) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np;
       r += gridDim.x * blockDim.x) {
    const int last = r / kSymChunk, Ir = r / kNB;
    double s = 0.0;
    for (int C = 0; C <= last; ++C) s += rowpart[(int64_t)C * np + r];
    for (int I = Ir; I < np / kNB; ++I) s += colpart[(int64_t)I * np + r];
    y[r] = s;
  }
}

// z (in/out, length n_pad): z := Z z with the root inverse held in S.
hipError_t root_sym_apply(Handle& h, double* z) {
  const int np = (int)h.an.n_pad;
  const int nch = (np + kSymChunk - 1) / kSymChunk;
  double* rowpart = h.vpart;
  double* colpart = h.vpart + (int64_t)nch * np;
  hipLaunchKernelGGL(k_symv_part, dim3(np / kNB, nch), dim3(256), 0, h.stream, h.S,
                     (int64_t)np, z, rowpart, colpart, np);
  hipLaunchKernelGGL(k_symv_reduce, dim3((np + 255) / 256), dim3(256), 0, h.stream,
                     rowpart, colpart, z, np);
  return hipGetLastError();
}

// the symmetric product's row partial sums (chunks x n_pad) and column
// partial sums (tile rows x n_pad); the triangular products use fewer
// (kMvChunk >= kSymChunk)
int64_t root_inv_part_size(int64_t np) {
  static_assert(kMvChunk >= kSymChunk, "partial-sum buffer sized for the symmetric product");
  return ((np + kSymChunk - 1) / kSymChunk) * np + (np / kNB) * np;
}

hipError_t root_trsv_fwd(Handle& h, double* z) {
  const int np = (int)h.an.n_pad;
  for (int c0 = 0; c0 < np; c0 += kTrsvChunk) {
    int c1 = std::min(np, c0 + kTrsvChunk);
    hipLaunchKernelGGL(k_trsv_fwd_chunk, dim3(1), dim3(256), 0, h.stream, h.S,
                       (int64_t)np, h.invd, z, c0, c1);
    if (c1 < np)
      hipLaunchKernelGGL(k_gemv_n, dim3((np - c1) / kNB), dim3(256), 0,
                         h.stream, h.S, (int64_t)np, z, c0, c1);
  }
  return hipGetLastError();
}

hipError_t root_trsv_bwd(Handle& h, double* z) {
  const int np = (int)h.an.n_pad;
  int nchunk = (np + kTrsvChunk - 1) / kTrsvChunk;
  for (int c = nchunk - 1; c >= 0; --c) {
    int c0 = c * kTrsvChunk, c1 = std::min(np, c0 + kTrsvChunk);
    hipLaunchKernelGGL(k_trsv_bwd_chunk, dim3(1), dim3(256), 0, h.stream, h.S,
                       (int64_t)np, h.invd, z, c0, c1);
    if (c0 > 0)
      hipLaunchKernelGGL(k_gemv_t, dim3((c0 + 3) / 4), dim3(256), 0, h.stream,
                         h.S, (int64_t)np, z, c0, c1);
  }
  return hipGetLastError();
}

}  // namespace spi

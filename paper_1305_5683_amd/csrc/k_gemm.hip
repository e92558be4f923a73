// Tiled GEMM on the gfx950 matrix cores, FP64 data in and out.
//
// The bulk of the root front's Cholesky factorisation, of the inversion of
// its factor and of the product giving the root block of A^-1 are dense
// contractions; they all go through this one kernel.  The compute type T is
// double (v_mfma_f64_16x16x4f64) or, for the mixed-precision path, float
// (v_mfma_f32_16x16x4f32): operands are rounded to T when staged in LDS and
// accumulated in T over the K range of one launch; the epilogue combines
// the result with C in FP64, so sums across launches (the panels of a
// blocked factorisation) are FP64.
//
// C[i, j] = beta * C[i, j] + alpha * sum_k opA(i, k) * opB(k, j)
// Operand access:
//   A, kXC: A(i, k) = A[i + k * lda]   (i contiguous)
//   A, kKC: A(i, k) = A[k + i * lda]   (k contiguous)
//   B, kXC: B(k, j) = B[j + k * ldb]   (j contiguous)
//   B, kKC: B(k, j) = B[k + j * ldb]   (k contiguous)
// Tiles are BM x BN, 256 threads = 4 waves in a 2 x 2 grid; each wave owns
// a (BM/2) x (BN/2) block of 16 x 16 accumulators.  K advances in slabs of
// kKT = 16, staged through two LDS buffers with a register prefetch.
// `kmask`: kGemmKStartCol (B lower triangular: k >= j only) and
// kGemmKEndRow (A lower triangular: k <= i only) trim the K range per tile.
// `lower`: only tiles with I >= J are enumerated (square tiles) and the
// diagonal tiles write their lower triangle only.  `kstart_diag`: the K
// range of tile (I, J) starts at I * BM (products whose left factor is lower
// triangular with zeros stored above the diagonal).  `diag_mask`: C's
// origin lies on the matrix diagonal and only its lower part (i >= j) is
// written; tiles entirely above the diagonal do nothing.  `skip`: tiles
// whose rows meet [r0, r1), whose columns meet [c0, c1), or whose rows and
// columns both meet [s0, s1) do nothing (the parts that other work owns at
// the same time).  `ksplit` (binary32 only, a kernel instantiation of its
// own): the products of k < ksplit and of k >= ksplit are summed apart in
// binary32 and added in binary64 in the epilogue.
#include <hip/hip_runtime.h>

#include "spi_internal.h"

namespace spi {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kKT = 16;
constexpr int kGroup = 8;      // tile rows per group of the launch order
// LDS layouts.  kXC slabs are [k][x] with the row padded so that a row's
// stride is 64 bytes mod 256: the four 16-lane groups of a fragment read
// (k = ks .. ks + 3) then start in four different quarters of the banks
// (8 elements of padding for double, 16 for float).  kKC slabs are [x][k]
// with stride kKT + 2 so the lanes of a fragment read spread over banks.
template <typename T> struct PadXC;
template <> struct PadXC<double> { static constexpr int v = 8; };
template <> struct PadXC<float> { static constexpr int v = 16; };
constexpr int kStrKC = kKT + 2;

struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int M, N, K;
  double alpha, beta;
  int lower, kstart_diag, diag_mask;
  int kmask;  // kGemmKStartCol / kGemmKEndRow: triangular operands
  int tiles_m, tiles_n, n_tiles;
  GemmSkip skip;
  int ksplit;  // binary32: the products of k < ksplit and of k >= ksplit are
               // summed apart and added in binary64 (K <= 2 ksplit)
};

// Logical tile t -> (I, J).  Tiles are visited in groups of kGroup tile
// rows, column by column inside a group; with xcd_remap<8> each XCD takes 8
// consecutive logical tiles of every 64 (one column of the group, sharing
// its panel of B), and every XCD gets an equal share of each part of the
// launch (tiles whose K range depends on the tile index stay balanced).
__device__ inline void tile_of(const GemmArgs& g, int t, int& I, int& J) {
  const int G = kGroup;
  if (!g.lower) {
    const int grp = t / (G * g.tiles_n);
    const int local = t - grp * G * g.tiles_n;
    const int gs = min(G, g.tiles_m - grp * G);
    I = grp * G + local % gs;
    J = local / gs;
    return;
  }
  // lower triangle: group grp holds rows [grp*G, grp*G + gs); columns
  // J < grp*G have gs tiles each, the diagonal block a triangle.
  int grp = 0, base = 0;
  for (;;) {
    const int gs = min(G, g.tiles_m - grp * G);
    const int cnt = grp * G * gs + gs * (gs + 1) / 2;
    if (t < base + cnt) break;
    base += cnt;
    ++grp;
  }
  const int gs = min(G, g.tiles_m - grp * G);
  int local = t - base;
  if (local < grp * G * gs) {
    J = local / gs;
    I = grp * G + local % gs;
    return;
  }
  local -= grp * G * gs;
  int d = 0;
  while (local >= gs - d) {
    local -= gs - d;
    ++d;
  }
  J = grp * G + d;
  I = J + local;
}

template <int BM, int BN, int OPA, int OPB, typename T, bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_gemm(GemmArgs g) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MI = WM / 16, NI = WN / 16;
  constexpr int kPadXC = PadXC<T>::v;
  constexpr int A_SZ = (OPA == kXC) ? kKT * (BM + kPadXC) : BM * kStrKC;
  constexpr int B_SZ = (OPB == kXC) ? kKT * (BN + kPadXC) : BN * kStrKC;
  __shared__ T As[2][A_SZ];
  __shared__ T Bs[2][B_SZ];

  int I, J;
  tile_of(g, xcd_remap<8>(blockIdx.x, g.n_tiles), I, J);
  const int i0 = I * BM, j0 = J * BN;
  if (g.diag_mask && i0 + BM - 1 < j0) return;  // tile above the diagonal
  if ((i0 < g.skip.r1 && i0 + BM > g.skip.r0) ||
      (j0 < g.skip.c1 && j0 + BN > g.skip.c0) ||
      (i0 < g.skip.s1 && i0 + BM > g.skip.s0 && j0 < g.skip.s1 && j0 + BN > g.skip.s0))
    return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // K range of the tile: an upper-triangular A starts at i0 (kstart_diag),
  // a lower-triangular B starts at j0, a lower-triangular A ends at i0 + BM
  int kbeg = g.kstart_diag ? i0 : 0;
  if (g.kmask & kGemmKStartCol) kbeg = max(kbeg, j0);
  const int kend = (g.kmask & kGemmKEndRow) ? min(g.K, i0 + BM) : g.K;

  // global -> register staging: each thread moves EA (EB) doubles per slab
  constexpr int EA = BM * kKT / 256, EB = BN * kKT / 256;
  double ra[EA], rb[EB];

  // kXC: a k-row of the slab is X contiguous doubles; X / 2 threads read it
  // as double2 (a wave covers whole rows), so both the global read and the
  // LDS write of one instruction are contiguous.  kKC: every x has kKT
  // contiguous k; kKT / E threads share one x.  Each thread's addresses are
  // formed once (slab kbeg) and advanced by one slab per iteration.
  auto first = [&](const double* base, int64_t ld, int x0, int op, int X,
                   int E) -> const double* {
    if (op == kXC) {
      const int tpr = X / 2, r0 = tid / tpr, x = (tid % tpr) * 2;
      return base + (int64_t)(x0 + x) + (int64_t)(kbeg + r0) * ld;
    }
    const int tpx = kKT / E, x = tid / tpx, kk = (tid % tpx) * E;
    return base + (int64_t)(kbeg + kk) + (int64_t)(x0 + x) * ld;
  };
  auto load = [&](const double* p, int64_t ld, int op, int X, int E, double* r) {
    if (op == kXC) {
      const int64_t st = (int64_t)(256 / (X / 2)) * ld;  // rows per pass
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        double2 v = *reinterpret_cast<const double2*>(p + i * st);
        r[2 * i] = v.x;
        r[2 * i + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; e += 2) {
        double2 v = *reinterpret_cast<const double2*>(p + e);
        r[e] = v.x;
        r[e + 1] = v.y;
      }
    }
  };
  auto store = [&](T* L, int op, int X, int E, const double* r) {
    if (op == kXC) {
      const int tpr = X / 2, rows = 256 / tpr;
      const int r0 = tid / tpr, x = (tid % tpr) * 2;
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        const int kk = r0 + i * rows;
        L[kk * (X + kPadXC) + x] = (T)r[2 * i];
        L[kk * (X + kPadXC) + x + 1] = (T)r[2 * i + 1];
      }
    } else {
      const int tpx = kKT / E;
      const int x = tid / tpx, kk = (tid % tpx) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) L[x * kStrKC + kk + e] = (T)r[e];
    }
  };

  typedef typename Acc<T>::type VA;
  // SPLIT (binary32 only): the sums of k < ksplit and k >= ksplit are kept
  // apart and added in binary64 (an instantiation of its own, since the
  // second accumulator set costs registers)
  constexpr bool kF32 = SPLIT && sizeof(T) == 4;
  VA acc[MI][NI];
  VA acc0[kF32 ? MI : 1][kF32 ? NI : 1];  // binary32: sums of k < ksplit
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b) acc[a][b] = VA{0, 0, 0, 0};
  if constexpr (kF32) {
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
      for (int b = 0; b < NI; ++b) acc0[a][b] = VA{0, 0, 0, 0};
  }

  const double* pa = first(g.A, g.lda, i0, OPA, BM, EA);
  const double* pb = first(g.B, g.ldb, j0, OPB, BN, EB);
  const int64_t stepA = (OPA == kXC) ? kKT * g.lda : kKT;
  const int64_t stepB = (OPB == kXC) ? kKT * g.ldb : kKT;
  // Two LDS buffers: slab s is read from buffer s & 1 while slab s + 1 is
  // stored into the other one (after the slab's products, so they are not
  // held up by the global loads), and the loads of slab s + 2 are issued;
  // one barrier per slab.
  if (kbeg < kend) {
    load(pa, g.lda, OPA, BM, EA, ra);
    load(pb, g.ldb, OPB, BN, EB, rb);
    store(As[0], OPA, BM, EA, ra);
    store(Bs[0], OPB, BN, EB, rb);
    if (kbeg + kKT < kend) {
      pa += stepA;
      pb += stepB;
      load(pa, g.lda, OPA, BM, EA, ra);
      load(pb, g.ldb, OPB, BN, EB, rb);
    }
  }
  const int lx = lane & 15, lk = lane >> 4;
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    if constexpr (kF32) {
      if (k0 == g.ksplit && k0 != 0) {  // start of the second binary32 sum
#pragma unroll
        for (int a = 0; a < MI; ++a)
#pragma unroll
          for (int b = 0; b < NI; ++b) {
            acc0[a][b] = acc[a][b];
            acc[a][b] = VA{0, 0, 0, 0};
          }
      }
    }
    __syncthreads();  // slab k0 complete in buf; buf ^ 1 no longer read
    const T* Ab = As[buf];
    const T* Bb = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < kKT; ks += 4) {
      T fa[MI], fb[NI];
#pragma unroll
      for (int a = 0; a < MI; ++a) {
        const int x = wm * WM + a * 16 + lx, kk = ks + lk;
        fa[a] = (OPA == kXC) ? Ab[kk * (BM + kPadXC) + x] : Ab[x * kStrKC + kk];
      }
#pragma unroll
      for (int b = 0; b < NI; ++b) {
        const int x = wn * WN + b * 16 + lx, kk = ks + lk;
        fb[b] = (OPB == kXC) ? Bb[kk * (BN + kPadXC) + x] : Bb[x * kStrKC + kk];
      }
      // D = Bfrag^T * Afrag, so lane (lx, lk) holds output row i = lx of
      // the 16 x 16 block (column-major stores of C stay contiguous over 16
      // rows).  Its column for item v follows the instruction's result
      // layout: FP64 puts D[r][c] in lane c + 16 (r % 4), item r / 4, so
      // j = 4 v + lk; FP32 puts it in lane c + 16 (r / 4), item r % 4, so
      // j = 4 lk + v.
#pragma unroll
      for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
    }
    if (k0 + kKT < kend) {
      store(As[buf ^ 1], OPA, BM, EA, ra);
      store(Bs[buf ^ 1], OPB, BN, EB, rb);
      if (k0 + 2 * kKT < kend) {
        pa += stepA;
        pb += stepB;
        load(pa, g.lda, OPA, BM, EA, ra);
        load(pb, g.ldb, OPB, BN, EB, rb);
      }
    }
    buf ^= 1;
  }

  // Epilogue, one row block of 16 at a time: all of its C loads are issued
  // before any store (a load after a store to the same array would wait for
  // the store), then the stores, predicated on the triangle mask.
  const bool mask_tile = (g.lower && I == J) || g.diag_mask;
#pragma unroll
  for (int a = 0; a < MI; ++a) {
    const int i = i0 + wm * WM + a * 16 + lx;
    double cv[NI][4];
    if (g.beta != 0.0) {
#pragma unroll
      for (int b = 0; b < NI; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = j0 + wn * WN + b * 16 +
                        (sizeof(T) == 8 ? v * 4 + lk : lk * 4 + v);
          cv[b][v] = g.C[(int64_t)i + (int64_t)j * g.ldc];
        }
    }
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + wn * WN + b * 16 +
                      (sizeof(T) == 8 ? v * 4 + lk : lk * 4 + v);
        double r;
        if constexpr (kF32)
          r = g.alpha * ((double)acc0[a][b][v] + (double)acc[a][b][v]);
        else
          r = g.alpha * (double)acc[a][b][v];
        if (g.beta != 0.0) r = fma(g.beta, cv[b][v], r);
        if (!(mask_tile && i < j)) g.C[(int64_t)i + (int64_t)j * g.ldc] = r;
      }
  }
}

template <int BM, int BN, int OPA, int OPB, typename T, bool SPLIT = false>
static hipError_t gemm_t(hipStream_t s, const GemmArgs& a0) {
  GemmArgs a = a0;
  a.tiles_m = a.M / BM;
  a.tiles_n = a.N / BN;
  a.n_tiles = a.lower ? a.tiles_m * (a.tiles_m + 1) / 2 : a.tiles_m * a.tiles_n;
  if (a.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<BM, BN, OPA, OPB, T, SPLIT>), dim3(a.n_tiles), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t gemm(hipStream_t s, int bm, int bn, int opA, int opB,
                const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc, int M, int N, int K, double alpha,
                double beta, bool lower, bool kstart_diag, bool diag_mask,
                bool f32, int kmask, GemmSkip skip, int ksplit) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (M % bm || N % bn || K % kKT || (lower && (bm != bn || M != N)))
    return hipErrorInvalidValue;
  if (ksplit < 0 || ksplit % kKT || (ksplit && (!f32 || K > 2 * ksplit)))
    return hipErrorInvalidValue;
  GemmArgs a{A, B, C, lda, ldb, ldc, M, N, K, alpha, beta, lower ? 1 : 0,
             kstart_diag ? 1 : 0, diag_mask ? 1 : 0, kmask, 0, 0, 0, skip, ksplit};
  if (ksplit) {  // the shapes of the sweep updates
    if (bm == 128 && bn == 128 && opA == kXC && opB == kXC)
      return gemm_t<128, 128, kXC, kXC, float, true>(s, a);
    if (bm == 64 && bn == 64 && opA == kXC && opB == kXC)
      return gemm_t<64, 64, kXC, kXC, float, true>(s, a);
    if (bm == 32 && bn == 32 && opA == kXC && opB == kXC)
      return gemm_t<32, 32, kXC, kXC, float, true>(s, a);
    return hipErrorInvalidValue;
  }
#define SPI_GEMM_CASE(BM_, BN_, OA, OB)                                   \
  if (bm == BM_ && bn == BN_ && opA == OA && opB == OB)                  \
    return f32 ? gemm_t<BM_, BN_, OA, OB, float>(s, a)                   \
               : gemm_t<BM_, BN_, OA, OB, double>(s, a);
#define SPI_GEMM_OPS(BM_, BN_)          \
  SPI_GEMM_CASE(BM_, BN_, kXC, kXC)     \
  SPI_GEMM_CASE(BM_, BN_, kXC, kKC)     \
  SPI_GEMM_CASE(BM_, BN_, kKC, kKC)
  SPI_GEMM_OPS(128, 128)
  SPI_GEMM_OPS(128, 64)
  SPI_GEMM_OPS(64, 128)
  SPI_GEMM_OPS(64, 64)
  SPI_GEMM_CASE(32, 32, kXC, kXC)
#undef SPI_GEMM_OPS
#undef SPI_GEMM_CASE
  return hipErrorInvalidValue;
}

}  // namespace spi

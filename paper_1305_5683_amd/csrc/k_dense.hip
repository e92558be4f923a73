// Dense kernels of the root front (gfx950, FP64 MFMA).
//
// The root front of the multifrontal factorisation (Sect. 3.2.2 of Bouchet
// et al.: a partial factorisation of a dense matrix at every node, here the
// complete factorisation at the root) is a dense SPD matrix stored
// column-major, n_pad x n_pad, padded with identity.  Its Cholesky factor,
// the inverse of that factor and the product giving the root block of A^-1
// are blocked algorithms whose bulk is one tiled GEMM kernel on the
// 16x16x4 FP64 matrix cores; the kNB x kNB diagonal blocks are factored and
// inverted by a single-workgroup kernel in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "spi_internal.h"

namespace spi {

typedef double v4d __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- GEMM
// C[i, j] = beta * C[i, j] + alpha * sum_k opA(i, k) * opB(k, j)
// Operand access:
//   A, kXC: A(i, k) = A[i + k * lda]   (i contiguous)
//   A, kKC: A(i, k) = A[k + i * lda]   (k contiguous)
//   B, kXC: B(k, j) = B[j + k * ldb]   (j contiguous)
//   B, kKC: B(k, j) = B[k + j * ldb]   (k contiguous)
// Tiles are BM x BN, 256 threads = 4 waves in a 2 x 2 grid, each wave owns a
// (BM/2) x (BN/2) block of 16 x 16 MFMA accumulators.  K advances in slabs
// of kKT = 16 staged through LDS (register prefetch of the next slab).
// `lower`: only tiles with I >= J are enumerated (square tiles) and the
// diagonal tiles write their lower triangle only.  `kstart_diag`: the K
// range of tile (I, J) starts at I * BM (products with a lower-triangular
// left factor whose upper part is stored as zeros).
constexpr int kKT = 16;

struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int M, N, K;
  double alpha, beta;
  int lower, kstart_diag;
  int tiles_m, tiles_n, n_tiles;
};

__device__ inline void tile_of(const GemmArgs& g, int t, int& I, int& J) {
  if (g.lower) {
    // t = I (I + 1) / 2 + J, J <= I
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
  } else {
    I = t % g.tiles_m;
    J = t / g.tiles_m;
  }
}

// Map the hardware workgroup index to a logical tile so that consecutive
// logical tiles (which share operand panels) run on the same XCD, whose L2
// they then share.  Workgroups are dispatched round-robin over 8 XCDs.
__device__ inline int xcd_remap(int w, int n) {
  const int nx = 8;
  int per = n / nx, rem = n % nx;
  int x = w % nx, local = w / nx;
  return x * per + min(x, rem) + local;
}

template <int BM, int BN, int OPA, int OPB>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MI = WM / 16, NI = WN / 16;
  // LDS layouts: kXC operands as [k][x], kKC operands as [x][k] (+1 pad)
  constexpr int A_SZ = (OPA == kXC) ? kKT * BM : BM * (kKT + 1);
  constexpr int B_SZ = (OPB == kXC) ? kKT * BN : BN * (kKT + 1);
  __shared__ double As[A_SZ];
  __shared__ double Bs[B_SZ];

  const int wg = xcd_remap(blockIdx.x, g.n_tiles);
  int I, J;
  tile_of(g, wg, I, J);
  const int i0 = I * BM, j0 = J * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  int kbeg = g.kstart_diag ? i0 : 0;
  const int kend = g.K;

  // global -> register staging: each thread moves EA (EB) doubles per slab
  constexpr int EA = BM * kKT / 256, EB = BN * kKT / 256;
  double ra[EA], rb[EB];

  auto load_a = [&](int k0) {
    if (OPA == kXC) {  // rows of the slab: kKT rows of BM contiguous doubles
      constexpr int TPR = BM / EA;  // threads per k-row
      int kk = tid / TPR, x = (tid % TPR) * EA;
      const double* p = g.A + (int64_t)(i0 + x) + (int64_t)(k0 + kk) * g.lda;
#pragma unroll
      for (int e = 0; e < EA; e += 2) {
        double2 v = *reinterpret_cast<const double2*>(p + e);
        ra[e] = v.x;
        ra[e + 1] = v.y;
      }
    } else {  // for each x: kKT contiguous k
      constexpr int TPX = kKT / EA;  // threads per x
      int x = tid / TPX, kk = (tid % TPX) * EA;
      const double* p = g.A + (int64_t)(k0 + kk) + (int64_t)(i0 + x) * g.lda;
#pragma unroll
      for (int e = 0; e < EA; e += 2) {
        double2 v = *reinterpret_cast<const double2*>(p + e);
        ra[e] = v.x;
        ra[e + 1] = v.y;
      }
    }
  };
  auto store_a = [&]() {
    if (OPA == kXC) {
      constexpr int TPR = BM / EA;
      int kk = tid / TPR, x = (tid % TPR) * EA;
#pragma unroll
      for (int e = 0; e < EA; ++e) As[kk * BM + x + e] = ra[e];
    } else {
      constexpr int TPX = kKT / EA;
      int x = tid / TPX, kk = (tid % TPX) * EA;
#pragma unroll
      for (int e = 0; e < EA; ++e) As[x * (kKT + 1) + kk + e] = ra[e];
    }
  };
  auto load_b = [&](int k0) {
    if (OPB == kXC) {
      constexpr int TPR = BN / EB;
      int kk = tid / TPR, x = (tid % TPR) * EB;
      const double* p = g.B + (int64_t)(j0 + x) + (int64_t)(k0 + kk) * g.ldb;
#pragma unroll
      for (int e = 0; e < EB; e += 2) {
        double2 v = *reinterpret_cast<const double2*>(p + e);
        rb[e] = v.x;
        rb[e + 1] = v.y;
      }
    } else {
      constexpr int TPX = kKT / EB;
      int x = tid / TPX, kk = (tid % TPX) * EB;
      const double* p = g.B + (int64_t)(k0 + kk) + (int64_t)(j0 + x) * g.ldb;
#pragma unroll
      for (int e = 0; e < EB; e += 2) {
        double2 v = *reinterpret_cast<const double2*>(p + e);
        rb[e] = v.x;
        rb[e + 1] = v.y;
      }
    }
  };
  auto store_b = [&]() {
    if (OPB == kXC) {
      constexpr int TPR = BN / EB;
      int kk = tid / TPR, x = (tid % TPR) * EB;
#pragma unroll
      for (int e = 0; e < EB; ++e) Bs[kk * BN + x + e] = rb[e];
    } else {
      constexpr int TPX = kKT / EB;
      int x = tid / TPX, kk = (tid % TPX) * EB;
#pragma unroll
      for (int e = 0; e < EB; ++e) Bs[x * (kKT + 1) + kk + e] = rb[e];
    }
  };
  auto frag_a = [&](int kk, int x) -> double {  // A(x, kk), x tile-local
    return (OPA == kXC) ? As[kk * BM + x] : As[x * (kKT + 1) + kk];
  };
  auto frag_b = [&](int kk, int x) -> double {  // B(kk, x)
    return (OPB == kXC) ? Bs[kk * BN + x] : Bs[x * (kKT + 1) + kk];
  };

  v4d acc[MI][NI];
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) {
    load_a(kbeg);
    load_b(kbeg);
  }
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    __syncthreads();
    store_a();
    store_b();
    __syncthreads();
    if (k0 + kKT < kend) {
      load_a(k0 + kKT);
      load_b(k0 + kKT);
    }
    const int lx = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < kKT; ks += 4) {
      double fa[MI], fb[NI];
#pragma unroll
      for (int a = 0; a < MI; ++a) fa[a] = frag_a(ks + lk, wm * WM + a * 16 + lx);
#pragma unroll
      for (int b = 0; b < NI; ++b) fb[b] = frag_b(ks + lk, wn * WN + b * 16 + lx);
      // D = Bfrag^T * Afrag.  The 16x16 result D[r][c] sits in lane
      // c + 16 * (r % 4), item r / 4; with the operands swapped, lane
      // (lx, lk) item v holds output row i = lx and column j = 4 * v + lk,
      // which keeps the stores of a column-major C contiguous over 16 rows.
#pragma unroll
      for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[b], fa[a],
                                                           acc[a][b], 0, 0, 0);
    }
  }

  // epilogue
  const int lx = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wm * WM + a * 16 + lx;
        int j = j0 + wn * WN + b * 16 + v * 4 + lk;
        if (g.lower && I == J && i < j) continue;
        double* c = g.C + (int64_t)i + (int64_t)j * g.ldc;
        double r = g.alpha * acc[a][b][v];
        if (g.beta != 0.0) r += g.beta * (*c);
        *c = r;
      }
}

template <int BM, int BN, int OPA, int OPB>
static hipError_t gemm_t(hipStream_t s, const GemmArgs& a0) {
  GemmArgs a = a0;
  a.tiles_m = a.M / BM;
  a.tiles_n = a.N / BN;
  a.n_tiles = a.lower ? a.tiles_m * (a.tiles_m + 1) / 2 : a.tiles_m * a.tiles_n;
  if (a.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<BM, BN, OPA, OPB>), dim3(a.n_tiles), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t gemm(hipStream_t s, int bm, int bn, int opA, int opB,
                const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc, int M, int N, int K, double alpha,
                double beta, bool lower, bool kstart_diag) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (M % bm || N % bn || K % kKT || (lower && (bm != bn || M != N)))
    return hipErrorInvalidValue;
  GemmArgs a{A, B, C, lda, ldb, ldc, M, N, K, alpha, beta, lower ? 1 : 0,
             kstart_diag ? 1 : 0, 0, 0, 0};
#define SPI_GEMM_CASE(BM_, BN_, OA, OB)                                   \
  if (bm == BM_ && bn == BN_ && opA == OA && opB == OB)                  \
    return gemm_t<BM_, BN_, OA, OB>(s, a);
#define SPI_GEMM_OPS(BM_, BN_)          \
  SPI_GEMM_CASE(BM_, BN_, kXC, kXC)     \
  SPI_GEMM_CASE(BM_, BN_, kXC, kKC)     \
  SPI_GEMM_CASE(BM_, BN_, kKC, kKC)
  SPI_GEMM_OPS(128, 128)
  SPI_GEMM_OPS(128, 64)
  SPI_GEMM_OPS(64, 128)
  SPI_GEMM_OPS(64, 64)
#undef SPI_GEMM_OPS
#undef SPI_GEMM_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------ diagonal block kernels
// Cholesky of the kNB x kNB diagonal block at (k0, k0) in LDS, then its
// triangular inverse.  Writes L back (lower triangle incl. diagonal) and the
// inverse, column-major with explicit zeros above the diagonal, to `inv`.
// A pivot that is not positive and finite records its elimination index
// (base + k0 + k) with atomicMin in `fail` and continues with pivot 1.
__global__ __launch_bounds__(256) void k_potrf_diag(double* S, int64_t ld,
                                                    int k0, double* inv,
                                                    int64_t* fail,
                                                    int64_t base) {
  __shared__ double T[kNB][kNB + 1];
  __shared__ double X[kNB][kNB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kNB * kNB; e += 256) {
    int i = e % kNB, j = e / kNB;
    T[i][j] = (i >= j) ? S[(int64_t)(k0 + i) + (int64_t)(k0 + j) * ld] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < kNB; ++k) {
    double d = T[k][k];
    bool bad = !(d > 0.0) || !isfinite(d);
    double lkk = bad ? 1.0 : sqrt(d);
    __syncthreads();
    if (t == 0) {
      if (bad) atomicMin((unsigned long long*)fail,
                         (unsigned long long)(base + k0 + k));
      T[k][k] = lkk;
    }
    if (t > k && t < kNB) T[t][k] /= lkk;
    __syncthreads();
    const int nt = kNB - 1 - k;
    for (int e = t; e < nt * nt; e += 256) {
      int i = k + 1 + e % nt, j = k + 1 + e / nt;
      if (i >= j) T[i][j] -= T[i][k] * T[j][k];
    }
    __syncthreads();
  }
  // X = T^-1 row by row: X[i][j] = (delta_ij - sum_{j<=q<i} T[i][q] X[q][j]) / T[i][i]
  for (int i = 0; i < kNB; ++i) {
    if (t < kNB) {
      int j = t;
      double v = 0.0;
      if (j <= i) {
        double s = (i == j) ? 1.0 : 0.0;
        for (int q = j; q < i; ++q) s -= T[i][q] * X[q][j];
        v = s / T[i][i];
      }
      X[i][j] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < kNB * kNB; e += 256) {
    int i = e % kNB, j = e / kNB;
    if (i >= j) S[(int64_t)(k0 + i) + (int64_t)(k0 + j) * ld] = T[i][j];
    inv[i + j * kNB] = X[i][j];
  }
}

// Copy a kNB x kNB column-major block (with its zeros) into a matrix.
__global__ void k_put_block(double* W, int64_t ld, int k0, const double* blk) {
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) {
    int i = e % kNB, j = e / kNB;
    W[(int64_t)(k0 + i) + (int64_t)(k0 + j) * ld] = blk[e];
  }
}

// Zero the whole root front and put 1 on the padded diagonal.
__global__ void k_root_fill(double* S, int64_t n_pad, int64_t n_root) {
  int64_t total = n_pad * n_pad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e % n_pad, j = e / n_pad;
    S[e] = (i == j && i >= n_root) ? 1.0 : 0.0;
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

hipError_t launch_root_fill(Handle& h) {
  if (!h.an.n_pad) return hipSuccess;
  hipLaunchKernelGGL(k_root_fill, dim3(fill_grid(h.an.n_pad * h.an.n_pad)),
                     dim3(256), 0, h.stream, h.S, h.an.n_pad, h.an.n_root);
  return hipGetLastError();
}

static int pick_bm(int M) { return (M % 128 == 0) ? 128 : 64; }

// Right-looking blocked Cholesky of the root front, block kNB.
hipError_t root_potrf(Handle& h) {
  const int np = (int)h.an.n_pad;
  const int64_t ld = np;
  hipError_t e = hipSuccess;
  const int64_t base = (int64_t)h.an.leaf_cols.size();
  for (int k0 = 0; k0 < np; k0 += kNB) {
    double* inv = h.invd + (int64_t)(k0 / kNB) * kNB * kNB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, h.stream, h.S, ld,
                       k0, inv, h.flag, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int rest = np - k0 - kNB;
    if (rest <= 0) break;
    double* P = h.S + (int64_t)(k0 + kNB) + (int64_t)k0 * ld;
    // panel: P := P * inv^T  (each tile owns whole rows of the panel)
    e = gemm(h.stream, pick_bm(rest), 64, kXC, kXC, P, ld, inv, kNB, P, ld,
             rest, kNB, kNB, 1.0, 0.0, false, false);
    if (e != hipSuccess) return e;
    // trailing update, lower triangle: S22 -= P P^T
    double* C = h.S + (int64_t)(k0 + kNB) * (ld + 1);
    int t = (rest % 128 == 0) ? 128 : 64;
    e = gemm(h.stream, t, t, kXC, kXC, P, ld, P, ld, C, ld, rest, rest, kNB,
             -1.0, 1.0, true, false);
    if (e != hipSuccess) return e;
  }
  return e;
}

// Inverse of the root factor (W = L^-1, in place on a copy of L) followed
// by Z = W^T W, the root block of A^-1 (lower triangle).
//
// Inversion by block columns, left to right.  With the first block columns
// already inverted, row block k to the left holds L_k,<k X_<k and the block
// rows below hold L_>k,<k X_<k.  Step k, with X_kk = L_kk^-1 (kept from the
// factorisation):
//   T      = L_>k,k X_kk              (becomes the state of block column k)
//   S_>k,<k -= T * S_k,<k
//   S_k,<k  = -X_kk * S_k,<k          (final row block k of L^-1)
//   S_kk    = X_kk
hipError_t root_trtri(Handle& h) {
  const int np = (int)h.an.n_pad;
  const int64_t ld = np;
  hipError_t e;
  hipLaunchKernelGGL(k_copy_lower, dim3(fill_grid((int64_t)np * np)), dim3(256),
                     0, h.stream, h.S, h.W, (int64_t)np);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k0 = 0; k0 < np; k0 += kNB) {
    const double* inv = h.invd + (int64_t)(k0 / kNB) * kNB * kNB;
    const int rest = np - k0 - kNB;
    double* W21 = h.W + (int64_t)(k0 + kNB) + (int64_t)k0 * ld;
    double* W10 = h.W + (int64_t)k0;
    double* W20 = h.W + (int64_t)(k0 + kNB);
    if (rest > 0) {
      e = gemm(h.stream, pick_bm(rest), 64, kXC, kKC, W21, ld, inv, kNB, W21,
               ld, rest, kNB, kNB, 1.0, 0.0, false, false);
      if (e != hipSuccess) return e;
      if (k0 > 0) {
        e = gemm(h.stream, pick_bm(rest), (k0 % 128 == 0) ? 128 : 64, kXC, kKC,
                 W21, ld, W10, ld, W20, ld, rest, k0, kNB, -1.0, 1.0, false,
                 false);
        if (e != hipSuccess) return e;
      }
    }
    if (k0 > 0) {
      e = gemm(h.stream, 64, (k0 % 128 == 0) ? 128 : 64, kXC, kKC, inv, kNB,
               W10, ld, W10, ld, kNB, k0, kNB, -1.0, 0.0, false, false);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_put_block, dim3(1), dim3(256), 0, h.stream, h.W, ld,
                       k0, inv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Z = W^T W (lower tiles); tile (I, J) sums over K >= I since W is lower
// triangular with stored zeros above the diagonal.
hipError_t root_lauum(Handle& h) {
  const int np = (int)h.an.n_pad;
  return gemm(h.stream, 128, 128, kKC, kKC, h.W, np, h.W, np, h.Z, np, np, np,
              np, 1.0, 0.0, true, true);
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

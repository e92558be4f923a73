// Learned preconditioner and FP32 preconditioned conjugate gradients.
//
// Many energy bands share the pattern of H (Sect. 2.2.3). Iterative
// solvers need a good preconditioner to converge (Sect. 3.1). The direct
// factor of a reference band, A_r = L L^T, is reused as the base
// preconditioner of later bands. A small network, applied to every unknown
// with shared weights, predicts a diagonal correction d:
//   M^-1 = D A_r^-1 D,   D = diag(d),   d_j = exp(g(f_j))
// Features of unknown j (band b against the reference r):
//   f0 = log(A_b,jj / A_r,jj),  f1 = [j is a root-front unknown],
//   f2 = mean of f0 over the unknowns of the same kind
// Network (hidden width HID, float32):
//   h1 = tanh(W1 f + b1), h2 = tanh(W2 h1 + b2), g = w3.h2 + b3 + wl.f
// Flat parameter layout:
//   [W1 (HID x 3, row-major), b1, W2 (HID x HID, row-major), b2, w3, b3, wl (3)]
// Training minimises, per band with direct solution x of A_b x = rhs,
//   L = e^T A_b e / (2 x^T rhs),   e = M^-1 rhs - x
// The network's forward and backward passes are these kernels; the
// parameter gradients are reduced per block in FP64, then over blocks in a
// fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "spi_internal.h"

namespace spi {

namespace {

constexpr int kF = 3;      // features per unknown
constexpr int kLpThreads = 256;

template <int HID>
struct NetLayout {
  static constexpr int oW1 = 0;
  static constexpr int ob1 = oW1 + HID * kF;
  static constexpr int oW2 = ob1 + HID;
  static constexpr int ob2 = oW2 + HID * HID;
  static constexpr int ow3 = ob2 + HID;
  static constexpr int ob3 = ow3 + HID;
  static constexpr int owl = ob3 + 1;
  static constexpr int P = owl + kF;
};

// Grid of a grid-stride kernel (capped: the kernel loops).
int grid_of(int64_t n, int per) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65535));
}

// Grid of a one-thread-per-unknown kernel: exact (n < 2^31).
int grid_exact(int64_t n) {
  return (int)std::max<int64_t>(1, (n + kLpThreads - 1) / kLpThreads);
}

}  // namespace

int64_t lp_param_count(int hidden) {
  return (int64_t)hidden * kF + hidden + (int64_t)hidden * hidden + hidden +
         hidden + 1 + kF;
}

// ------------------------------------------------------------- features
// f0, f1 and per-block sums of f0 by kind: part[4 b + {0,1,2,3}] =
// (sum over leaf unknowns, count, sum over root unknowns, count).
__global__ __launch_bounds__(kLpThreads) void k_lp_f0(
    const double* __restrict__ diag_b, const double* __restrict__ diag_r,
    const int32_t* __restrict__ root_of_col, float* __restrict__ phi,
    double* __restrict__ part, int64_t n) {
  __shared__ double red[4][kLpThreads / 64];
  const int64_t j = (int64_t)blockIdx.x * kLpThreads + threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < n) {
    const double f0 = log(diag_b[j] / diag_r[j]);
    const int root = root_of_col[j] >= 0;
    phi[3 * j] = (float)f0;
    phi[3 * j + 1] = root ? 1.0f : 0.0f;
    s[2 * root] = f0;
    s[2 * root + 1] = 1.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = s[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < kLpThreads / 64; ++w) v += red[threadIdx.x][w];
    part[4 * blockIdx.x + threadIdx.x] = v;
  }
}

// f2 = mean of f0 over the unknown's kind (every block re-reduces the
// per-block sums in the same order, so all blocks agree).
__global__ __launch_bounds__(kLpThreads) void k_lp_f2(
    const double* __restrict__ part, int nblocks,
    const int32_t* __restrict__ root_of_col, float* __restrict__ phi, int64_t n) {
  __shared__ float mean[2];
  if (threadIdx.x < 2) {
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      s += part[4 * b + 2 * threadIdx.x];
      c += part[4 * b + 2 * threadIdx.x + 1];
    }
    mean[threadIdx.x] = c > 0.0 ? (float)(s / c) : 0.0f;
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kLpThreads + threadIdx.x;
  if (j < n) phi[3 * j + 2] = mean[root_of_col[j] >= 0 ? 1 : 0];
}

// ------------------------------------------------------------- network
template <int HID>
__device__ inline float net_forward(const float* prm, const float* f, float* h1,
                                    float* h2) {
  using N = NetLayout<HID>;
#pragma unroll
  for (int i = 0; i < HID; ++i) {
    float a = prm[N::ob1 + i];
#pragma unroll
    for (int q = 0; q < kF; ++q) a += prm[N::oW1 + i * kF + q] * f[q];
    h1[i] = tanhf(a);
  }
#pragma unroll
  for (int i = 0; i < HID; ++i) {
    float a = prm[N::ob2 + i];
#pragma unroll
    for (int k = 0; k < HID; ++k) a += prm[N::oW2 + i * HID + k] * h1[k];
    h2[i] = tanhf(a);
  }
  float g = prm[N::ob3];
#pragma unroll
  for (int i = 0; i < HID; ++i) g += prm[N::ow3 + i] * h2[i];
#pragma unroll
  for (int q = 0; q < kF; ++q) g += prm[N::owl + q] * f[q];
  return g;
}

// d_j = exp(g_j) (FP64 output; the network runs in FP32).
template <int HID>
__global__ __launch_bounds__(kLpThreads) void k_lp_forward(
    const float* __restrict__ params, const float* __restrict__ phi,
    double* __restrict__ d, int64_t n) {
  using N = NetLayout<HID>;
  __shared__ float prm[N::P];
  for (int p = threadIdx.x; p < N::P; p += kLpThreads) prm[p] = params[p];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kLpThreads + threadIdx.x;
  if (j >= n) return;
  float f[kF] = {phi[3 * j], phi[3 * j + 1], phi[3 * j + 2]};
  float h1[HID], h2[HID];
  d[j] = exp((double)net_forward<HID>(prm, f, h1, h2));
}

// Parameter gradient of sum_j dg_j g_j, dg_j = dL/dd_j * d_j: the forward
// pass is recomputed per unknown, each parameter's contributions are summed
// over the block in FP64 and written to part[block * P + p].
template <int HID>
__global__ __launch_bounds__(kLpThreads) void k_lp_backward(
    const float* __restrict__ params, const float* __restrict__ phi,
    const double* __restrict__ dLdd, const double* __restrict__ d,
    double* __restrict__ part, int64_t n) {
  using N = NetLayout<HID>;
  constexpr int NW = kLpThreads / 64;
  __shared__ float prm[N::P];
  __shared__ double red[NW][N::P];
  for (int p = threadIdx.x; p < N::P; p += kLpThreads) prm[p] = params[p];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * kLpThreads + threadIdx.x;
  const bool live = j < n;
  float f[kF] = {0.f, 0.f, 0.f}, h1[HID], h2[HID];
  float dg = 0.0f;
  if (live) {
    f[0] = phi[3 * j];
    f[1] = phi[3 * j + 1];
    f[2] = phi[3 * j + 2];
    dg = (float)(dLdd[j] * d[j]);
  }
  net_forward<HID>(prm, f, h1, h2);
  float d2[HID], d1[HID];
#pragma unroll
  for (int i = 0; i < HID; ++i) d2[i] = dg * prm[N::ow3 + i] * (1.0f - h2[i] * h2[i]);
#pragma unroll
  for (int k = 0; k < HID; ++k) {
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < HID; ++i) s += d2[i] * prm[N::oW2 + i * HID + k];
    d1[k] = s * (1.0f - h1[k] * h1[k]);
  }
  if (!live) {
#pragma unroll
    for (int i = 0; i < HID; ++i) d1[i] = d2[i] = 0.0f;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto put = [&](int p, float c) {
    double v = (double)c;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][p] = v;
  };
#pragma unroll
  for (int i = 0; i < HID; ++i) {
#pragma unroll
    for (int q = 0; q < kF; ++q) put(N::oW1 + i * kF + q, d1[i] * f[q]);
    put(N::ob1 + i, d1[i]);
  }
#pragma unroll
  for (int i = 0; i < HID; ++i) {
#pragma unroll
    for (int k = 0; k < HID; ++k) put(N::oW2 + i * HID + k, d2[i] * h1[k]);
    put(N::ob2 + i, d2[i]);
    put(N::ow3 + i, live ? dg * h2[i] : 0.0f);
  }
  put(N::ob3, dg);
#pragma unroll
  for (int q = 0; q < kF; ++q) put(N::owl + q, dg * f[q]);
  __syncthreads();
  for (int p = threadIdx.x; p < N::P; p += kLpThreads) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += red[w][p];
    part[(int64_t)blockIdx.x * N::P + p] = v;
  }
}

// grad[p] = sum over blocks (fixed order).
__global__ void k_lp_reduce(const double* __restrict__ part, int nblocks, int P,
                            double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double v = 0.0;
  for (int b = 0; b < nblocks; ++b) v += part[(int64_t)b * P + p];
  grad[p] = v;
}

// Adam step (Kingma & Ba), bias-corrected, in FP32.
__global__ void k_lp_adam(float* __restrict__ params, const double* __restrict__ grad,
                          float* __restrict__ m, float* __restrict__ v, int P,
                          float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float g = (float)grad[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

// ---------------------------------------------------- FP64 vector kernels
#define SPI_GRID_STRIDE(i, n)                                                 \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_vmul(const double* a, const double* b, double* out, int64_t n) {
  SPI_GRID_STRIDE(i, n) out[i] = a[i] * b[i];
}
// e = d v - x
__global__ void k_lp_err(const double* d, const double* v, const double* x,
                         double* e, int64_t n) {
  SPI_GRID_STRIDE(i, n) e[i] = d[i] * v[i] - x[i];
}
// u = d q s
__global__ void k_lp_u(const double* d, const double* q, double s, double* u,
                       int64_t n) {
  SPI_GRID_STRIDE(i, n) u[i] = d[i] * (q[i] * s);
}
// dL/dd = (q s) v + rhs w
__global__ void k_lp_dldd(const double* q, double s, const double* v,
                          const double* rhs, const double* w, double* out,
                          int64_t n) {
  SPI_GRID_STRIDE(i, n) out[i] = (q[i] * s) * v[i] + rhs[i] * w[i];
}
// y = -x
__global__ void k_neg(const double* x, double* y, int64_t n) {
  SPI_GRID_STRIDE(i, n) y[i] = -x[i];
}
__global__ void k_fill1(double* x, int64_t n) {
  SPI_GRID_STRIDE(i, n) x[i] = 1.0;
}

// Dot products: per-block partial sums in FP64 (host adds them in order).
template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* __restrict__ a,
                                             const T* __restrict__ b,
                                             double* __restrict__ part, int64_t n) {
  __shared__ double red[4];
  double s = 0.0;
  SPI_GRID_STRIDE(i, n) s += (double)a[i] * (double)b[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------- FP32 PCG kernels
// val32 = H's values in binary32, undoing the (power-of-two) column scale.
__global__ void k_val32(const double* __restrict__ val, const int32_t* __restrict__ col,
                        const double* __restrict__ scale, float* __restrict__ v32,
                        int64_t nnz) {
  SPI_GRID_STRIDE(e, nnz) v32[e] = (float)(scale ? val[e] / scale[col[e]] : val[e]);
}
// t_r = w_r sum_e h_re p_col(e) (one wave per row, FP32 products, FP32 sum)
__global__ __launch_bounds__(256) void k_hx_f32(const int64_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const float* __restrict__ v32,
                                                const double* __restrict__ w,
                                                const float* __restrict__ p,
                                                float* __restrict__ t, int64_t m) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  float s = 0.0f;
  for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) s += v32[e] * p[col[e]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) t[r] = (float)w[r] * s;
}
// q_c = sum_r h_rc t_r (one wave per column)
__global__ __launch_bounds__(256) void k_htt_f32(const int64_t* __restrict__ colptr,
                                                 const int64_t* __restrict__ csc_pos,
                                                 const int32_t* __restrict__ csc_row,
                                                 const float* __restrict__ v32,
                                                 const float* __restrict__ t,
                                                 float* __restrict__ q, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  float s = 0.0f;
  for (int64_t k = colptr[c] + lane; k < colptr[c + 1]; k += 64)
    s += v32[csc_pos[k]] * t[csc_row[k]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) q[c] = s;
}
// out64 = in32 * d ; out32 = in64 * d (d may be null = 1)
__global__ void k_to64(const float* in, const double* d, double* out, int64_t n) {
  SPI_GRID_STRIDE(i, n) out[i] = d ? (double)in[i] * d[i] : (double)in[i];
}
__global__ void k_to32(const double* in, const double* d, float* out, int64_t n) {
  SPI_GRID_STRIDE(i, n) out[i] = (float)(d ? in[i] * d[i] : in[i]);
}
// y += a x (FP32)
__global__ void k_axpy32(float a, const float* x, float* y, int64_t n) {
  SPI_GRID_STRIDE(i, n) y[i] += a * x[i];
}
// y = x + b y (FP32)
__global__ void k_xpby32(const float* x, float b, float* y, int64_t n) {
  SPI_GRID_STRIDE(i, n) y[i] = x[i] + b * y[i];
}
// x64 += e32
__global__ void k_acc64(const float* e, double* x, int64_t n) {
  SPI_GRID_STRIDE(i, n) x[i] += (double)e[i];
}
// e32 = 0
__global__ void k_zero32(float* e, int64_t n) {
  SPI_GRID_STRIDE(i, n) e[i] = 0.0f;
}

// ------------------------------------------------------------ launchers
constexpr int kVecBlocks = 256;

#define SPI_LAUNCH_VEC(kern, n, ...)                                          \
  hipLaunchKernelGGL(kern, dim3(grid_of((n), 256)), dim3(256), 0, s, __VA_ARGS__)

hipError_t lp_features(hipStream_t s, const double* diag_b, const double* diag_r,
                       const int32_t* root_of_col, float* phi, double* part,
                       int64_t n) {
  const int nb = grid_exact(n);
  hipLaunchKernelGGL(k_lp_f0, dim3(nb), dim3(kLpThreads), 0, s, diag_b, diag_r,
                     root_of_col, phi, part, n);
  hipLaunchKernelGGL(k_lp_f2, dim3(nb), dim3(kLpThreads), 0, s, part, nb,
                     root_of_col, phi, n);
  return hipGetLastError();
}

int lp_backward_blocks(int64_t n) { return grid_exact(n); }

#define SPI_LP_HID(H, call)       \
  switch (H) {                    \
    case 8: call(8); break;       \
    case 16: call(16); break;     \
    case 32: call(32); break;     \
    default: return hipErrorInvalidValue; \
  }

hipError_t lp_forward(hipStream_t s, int hidden, const float* params,
                      const float* phi, double* d, int64_t n) {
#define SPI_FWD(H)                                                              \
  hipLaunchKernelGGL(k_lp_forward<H>, dim3(grid_exact(n)),                    \
                     dim3(kLpThreads), 0, s, params, phi, d, n)
  SPI_LP_HID(hidden, SPI_FWD)
#undef SPI_FWD
  return hipGetLastError();
}

hipError_t lp_backward(hipStream_t s, int hidden, const float* params,
                       const float* phi, const double* dLdd, const double* d,
                       double* part, double* grad, int64_t n) {
  const int nb = grid_exact(n);
#define SPI_BWD(H)                                                              \
  hipLaunchKernelGGL(k_lp_backward<H>, dim3(nb), dim3(kLpThreads), 0, s,       \
                     params, phi, dLdd, d, part, n)
  SPI_LP_HID(hidden, SPI_BWD)
#undef SPI_BWD
  const int P = (int)lp_param_count(hidden);
  hipLaunchKernelGGL(k_lp_reduce, dim3((P + 255) / 256), dim3(256), 0, s, part,
                     nb, P, grad);
  return hipGetLastError();
}

hipError_t lp_adam(hipStream_t s, float* params, const double* grad, float* m,
                   float* v, int P, float lr, int step) {
  const float c1 = 1.0f - powf(0.9f, (float)step);
  const float c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_lp_adam, dim3((P + 255) / 256), dim3(256), 0, s, params,
                     grad, m, v, P, lr, c1, c2);
  return hipGetLastError();
}

hipError_t vec_mul(hipStream_t s, const double* a, const double* b, double* out,
                   int64_t n) {
  SPI_LAUNCH_VEC(k_vmul, n, a, b, out, n);
  return hipGetLastError();
}
hipError_t lp_err(hipStream_t s, const double* d, const double* v, const double* x,
                  double* e, int64_t n) {
  SPI_LAUNCH_VEC(k_lp_err, n, d, v, x, e, n);
  return hipGetLastError();
}
hipError_t lp_u(hipStream_t s, const double* d, const double* q, double sc,
                double* u, int64_t n) {
  SPI_LAUNCH_VEC(k_lp_u, n, d, q, sc, u, n);
  return hipGetLastError();
}
hipError_t lp_dldd(hipStream_t s, const double* q, double sc, const double* v,
                   const double* rhs, const double* w, double* out, int64_t n) {
  SPI_LAUNCH_VEC(k_lp_dldd, n, q, sc, v, rhs, w, out, n);
  return hipGetLastError();
}
hipError_t vec_neg(hipStream_t s, const double* x, double* y, int64_t n) {
  SPI_LAUNCH_VEC(k_neg, n, x, y, n);
  return hipGetLastError();
}
hipError_t vec_ones(hipStream_t s, double* x, int64_t n) {
  SPI_LAUNCH_VEC(k_fill1, n, x, n);
  return hipGetLastError();
}
hipError_t dot_partials64(hipStream_t s, const double* a, const double* b,
                          double* part, int64_t n) {
  hipLaunchKernelGGL(k_dot<double>, dim3(kVecBlocks), dim3(256), 0, s, a, b, part, n);
  return hipGetLastError();
}
hipError_t dot_partials32(hipStream_t s, const float* a, const float* b,
                          double* part, int64_t n) {
  hipLaunchKernelGGL(k_dot<float>, dim3(kVecBlocks), dim3(256), 0, s, a, b, part, n);
  return hipGetLastError();
}
int dot_blocks() { return kVecBlocks; }

hipError_t pcg_val32(Handle& h, float* v32) {
  hipStream_t s = h.stream;
  const int64_t nnz = h.an.nnz;
  if (!nnz) return hipSuccess;
  SPI_LAUNCH_VEC(k_val32, nnz, h.val, h.d.col,
                 h.opts.equilibrate ? h.colscale : nullptr, v32, nnz);
  return hipGetLastError();
}
// q = A p = H^T W H p in FP32 (t: m floats of scratch)
hipError_t pcg_spmv32(Handle& h, const float* v32, const float* p, float* t,
                      float* q) {
  const Analysis& a = h.an;
  hipLaunchKernelGGL(k_hx_f32, dim3((unsigned)((a.m + 3) / 4)), dim3(256), 0,
                     h.stream, h.d.rowptr, h.d.col, v32, h.w, p, t, a.m);
  hipLaunchKernelGGL(k_htt_f32, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0,
                     h.stream, h.d.colptr, h.d.csc_pos, h.d.csc_row, v32, t, q,
                     a.n);
  return hipGetLastError();
}
hipError_t vec_to64(hipStream_t s, const float* in, const double* d, double* out,
                    int64_t n) {
  SPI_LAUNCH_VEC(k_to64, n, in, d, out, n);
  return hipGetLastError();
}
hipError_t vec_to32(hipStream_t s, const double* in, const double* d, float* out,
                    int64_t n) {
  SPI_LAUNCH_VEC(k_to32, n, in, d, out, n);
  return hipGetLastError();
}
hipError_t vec_axpy32(hipStream_t s, float a, const float* x, float* y, int64_t n) {
  SPI_LAUNCH_VEC(k_axpy32, n, a, x, y, n);
  return hipGetLastError();
}
hipError_t vec_xpby32(hipStream_t s, const float* x, float b, float* y, int64_t n) {
  SPI_LAUNCH_VEC(k_xpby32, n, x, b, y, n);
  return hipGetLastError();
}
hipError_t vec_acc64(hipStream_t s, const float* e, double* x, int64_t n) {
  SPI_LAUNCH_VEC(k_acc64, n, e, x, n);
  return hipGetLastError();
}
hipError_t vec_zero32(hipStream_t s, float* e, int64_t n) {
  SPI_LAUNCH_VEC(k_zero32, n, e, n);
  return hipGetLastError();
}

}  // namespace spi

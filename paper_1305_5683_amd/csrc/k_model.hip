// Kernels of the model-level loops around the solver: the empty-field
// (detector pattern) update of App. A.4 and the Poisson-likelihood terms of
// App. A.1-A.2.  Every reduction runs in a fixed order (lane-strided sums,
// then a shuffle tree; fixed block partitions), so results repeat bit for
// bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "spi_internal.h"

namespace spi {

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return __shfl(v, 0, 64);
}

static unsigned waves4(int64_t items) {
  return (unsigned)std::max<int64_t>(1, (items + 3) / 4);
}

// ------------------------------------------------------------ empty field
// One wave per row i: e_i = (H x)_i with H's current (unscaled) values, the
// source counts s_i = e_i minus the background term, chi_i = w_i (y_i -
// e_i)^2, and the row's shares of the closed-form pattern update (App.
// A.4): with g_i = I_i t_i (I_i = x at the background column),
//   LSQ: num_i = (y_i - s_i) g_i w_i, den_i = g_i^2 w_i;
//   MLE: num_i = y_i - s_i,           den_i = g_i.
// Rows without a background entry give num = den = 0.
__global__ __launch_bounds__(256) void k_ef_rows(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ w,
    const double* __restrict__ y, const double* __restrict__ x,
    const int64_t* __restrict__ bg_pos, const double* __restrict__ t, int stat,
    double* __restrict__ numden, double* __restrict__ chi, int64_t m) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  double e = 0.0;
  for (int64_t k = rowptr[r] + lane; k < rowptr[r + 1]; k += 64) e += val[k] * x[col[k]];
  e = wave_sum(e);
  if (lane != 0) return;
  const int64_t b = bg_pos[r];
  const double yr = y[r], wr = w[r];
  const double res = yr - e;
  chi[r] = wr * res * res;
  double num = 0.0, den = 0.0;
  if (b >= 0) {
    const double I = x[col[b]];
    const double s = e - val[b] * I;
    const double g = I * t[r];
    if (stat == 0) {
      num = (yr - s) * g * wr;
      den = g * g * wr;
    } else {
      num = yr - s;
      den = g;
    }
  }
  numden[2 * r] = num;
  numden[2 * r + 1] = den;
}

// One wave per pattern unit u: U_u = sum num / sum den over the unit's rows
// (kept when the sum of den is zero), then the unit's background entries
// val[bg_pos[i]] = U_u t_i.
__global__ __launch_bounds__(256) void k_ef_units(
    const int64_t* __restrict__ grp_ptr, const int32_t* __restrict__ grp_rows,
    const double* __restrict__ numden, const int64_t* __restrict__ bg_pos,
    const double* __restrict__ t, double* __restrict__ U, double* __restrict__ val,
    int n_u, int update) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= n_u) return;
  const int64_t q0 = grp_ptr[u], q1 = grp_ptr[u + 1];
  double Uu = U[u];
  if (update) {
    double num = 0.0, den = 0.0;
    for (int64_t q = q0 + lane; q < q1; q += 64) {
      const int32_t r = grp_rows[q];
      num += numden[2 * r];
      den += numden[2 * r + 1];
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (den != 0.0) Uu = num / den;
    if (lane == 0) U[u] = Uu;
  }
  for (int64_t q = q0 + lane; q < q1; q += 64) {
    const int32_t r = grp_rows[q];
    const int64_t b = bg_pos[r];
    if (b >= 0) val[b] = Uu * t[r];
  }
}

// Fixed-order sum of v[0..n): block b of kSumBlocks sums the b-th of
// kSumBlocks equal ranges (thread-strided, then a tree), part[b]; one more
// block sums the parts.
constexpr int kSumBlocks = 256;

__global__ __launch_bounds__(256) void k_sum_part(const double* __restrict__ v,
                                                  int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t chunk = (n + kSumBlocks - 1) / kSumBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = std::min<int64_t>(n, lo + chunk);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += v[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sum_final(double* __restrict__ part) {
  __shared__ double red[4];
  double s = threadIdx.x < kSumBlocks ? part[threadIdx.x] : 0.0;
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[kSumBlocks] = (red[0] + red[1]) + (red[2] + red[3]);
}

int64_t sum_scratch_size() { return kSumBlocks + 1; }

hipError_t launch_sum(hipStream_t s, const double* v, int64_t n, double* part) {
  hipLaunchKernelGGL(k_sum_part, dim3(kSumBlocks), dim3(256), 0, s, v, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part);
  return hipGetLastError();
}

hipError_t launch_ef_rows(Handle& h, const double* val, const double* y,
                          const double* x, const int64_t* bg_pos, const double* t,
                          int stat) {
  const int64_t m = h.an.m;
  hipLaunchKernelGGL(k_ef_rows, dim3(waves4(m)), dim3(256), 0, h.stream, h.d.rowptr,
                     h.d.col, val, h.w, y, x, bg_pos, t, stat, h.vdd, h.vrow, m);
  return hipGetLastError();
}

hipError_t launch_ef_units(Handle& h, const int64_t* grp_ptr, const int32_t* grp_rows,
                           int n_u, const int64_t* bg_pos, const double* t, double* U,
                           double* val, bool update) {
  if (n_u <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ef_units, dim3(waves4(n_u)), dim3(256), 0, h.stream, grp_ptr,
                     grp_rows, h.vdd, bg_pos, t, U, val, n_u, update ? 1 : 0);
  return hipGetLastError();
}

}  // namespace spi

namespace spi {

// ------------------------------------------------- Poisson likelihood terms
// One wave per row i, with e_i = (H x)_i: the likelihood term
// c_i = 2 (e_i - d_i ln e_i) (2 e_i where d_i = 0), the Newton weight
// w_i = d_i / e_i^2 and r_i = d_i / e_i - 1.  A row with e_i <= 0 is not a
// valid model: it sets *bad and gives c_i = 0.
__global__ __launch_bounds__(256) void k_cash_rows(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ x,
    const double* __restrict__ y, double* __restrict__ c, double* __restrict__ w,
    double* __restrict__ r, int64_t* bad, int64_t m) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  double e = 0.0;
  for (int64_t k = rowptr[i] + lane; k < rowptr[i + 1]; k += 64) e += val[k] * x[col[k]];
  e = wave_sum(e);
  if (lane != 0) return;
  const double d = y[i];
  if (!(e > 0.0)) {
    atomicOr((unsigned long long*)bad, 1ull);
    c[i] = 0.0;
    w[i] = 0.0;
    r[i] = 0.0;
    return;
  }
  c[i] = d > 0.0 ? 2.0 * (e - d * log(e)) : 2.0 * e;
  const double q = d / e;
  w[i] = q / e;
  r[i] = q - 1.0;
}

// g_j = sum_i H_ij r_i over column j (one wave per column; the column-ordered
// values are equilibrated, H S, and the power-of-two scale is divided out
// exactly).
__global__ __launch_bounds__(256) void k_htr(const int64_t* __restrict__ colptr,
                                             const int32_t* __restrict__ csc_row,
                                             const double* __restrict__ valc,
                                             const double* __restrict__ scale,
                                             const double* __restrict__ r,
                                             double* __restrict__ g, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double s = 0.0;
  for (int64_t k = colptr[j] + lane; k < colptr[j + 1]; k += 64) s += valc[k] * r[csc_row[k]];
  s = wave_sum(s);
  if (lane == 0) g[j] = scale ? s / scale[j] : s;
}

__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] * b[i];
}

// xt = x + a * dx
__global__ void k_axpy_to(const double* __restrict__ x, double a,
                          const double* __restrict__ dx, double* __restrict__ xt,
                          int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    xt[i] = x[i] + a * dx[i];
}

// max_i |a dx_i| and max_i |x_i| into nm[0..1] (ordered bit patterns of
// non-negative doubles, reduced with atomicMax; nm zeroed first)
__global__ void k_maxabs2(const double* __restrict__ dx, double a,
                          const double* __restrict__ x, unsigned long long* nm,
                          int64_t n) {
  double m0 = 0.0, m1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    m0 = fmax(m0, fabs(a * dx[i]));
    m1 = fmax(m1, fabs(x[i]));
  }
  for (int off = 32; off > 0; off >>= 1) {
    m0 = fmax(m0, __shfl_down(m0, off, 64));
    m1 = fmax(m1, __shfl_down(m1, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&nm[0], (unsigned long long)__double_as_longlong(m0));
    atomicMax(&nm[1], (unsigned long long)__double_as_longlong(m1));
  }
}

static unsigned vec_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

hipError_t launch_cash_rows(Handle& h, const double* val, const double* x,
                            const double* y, double* w, double* r) {
  const int64_t m = h.an.m;
  hipLaunchKernelGGL(k_cash_rows, dim3(waves4(m)), dim3(256), 0, h.stream, h.d.rowptr,
                     h.d.col, val, x, y, h.vrow, w, r, h.flag + 3, m);
  return hipGetLastError();
}

hipError_t launch_htr(Handle& h, const double* r, double* g) {
  hipLaunchKernelGGL(k_htr, dim3(waves4(h.an.n)), dim3(256), 0, h.stream, h.d.colptr,
                     h.d.csc_row, h.valc, h.opts.equilibrate ? h.colscale : nullptr, r,
                     g, h.an.n);
  return hipGetLastError();
}

hipError_t launch_dot(Handle& h, const double* a, const double* b, double* tmp,
                      int64_t n) {
  hipLaunchKernelGGL(k_mul, dim3(vec_grid(n)), dim3(256), 0, h.stream, a, b, tmp, n);
  return launch_sum(h.stream, tmp, n, h.vsum);
}

hipError_t launch_axpy_to(Handle& h, const double* x, double a, const double* dx,
                          double* xt) {
  hipLaunchKernelGGL(k_axpy_to, dim3(vec_grid(h.an.n)), dim3(256), 0, h.stream, x, a,
                     dx, xt, h.an.n);
  return hipGetLastError();
}

hipError_t launch_maxabs2(Handle& h, const double* dx, double a, const double* x,
                          double* nm) {
  hipLaunchKernelGGL(k_maxabs2, dim3(vec_grid(h.an.n)), dim3(256), 0, h.stream, dx, a,
                     x, (unsigned long long*)nm, h.an.n);
  return hipGetLastError();
}

}  // namespace spi

// C ABI of the learned preconditioner and of FP32 preconditioned conjugate
// gradients (declared in include/spi.h).  Kernels in k_learned.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "spi_internal.h"

using namespace spi;

struct spi_lp {
  int hidden = 0;
  int P = 0;
  int step = 0;
  float* params = nullptr;  // device, P
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  double* grad = nullptr;   // device, P
  double* part = nullptr;   // device, blocks x P
  int part_blocks = 0;
};

namespace spi {

void free_lp_work(Handle& h) {
  Handle::LpWork& w = h.lp;
  void* ptrs[] = {w.v32, w.r, w.z, w.p, w.q, w.e, w.t, w.d, w.x, w.r64,
                  w.u, w.v, w.w, w.g, w.part, w.phi, w.fpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  w = Handle::LpWork{};
}

}  // namespace spi

namespace {

template <class T>
hipError_t alloc(T*& p, int64_t count) {
  if (p || count <= 0) return hipSuccess;
  return hipMalloc((void**)&p, (size_t)count * sizeof(T));
}

hipError_t ensure_lp_work(Handle& h) {
  Handle::LpWork& w = h.lp;
  const int64_t n = h.an.n, m = h.an.m;
  hipError_t e = hipSuccess;
#define A_(p, c) \
  if (e == hipSuccess) e = alloc(w.p, c)
  A_(v32, h.an.nnz); A_(r, n); A_(z, n); A_(p, n); A_(q, n); A_(e, n); A_(t, m);
  A_(d, n); A_(x, n); A_(r64, n); A_(u, n); A_(v, n); A_(w, n); A_(g, n);
  A_(part, dot_blocks()); A_(phi, 3 * n);
  A_(fpart, 4 * (int64_t)lp_backward_blocks(n));
#undef A_
  return e;
}

// Sum of the per-block dot partials on the host (synchronises the stream).
hipError_t host_sum(Handle& h, double* out) {
  std::vector<double> buf(dot_blocks());
  hipError_t e = hipMemcpyAsync(buf.data(), h.lp.part, buf.size() * sizeof(double),
                                hipMemcpyDeviceToHost, h.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h.stream);
  double s = 0.0;
  for (double v : buf) s += v;
  *out = s;
  return e;
}

hipError_t dot64(Handle& h, const double* a, const double* b, double* out) {
  hipError_t e = dot_partials64(h.stream, a, b, h.lp.part, h.an.n);
  return e == hipSuccess ? host_sum(h, out) : e;
}

hipError_t dot32(Handle& h, const float* a, const float* b, double* out) {
  hipError_t e = dot_partials32(h.stream, a, b, h.lp.part, h.an.n);
  return e == hipSuccess ? host_sum(h, out) : e;
}

// out = A_ref^-1 in with the reference factor (its column scaling undone).
hipError_t apply_ref_inv(Handle& pre, const double* in, double* out) {
  if (!pre.opts.equilibrate) return launch_solve_pass(pre, in, out);
  hipError_t e = launch_scale_vec(pre, in, pre.vbh, 0);
  if (e == hipSuccess) e = launch_solve_pass(pre, pre.vbh, pre.vxh);
  if (e == hipSuccess) e = launch_scale_vec(pre, pre.vxh, out, 0);
  return e;
}

// out = A x (FP64, double-double accumulation from H; tmp: n scratch).
// With equilibration A x = S^-1 (H S)^T W (H S) (S^-1 x).
hipError_t apply_A64(Handle& h, const double* x, double* out, double* tmp) {
  hipError_t e;
  if (!h.opts.equilibrate) {
    e = launch_residual_dd(h, nullptr, x, tmp);  // tmp = -A x
    return e == hipSuccess ? vec_neg(h.stream, tmp, out, h.an.n) : e;
  }
  e = launch_scale_vec(h, x, out, 1);
  if (e == hipSuccess) e = launch_residual_dd(h, nullptr, out, tmp);
  if (e == hipSuccess) e = vec_neg(h.stream, tmp, tmp, h.an.n);
  if (e == hipSuccess) e = launch_scale_vec(h, tmp, out, 1);
  return e;
}

// r = b - A x in FP64 (double-double accumulation).
hipError_t residual64(Handle& h, const double* b, const double* x, double* r,
                      double* tmp) {
  hipError_t e;
  if (!h.opts.equilibrate) return launch_residual_dd(h, b, x, r);
  // S^-1 (S b - (H S)^T W (H S) S^-1 x)
  e = launch_scale_vec(h, x, tmp, 1);
  if (e == hipSuccess) e = launch_scale_vec(h, b, h.vbh, 0);
  if (e == hipSuccess) e = launch_residual_dd(h, h.vbh, tmp, r);
  if (e == hipSuccess) e = launch_scale_vec(h, r, r, 1);
  return e;
}

int check_pair(Handle& h, Handle& pre) {
  if (h.an.n != pre.an.n || h.an.m != pre.an.m || h.an.nnz != pre.an.nnz)
    return fail(h, SPI_E_ARG, hipSuccess, "band and reference patterns differ");
  if (h.stream != pre.stream)
    return fail(h, SPI_E_ARG, hipSuccess,
                "band and reference handles must share one stream");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "band has no values");
  if (!pre.have_factor)
    return fail(h, SPI_E_STATE, hipSuccess, "reference handle is not factored");
  return SPI_OK;
}

// d = exp(g(features)) for band h against the reference (or d = 1).
int correction(Handle& h, Handle& pre, const spi_lp* lp) {
  Handle::LpWork& w = h.lp;
  const int64_t n = h.an.n;
  if (!lp) {
    SPI_CK(vec_ones(h.stream, w.d, n), "unit correction");
    return SPI_OK;
  }
  SPI_CK(lp_features(h.stream, h.diagA, pre.diagA, h.d.root_of_col, w.phi,
                     w.fpart, n), "features");
  SPI_CK(lp_forward(h.stream, lp->hidden, lp->params, w.phi, w.d, n),
         "network forward");
  return SPI_OK;
}

// Loss of one band and (optionally) the parameter gradient into lp->grad.
int loss_and_grad(spi_lp* lp, Handle& h, Handle& pre, const double* rhs,
                  const double* x, double* loss, bool want_grad) {
  int st = check_pair(h, pre);
  if (st != SPI_OK) return st;
  SPI_CK(ensure_lp_work(h), "learned-preconditioner scratch");
  Handle::LpWork& w = h.lp;
  const int64_t n = h.an.n;
  if ((st = correction(h, pre, lp)) != SPI_OK) return st;
  // v = A_r^-1 (d rhs); e = d v - x; q = A_b e
  SPI_CK(vec_mul(h.stream, w.d, rhs, w.u, n), "d rhs");
  SPI_CK(apply_ref_inv(pre, w.u, w.v), "reference solve");
  SPI_CK(lp_err(h.stream, w.d, w.v, x, w.r64, n), "error");
  SPI_CK(apply_A64(h, w.r64, w.g, w.x), "A e");
  double eq = 0.0, xr = 0.0;
  SPI_CK(dot64(h, w.r64, w.g, &eq), "e^T A e");
  SPI_CK(dot64(h, x, rhs, &xr), "x^T rhs");
  if (!(xr > 0.0)) return fail(h, SPI_E_ARG, hipSuccess, "x^T rhs must be > 0");
  *loss = 0.5 * eq / xr;
  if (!want_grad) return SPI_OK;
  // dL/df = q / xr; dL/dd = dL/df v + rhs A_r^-1 (d dL/df)
  SPI_CK(lp_u(h.stream, w.d, w.g, 1.0 / xr, w.u, n), "d dL/df");
  SPI_CK(apply_ref_inv(pre, w.u, w.w), "reference solve (adjoint)");
  SPI_CK(lp_dldd(h.stream, w.g, 1.0 / xr, w.v, rhs, w.w, w.u, n), "dL/dd");
  SPI_CK(lp_backward(h.stream, lp->hidden, lp->params, w.phi, w.u, w.d,
                     lp->part, lp->grad, n), "network backward");
  return SPI_OK;
}

}  // namespace

extern "C" {

int64_t spi_lp_param_count(int32_t hidden) {
  if (hidden != 8 && hidden != 16 && hidden != 32) return -1;
  return lp_param_count(hidden);
}

int spi_lp_create(spi_lp** out, int32_t hidden, const float* params) {
  if (!out) return SPI_E_ARG;
  *out = nullptr;
  const int64_t P = spi_lp_param_count(hidden);
  if (P < 0 || !params) return SPI_E_ARG;
  spi_lp* lp = new (std::nothrow) spi_lp();
  if (!lp) return SPI_E_OOM;
  lp->hidden = hidden;
  lp->P = (int)P;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&lp->params, P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&lp->m, P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&lp->v, P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&lp->grad, P * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(lp->params, params, P * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(lp->m, 0, P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(lp->v, 0, P * sizeof(float));
  if (e != hipSuccess) {
    spi_lp_destroy(lp);
    return e == hipErrorOutOfMemory ? SPI_E_OOM : SPI_E_HIP;
  }
  *out = lp;
  return SPI_OK;
}

int spi_lp_get_params(const spi_lp* lp, float* params) {
  if (!lp || !params) return SPI_E_ARG;
  hipError_t e = hipMemcpy(params, lp->params, lp->P * sizeof(float),
                           hipMemcpyDeviceToHost);
  return e == hipSuccess ? SPI_OK : SPI_E_HIP;
}

static int ensure_part(spi_lp* lp, int64_t n) {
  const int nb = lp_backward_blocks(n);
  if (lp->part && lp->part_blocks >= nb) return SPI_OK;
  if (lp->part) (void)hipFree(lp->part);
  lp->part = nullptr;
  if (hipMalloc((void**)&lp->part, (size_t)nb * lp->P * sizeof(double)) != hipSuccess)
    return SPI_E_OOM;
  lp->part_blocks = nb;
  return SPI_OK;
}

int spi_lp_loss_grad(spi_lp* lp, spi_handle* band, spi_handle* ref,
                     const double* rhs, const double* x, double* loss,
                     double* grad) {
  if (!lp || !band || !ref || !rhs || !x || !loss) return SPI_E_ARG;
  Handle& h = band->h;
  int st = ensure_part(lp, h.an.n);
  if (st != SPI_OK) return fail(h, st, hipSuccess, "gradient scratch");
  st = loss_and_grad(lp, h, ref->h, rhs, x, loss, grad != nullptr);
  if (st != SPI_OK || !grad) return st;
  SPI_CK(hipMemcpyAsync(grad, lp->grad, lp->P * sizeof(double),
                        hipMemcpyDeviceToHost, h.stream), "gradient readback");
  SPI_CK(hipStreamSynchronize(h.stream), "gradient");
  return SPI_OK;
}

int spi_lp_train_step(spi_lp* lp, spi_handle* band, spi_handle* ref,
                      const double* rhs, const double* x, double lr,
                      double* loss) {
  if (!lp || !band || !ref || !rhs || !x || !loss || !(lr > 0.0)) return SPI_E_ARG;
  Handle& h = band->h;
  int st = ensure_part(lp, h.an.n);
  if (st != SPI_OK) return fail(h, st, hipSuccess, "gradient scratch");
  st = loss_and_grad(lp, h, ref->h, rhs, x, loss, true);
  if (st != SPI_OK) return st;
  lp->step += 1;
  SPI_CK(lp_adam(h.stream, lp->params, lp->grad, lp->m, lp->v, lp->P, (float)lr,
                 lp->step), "Adam step");
  return SPI_OK;
}

void spi_lp_destroy(spi_lp* lp) {
  if (!lp) return;
  void* ptrs[] = {lp->params, lp->m, lp->v, lp->grad, lp->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete lp;
}

int spi_pcg_solve(spi_handle* band, spi_handle* ref, const spi_lp* lp,
                  const double* b, double* x, double tol, int32_t maxit,
                  spi_pcg_info* info) {
  if (!band || !ref || !b || !x || !(tol > 0.0) || maxit < 1) return SPI_E_ARG;
  Handle& h = band->h;
  Handle& pre = ref->h;
  int st = check_pair(h, pre);
  if (st != SPI_OK) return st;
  SPI_CK(ensure_lp_work(h), "PCG scratch");
  Handle::LpWork& w = h.lp;
  const int64_t n = h.an.n;
  hipStream_t s = h.stream;
  if ((st = correction(h, pre, lp)) != SPI_OK) return st;
  if (!h.val32_ok) {
    SPI_CK(pcg_val32(h, w.v32), "binary32 values");
    h.val32_ok = true;
  }
  spi_pcg_info out{};
  double nb2 = 0.0;
  SPI_CK(dot64(h, b, b, &nb2), "||b||");
  const double nb = std::sqrt(nb2);
  // x = 0, r = b (FP64)
  SPI_CK(fill_f64(s, x, 0.0, n), "x0");
  SPI_CK(hipMemcpyAsync(w.r64, b, n * sizeof(double), hipMemcpyDeviceToDevice, s),
         "r0");
  double rn = nb;
  bool converged = nb == 0.0;
  // Outer FP64 loop: correction equation A e = r solved by FP32 PCG to a
  // relative residual of kInner (binary32 cannot go much below), x += e,
  // then the true residual in FP64.
  const double kInner = 1e-5;
  int total = 0, outer = 0;
  while (!converged && total < maxit && outer < 64) {
    ++outer;
    SPI_CK(vec_to32(s, w.r64, nullptr, w.r, n), "r32");
    SPI_CK(vec_zero32(s, w.e, n), "e0");
    // z = D A_r^-1 D r
    auto precond = [&](const float* r32, float* z32) -> hipError_t {
      hipError_t e = vec_to64(s, r32, w.d, w.u, n);
      if (e == hipSuccess) e = apply_ref_inv(pre, w.u, w.v);
      if (e == hipSuccess) e = vec_to32(s, w.v, w.d, z32, n);
      return e;
    };
    SPI_CK(precond(w.r, w.z), "preconditioner");
    SPI_CK(hipMemcpyAsync(w.p, w.z, n * sizeof(float), hipMemcpyDeviceToDevice, s),
           "p0");
    double rz = 0.0, rr0 = 0.0;
    SPI_CK(dot32(h, w.r, w.z, &rz), "r^T z");
    SPI_CK(dot32(h, w.r, w.r, &rr0), "r^T r");
    const double stop2 = kInner * kInner * rr0;
    while (total < maxit) {
      SPI_CK(pcg_spmv32(h, w.v32, w.p, w.t, w.q), "A p");
      double pq = 0.0;
      SPI_CK(dot32(h, w.p, w.q, &pq), "p^T A p");
      if (!(pq > 0.0)) break;
      const double alpha = rz / pq;
      SPI_CK(vec_axpy32(s, (float)alpha, w.p, w.e, n), "e += a p");
      SPI_CK(vec_axpy32(s, (float)-alpha, w.q, w.r, n), "r -= a q");
      ++total;
      double rr = 0.0;
      SPI_CK(dot32(h, w.r, w.r, &rr), "r^T r");
      if (rr <= stop2) break;
      SPI_CK(precond(w.r, w.z), "preconditioner");
      double rz_new = 0.0;
      SPI_CK(dot32(h, w.r, w.z, &rz_new), "r^T z");
      SPI_CK(vec_xpby32(s, w.z, (float)(rz_new / rz), w.p, n), "p = z + b p");
      rz = rz_new;
    }
    SPI_CK(vec_acc64(s, w.e, x, n), "x += e");
    SPI_CK(residual64(h, b, x, w.r64, w.g), "FP64 residual");
    double r2 = 0.0;
    SPI_CK(dot64(h, w.r64, w.r64, &r2), "||r||");
    rn = std::sqrt(r2);
    converged = rn <= tol * nb;
  }
  out.iterations = total;
  out.outer = outer;
  out.rel_residual = nb > 0.0 ? rn / nb : 0.0;
  if (!converged) {
    // multifrontal fallback on the band itself
    out.fell_back = 1;
    int fs = spi_factor(band);
    if (fs != SPI_OK) {
      if (info) *info = out;
      return fs;
    }
    fs = spi_solve(band, b, x, 1, n);
    if (fs != SPI_OK && fs != SPI_E_NOCONV) {
      if (info) *info = out;
      return fs;
    }
    SPI_CK(residual64(h, b, x, w.r64, w.g), "FP64 residual");
    double r2 = 0.0;
    SPI_CK(dot64(h, w.r64, w.r64, &r2), "||r||");
    out.rel_residual = nb > 0.0 ? std::sqrt(r2) / nb : 0.0;
    if (out.rel_residual > tol) {
      if (info) *info = out;
      return fail(h, SPI_E_NOCONV, hipSuccess,
                  "PCG and its direct fallback both missed the tolerance");
    }
  }
  if (info) *info = out;
  return SPI_OK;
}

}  // extern "C"

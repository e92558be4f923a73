// C ABI of the model-level loops around the solver (declared in
// include/spi.h): the empty-field (detector pattern) loop of App. A.4-A.5
// and the Poisson likelihood fit by Newton's method of App. A.1-A.2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "spi_internal.h"

using namespace spi;

namespace {

int check_ef_args(Handle& h, const double* val, const double* y, const int64_t* bg_pos,
                  const double* t, const int64_t* grp_ptr, const int32_t* grp_rows,
                  int32_t n_u, int32_t stat, const double* U) {
  if (!val || !y || !bg_pos || !t || !grp_ptr || !grp_rows || !U || n_u < 1 ||
      (stat != 0 && stat != 1))
    return fail(h, SPI_E_ARG, hipSuccess, "invalid empty-field arguments");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "empty-field call before spi_set_values");
  return SPI_OK;
}

// chi^2 of x with the values `val` and the rows' update shares; reads chi^2
// back (synchronises).
int ef_rows_chi2(Handle& h, const double* val, const double* y, const double* x,
                 const int64_t* bg_pos, const double* t, int32_t stat, double* chi2) {
  SPI_CK(launch_ef_rows(h, val, y, x, bg_pos, t, stat), "empty-field rows");
  SPI_CK(launch_sum(h.stream, h.vrow, h.an.m, h.vsum), "chi^2");
  SPI_CK(hipMemcpyAsync(chi2, h.vsum + sum_scratch_size() - 1, sizeof(double),
                        hipMemcpyDeviceToHost, h.stream), "chi^2 readback");
  SPI_CK(hipStreamSynchronize(h.stream), "chi^2");
  return SPI_OK;
}

// Likelihood terms at x: C (host), the weights y/e^2 into w and
// r = y/e - 1 into r; returns false in *ok if some e_i <= 0.
int cash_terms(Handle& h, const double* val, const double* y, const double* x,
               double* w, double* r, double* C, bool* ok) {
  SPI_CK(fill_i64(h.stream, h.flag + 3, 0, 1), "model flag");
  SPI_CK(launch_cash_rows(h, val, x, y, w, r), "likelihood terms");
  SPI_CK(launch_sum(h.stream, h.vrow, h.an.m, h.vsum), "likelihood sum");
  double c = 0.0;
  uint64_t bad = 0;
  SPI_CK(hipMemcpyAsync(&c, h.vsum + sum_scratch_size() - 1, sizeof(double),
                        hipMemcpyDeviceToHost, h.stream), "likelihood readback");
  SPI_CK(hipMemcpyAsync(&bad, h.flag + 3, sizeof(bad), hipMemcpyDeviceToHost,
                        h.stream), "model flag readback");
  SPI_CK(hipStreamSynchronize(h.stream), "likelihood");
  *ok = bad == 0;
  *C = *ok ? c : HUGE_VAL;
  return SPI_OK;
}

double read_sum(Handle& h, int* st) {
  double v = 0.0;
  hipError_t e = hipMemcpyAsync(&v, h.vsum + sum_scratch_size() - 1, sizeof(double),
                                hipMemcpyDeviceToHost, h.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h.stream);
  *st = e == hipSuccess ? SPI_OK : fail(h, SPI_E_HIP, e, "sum readback");
  return v;
}

}  // namespace

extern "C" {

int spi_mle_terms(spi_handle* H, const double* val, const double* y, const double* x,
                  double* w, double* g, double* cash) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!val || !y || !x || !w || !g)
    return fail(h, SPI_E_ARG, hipSuccess, "null likelihood argument");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_mle_terms before spi_set_values");
  double C = 0.0;
  bool ok = false;
  int st = cash_terms(h, val, y, x, w, h.vr, &C, &ok);
  if (st != SPI_OK) return st;
  if (cash) *cash = C;
  if (!ok) return fail(h, SPI_E_ARG, hipSuccess, "the model H x is not positive");
  SPI_CK(launch_htr(h, h.vr, g), "gradient");
  return SPI_OK;
}

int spi_mle_newton(spi_handle* H, const double* val, const double* y, double* x,
                   int32_t itermax, double tol, double* d, double* cash_hist,
                   int32_t* steps) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!val || !y || !x || itermax < 1 || !(tol >= 0.0))
    return fail(h, SPI_E_ARG, hipSuccess, "invalid likelihood-fit arguments");
  if (!h.have_values)
    return fail(h, SPI_E_STATE, hipSuccess, "spi_mle_newton before spi_set_values");
  const int64_t n = h.an.n;
  double* g = h.vb2;      // -G/2 = H^T (y/e - 1)
  double* dx = h.vm1;     // Newton step
  double* xt = h.vm2;     // trial point
  double C = 0.0;
  bool ok = false;
  int st = cash_terms(h, val, y, x, h.vw, h.vr, &C, &ok);
  if (st != SPI_OK) return st;
  if (!ok) return fail(h, SPI_E_ARG, hipSuccess, "the start's model H x is not positive");
  if (cash_hist) cash_hist[0] = C;
  int done = 0;
  for (int it = 0; it < itermax; ++it) {
    // Newton step: (H^T [y/e^2] H) dx = H^T (y/e - 1) at the current x
    SPI_CK(launch_htr(h, h.vr, g), "gradient");
    if ((st = spi_set_values(H, val, h.vw)) != SPI_OK) return st;
    if ((st = spi_factor(H)) != SPI_OK) return st;
    st = spi_solve(H, g, dx, 1, n);
    if (st != SPI_OK && st != SPI_E_NOCONV) return st;
    SPI_CK(launch_dot(h, dx, g, xt, n), "decrement");
    const double dec = read_sum(h, &st);
    if (st != SPI_OK) return st;
    const bool small = 2.0 * dec <= 1e-12 * std::fabs(C);
    double a = 1.0, Ct = 0.0;
    for (;;) {
      SPI_CK(launch_axpy_to(h, x, a, dx, xt), "trial point");
      if ((st = cash_terms(h, val, y, xt, h.vw, h.vr, &Ct, &ok)) != SPI_OK) return st;
      if (ok && (small || Ct <= C - 1e-4 * a * 2.0 * dec)) break;
      a *= 0.5;
      if (a < 1e-10)
        return fail(h, SPI_E_NOCONV, hipSuccess, "likelihood line search failed");
    }
    SPI_CK(hipMemcpyAsync(x, xt, n * sizeof(double), hipMemcpyDeviceToDevice,
                          h.stream), "accept step");
    C = Ct;
    done = it + 1;
    if (cash_hist) cash_hist[done] = C;
    // stop after a step below tol of max|x|
    SPI_CK(fill_f64(h.stream, h.vnorm, 0.0, 2), "norms");
    SPI_CK(launch_maxabs2(h, dx, a, x, h.vnorm), "step size");
    double nm[2] = {0.0, 0.0};
    SPI_CK(hipMemcpyAsync(nm, h.vnorm, sizeof(nm), hipMemcpyDeviceToHost, h.stream),
           "step size readback");
    SPI_CK(hipStreamSynchronize(h.stream), "step size");
    if (nm[0] <= tol * nm[1]) break;
  }
  if (steps) *steps = done;
  // the Hessian at the solution (weights y/e^2 of the accepted x, left in
  // h.vw by its likelihood terms) and its inverse's diagonal
  if (d) {
    if ((st = spi_set_values(H, val, h.vw)) != SPI_OK) return st;
    if ((st = spi_factor(H)) != SPI_OK) return st;
    if ((st = spi_diag_inv(H, d)) != SPI_OK) return st;
  }
  return SPI_OK;
}

int spi_empty_field_update(spi_handle* H, double* val, const double* y,
                           const double* x, const int64_t* bg_pos, const double* t,
                           const int64_t* grp_ptr, const int32_t* grp_rows,
                           int32_t n_u, int32_t stat, double* U, double* chi2) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  int st = check_ef_args(h, val, y, bg_pos, t, grp_ptr, grp_rows, n_u, stat, U);
  if (st != SPI_OK) return st;
  if (!x) return fail(h, SPI_E_ARG, hipSuccess, "null solution");
  double c = 0.0;
  if ((st = ef_rows_chi2(h, val, y, x, bg_pos, t, stat, &c)) != SPI_OK) return st;
  if (chi2) *chi2 = c;
  SPI_CK(launch_ef_units(h, grp_ptr, grp_rows, n_u, bg_pos, t, U, val, true),
         "pattern update");
  return SPI_OK;
}

int spi_empty_field_loop(spi_handle* H, double* val, const double* y,
                         const int64_t* bg_pos, const double* t,
                         const int64_t* grp_ptr, const int32_t* grp_rows, int32_t n_u,
                         int32_t stat, int32_t itermax, double rtol, double* U,
                         double* x, double* d, double* chi2_hist, int32_t* passes) {
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  int st = check_ef_args(h, val, y, bg_pos, t, grp_ptr, grp_rows, n_u, stat, U);
  if (st != SPI_OK) return st;
  if (!x || itermax < 1 || !(rtol >= 0.0))
    return fail(h, SPI_E_ARG, hipSuccess, "invalid empty-field loop arguments");
  const int64_t n = h.an.n;
  // the pattern the first pass uses: background entries U_u t_i
  SPI_CK(launch_ef_units(h, grp_ptr, grp_rows, n_u, bg_pos, t, U, val, false),
         "initial pattern");
  double prev = 0.0;
  int done = 0;
  for (int it = 0; it < itermax; ++it) {
    if ((st = spi_set_leaf_values(H, val)) != SPI_OK) return st;
    if ((st = spi_factor(H)) != SPI_OK) return st;
    if ((st = spi_rhs(H, y, h.vb2)) != SPI_OK) return st;
    st = spi_solve(H, h.vb2, x, 1, n);
    if (st != SPI_OK && st != SPI_E_NOCONV) return st;
    double c = 0.0;
    if ((st = ef_rows_chi2(h, val, y, x, bg_pos, t, stat, &c)) != SPI_OK) return st;
    if (chi2_hist) chi2_hist[it] = c;
    done = it + 1;
    // stop once chi^2 decreases by no more than rtol: x, U and the factor
    // are then those of this pass
    if (it > 0 && prev - c <= rtol * prev) break;
    prev = c;
    if (it + 1 == itermax) break;
    SPI_CK(launch_ef_units(h, grp_ptr, grp_rows, n_u, bg_pos, t, U, val, true),
           "pattern update");
  }
  if (passes) *passes = done;
  // variances from the last pass's factor (the Hessian at the solution)
  if (d && (st = spi_diag_inv(H, d)) != SPI_OK) return st;
  return SPI_OK;
}

}  // extern "C"

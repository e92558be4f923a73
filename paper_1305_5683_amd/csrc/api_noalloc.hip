// spi_diag_inv_noalloc: spi_diag_inv whose scratch memory (the partial sums
// of the leaf selected inversion) lives in a fixed array of device memory
// defined here, instead of in a buffer of the handle.  For callers that
// cannot allocate (declared in include/spi.h).
//
// The array is file-scope device memory: each GPU the library runs on holds
// its own copy, of kScratchDoubles doubles, until the process ends.  Host
// code never passes the array's name to a kernel (in host code the name is
// a host-side stand-in, not a device address): the device address is taken
// once per device with hipGetSymbolAddress, with that device current, and
// kept in scratch_dev[].  Every call on one GPU shares that GPU's array, so
// calls that overlap on one GPU (different streams, different threads)
// race.  Nothing in the array needs clearing: every partial sum the
// reduction reads is written first by the same call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <sstream>

#include "spi_internal.h"

namespace {

// 2^23 doubles = 64 MiB (the medium workload needs 38 MiB).
constexpr int64_t kScratchDoubles = int64_t(1) << 23;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, taken once per device.
hipError_t scratch_ptr(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!scratch_dev[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    scratch_dev[device] = static_cast<double*>(p);
  }
  *out = scratch_dev[device];
  return hipSuccess;
}

}  // namespace

extern "C" int spi_diag_inv_noalloc(spi_handle* H, double* d) {
  using namespace spi;
  if (!H) return SPI_E_ARG;
  Handle& h = H->h;
  if (!d) return fail(h, SPI_E_ARG, hipSuccess, "null output");
  if (!h.have_factor)
    return fail(h, SPI_E_STATE, hipSuccess,
                "spi_diag_inv_noalloc without a valid factor");
  const int64_t need = h.an.task_part_off.back();
  if (need > kScratchDoubles) {
    std::ostringstream os;
    os << "spi_diag_inv_noalloc: the selected inversion needs " << need
       << " doubles of scratch, above the fixed maximum of " << kScratchDoubles
       << " (use spi_diag_inv)";
    return fail(h, SPI_E_ARG, hipSuccess, os.str().c_str());
  }
  double* part = nullptr;
  SPI_CK(scratch_ptr(h.device, &part), "scratch address");
  // no phase timing here: its events are created on first use
  const int timing = h.opts.timing;
  h.opts.timing = 0;
  const int st = diag_enqueue(h, d, part);
  h.opts.timing = timing;
  return st;
}

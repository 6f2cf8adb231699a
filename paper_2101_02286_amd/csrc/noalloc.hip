// cb_solve_noalloc: cb_solve for callers that cannot allocate device memory.
//
// The only device memory a solve needs beyond its input and output is the
// partition scratch of lines split over P > 1 workgroups (3r values per
// line and partition, written by phase A, read by phases B and C).  Here it
// lives in a fixed array of this library, one copy per GPU, held until the
// process ends.  Its device address is resolved once per device, on the
// first call with that device current; host code passes that address to
// the kernels (the array's name is only a host-side handle).  Phase A writes
// every scratch value that phases B and C read, so nothing is cleared
// between calls.  All calls on one GPU share the array: calls that overlap
// in time on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/cb.h"
#include "launch.h"

static __device__ __align__(256) double scratch[CB_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, resolved on first use.
cb_status scratch_of_current_device(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return cb::set_error(CB_ERR_HIP, (std::string("cb_solve_noalloc: hipGetDevice: ") + hipGetErrorString(e)).c_str());
  if (dev < 0 || dev >= kMaxDevices) return cb::set_error(CB_ERR_UNSUPPORTED, "cb_solve_noalloc: device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cb::set_error(CB_ERR_HIP, (std::string("cb_solve_noalloc: hipGetSymbolAddress: ") +
                                        hipGetErrorString(e)).c_str());
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return CB_OK;
}

}  // namespace

extern "C" cb_status cb_solve_noalloc(cb_plan_t plan, const cb_grid *grid, int32_t axis, const double *b, double *x,
                                      void *stream) {
  void *p = nullptr;
  cb_status s = scratch_of_current_device(&p);
  if (s != CB_OK) return s;
  const cb::FixedScratch fs{p, CB_NOALLOC_SCRATCH_BYTES};
  return cb::solve_entry(plan, grid, axis, b, x, stream, &fs);
}

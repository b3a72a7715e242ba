// lbm_static.hip -- an entry point that allocates nothing: the FP64 mass and
// momentum of a population buffer the caller owns, with the reduction's
// partial sums in a fixed device array of this file instead of memory the
// library allocates.  For callers that cannot call hipMalloc (work under HIP
// graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace {

// Partial quadruples of the fixed-order reduction (kStaticBlocks blocks) and
// the four totals.  One copy per device, held until the process ends.
constexpr int kStaticBlocks = 1024;
constexpr size_t kScratchDoubles = size_t(kStaticBlocks) * 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device
std::mutex g_scratch_mutex;

// Address of this device's scratch array.  In host code the array's name is
// a host-side stand-in, so the device address is looked up once per device
// (with that device current) and kept.
lbm_status scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return lbm::set_error(LBM_ERR_STATE, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return lbm::set_error(LBM_ERR_HIP, "hipGetSymbolAddress of the static scratch: %s", hipGetErrorString(e));
    g_scratch[dev] = static_cast<double *>(p);
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_totals_static(const void *f, int nx, int ny, int nz, lbm_storage storage, int layout,
                             void *hip_stream, double *out_device) {
  if (!f || !out_device) return lbm::set_error(LBM_ERR_ARG, "NULL pointer");
  if (nx < 1 || ny < 1 || nz < 1) return lbm::set_error(LBM_ERR_ARG, "lattice sizes must be >= 1");
  const double n = double(nx) * double(ny) * double(nz);
  if (n >= 2147483648.0)
    return lbm::set_error(LBM_ERR_ARG, "lattice has %.0f nodes; at most 2^31 - 1 fit the static reduction", n);
  const size_t esize = lbm_element_bytes(storage);
  if (esize == 0) return lbm::set_error(LBM_ERR_ARG, "invalid storage form %d", int(storage));
  if (layout != LBM_LAYOUT_POPULATION_MAJOR && layout != LBM_LAYOUT_ROW_MAJOR)
    return lbm::set_error(LBM_ERR_ARG, "layout must be LBM_LAYOUT_POPULATION_MAJOR or LBM_LAYOUT_ROW_MAJOR");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  double *partials = nullptr;
  lbm_status st = scratch_on(dev, &partials);
  if (st != LBM_OK) return st;
  const size_t N = size_t(nx) * size_t(ny) * size_t(nz);
  const lbm::PopLayout lay =
      layout == LBM_LAYOUT_ROW_MAJOR ? lbm::row_major(nx, esize) : lbm::population_major(N, nx);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // every block writes its partial quadruple (zeros when it has no node), so
  // nothing left by an earlier call needs clearing
  e = lbm::launch_moments(int(storage), f, lay, 0, N, nullptr, nullptr, partials, kStaticBlocks, s);
  if (e == hipSuccess) e = lbm::launch_reduce(partials, kStaticBlocks, out_device, s);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, "totals launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

}  // extern "C"

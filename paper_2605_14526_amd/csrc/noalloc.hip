// The allocation-free variant of the global solve x = A~^{-1} r (Sec. 4.6):
// the same kernels as pd_debug_apply_Ainv, with their scratch vectors in a
// file-scope device array instead of scene-owned buffers, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  Each device holds its own copy of the array; its address is taken
// once per device with hipGetSymbolAddress and kept, because the array's
// name in host code is only a host-side stand-in, not a device address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pdhot.h"
#include "pd_internal.h"

namespace {

// 2^21 doubles (16 MiB): the staging vectors (6 per vertex) plus the interface
// vectors fit meshes of up to about 300k vertices
constexpr size_t kScratchDoubles = size_t(1) << 21;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mtx;

// the current device's copy of the array (looked up once per device)
int scratch_for_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    pdhot::set_last_error("no usable current HIP device");
    return PD_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mtx);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      pdhot::set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return PD_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PD_OK;
}

}  // namespace

extern "C" int pd_apply_Ainv_noalloc(pd_scene* scene, const double* r, double* x, void* stream) {
  double* ws = nullptr;
  const int rc = scratch_for_current_device(&ws);
  if (rc != PD_OK) return rc;
  return pdhot::apply_Ainv_ws(scene, r, x, ws, kScratchDoubles, stream);
}

// Allocation-free Gauss-Newton Hessian-vector product: fwi_gn_hvp with its
// workspace in a fixed device array of this library instead of caller
// memory, for callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds one copy, at its own address, until the process ends.  Host code
// never uses the array's name as an address (on the host it is only a
// stand-in); the device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <mutex>
#include <string>

#include "../../include/fwi.h"
#include "fwi_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[FWI_NOALLOC_MAX_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fwi::set_error(FWI_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fwi::set_error(FWI_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fwi::set_error(FWI_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return FWI_OK;
}

}  // namespace

extern "C" int fwi_gn_hvp_noalloc(fwi_plan *p, const float *m, const float *v, int B, float *hv,
                                  void *stream) {
  if (!p) return fwi::set_error(FWI_EINVAL, "plan is null");
  size_t need = 0;
  if (int rc = fwi_workspace_size(p, FWI_OP_GN_HVP, B, &need)) return rc;
  if (need > (size_t)FWI_NOALLOC_MAX_BYTES)
    return fwi::set_error(FWI_ENOMEM, "fwi_gn_hvp_noalloc: this problem needs " +
                                          std::to_string(need) + " bytes of scratch, the fixed "
                                          "array holds " + std::to_string(FWI_NOALLOC_MAX_BYTES) +
                                          " (use fwi_gn_hvp with a caller workspace)");
  void *ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  return fwi_gn_hvp(p, m, v, B, hv, ws, (size_t)FWI_NOALLOC_MAX_BYTES, stream);
}

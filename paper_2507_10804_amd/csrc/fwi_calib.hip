// Bandwidth calibration: a STREAM-style device copy of known size.  Its
// duration gives the HBM rate a plain streaming kernel attains on the
// device (the practical ceiling quoted beside the 8 TB/s peak), and its
// FETCH_SIZE / WRITE_SIZE counter readings the scale from counter units to
// bytes.  Not part of the Hessian computation.
#include <string>

#include "../../include/fwi_calib.h"
#include "fwi_internal.h"

namespace {

constexpr int CT = 256;  // threads per workgroup

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load16(const float4 *p, bool nt) {
  if (!nt) return *p;
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store16(float4 *p, float4 v, bool nt) {
  if (nt) {
    const f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(p));
  } else {
    *p = v;
  }
}

// Each thread moves U 16-byte elements per pass (all loads issued before
// the stores); the grid strides over the array.
template <bool NT, int U>
__global__ __launch_bounds__(CT) void k_copy16(float4 *__restrict__ dst,
                                               const float4 *__restrict__ src, long long n) {
  const long long stride = (long long)gridDim.x * CT * U;
  for (long long base = (long long)blockIdx.x * CT * U + threadIdx.x; base < n; base += stride) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long q = base + (long long)u * CT;
      v[u] = q < n ? load16(src + q, NT) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long q = base + (long long)u * CT;
      if (q < n) store16(dst + q, v[u], NT);
    }
  }
}

template <bool NT, int U>
void launch(float4 *dst, const float4 *src, long long n, int grid_mode, hipStream_t st) {
  const long long one_pass = (n + (long long)CT * U - 1) / ((long long)CT * U);
  long long grid = grid_mode == 0 ? one_pass : (long long)256 * (grid_mode == 1 ? 8 : 32);
  if (grid > one_pass) grid = one_pass;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_copy16<NT, U>), dim3((unsigned)grid), dim3(CT), 0, st, dst, src, n);
}

}  // namespace

extern "C" int fwi_calib_copy(void *dst, const void *src, size_t bytes, int variant,
                              void *stream) {
  if (!dst || !src) return fwi::set_error(FWI_EINVAL, "null pointer");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fwi::set_error(FWI_EINVAL, "size and pointers must be multiples of 16 bytes");
  if (variant < 0 || variant > 11) return fwi::set_error(FWI_EINVAL, "variant must be in [0, 11]");
  const long long n = (long long)(bytes / 16);
  if (n == 0) return FWI_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool nt = variant & 1, unroll = (variant >> 1) & 1;
  const int grid_mode = variant >> 2;
  auto *d = static_cast<float4 *>(dst);
  auto *s = static_cast<const float4 *>(src);
  if (nt && unroll) launch<true, 4>(d, s, n, grid_mode, st);
  else if (nt) launch<true, 1>(d, s, n, grid_mode, st);
  else if (unroll) launch<false, 4>(d, s, n, grid_mode, st);
  else launch<false, 1>(d, s, n, grid_mode, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fwi::set_error(FWI_EHIP, std::string("copy launch: ") + hipGetErrorString(e));
  return FWI_OK;
}

// Vector algebra of the L-BFGS and gpCN drivers on gfx950 (Section 2.1 and
// 2.3; the ABI is in fwi_opt.h).  Every operation streams its vectors once:
// a grid-stride pass with FP64 accumulation per workgroup, then one
// workgroup that adds the partials in index order and forms the scalar the
// next update needs (alpha_i, the loop-2 coefficient, rho and gamma), so
// the two-loop recursion runs without host round trips.  Bandwidth-bound
// BLAS-1 work.
#include "fwi.h"
#include "fwi_internal.h"
#include "fwi_opt.h"

#include <algorithm>
#include <string>

namespace fwi {
namespace {

constexpr int VT = 256;      // threads per workgroup
constexpr int VPART = 1024;  // most partial sums

int vec_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(VPART, (n + 4 * VT - 1) / (4 * VT)));
}

__device__ inline double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < VT / 64; ++i) s += red[i];
  return s;  // valid in thread 0
}

// part[blk] = sum over the block's grid-stride share of x.y1 (and x.y2).
__global__ __launch_bounds__(VT) void k_dot_part(int64_t n, const float *__restrict__ x,
                                                 const float *__restrict__ y1,
                                                 const float *__restrict__ y2,
                                                 double *__restrict__ part) {
  __shared__ double red[VT / 64];
  double a = 0.0, b = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VT;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += stride) {
    const double xv = x[i];
    a += xv * (double)y1[i];
    if (y2) b += xv * (double)y2[i];
  }
  const double sa = block_sum(a, red);
  __syncthreads();
  const double sb = y2 ? block_sum(b, red) : 0.0;
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sa;
    if (y2) part[VPART + blockIdx.x] = sb;
  }
}

enum { FIN_DOT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_PAIR = 3 };

// Sum of the partials in index order, then the derived scalar:
//   FIN_DOT:   out[0] = d
//   FIN_ALPHA: out[0] = rho[0] d              (alpha_i)
//   FIN_BETA:  out[0] = alpha[0] - rho[0] d   (loop-2 coefficient)
//   FIN_PAIR:  out[0] = 1 / d, out2[0] = d / d2  (rho, gamma)
__global__ __launch_bounds__(64) void k_dot_fin(int nb, const double *__restrict__ part, int mode,
                                                const double *__restrict__ rho,
                                                const double *__restrict__ alpha,
                                                double *__restrict__ out,
                                                double *__restrict__ out2) {
  if (threadIdx.x != 0) return;
  double d = 0.0, d2 = 0.0;
  for (int i = 0; i < nb; ++i) d += part[i];
  if (mode == FIN_PAIR)
    for (int i = 0; i < nb; ++i) d2 += part[VPART + i];
  if (mode == FIN_DOT) out[0] = d;
  else if (mode == FIN_ALPHA) out[0] = rho[0] * d;
  else if (mode == FIN_BETA) out[0] = alpha[0] - rho[0] * d;
  else {
    out[0] = 1.0 / d;
    out2[0] = d / d2;
  }
}

__global__ __launch_bounds__(VT) void k_update(int64_t n, double a, const double *__restrict__ ad,
                                               const float *x, double b, float *y) {
  const double s = a * (ad ? ad[0] : 1.0);
  const int64_t stride = (int64_t)gridDim.x * VT;
  if (b == 0.0) {  // y is not read (it may be uninitialised)
    for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += stride)
      y[i] = (float)(s * (double)x[i]);
  } else {
    for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += stride)
      y[i] = (float)(s * (double)x[i] + b * (double)y[i]);
  }
}

}  // namespace
}  // namespace fwi

using namespace fwi;

namespace {

#define OP_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(FWI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

size_t ws_need() { return sizeof(double) * (2 * VPART + 64); }

int check_n(int64_t n) {
  if (n < 1 || n >= ((int64_t)1 << 31)) return set_error(FWI_EINVAL, "vector length must be in [1, 2^31)");
  return FWI_OK;
}

int check_ws(void *ws, size_t bytes) {
  if (!ws) return set_error(FWI_EINVAL, "null workspace");
  if (bytes < ws_need()) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(ws_need()));
  return FWI_OK;
}

// dot of x with y1 (and y2) finished in `mode`.
int dot(int64_t n, const float *x, const float *y1, const float *y2, int mode, const double *rho,
        const double *alpha, double *out, double *out2, void *ws, hipStream_t st) {
  double *part = static_cast<double *>(ws);
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(VT), 0, st, n, x, y1, y2, part);
  OP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(64), 0, st, nb, part, mode, rho, alpha, out, out2);
  OP_TRY(hipGetLastError());
  return FWI_OK;
}

int update(int64_t n, double a, const double *ad, const float *x, double b, float *y,
           hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3(vec_blocks(n)), dim3(VT), 0, st, n, a, ad, x, b, y);
  OP_TRY(hipGetLastError());
  return FWI_OK;
}

int check_order(int m, const int *order) {
  if (m < 0 || m > 64) return set_error(FWI_EINVAL, "number of pairs must be in [0, 64]");
  if (m > 0 && !order) return set_error(FWI_EINVAL, "null order");
  for (int i = 0; i < m; ++i)
    if (order[i] < 0 || order[i] >= 64) return set_error(FWI_EINVAL, "pair slot out of [0, 64)");
  return FWI_OK;
}

}  // namespace

extern "C" {

int fwi_vec_workspace_size(int64_t n, size_t *bytes) {
  if (!bytes) return set_error(FWI_EINVAL, "null argument");
  if (int rc = check_n(n)) return rc;
  *bytes = ws_need();
  return FWI_OK;
}

int fwi_vec_dot(int64_t n, const float *x, const float *y, double *out, void *ws,
                size_t ws_bytes, void *stream) {
  if (int rc = check_n(n)) return rc;
  if (int rc = check_ws(ws, ws_bytes)) return rc;
  if (!x || !y || !out) return set_error(FWI_EINVAL, "fwi_vec_dot: null array");
  return dot(n, x, y, nullptr, FIN_DOT, nullptr, nullptr, out, nullptr, ws,
             static_cast<hipStream_t>(stream));
}

int fwi_vec_update(int64_t n, double a, const double *ad, const float *x, double b, float *y,
                   void *stream) {
  if (int rc = check_n(n)) return rc;
  if (!x || !y) return set_error(FWI_EINVAL, "fwi_vec_update: null array");
  return update(n, a, ad, x, b, y, static_cast<hipStream_t>(stream));
}

int fwi_lbfgs_pair(int64_t n, const float *s, const float *y, double *rho, double *gamma,
                   void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_n(n)) return rc;
  if (int rc = check_ws(ws, ws_bytes)) return rc;
  if (!s || !y || !rho || !gamma) return set_error(FWI_EINVAL, "fwi_lbfgs_pair: null array");
  // x = y: y^T s and y^T y
  return dot(n, y, s, y, FIN_PAIR, nullptr, nullptr, rho, gamma, ws,
             static_cast<hipStream_t>(stream));
}

int fwi_lbfgs_loop1(int64_t n, int m, const int *order, const float *S, const float *Y,
                    const double *rho, float *q, double *alpha, void *ws, size_t ws_bytes,
                    void *stream) {
  if (int rc = check_n(n)) return rc;
  if (int rc = check_ws(ws, ws_bytes)) return rc;
  if (int rc = check_order(m, order)) return rc;
  if (m > 0 && (!S || !Y || !rho || !q || !alpha)) return set_error(FWI_EINVAL, "fwi_lbfgs_loop1: null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int k = 0; k < m; ++k) {
    const int i = order[k];
    if (int rc = dot(n, S + (int64_t)i * n, q, nullptr, FIN_ALPHA, rho + i, nullptr, alpha + i,
                     nullptr, ws, st))
      return rc;
    if (int rc = update(n, -1.0, alpha + i, Y + (int64_t)i * n, 1.0, q, st)) return rc;
  }
  return FWI_OK;
}

int fwi_lbfgs_loop2(int64_t n, int m, const int *order, const float *S, const float *Y,
                    const double *rho, const double *alpha, float *r, void *ws, size_t ws_bytes,
                    void *stream) {
  if (int rc = check_n(n)) return rc;
  if (int rc = check_ws(ws, ws_bytes)) return rc;
  if (int rc = check_order(m, order)) return rc;
  if (m > 0 && (!S || !Y || !rho || !r || !alpha)) return set_error(FWI_EINVAL, "fwi_lbfgs_loop2: null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  double *coef = static_cast<double *>(ws) + 2 * VPART;
  for (int k = m - 1; k >= 0; --k) {
    const int i = order[k];
    if (int rc = dot(n, Y + (int64_t)i * n, r, nullptr, FIN_BETA, rho + i, alpha + i, coef + k,
                     nullptr, ws, st))
      return rc;
    if (int rc = update(n, 1.0, coef + k, S + (int64_t)i * n, 1.0, r, st)) return rc;
  }
  return FWI_OK;
}

}  // extern "C"

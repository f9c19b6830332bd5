// Matern prior operators and the low-rank (randomized) Hessian approximation
// on gfx950 (Sections 2 and 3.1; the ABI and the exact formulas are in
// fwi_lowrank.h).
//
// Everything here is small next to the Hessian products that feed it (one
// 921 x 301 product is about half a second; the dense algebra of a rank-100
// approximation is milliseconds), so the kernels favour accuracy:
// * GEMMs read FP32 operands with arbitrary strides, tile them through LDS
//   and accumulate in FP64 (the prior's inverse amplifies low frequencies by
//   up to cond(R), and long inner products over the grid lose digits in FP32
//   sums).  FP32 MFMA would not be faster than the vector unit on this chip
//   (the same 157 TFLOP/s peak), and FP64 is what the accuracy needs;
// * Gram matrices over the grid are split along the grid into chunks whose
//   FP64 partials are summed in a fixed order (deterministic);
// * the k x k symmetric eigenproblems run as parallel cyclic Jacobi in FP64
//   in one workgroup, with a bounded number of sweeps.
#include "fwi.h"
#include "fwi_internal.h"
#include "fwi_lowrank.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace fwi {
namespace {

constexpr size_t LR_ALIGN = 256;
size_t lr_align(size_t v) { return (v + LR_ALIGN - 1) / LR_ALIGN * LR_ALIGN; }

// --------------------------------------------------------------------- GEMM
constexpr int GT = 64;   // output tile edge
constexpr int GK = 16;   // inner-dimension slice staged per step

__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ float As[GK][GT + 1];
  __shared__ float Bs[GK][GT + 1];
  const int z = blockIdx.z;
  const bool split = g.part != nullptr;
  const float *A = g.A + (split ? 0 : z * g.ab);
  const float *B = g.B + (split ? 0 : z * g.bb);
  const int p_lo = split ? z * g.kchunk : 0;
  const int p_hi = split ? min(g.K, p_lo + g.kchunk) : g.K;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const bool a_krow = g.ak == 1;  // A contiguous along the inner dimension
  const bool b_nrow = g.bn == 1;  // B contiguous along the output columns
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int p0 = p_lo; p0 < p_hi; p0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int ii = a_krow ? e / GK : e % GT, pp = a_krow ? e % GK : e / GT;
      const int i = i0 + ii, p = p0 + pp;
      As[pp][ii] = (i < g.M && p < p_hi) ? A[i * g.am + p * g.ak] : 0.0f;
      const int jj = b_nrow ? e % GT : e / GK, qq = b_nrow ? e / GT : e % GK;
      const int j = j0 + jj, q = p0 + qq;
      Bs[qq][jj] = (j < g.N && q < p_hi) ? B[q * g.bk + j * g.bn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int pp = 0; pp < GK; ++pp) {
      double av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[pp][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[pp][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_fma(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty * 4 + r;
    if (i >= g.M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx * 4 + c;
      if (j >= g.N) continue;
      if (split) {
        g.part[((long long)z * g.M + i) * g.N + j] = acc[r][c];
      } else {
        float *cp = g.C + z * g.cb + i * g.cm + j * g.cn;
        const double v = (double)g.alpha * acc[r][c] + (g.beta != 0.0f ? (double)g.beta * *cp : 0.0);
        *cp = (float)v;
      }
    }
  }
}

// out[i] = sum over chunks of part[chunk][i], in chunk order.
__global__ void k_sum_parts(const double *__restrict__ part, int nchunk, long long n,
                            double *__restrict__ out) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[c * n + e];
    out[e] = s;
  }
}

}  // namespace

hipError_t gemm(const Gemm &g, int batch, hipStream_t st) {
  const dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT),
                  (unsigned)batch);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

int nchunks(long long K) { return (int)((K + KCHUNK - 1) / KCHUNK); }

// FP64 product over a long inner dimension: out[M][N] (FP64) = A B.
hipError_t gemm_long(Gemm g, double *part, double *out, hipStream_t st) {
  g.part = part;
  g.kchunk = KCHUNK;
  const int nc = nchunks(g.K);
  hipError_t e = gemm(g, nc, st);
  if (e != hipSuccess) return e;
  const long long n = (long long)g.M * g.N;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)),
                     dim3(256), 0, st, part, nc, n, out);
  return hipGetLastError();
}

Gemm plain(int M, int N, int K) {
  Gemm g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = 1.0f;
  g.beta = 0.0f;
  return g;
}

namespace {

// ------------------------------------------------------------------- prior
struct PriorGeo {
  int nz, nx;
  float ih2;       // 1 / h^2
  float delta, gamma;
};

// out = A v = delta v - gamma Lap_h v, mirrored edges, for B planes.
__global__ void k_prior_a(PriorGeo g, const float *__restrict__ v, int B, float *__restrict__ out) {
  const long long plane = (long long)g.nz * g.nx, n = plane * B;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long b = e / plane;
    const int rem = (int)(e - b * plane);
    const int i = rem / g.nx, j = rem - i * g.nx;
    const float *p = v + b * plane;
    const float c = p[rem];
    const float up = p[max(i - 1, 0) * g.nx + j], dn = p[min(i + 1, g.nz - 1) * g.nx + j];
    const float lf = p[i * g.nx + max(j - 1, 0)], rt = p[i * g.nx + min(j + 1, g.nx - 1)];
    const float lap = (((up - c) + (dn - c)) + ((lf - c) + (rt - c))) * g.ih2;
    out[e] = __builtin_fmaf(-g.gamma, lap, g.delta * c);
  }
}

// x[b][p][q] /= spec[p][q]^power (power 1 or 2).
__global__ void k_prior_scale(const float *__restrict__ spec, long long plane, int B, int power,
                              float *__restrict__ x) {
  const long long n = plane * B;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double s = spec[e % plane];
    x[e] = (float)((double)x[e] / (power == 2 ? s * s : s));
  }
}

// --------------------------------------------------------- small symmetric
// Eigenpairs of the symmetric k x k FP64 matrix A (overwritten) by parallel
// cyclic Jacobi (round-robin pairing: every round rotates k/2 disjoint
// pairs).  A round is A <- J^T A J with J block-diagonal over the pairs, so
// every 2 x 2 block {p, q} x {p', q'} of A updates on its own as
// R_pq A_block R_p'q'^T: one pass over A per round, no barrier between the
// row and the column rotations.  The eigenvector matrix is kept transposed
// (Z = V^T), which makes its update a row rotation with contiguous access.
// Outputs the eigenvalues in descending order in w[k] and the matching
// eigenvectors as the columns of Zs (k x k); Z is scratch.  At most
// max_sweeps sweeps; stops when the off-diagonal Frobenius norm is below tol
// times the whole norm.
constexpr int EIG_T = 1024;

__global__ __launch_bounds__(EIG_T) void k_symeig(int k, double *__restrict__ A,
                                                  double *__restrict__ Z, double *__restrict__ w,
                                                  double *__restrict__ Zs, int max_sweeps,
                                                  double tol) {
  __shared__ double cs[EIG_KMAX / 2], sn[EIG_KMAX / 2];
  __shared__ int pp[EIG_KMAX / 2], qq[EIG_KMAX / 2];
  __shared__ double red[EIG_T / 64], diag[EIG_KMAX];
  __shared__ int stop, perm[EIG_KMAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = EIG_T / 64;
  const int n = k + (k & 1);  // even count; index k is a placeholder when k is odd
  const int half = n / 2;
  for (int i = wave; i < k; i += NW) {
    for (int j = lane; j < k; j += 64) {
      Z[i * k + j] = i == j ? 1.0 : 0.0;
      if (i < j) {  // exact symmetry of the input
        const double sy = 0.5 * (A[i * k + j] + A[j * k + i]);
        A[i * k + j] = sy;
        A[j * k + i] = sy;
      }
    }
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = wave; i < k; i += NW) {
      for (int j = lane; j < k; j += 64) {
        const double a = A[i * k + j] * A[i * k + j];
        tot += a;
        if (i != j) off += a;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      tot += __shfl_down(tot, o, 64);
    }
    if (lane == 0) red[wave] = off;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int q = 0; q < NW; ++q) sum += red[q];
      red[0] = sum;
    }
    __syncthreads();
    const double offs = red[0];
    __syncthreads();
    if (lane == 0) red[wave] = tot;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int q = 0; q < NW; ++q) sum += red[q];
      stop = (offs <= tol * tol * sum) ? 1 : 0;
    }
    __syncthreads();
    if (stop) break;
    for (int round = 0; round < n - 1; ++round) {
      if (tid < half) {
        auto pos = [&](int x) { return x == 0 ? 0 : (x - 1 + round) % (n - 1) + 1; };
        int p = pos(tid), q = pos(n - 1 - tid);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, sr = 0.0;
        if (q < k) {
          const double apq = A[p * k + q];
          if (apq != 0.0) {
            const double tau = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
            // smaller root of t^2 + 2 tau t - 1 = 0; 1/(2 tau) once tau^2 would overflow
            const double t = fabs(tau) < 1e150
                                 ? (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau))
                                 : 0.5 / tau;
            c = 1.0 / sqrt(1.0 + t * t);
            sr = t * c;
          }
        }
        pp[tid] = p;
        qq[tid] = q < k ? q : -1;  // placeholder partner: a 1-wide block
        cs[tid] = c;
        sn[tid] = q < k ? sr : 0.0;
      }
      __syncthreads();
      // A: the 2 x 2 blocks (pair r rows, pair u columns); 32 lanes per r.
      // A thread issues the loads of UB blocks before their arithmetic, so a
      // round costs a few memory round trips instead of one per block.
      constexpr int UB = 4;
      for (int r = tid >> 5; r < half; r += EIG_T >> 5) {
        const int p = pp[r], q = qq[r];
        const double c = cs[r], sr = sn[r];
        for (int u0 = tid & 31; u0 < half; u0 += 32 * UB) {
          double a00[UB], a01[UB], a10[UB], a11[UB];
#pragma unroll
          for (int i = 0; i < UB; ++i) {
            const int u = u0 + 32 * i;
            if (u < half) {
              const int pu = pp[u], qu = qq[u];
              a00[i] = A[p * k + pu];
              a01[i] = qu >= 0 ? A[p * k + qu] : 0.0;
              a10[i] = q >= 0 ? A[q * k + pu] : 0.0;
              a11[i] = (q >= 0 && qu >= 0) ? A[q * k + qu] : 0.0;
            }
          }
#pragma unroll
          for (int i = 0; i < UB; ++i) {
            const int u = u0 + 32 * i;
            if (u < half) {
              const int pu = pp[u], qu = qq[u];
              const double cu = cs[u], su = sn[u];
              const double b00 = c * a00[i] - sr * a10[i], b01 = c * a01[i] - sr * a11[i];
              const double b10 = sr * a00[i] + c * a10[i], b11 = sr * a01[i] + c * a11[i];
              A[p * k + pu] = b00 * cu - b01 * su;
              if (qu >= 0) A[p * k + qu] = b00 * su + b01 * cu;
              if (q >= 0) {
                A[q * k + pu] = b10 * cu - b11 * su;
                if (qu >= 0) A[q * k + qu] = b10 * su + b11 * cu;
              }
            }
          }
        }
      }
      // Z = V^T: rows p, q rotate like the rows of A (loads batched likewise)
      for (int r = wave; r < half; r += NW) {
        const int p = pp[r], q = qq[r];
        if (q < 0) continue;
        const double c = cs[r], sr = sn[r];
        for (int j0 = lane; j0 < k; j0 += 64 * UB) {
          double zp[UB], zq[UB];
#pragma unroll
          for (int i = 0; i < UB; ++i) {
            const int j = j0 + 64 * i;
            if (j < k) {
              zp[i] = Z[p * k + j];
              zq[i] = Z[q * k + j];
            }
          }
#pragma unroll
          for (int i = 0; i < UB; ++i) {
            const int j = j0 + 64 * i;
            if (j < k) {
              Z[p * k + j] = c * zp[i] - sr * zq[i];
              Z[q * k + j] = sr * zp[i] + c * zq[i];
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // order by descending eigenvalue: stable rank of each diagonal entry
  for (int i = tid; i < k; i += EIG_T) diag[i] = A[i * k + i];
  __syncthreads();
  for (int i = tid; i < k; i += EIG_T) {
    const double d = diag[i];
    int rank = 0;
    for (int j = 0; j < k; ++j) rank += (diag[j] > d) || (diag[j] == d && j < i);
    perm[rank] = i;
  }
  __syncthreads();
  for (int j = wave; j < k; j += NW) {
    const int src = perm[j];
    for (int i = lane; i < k; i += 64) Zs[i * k + j] = Z[src * k + i];
  }
  for (int i = tid; i < k; i += EIG_T) w[i] = diag[perm[i]];
}

// Orthonormalising transform from the eigenpairs (w descending, columns of Zs)
// of a Gram matrix: T[j][:] = Zs[:, j] / sqrt(w_j) for w_j > tol * w_0, zero
// rows otherwise; *kept = number of kept directions.
__global__ void k_orth_rows(int k, const double *__restrict__ w, const double *__restrict__ Zs,
                            double tol, float *__restrict__ T, int *__restrict__ kept) {
  const double top = w[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) {
    const int j = e / k, i = e % k;
    const bool keep = top > 0.0 && w[j] > tol * top;
    T[e] = keep ? (float)(Zs[i * k + j] / sqrt(w[j])) : 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int n = 0;
    while (n < k && top > 0.0 && w[n] > tol * top) ++n;
    *kept = n;
  }
}

// Ur[i][p] = Zs[p][i] (FP32) for the r leading eigenvectors, lambda[i] = w[i].
__global__ void k_lead_rows(int k, int r, const double *__restrict__ w,
                            const double *__restrict__ Zs, float *__restrict__ Ur,
                            double *__restrict__ lambda) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r * k; e += gridDim.x * blockDim.x) {
    const int i = e / k, p = e % k;
    Ur[e] = (float)Zs[p * k + i];
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < r; i += blockDim.x) lambda[i] = w[i];
}

// c[i][b] *= f(lambda_i): op 0 lambda, 1 lambda/(lambda+1), 2 1-(lambda+1)^-1/2;
// also writes the FP32 copy cf.
__global__ void k_coef(int r, int B, int op, const double *__restrict__ lambda,
                       double *__restrict__ c, float *__restrict__ cf) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r * B; e += gridDim.x * blockDim.x) {
    const double l = lambda[e / B];
    const double f = op == 0 ? l : op == 1 ? l / (l + 1.0) : 1.0 - 1.0 / sqrt(l + 1.0);
    c[e] *= f;
    cf[e] = (float)c[e];
  }
}

__global__ void k_copy_f(float *__restrict__ dst, const float *__restrict__ src, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

unsigned blocks(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 16384); }

}  // namespace

hipError_t sym_eig(int k, double *A, double *Z, double *w, double *Zs, hipStream_t st) {
  hipLaunchKernelGGL(k_symeig, dim3(1), dim3(EIG_T), 0, st, k, A, Z, w, Zs, 60, 1e-14);
  return hipGetLastError();
}

}  // namespace fwi

using namespace fwi;

struct fwi_prior {
  PriorGeo g{};
  double h = 1.0, delta = 0.0, gamma = 0.0;
  std::vector<float> host;  // C_z [nz][nz], C_x [nx][nx], spectrum [nz][nx]
  size_t off_cz = 0, off_cx = 0, off_spec = 0;
  void *dev = nullptr;
};

namespace {

template <class T>
T *at_(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

#define LR_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(FWI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Orthonormal DCT-II matrix C[p][i] = sqrt(2/n) c_p cos(pi p (i + 1/2) / n).
void dct_matrix(int n, float *C) {
  for (int p = 0; p < n; ++p) {
    const double cp = (p == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n));
    for (int i = 0; i < n; ++i) C[(size_t)p * n + i] = (float)(cp * std::cos(M_PI * p * (i + 0.5) / n));
  }
}

// R^-1 (power 2) or A^-1 (power 1) of B planes: DCT along x and z as GEMMs,
// division by the spectrum, inverse DCT.  ws: B planes of scratch.
int prior_inverse(fwi_prior *p, int power, const float *v, int B, float *out, float *ws,
                  hipStream_t st) {
  const int nz = p->g.nz, nx = p->g.nx;
  const long long plane = (long long)nz * nx;
  const float *Cz = at_<float>(p->dev, p->off_cz), *Cx = at_<float>(p->dev, p->off_cx);
  const float *spec = at_<float>(p->dev, p->off_spec);
  {  // ws = V Cx^T (rows of every plane)
    Gemm g = plain(B * nz, nx, nx);
    g.A = v; g.am = nx; g.ak = 1;
    g.B = Cx; g.bk = 1; g.bn = nx;
    g.C = ws; g.cm = nx; g.cn = 1;
    LR_TRY(gemm(g, 1, st));
  }
  {  // out_b = Cz ws_b
    Gemm g = plain(nz, nx, nz);
    g.A = Cz; g.am = nz; g.ak = 1; g.ab = 0;
    g.B = ws; g.bk = nx; g.bn = 1; g.bb = plane;
    g.C = out; g.cm = nx; g.cn = 1; g.cb = plane;
    LR_TRY(gemm(g, B, st));
  }
  hipLaunchKernelGGL(k_prior_scale, dim3(blocks(plane * B)), dim3(256), 0, st, spec, plane, B,
                     power, out);
  LR_TRY(hipGetLastError());
  {  // ws_b = Cz^T out_b
    Gemm g = plain(nz, nx, nz);
    g.A = Cz; g.am = 1; g.ak = nz; g.ab = 0;
    g.B = out; g.bk = nx; g.bn = 1; g.bb = plane;
    g.C = ws; g.cm = nx; g.cn = 1; g.cb = plane;
    LR_TRY(gemm(g, B, st));
  }
  {  // out = ws Cx
    Gemm g = plain(B * nz, nx, nx);
    g.A = ws; g.am = nx; g.ak = 1;
    g.B = Cx; g.bk = nx; g.bn = 1;
    g.C = out; g.cm = nx; g.cn = 1;
    LR_TRY(gemm(g, 1, st));
  }
  return FWI_OK;
}

int prior_r(fwi_prior *p, const float *v, int B, float *out, float *ws, hipStream_t st) {
  const long long n = (long long)p->g.nz * p->g.nx * B;
  hipLaunchKernelGGL(k_prior_a, dim3(blocks(n)), dim3(256), 0, st, p->g, v, B, ws);
  LR_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_prior_a, dim3(blocks(n)), dim3(256), 0, st, p->g, ws, B, out);
  LR_TRY(hipGetLastError());
  return FWI_OK;
}

int check_prior(const fwi_prior *p) {
  if (!p) return set_error(FWI_EINVAL, "prior is null");
  if (!p->dev) return set_error(FWI_EUNBOUND, "prior has no device block: call fwi_prior_bind");
  return FWI_OK;
}

}  // namespace

extern "C" {

int fwi_prior_create(int32_t nz, int32_t nx, double h, double delta, double gamma,
                     fwi_prior **out) {
  if (!out) return set_error(FWI_EINVAL, "null argument");
  *out = nullptr;
  if (nz < 1 || nx < 1 || (long long)nz * nx >= (1LL << 31) || nz > 8192 || nx > 8192)
    return set_error(FWI_EINVAL, "prior: nz, nx must be in [1, 8192]");
  if (!(h > 0.0) || !(delta > 0.0) || !(gamma > 0.0) || !std::isfinite(h) ||
      !std::isfinite(delta) || !std::isfinite(gamma))
    return set_error(FWI_EINVAL, "prior: h, delta and gamma must be positive");
  fwi_prior *p = new fwi_prior();
  p->g.nz = nz;
  p->g.nx = nx;
  p->g.ih2 = (float)(1.0 / (h * h));
  p->g.delta = (float)delta;
  p->g.gamma = (float)gamma;
  p->h = h;
  p->delta = delta;
  p->gamma = gamma;
  const size_t ncz = (size_t)nz * nz, ncx = (size_t)nx * nx, nsp = (size_t)nz * nx;
  p->off_cz = 0;
  p->off_cx = lr_align(ncz * sizeof(float));
  p->off_spec = p->off_cx + lr_align(ncx * sizeof(float));
  p->host.assign((p->off_spec + lr_align(nsp * sizeof(float))) / sizeof(float), 0.0f);
  dct_matrix(nz, p->host.data() + p->off_cz / sizeof(float));
  dct_matrix(nx, p->host.data() + p->off_cx / sizeof(float));
  float *spec = p->host.data() + p->off_spec / sizeof(float);
  for (int i = 0; i < nz; ++i) {
    const double sz = std::sin(M_PI * i / (2.0 * nz));
    for (int j = 0; j < nx; ++j) {
      const double sx = std::sin(M_PI * j / (2.0 * nx));
      spec[(size_t)i * nx + j] = (float)(delta + gamma * (4.0 / (h * h)) * (sz * sz + sx * sx));
    }
  }
  *out = p;
  return FWI_OK;
}

void fwi_prior_destroy(fwi_prior *p) { delete p; }

int fwi_prior_device_bytes(const fwi_prior *p, size_t *bytes) {
  if (!p || !bytes) return set_error(FWI_EINVAL, "null argument");
  *bytes = p->host.size() * sizeof(float);
  return FWI_OK;
}

int fwi_prior_bind(fwi_prior *p, void *dev, size_t bytes, void *stream) {
  if (!p || !dev) return set_error(FWI_EINVAL, "null argument");
  if (bytes < p->host.size() * sizeof(float))
    return set_error(FWI_ENOMEM, "prior device block too small");
  if (reinterpret_cast<uintptr_t>(dev) % LR_ALIGN)
    return set_error(FWI_EINVAL, "prior device block must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  LR_TRY(hipMemcpyAsync(dev, p->host.data(), p->host.size() * sizeof(float),
                        hipMemcpyHostToDevice, st));
  LR_TRY(hipStreamSynchronize(st));
  p->dev = dev;
  return FWI_OK;
}

int fwi_prior_workspace_size(const fwi_prior *p, int B, size_t *bytes) {
  if (!p || !bytes) return set_error(FWI_EINVAL, "null argument");
  if (B < 1 || B > 65535) return set_error(FWI_EINVAL, "B must be in [1, 65535]");
  *bytes = lr_align((size_t)B * p->g.nz * p->g.nx * sizeof(float));
  return FWI_OK;
}

int fwi_prior_apply(fwi_prior *p, int op, const float *v, int B, float *out, void *ws,
                    size_t ws_bytes, void *stream) {
  if (int rc = check_prior(p)) return rc;
  if (!v || !out || !ws) return set_error(FWI_EINVAL, "fwi_prior_apply: null array");
  if (v == out) return set_error(FWI_EINVAL, "fwi_prior_apply: out must not alias v");
  size_t need = 0;
  if (int rc = fwi_prior_workspace_size(p, B, &need)) return rc;
  if (ws_bytes < need) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(need));
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *w = static_cast<float *>(ws);
  switch (op) {
    case FWI_PRIOR_R: return prior_r(p, v, B, out, w, st);
    case FWI_PRIOR_RINV: return prior_inverse(p, 2, v, B, out, w, st);
    case FWI_PRIOR_AINV: return prior_inverse(p, 1, v, B, out, w, st);
    default: return set_error(FWI_EINVAL, "fwi_prior_apply: unknown op");
  }
}

}  // extern "C"

// ------------------------------------------------------------ low rank
// Workspace layout of the low-rank calls (k probes, B vectors, r ranks).
struct LrLayout {
  size_t tmp, tmp2, part, G, Z, Zs, w, T, kept, c, cf, total;
};

static LrLayout lr_layout(const fwi_prior *p, int k, int B, int r) {
  const size_t plane = (size_t)p->g.nz * p->g.nx;
  const size_t rows = (size_t)std::max(std::max(k, B), r);
  const size_t mm = (size_t)std::max(k, r) * (size_t)std::max(k, B);
  const size_t nc = (size_t)nchunks((long long)plane);
  LrLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t at = o; o = lr_align(o + b); return at; };
  L.tmp = take(rows * plane * sizeof(float));
  L.tmp2 = take(rows * plane * sizeof(float));
  L.part = take(nc * mm * sizeof(double));
  L.G = take((size_t)k * k * sizeof(double));
  L.Z = take((size_t)k * k * sizeof(double));
  L.Zs = take((size_t)k * k * sizeof(double));
  L.w = take((size_t)k * sizeof(double));
  L.T = take((size_t)k * k * sizeof(float));
  L.kept = take(sizeof(int));
  L.c = take(mm * sizeof(double));
  L.cf = take(mm * sizeof(float));
  L.total = o;
  return L;
}

static int lr_check(const fwi_prior *p, int k, void *ws, size_t ws_bytes, int B, int r) {
  if (int rc = check_prior(p)) return rc;
  if (k < 1 || k > EIG_KMAX) return set_error(FWI_EINVAL, "k must be in [1, 512]");
  if (B < 1 || B > 65535 || r < 0 || r > k) return set_error(FWI_EINVAL, "bad batch or rank");
  if (!ws) return set_error(FWI_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % LR_ALIGN)
    return set_error(FWI_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = lr_layout(p, k, B, r).total;
  if (ws_bytes < need) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(need));
  return FWI_OK;
}

// Gram G = X Y^T of k rows of length n (FP64), into ws G.
static int gram(int k, long long n, const float *X, const float *Y, void *ws, const LrLayout &L,
                hipStream_t st) {
  Gemm g = plain(k, k, (int)n);
  g.A = X; g.am = n; g.ak = 1;
  g.B = Y; g.bk = 1; g.bn = n;
  LR_TRY(gemm_long(g, at_<double>(ws, L.part), at_<double>(ws, L.G), st));
  return FWI_OK;
}

static int symeig(int k, void *ws, const LrLayout &L, hipStream_t st) {
  LR_TRY(sym_eig(k, at_<double>(ws, L.G), at_<double>(ws, L.Z), at_<double>(ws, L.w),
                 at_<double>(ws, L.Zs), st));
  return FWI_OK;
}

// rows' = T rows (k x k times k x n), into out.
static int transform_rows(int k, long long n, const float *T, const float *X, float *out,
                          hipStream_t st) {
  Gemm g = plain(k, (int)n, k);
  g.A = T; g.am = k; g.ak = 1;
  g.B = X; g.bk = n; g.bn = 1;
  g.C = out; g.cm = n; g.cn = 1;
  LR_TRY(gemm(g, 1, st));
  return FWI_OK;
}

extern "C" {

int fwi_lowrank_workspace_size(const fwi_prior *p, int k, int B, int r, size_t *bytes) {
  if (!p || !bytes) return set_error(FWI_EINVAL, "null argument");
  if (k < 1 || k > EIG_KMAX || B < 1 || B > 65535 || r < 0 || r > k)
    return set_error(FWI_EINVAL, "bad k, B or r");
  *bytes = lr_layout(p, k, B, r).total;
  return FWI_OK;
}

int fwi_lowrank_range(fwi_prior *p, int k, const float *ybar, double tol, float *Q, float *RQ,
                      int *kept, void *ws, size_t ws_bytes, void *stream) {
  if (int rc = lr_check(p, k, ws, ws_bytes, 1, 0)) return rc;
  if (!ybar || !Q || !RQ || !kept) return set_error(FWI_EINVAL, "fwi_lowrank_range: null array");
  if (!(tol > 0.0) || !(tol < 1.0)) return set_error(FWI_EINVAL, "tol must be in (0, 1)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LrLayout L = lr_layout(p, k, 1, 0);
  const long long n = (long long)p->g.nz * p->g.nx;
  float *Y = at_<float>(ws, L.tmp), *Yb = at_<float>(ws, L.tmp2);
  // Y = R^-1 ybar (Q serves as scratch), Yb = ybar
  if (int rc = prior_inverse(p, 2, ybar, k, Y, Q, st)) return rc;
  hipLaunchKernelGGL(k_copy_f, dim3(blocks(n * k)), dim3(256), 0, st, Yb, ybar, n * k);
  LR_TRY(hipGetLastError());
  // pass 0: (Y, Yb) -> (Q, RQ); pass 1: (Q, RQ) -> (Y, Yb), copied back
  for (int pass = 0; pass < 2; ++pass) {
    const float *sx = pass == 0 ? Y : Q, *sr = pass == 0 ? Yb : RQ;
    float *dx = pass == 0 ? Q : Y, *dr = pass == 0 ? RQ : Yb;
    if (int rc = gram(k, n, sx, sr, ws, L, st)) return rc;
    if (int rc = symeig(k, ws, L, st)) return rc;
    hipLaunchKernelGGL(k_orth_rows, dim3(blocks((long long)k * k)), dim3(256), 0, st, k,
                       at_<double>(ws, L.w), at_<double>(ws, L.Zs), tol, at_<float>(ws, L.T),
                       kept);
    LR_TRY(hipGetLastError());
    if (int rc = transform_rows(k, n, at_<float>(ws, L.T), sx, dx, st)) return rc;
    if (int rc = transform_rows(k, n, at_<float>(ws, L.T), sr, dr, st)) return rc;
  }
  hipLaunchKernelGGL(k_copy_f, dim3(blocks(n * k)), dim3(256), 0, st, Q, Y, n * k);
  LR_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_copy_f, dim3(blocks(n * k)), dim3(256), 0, st, RQ, Yb, n * k);
  LR_TRY(hipGetLastError());
  return FWI_OK;
}

int fwi_lowrank_project(fwi_prior *p, int k, const float *Q, const float *HQ, int r,
                        double *lambda, float *V, void *ws, size_t ws_bytes, void *stream) {
  if (int rc = lr_check(p, k, ws, ws_bytes, 1, r)) return rc;
  if (!Q || !HQ || !lambda || !V || r < 1) return set_error(FWI_EINVAL, "fwi_lowrank_project: bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LrLayout L = lr_layout(p, k, 1, r);
  const long long n = (long long)p->g.nz * p->g.nx;
  if (int rc = gram(k, n, Q, HQ, ws, L, st)) return rc;
  if (int rc = symeig(k, ws, L, st)) return rc;
  float *Ur = at_<float>(ws, L.T);
  hipLaunchKernelGGL(k_lead_rows, dim3(blocks((long long)r * k)), dim3(256), 0, st, k, r,
                     at_<double>(ws, L.w), at_<double>(ws, L.Zs), Ur, lambda);
  LR_TRY(hipGetLastError());
  Gemm g = plain(r, (int)n, k);
  g.A = Ur; g.am = k; g.ak = 1;
  g.B = Q; g.bk = n; g.bn = 1;
  g.C = V; g.cm = n; g.cn = 1;
  LR_TRY(gemm(g, 1, st));
  return FWI_OK;
}

int fwi_lowrank_apply(fwi_prior *p, int op, const double *lambda, const float *V, int r,
                      const float *v, int B, float *out, void *ws, size_t ws_bytes,
                      void *stream) {
  if (int rc = lr_check(p, std::max(r, 1), ws, ws_bytes, B, r)) return rc;
  if (!lambda || !V || !v || !out || r < 1) return set_error(FWI_EINVAL, "fwi_lowrank_apply: bad argument");
  if (v == out) return set_error(FWI_EINVAL, "fwi_lowrank_apply: out must not alias v");
  if (op < FWI_LOWRANK_HESSIAN || op > FWI_LOWRANK_SAMPLE)
    return set_error(FWI_EINVAL, "fwi_lowrank_apply: unknown op");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LrLayout L = lr_layout(p, r, B, r);
  const long long n = (long long)p->g.nz * p->g.nx;
  float *t1 = at_<float>(ws, L.tmp), *t2 = at_<float>(ws, L.tmp2);
  const float *x = nullptr;     // the vectors projected on V
  const float *basis = V;       // the expansion basis
  float sign = -1.0f;
  if (op == FWI_LOWRANK_HESSIAN) {
    if (int rc = prior_r(p, v, B, out, t1, st)) return rc;   // out = R v
    if (int rc = prior_r(p, V, r, t2, t1, st)) return rc;    // t2 = R V
    x = out;
    basis = t2;
    sign = 1.0f;
  } else if (op == FWI_LOWRANK_INVERSE) {
    if (int rc = prior_inverse(p, 2, v, B, out, t1, st)) return rc;  // out = R^-1 v
    x = v;
  } else {
    if (int rc = prior_inverse(p, 1, v, B, out, t1, st)) return rc;  // out = z = A^-1 w
    if (int rc = prior_r(p, out, B, t2, t1, st)) return rc;          // t2 = R z
    x = t2;
  }
  {  // c[r][B] = V x^T (FP64)
    Gemm g = plain(r, B, (int)n);
    g.A = V; g.am = n; g.ak = 1;
    g.B = x; g.bk = 1; g.bn = n;
    LR_TRY(gemm_long(g, at_<double>(ws, L.part), at_<double>(ws, L.c), st));
  }
  hipLaunchKernelGGL(k_coef, dim3(blocks((long long)r * B)), dim3(256), 0, st, r, B,
                     op == FWI_LOWRANK_HESSIAN ? 0 : op == FWI_LOWRANK_INVERSE ? 1 : 2, lambda,
                     at_<double>(ws, L.c), at_<float>(ws, L.cf));
  LR_TRY(hipGetLastError());
  {  // out += sign basis^T c
    Gemm g = plain(B, (int)n, r);
    g.A = at_<float>(ws, L.cf); g.am = 1; g.ak = B;
    g.B = basis; g.bk = n; g.bn = 1;
    g.C = out; g.cm = n; g.cn = 1;
    g.alpha = sign;
    g.beta = 1.0f;
    LR_TRY(gemm(g, 1, st));
  }
  return FWI_OK;
}

}  // extern "C"

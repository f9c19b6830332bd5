// Point-spread-function approximation of the misfit Hessian on gfx950:
// PSF extraction from comb products and the symbol-row (PsiDO) apply
// (Sections 3.2 and 3.5; the ABI and the exact sums are in fwi_psf.h).
//
// Apply kernel.  The model grid is cut into the cells of the centre lattice
// (between consecutive centre rows and columns, plus the strips before the
// first and after the last centre).  Every output y of one cell blends the
// same four PSFs -- the cell's corners -- so a workgroup owns a 32 x 32
// sub-tile of one cell and computes, per output, the four correlations
//     a_c(y) = sum_d p_c(d) v(y + d)
// before blending them with the tent weights at y.  The four PSFs are
// interleaved in LDS as float4 (one broadcast read per tap) and the input
// window (sub-tile plus a half-width ring) is staged once per vector.  Each
// thread owns four consecutive rows of one column: for a fixed tap column the
// four inputs slide down the window, so one LDS read feeds 16 FMAs.  This is
// plain FP32 vector arithmetic: the contraction has only four "columns" (the
// corners), too narrow for MFMA tiles.
#include "fwi.h"
#include "fwi_internal.h"
#include "fwi_psf.h"

#include <algorithm>
#include <string>

namespace fwi {
namespace {

constexpr int PT = 32;                 // sub-tile edge (outputs)
constexpr int PHMAX = 32;              // largest half-width
constexpr int PDZ = 8;                 // PSF rows staged per chunk
constexpr int PNT = 256;               // threads: 32 columns x 8 groups of 4 rows
constexpr int PRZ = 4;                 // rows per thread
constexpr int LVP = PT + 2 * PHMAX;    // LDS pitch of the input window
constexpr int LPP = 2 * PHMAX + 1;     // LDS pitch of the staged PSF rows

// Dynamic LDS of the apply kernel: PDZ x LPP float4 taps, then the input
// window of (PT - PRZ + 3 + Wp) rows of LVP floats, Wp = W rounded up to
// whole chunks (rows past the window are zero).
__host__ __device__ inline int psf_window_rows(int W) {
  return PT - PRZ + 3 + (W + PDZ - 1) / PDZ * PDZ;
}

struct PsfGeo {
  int nz, nx, oz, ox, sz, sx, nzc, nxc, half, W, stride;
  int ncz, ncx;  // cell rows / columns of the lattice (nzc + 1, nxc + 1)
  int stz, stx;  // sub-tiles per cell along z / x
};

// Cell c in [0, count] of one axis: [0, first), [c_{c-1}, c_c) between
// centres, or [c_last, n); its two corner centres and whether the second
// corner carries weight (interior cells only).
__device__ __forceinline__ void cell_of(int c, int first, int spacing, int count, int n,
                                        int &lo, int &hi, int &p0, int &p1, bool &interior) {
  if (c == 0) {
    lo = 0; hi = first; p0 = p1 = 0; interior = false;
  } else if (c == count) {
    lo = first + (count - 1) * spacing; hi = n; p0 = p1 = count - 1; interior = false;
  } else {
    lo = first + (c - 1) * spacing; hi = lo + spacing; p0 = c - 1; p1 = c; interior = true;
  }
}

__global__ __launch_bounds__(PNT) void k_psf_rows(PsfGeo g, const float *__restrict__ psf,
                                                   const float *__restrict__ v,
                                                   float *__restrict__ out) {
  extern __shared__ float4 LDS4[];
  const int h = g.half, W = g.W;
  const int rows = psf_window_rows(W);
  float4 *LP = LDS4;                                 // [PDZ][LPP] corner taps
  float *LV = reinterpret_cast<float *>(LDS4 + PDZ * LPP);  // [rows][LVP] input window

  int bid = blockIdx.x;
  const int si = bid % g.stx; bid /= g.stx;
  const int sj = bid % g.stz; bid /= g.stz;
  const int cx = bid % g.ncx, cz = bid / g.ncx;
  int zlo, zhi, p0, p1, xlo, xhi, q0, q1;
  bool zin, xin;
  cell_of(cz, g.oz, g.sz, g.nzc, g.nz, zlo, zhi, p0, p1, zin);
  cell_of(cx, g.ox, g.sx, g.nxc, g.nx, xlo, xhi, q0, q1, xin);
  const int y0 = zlo + sj * PT, x0 = xlo + si * PT;
  if (y0 >= zhi || x0 >= xhi) return;  // empty sub-tile (uniform over the workgroup)

  // input window: rows y0-h.., columns x0-h..; zero outside the model and
  // in the rows that only padded taps reach
  const long long plane = (long long)g.nz * g.nx;
  const float *vb = v + blockIdx.y * plane;
  const int VW = PT + 2 * h;
  for (int e = threadIdx.x; e < rows * VW; e += PNT) {
    const int r = e / VW, c = e - r * VW;
    const int z = y0 - h + r, x = x0 - h + c;
    const bool ok = r < VW && z >= 0 && z < g.nz && x >= 0 && x < g.nx;
    LV[r * LVP + c] = ok ? vb[(long long)z * g.nx + x] : 0.0f;
  }

  const long long W2 = (long long)W * W;
  const float *P00 = psf + (long long)(p0 * g.nxc + q0) * W2;
  const float *P01 = psf + (long long)(p0 * g.nxc + q1) * W2;
  const float *P10 = psf + (long long)(p1 * g.nxc + q0) * W2;
  const float *P11 = psf + (long long)(p1 * g.nxc + q1) * W2;
  const int tx = threadIdx.x % PT, ty = (threadIdx.x / PT) * PRZ;

  float a[PRZ][4];
#pragma unroll
  for (int j = 0; j < PRZ; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) a[j][c] = 0.0f;

  for (int dz0 = 0; dz0 < W; dz0 += PDZ) {
    __syncthreads();  // previous chunk consumed (and, first time, LV written)
    for (int e = threadIdx.x; e < PDZ * W; e += PNT) {
      const int r = e / W, c = e - r * W;
      const long long off = (long long)(dz0 + r) * W + c;
      LP[r * LPP + c] = dz0 + r < W ? make_float4(P00[off], P01[off], P10[off], P11[off])
                                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    for (int dx = 0; dx < W; ++dx) {
      // window row ty + j + dz0 + r feeds output row j at tap row dz0 + r
      const float *col = LV + (ty + dz0) * LVP + tx + dx;
      const float4 *pc = LP + dx;
      // all loads of the chunk first (they overlap), then 16 FMAs per tap row
      float w[PDZ + PRZ - 1];
      float4 p[PDZ];
#pragma unroll
      for (int r = 0; r < PDZ + PRZ - 1; ++r) w[r] = col[r * LVP];
#pragma unroll
      for (int r = 0; r < PDZ; ++r) p[r] = pc[r * LPP];
#pragma unroll
      for (int r = 0; r < PDZ; ++r) {
#pragma unroll
        for (int j = 0; j < PRZ; ++j) {
          a[j][0] = __builtin_fmaf(p[r].x, w[r + j], a[j][0]);
          a[j][1] = __builtin_fmaf(p[r].y, w[r + j], a[j][1]);
          a[j][2] = __builtin_fmaf(p[r].z, w[r + j], a[j][2]);
          a[j][3] = __builtin_fmaf(p[r].w, w[r + j], a[j][3]);
        }
      }
    }
  }

  // tent weights at y: second corner gets (y - c_first_corner) / spacing
  const int x = x0 + tx;
  const float fx = xin ? (float)(x - (g.ox + q0 * g.sx)) / (float)g.sx : 0.0f;
  float *ob = out + blockIdx.y * plane;
#pragma unroll
  for (int j = 0; j < PRZ; ++j) {
    const int y = y0 + ty + j;
    if (y < zhi && x < xhi) {
      const float fz = zin ? (float)(y - (g.oz + p0 * g.sz)) / (float)g.sz : 0.0f;
      const float top = __builtin_fmaf(fx, a[j][1], (1.0f - fx) * a[j][0]);
      const float bot = __builtin_fmaf(fx, a[j][3], (1.0f - fx) * a[j][2]);
      ob[(long long)y * g.nx + x] = __builtin_fmaf(fz, bot, (1.0f - fz) * top);
    }
  }
}

__global__ void k_psf_extract(PsfGeo g, const float *__restrict__ hv, float *__restrict__ psf) {
  const long long W2 = (long long)g.W * g.W;
  const long long total = W2 * g.nzc * g.nxc;
  const long long plane = (long long)g.nz * g.nx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / W2);
    const int t = (int)(e - k * W2);
    const int i = t / g.W, j = t - i * g.W;
    const int p = k / g.nxc, q = k - p * g.nxc;
    const int comb = (p % g.stride) * g.stride + q % g.stride;
    const int z = g.oz + p * g.sz + i - g.half, x = g.ox + q * g.sx + j - g.half;
    const bool ok = z >= 0 && z < g.nz && x >= 0 && x < g.nx;
    psf[e] = ok ? hv[comb * plane + (long long)z * g.nx + x] : 0.0f;
  }
}

int check_grid(const fwi_psf_grid *gi, PsfGeo &g) {
  if (!gi) return set_error(FWI_EINVAL, "psf grid is null");
  const fwi_psf_grid &G = *gi;
  if (G.nz < 1 || G.nx < 1) return set_error(FWI_EINVAL, "psf grid: nz and nx must be >= 1");
  if (G.sz < 1 || G.sx < 1) return set_error(FWI_EINVAL, "psf grid: spacing must be >= 1");
  if (G.nzc < 1 || G.nxc < 1) return set_error(FWI_EINVAL, "psf grid: need at least one centre");
  if (G.oz < 0 || G.ox < 0 || (long long)G.oz + (long long)(G.nzc - 1) * G.sz >= G.nz ||
      (long long)G.ox + (long long)(G.nxc - 1) * G.sx >= G.nx)
    return set_error(FWI_EINVAL, "psf grid: every centre must lie inside the model grid");
  if (G.half < 0 || G.half > PHMAX)
    return set_error(FWI_EINVAL, "psf grid: half must be in [0, " + std::to_string(PHMAX) + "]");
  if (G.stride < 1 || G.stride > 64) return set_error(FWI_EINVAL, "psf grid: stride must be in [1, 64]");
  const long long W = 2LL * G.half + 1;
  if ((long long)G.nz * G.nx >= (1LL << 40) || W * W * G.nzc * G.nxc >= (1LL << 40))
    return set_error(FWI_EINVAL, "psf grid: arrays too large");
  g.nz = G.nz; g.nx = G.nx; g.oz = G.oz; g.ox = G.ox; g.sz = G.sz; g.sx = G.sx;
  g.nzc = G.nzc; g.nxc = G.nxc; g.half = G.half; g.W = (int)W; g.stride = G.stride;
  g.ncz = G.nzc + 1;
  g.ncx = G.nxc + 1;
  const int last_z = G.oz + (G.nzc - 1) * G.sz, last_x = G.ox + (G.nxc - 1) * G.sx;
  const int mz = std::max({G.oz, G.nzc > 1 ? G.sz : 0, G.nz - last_z});
  const int mx = std::max({G.ox, G.nxc > 1 ? G.sx : 0, G.nx - last_x});
  g.stz = (mz + PT - 1) / PT;
  g.stx = (mx + PT - 1) / PT;
  if ((long long)g.ncz * g.ncx * g.stz * g.stx >= (1LL << 31))
    return set_error(FWI_EINVAL, "psf grid: too many cells");
  return FWI_OK;
}

}  // namespace
}  // namespace fwi

using namespace fwi;

extern "C" int fwi_psf_check(const fwi_psf_grid *gi) {
  PsfGeo g;
  return check_grid(gi, g);
}

extern "C" int fwi_psf_extract(const fwi_psf_grid *gi, const float *hv, float *psf,
                               void *stream) {
  PsfGeo g;
  if (int rc = check_grid(gi, g)) return rc;
  if (!hv || !psf) return set_error(FWI_EINVAL, "fwi_psf_extract: null array");
  const long long total = (long long)g.W * g.W * g.nzc * g.nxc;
  const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_psf_extract, dim3(blocks), dim3(256), 0, (hipStream_t)stream, g, hv, psf);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(FWI_EHIP, std::string("k_psf_extract: ") + hipGetErrorString(e));
  return FWI_OK;
}

extern "C" int fwi_psf_apply(const fwi_psf_grid *gi, const float *psf, const float *v, int B,
                             float *out, void *stream) {
  PsfGeo g;
  if (int rc = check_grid(gi, g)) return rc;
  if (!psf || !v || !out) return set_error(FWI_EINVAL, "fwi_psf_apply: null array");
  if (B < 1 || B > 65535) return set_error(FWI_EINVAL, "fwi_psf_apply: B must be in [1, 65535]");
  if (v == out) return set_error(FWI_EINVAL, "fwi_psf_apply: out must not alias v");
  const size_t lds = sizeof(float4) * PDZ * LPP + sizeof(float) * psf_window_rows(g.W) * LVP;
  const dim3 grid((unsigned)(g.ncz * g.ncx * g.stz * g.stx), (unsigned)B);
  hipLaunchKernelGGL(k_psf_rows, grid, dim3(PNT), lds, (hipStream_t)stream, g, psf, v, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(FWI_EHIP, std::string("k_psf_rows: ") + hipGetErrorString(e));
  return FWI_OK;
}

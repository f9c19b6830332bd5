// Low-rank symbol approximations of the misfit Hessian on gfx950: the FFT
// apply of Section 3.3 (eq. "lr-psido"), PDO probing (Section 3.4, Appendix
// A) and the PSF+ least squares (Section 3.6).  The ABI and the exact
// definitions are in fwi_symbol.h.
//
// FFT engine.  Complex FP32 transforms of lengths up to 2048 with factors 2,
// 3 and 5, done in LDS: a workgroup stages whole lines -- one row, or a band
// of adjacent columns read row by row so that global reads stay contiguous --
// and runs self-sorting Stockham stages (radix 8, 9, 15, 4, 2, 3, 5; 9 and 15
// as one Cooley-Tukey step over the radix-3 and radix-5 butterflies) between
// two LDS buffers, or -- in the blend -- in place in one line per wavefront,
// with no workgroup barrier between stages.  A 2-D transform is a row pass
// and a column pass.  The zero
// padding of the FFT grid is never read (rows beyond the data are filled in
// LDS) and the inverse passes store only model-grid rows and columns.  The
// pointwise products with the symbol tables happen on the loads of the
// inverse column pass, and the blend sum_t Re(A_t z_t) on the stores of the
// inverse row pass, so an apply is four launches.  These are HBM/L2-bound
// data movements with O(log n) flops per element: no dense contraction, no
// MFMA.
#include "fwi.h"
#include "fwi_internal.h"
#include "fwi_psf.h"
#include "fwi_symbol.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

namespace fwi {
namespace {

constexpr int FFT_MAXN = 2048;
constexpr int FFT_MAXST = 12;
constexpr int SYM_RMAX = 16;   // PDO directions
constexpr int PP_RANK = 32;    // PSF+ rank
constexpr int NTH = 256;
constexpr int CNT = 512;  // threads of the column passes (8 waves per band)
constexpr int LDS_BUDGET = 65536;
constexpr double TIE = 1e-9;   // relative distance tolerance of the separation

struct Fft1 {
  int n, ns;
  int radix[FFT_MAXST];
  const float2 *tw;  // e^{-2 pi i m / n}, m < n
};

struct SymGeo {
  int nz, nx, mz, mx, r;
  double h, rho0;
  Fft1 fz, fx;
  double sx[SYM_RMAX / 2], sz[SYM_RMAX / 2];  // xi_k for k = 1..r/2
};

typedef float f2v __attribute__((ext_vector_type(2)));  // for the non-temporal builtins

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// i z (forward sign folded by the caller)
__device__ inline float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }

template <int R, bool INV>
__device__ inline void dft(float2 *v);

// N = R1 * R2 point DFT by one Cooley-Tukey step: R2 DFTs of size R1 over
// v[m + R2 k], twiddles w_N^{m k'} (cos and sin tables of 2 pi e / N), R1
// DFTs of size R2; output index k' + R1 m'.
template <int R1, int R2, bool INV>
__device__ inline void dft_ct(float2 *v, const float *cw, const float *sw) {
  constexpr int N = R1 * R2;
  float2 w[N];
#pragma unroll
  for (int m = 0; m < R2; ++m) {
    float2 t[R1];
#pragma unroll
    for (int k = 0; k < R1; ++k) t[k] = v[m + R2 * k];
    dft<R1, INV>(t);
#pragma unroll
    for (int kp = 0; kp < R1; ++kp) {
      const int e = (m * kp) % N;
      w[m + R2 * kp] = e == 0 ? t[kp] : cmul(t[kp], make_float2(cw[e], INV ? sw[e] : -sw[e]));
    }
  }
#pragma unroll
  for (int kp = 0; kp < R1; ++kp) {
    float2 t2[R2];
#pragma unroll
    for (int m = 0; m < R2; ++m) t2[m] = w[m + R2 * kp];
    dft<R2, INV>(t2);
#pragma unroll
    for (int mp = 0; mp < R2; ++mp) v[kp + R1 * mp] = t2[mp];
  }
}

// R-point DFT in place, sign - (forward) or + (inverse).
template <int R, bool INV>
__device__ inline void dft(float2 *v) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    const float2 it3 = INV ? cmuli(t3) : cmuli(make_float2(-t3.x, -t3.y));  // +-i t3
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, it3);
    v[3] = csub(t1, it3);
  } else if constexpr (R == 3) {
    const float c = -0.5f;
    const float s = INV ? 0.86602540378443865f : -0.86602540378443865f;
    const float2 a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    const float2 m = make_float2(fmaf(c, a.x, v[0].x), fmaf(c, a.y, v[0].y));
    const float2 ib = cscale(cmuli(b), s);
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, ib);
    v[2] = csub(m, ib);
  } else if constexpr (R == 9) {
    constexpr float c[9] = {1.0f, 0.76604444311897801f, 0.17364817766693041f,
                            -0.49999999999999978f, -0.93969262078590832f, -0.93969262078590843f,
                            -0.50000000000000044f, 0.17364817766692997f, 0.76604444311897779f};
    constexpr float sn[9] = {0.0f, 0.64278760968653925f, 0.98480775301220802f,
                             0.86602540378443871f, 0.34202014332566888f, -0.34202014332566866f,
                             -0.86602540378443837f, -0.98480775301220813f, -0.64278760968653958f};
    dft_ct<3, 3, INV>(v, c, sn);
  } else if constexpr (R == 15) {
    constexpr float c[15] = {1.0f, 0.91354545764260087f, 0.66913060635885824f,
                             0.30901699437494745f, -0.10452846326765333f, -0.49999999999999978f,
                             -0.80901699437494734f, -0.97814760073380569f, -0.97814760073380569f,
                             -0.80901699437494756f, -0.50000000000000044f, -0.10452846326765423f,
                             0.30901699437494723f, 0.66913060635885846f, 0.91354545764260098f};
    constexpr float sn[15] = {0.0f, 0.40673664307580015f, 0.74314482547739413f,
                              0.95105651629515353f, 0.9945218953682734f, 0.86602540378443871f,
                              0.58778525229247325f, 0.20791169081775931f, -0.20791169081775907f,
                              -0.58778525229247303f, -0.86602540378443837f, -0.99452189536827329f,
                              -0.95105651629515364f, -0.74314482547739402f, -0.40673664307580015f};
    dft_ct<3, 5, INV>(v, c, sn);
  } else if constexpr (R == 8) {
    // two radix-4 DFTs: of a_k = v_k + v_{k+4} (even outputs) and of
    // b_k = (v_k - v_{k+4}) w^k (odd outputs), w = e^{-+ i pi / 4}
    const float h = 0.70710678118654752f;
    const float sg = INV ? 1.0f : -1.0f;
    float2 a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = cadd(v[k], v[k + 4]);
      b[k] = csub(v[k], v[k + 4]);
    }
    {
      const float2 d1 = b[1], d2 = b[2], d3 = b[3];
      b[1] = make_float2(h * (d1.x - sg * d1.y), h * (d1.y + sg * d1.x));   // h (1 + s i) d1
      b[2] = make_float2(-sg * d2.y, sg * d2.x);                            // s i d2
      b[3] = make_float2(h * (-d3.x - sg * d3.y), h * (-d3.y + sg * d3.x)); // h (-1 + s i) d3
    }
    dft<4, INV>(a);
    dft<4, INV>(b);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  } else {  // R == 5
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = INV ? 0.95105651629515357f : -0.95105651629515357f;
    const float s2 = INV ? 0.58778525229247313f : -0.58778525229247313f;
    const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const float2 m1 = make_float2(v[0].x + fmaf(c1, a1.x, c2 * a2.x), v[0].y + fmaf(c1, a1.y, c2 * a2.y));
    const float2 m2 = make_float2(v[0].x + fmaf(c2, a1.x, c1 * a2.x), v[0].y + fmaf(c2, a1.y, c1 * a2.y));
    const float2 n1 = cmuli(make_float2(fmaf(s1, b1.x, s2 * b2.x), fmaf(s1, b1.y, s2 * b2.y)));
    const float2 n2 = cmuli(make_float2(fmaf(s2, b1.x, -s1 * b2.x), fmaf(s2, b1.y, -s1 * b2.y)));
    v[0] = make_float2(v[0].x + a1.x + a2.x, v[0].y + a1.y + a2.y);
    v[1] = cadd(m1, n1);
    v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2);
    v[3] = csub(m2, n2);
  }
}

// float2 loads and stores at a byte offset from a workgroup-uniform base, as
// raw buffer accesses: the base lives in a scalar descriptor and each access
// needs one 32-bit offset (a pointer costs a 64-bit address computation per
// access, and the column passes issue VALU work at the SIMDs' capacity).
// Offsets stay below 2^31: at most 2048 x 2048 values of 8 bytes per plane.
// Descriptor word 3 is the gfx9-family raw-buffer format.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t brsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, 0x7fffffff, 0x00020000);
}
__device__ inline float2 bld2(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <int POLICY = 0>  // 2: non-temporal
__device__ inline void bst2(__amdgpu_buffer_rsrc_t r, int off, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, POLICY);
}

// a / b for 0 <= a < 2^20 and 1 <= b <= 2^16, rb = 1/b in FP32: the estimate
// is off by at most one and is corrected exactly (a runtime integer division
// costs dozens of instructions, this five).
__device__ inline int qdiv(int a, int b, float rb) {
  int q = (int)((float)a * rb);
  const int r = a - q * b;
  q += (r >= b) - (r < 0);
  return q;
}

// One Stockham stage of radix R over `nlines` lines of length n (pitch
// apart): sub-transforms of length Ns become length Ns*R, output in natural
// order after the last stage.
template <int R, bool INV>
__device__ inline void stage(const float2 *src, float2 *dst, int pitch, int nlines, int n, int Ns,
                             const float2 *tw) {
  const int nR = n / R;
  const int tstep = n / (Ns * R);
  const float rnR = 1.0f / (float)nR, rNs = 1.0f / (float)Ns;
  for (int e = threadIdx.x; e < nlines * nR; e += blockDim.x) {
    const int line = qdiv(e, nR, rnR);
    const int j = e - line * nR;
    const float2 *x = src + line * pitch;
    float2 *y = dst + line * pitch;
    const int k = j - qdiv(j, Ns, rNs) * Ns;
    float2 v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = x[j + t * nR];
    if (Ns > 1) {
#pragma unroll
      for (int t = 1; t < R; ++t) {
        float2 w = tw[k * t * tstep];
        if (INV) w.y = -w.y;
        v[t] = cmul(v[t], w);
      }
    }
    dft<R, INV>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) y[base + t * Ns] = v[t];
  }
}

// All stages; returns the buffer that holds the result.  Every thread of the
// workgroup must call it (it synchronises after each stage).
// BIG compiles the radix-15 and radix-9 stages in (their registers count
// against every kernel that contains them): the column passes use them, the
// row passes, whose lengths factor without them, do not.
template <bool INV, bool BIG = false>
__device__ float2 *fft_lines(float2 *a, float2 *b, int pitch, int nlines, const Fft1 &f,
                             const float2 *tw) {
  int Ns = 1;
  for (int s = 0; s < f.ns; ++s) {
    const int R = f.radix[s];
    if (R == 8) stage<8, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else if (BIG && R == 15) stage<15, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else if (BIG && R == 9) stage<9, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else if (R == 4) stage<4, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else if (R == 2) stage<2, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else if (R == 3) stage<3, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    else stage<5, INV>(a, b, pitch, nlines, f.n, Ns, tw);
    __syncthreads();
    float2 *t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// One Stockham stage of one line run by one wavefront: lanes stride over the
// butterflies.
template <int R, bool INV>
__device__ inline void wave_stage(const float2 *a, float2 *b, int n, int Ns, const float2 *tw) {
  const int lane = threadIdx.x & 63;
  const int nR = n / R, tstep = n / (Ns * R);
  const float rNs = 1.0f / (float)Ns;
  for (int j = lane; j < nR; j += 64) {
    const int k = j - qdiv(j, Ns, rNs) * Ns;
    float2 v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = a[j + t * nR];
    if (Ns > 1) {
#pragma unroll
      for (int t = 1; t < R; ++t) {
        float2 w = tw[k * t * tstep];
        if (INV) w.y = -w.y;
        v[t] = cmul(v[t], w);
      }
    }
    dft<R, INV>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) b[base + t * Ns] = v[t];
  }
}

// The stages of one line run by one wavefront alone; a stage's LDS writes
// are ordered before the next stage's reads by a wavefront fence (a
// wavefront issues its LDS operations in order; no workgroup barrier is
// needed).  Returns the buffer holding the result.
template <bool INV>
__device__ float2 *fft_wave(float2 *a, float2 *b, const Fft1 &f, const float2 *tw) {
  int Ns = 1;
  for (int s = 0; s < f.ns; ++s) {
    const int R = f.radix[s];
    if (R == 8) wave_stage<8, INV>(a, b, f.n, Ns, tw);
    else if (R == 15) wave_stage<15, INV>(a, b, f.n, Ns, tw);
    else if (R == 9) wave_stage<9, INV>(a, b, f.n, Ns, tw);
    else if (R == 4) wave_stage<4, INV>(a, b, f.n, Ns, tw);
    else if (R == 2) wave_stage<2, INV>(a, b, f.n, Ns, tw);
    else if (R == 3) wave_stage<3, INV>(a, b, f.n, Ns, tw);
    else wave_stage<5, INV>(a, b, f.n, Ns, tw);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float2 *t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// One Stockham stage with compile-time sizes (line length N, radix R,
// sub-transform length NS), run by one wavefront: the read and write offsets
// t nR and t NS become immediate LDS offsets and j mod NS a multiply by a
// constant, which matters because the column passes issue VALU work at the
// SIMDs' capacity.  Same arithmetic, in the same order, as wave_stage.
template <int R, bool INV, int N, int NS>
__device__ inline void wave_stage_c(const float2 *a, float2 *b, const float2 *tw) {
  constexpr int nR = N / R, tstep = N / (NS * R);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int it = 0; it < (nR + 63) / 64; ++it) {
    const int j = lane + 64 * it;
    if (j < nR) {
      const int k = j % NS;
      float2 v[R];
#pragma unroll
      for (int t = 0; t < R; ++t) v[t] = a[j + t * nR];
      if (NS > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          float2 w = tw[k * t * tstep];
          if (INV) w.y = -w.y;
          v[t] = cmul(v[t], w);
        }
      }
      dft<R, INV>(v);
      float2 *y = b + (j - k) * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) y[t * NS] = v[t];
    }
  }
}

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 360-point column line (the FFT grid of the 921 x 301 model) as
// 8 x 9 x 5 with compile-time sizes; the radix order the host factors 360
// into, so the result matches the generic path exactly.  Result in b.
template <bool INV>
__device__ void fft_wave_360(float2 *a, float2 *b, const float2 *tw) {
  wave_stage_c<8, INV, 360, 1>(a, b, tw);
  wave_fence();
  wave_stage_c<9, INV, 360, 8>(b, a, tw);
  wave_fence();
  wave_stage_c<5, INV, 360, 72>(a, b, tw);
  wave_fence();
}

__device__ inline void load_tw(float2 *dst, const Fft1 &f) {
  for (int i = threadIdx.x; i < f.n; i += blockDim.x) dst[i] = f.tw[i];
}

// Copy `tot` elements global -> LDS as put(e, get(e)) with U independent
// loads in flight per thread before the first LDS store: a plain loop would
// wait out one memory latency per element.
template <int U, int NT = NTH, class Get, class Put>
__device__ inline void staged(int tot, Get get, Put put) {
  for (int base = threadIdx.x; base < tot; base += U * NT) {
    float2 tmp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT;
      tmp[u] = e < tot ? get(e) : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT;
      if (e < tot) put(e, tmp[u]);
    }
  }
}

// ------------------------------------------------------------- 2-D passes

// The C lines of a column band: one wavefront per line when the band has as
// many lines as the workgroup has wavefronts (then no workgroup barrier
// between stages), else all threads share every stage.  Ends with a
// workgroup barrier either way; returns the result buffer.
template <bool INV>
__device__ const float2 *cols_fft(float2 *a, float2 *b, int pitch, int C, const Fft1 &f,
                                  const float2 *tw) {
  if (C == CNT / 64) {
    const int w = threadIdx.x >> 6;
    if (f.n == 360 && f.ns == 3 && f.radix[0] == 8 && f.radix[1] == 9 && f.radix[2] == 5) {
      fft_wave_360<INV>(a + w * pitch, b + w * pitch, tw);
      __syncthreads();
      return b;
    }
    const float2 *r = fft_wave<INV>(a + w * pitch, b + w * pitch, f, tw);
    __syncthreads();
    return r - w * pitch;  // the same buffer for every line (same stage count)
  }
  return fft_lines<INV, true>(a, b, pitch, C, f, tw);
}

// Column band of a workgroup: consecutive workgroup ids go round-robin to the
// 8 XCDs (each with its own L2), so ids are remapped to give every XCD a
// contiguous run of bands -- neighbouring bands share 128-byte lines.
__device__ inline int xcd_band(int id, int nbands) {
  const int per = (nbands + 7) / 8;
  const int band = (id & 7) * per + (id >> 3);
  return band < nbands ? band : -1;
}

// Work item of a workgroup in a one-dimensional grid of units x `per`
// items: consecutive workgroup ids go round-robin to the 8 XCDs, so ids are
// remapped to give every XCD a contiguous run, in which the `per` items of
// one unit are consecutive -- operands the items of a unit share come from
// that XCD's L2 after the first read.
__device__ inline void xcd_run(int per, int &unit, int &item) {
  const int n = gridDim.x, id = blockIdx.x;
  const int q = n / 8, rem = n % 8, x = id % 8, slot = id / 8;
  const int lid = x < rem ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
  unit = lid / per;
  item = lid - unit * per;
}

// Forward row transforms of B real planes in[b][rows][cols] (cols <= mx, zero
// beyond): out[b][rows][mx].  One row per workgroup.
__global__ __launch_bounds__(NTH) void k_rows_fwd(SymGeo g, const float *__restrict__ in, int rows,
                                                  int cols, float2 *__restrict__ out) {
  extern __shared__ float2 sm[];
  const int n = g.mx;
  float2 *a = sm, *b = sm + n;
  const float2 *tw = g.fx.tw;  // row tables outweigh a row: read through the cache
  const long long row = (long long)blockIdx.y * rows + blockIdx.x;
  const float *src = in + row * cols;
  staged<8>(n, [&](int i) { return make_float2(i < cols ? src[i] : 0.0f, 0.0f); },
            [&](int i, float2 v) { a[i] = v; });
  __syncthreads();
  const float2 *res = fft_lines<false>(a, b, n, 1, g.fx, tw);
  float2 *dst = out + row * n;
  for (int i = threadIdx.x; i < n; i += NTH) dst[i] = res[i];
}

// Forward column transforms: in[b][rows_in][mx] (rows beyond rows_in are
// zero) to out[b][mz][mx].  A band of C adjacent columns per workgroup.
__global__ __launch_bounds__(CNT) void k_cols_fwd(SymGeo g, const float2 *__restrict__ in,
                                                  int rows_in, int cs, float2 *__restrict__ out) {
  extern __shared__ float2 sm[];
  const int C = 1 << cs, n = g.mz, pitch = n + 1, mx = g.mx;
  float2 *tw = sm, *a = sm + n, *b = a + C * pitch;
  const int band = xcd_band(blockIdx.x, (mx + C - 1) >> cs);
  if (band < 0) return;  // grid padding (whole workgroup, before any barrier)
  load_tw(tw, g.fz);
  const int col0 = band * C;
  const long long bz = blockIdx.y;
  const __amdgpu_buffer_rsrc_t rin = brsrc(in + bz * rows_in * mx), rout = brsrc(out + bz * n * mx);
  staged<8, CNT>(n * C,
            [&](int e) {
              const int i = e >> cs, c = e & (C - 1);
              return (i < rows_in && col0 + c < mx) ? bld2(rin, (i * mx + col0 + c) << 3)
                                                    : make_float2(0.0f, 0.0f);
            },
            [&](int e, float2 v) { a[(e & (C - 1)) * pitch + (e >> cs)] = v; });
  __syncthreads();
  const float2 *res = cols_fft<false>(a, b, pitch, C, g.fz, tw);
  for (int e = threadIdx.x; e < n * C; e += CNT) {
    const int i = e >> cs, c = e & (C - 1);
    if (col0 + c < mx) bst2(rout, (i * mx + col0 + c) << 3, res[c * pitch + i]);
  }
}

// Inverse column transforms of Mt[t] . spec[b], model rows stored:
// z[b][t][nz][mx].  Grid (column bands, T, B); bands of C = 2^cs columns.
__global__ __launch_bounds__(CNT) void k_cols_inv(SymGeo g, const float2 *__restrict__ spec,
                                                  const float2 *__restrict__ Mt, int T, int cs,
                                                  float2 *__restrict__ z) {
  extern __shared__ float2 sm[];
  const int C = 1 << cs, n = g.mz, pitch = n + 1, mx = g.mx;
  float2 *tw = sm, *a = sm + n, *b = a + C * pitch;
  const int band = xcd_band(blockIdx.x, (mx + C - 1) >> cs);
  if (band < 0) return;  // grid padding (whole workgroup, before any barrier)
  load_tw(tw, g.fz);
  const int col0 = band * C;
  const long long t = blockIdx.y, bv = blockIdx.z;
  const __amdgpu_buffer_rsrc_t rS = brsrc(spec + bv * n * mx), rW = brsrc(Mt + t * n * mx);
  const float2 *res;
  if (n == 360 && C == CNT / 64 && g.fz.ns == 3 && g.fz.radix[0] == 8 && g.fz.radix[1] == 9 &&
      g.fz.radix[2] == 5) {
    // 360-point lines: thread (column c, butterfly j < 45) loads its radix-8
    // inputs, rows j + 45 t, straight from global memory and writes the first
    // Stockham stage's outputs 8 j + t (the same values in the same order as
    // staging the products and running that stage from LDS, one LDS round
    // trip less); the wavefronts then run stages 9 and 5 on their columns.
    const int c = threadIdx.x & (CNT / 64 - 1), j = threadIdx.x / (CNT / 64);
    if (j < 45) {
      float2 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int o = ((j + 45 * k) * mx + col0 + c) << 3;
        v[k] = col0 + c < mx ? cmul(bld2(rS, o), bld2(rW, o)) : make_float2(0.0f, 0.0f);
      }
      dft<8, true>(v);
#pragma unroll
      for (int k = 0; k < 8; ++k) b[c * pitch + 8 * j + k] = v[k];
    }
    __syncthreads();  // a column's first stage came from several wavefronts; the twiddles
    const int w = threadIdx.x >> 6;
    wave_stage_c<9, true, 360, 8>(b + w * pitch, a + w * pitch, tw);
    wave_fence();
    wave_stage_c<5, true, 360, 72>(a + w * pitch, b + w * pitch, tw);
    __syncthreads();
    res = b;
  } else {
    staged<4, CNT>(n * C,
              [&](int e) {
                const int i = e >> cs, c = e & (C - 1);
                if (col0 + c >= mx) return make_float2(0.0f, 0.0f);
                const int o = (i * mx + col0 + c) << 3;
                return cmul(bld2(rS, o), bld2(rW, o));
              },
              [&](int e, float2 v) { a[(e & (C - 1)) * pitch + (e >> cs)] = v; });
    __syncthreads();
    res = cols_fft<true>(a, b, pitch, C, g.fz, tw);
  }
  // streaming stores: the partial transforms are read once, by the next pass;
  // allocating them in L2 would evict the table and spectrum bands that the
  // other vectors' and terms' workgroups re-read
  const __amdgpu_buffer_rsrc_t rZ = brsrc(z + (bv * T + t) * (long long)g.nz * mx);
  for (int e = threadIdx.x; e < g.nz * C; e += CNT) {
    const int i = e >> cs, c = e & (C - 1);
    if (col0 + c < mx) bst2<2>(rZ, (i * mx + col0 + c) << 3, res[c * pitch + i]);
  }
}

// Orders a wavefront's LDS accesses: those before complete before those
// after (a wavefront issues its LDS operations in order; the fences stop the
// compiler moving accesses across).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Stockham stage of radix R of one line of length n <= NMAX, in place,
// run by one wavefront: every lane holds the inputs of all its butterflies
// in registers before any lane writes.
template <int R, bool INV, int NMAX>
__device__ inline void wave_stage_ip(float2 *a, int n, int Ns, const float2 *tw) {
  constexpr int IT = (NMAX / R + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int nR = n / R, tstep = n / (Ns * R);
  const float rNs = 1.0f / (float)Ns;
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = lane + 64 * it;
    if (j < nR) {
#pragma unroll
      for (int t = 0; t < R; ++t) v[it][t] = a[j + t * nR];
    }
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = lane + 64 * it;
    if (j < nR) {
      const int k = j - qdiv(j, Ns, rNs) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          float2 w = tw[k * t * tstep];
          if (INV) w.y = -w.y;
          v[it][t] = cmul(v[it][t], w);
        }
      }
      dft<R, INV>(v[it]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) a[base + t * Ns] = v[it][t];
    }
  }
  wave_sync();
}

// All stages of one row line in place (result in natural order in `a`).
// Row lengths are factored without the radix-15 and radix-9 stages, whose
// register arrays would bound the occupancy of every kernel holding them.
template <bool INV, int NMAX>
__device__ void fft_wave_ip(float2 *a, const Fft1 &f, const float2 *tw) {
  int Ns = 1;
  for (int s = 0; s < f.ns; ++s) {
    const int R = f.radix[s];
    if (R == 8) wave_stage_ip<8, INV, NMAX>(a, f.n, Ns, tw);
    else if (R == 4) wave_stage_ip<4, INV, NMAX>(a, f.n, Ns, tw);
    else if (R == 2) wave_stage_ip<2, INV, NMAX>(a, f.n, Ns, tw);
    else if (R == 3) wave_stage_ip<3, INV, NMAX>(a, f.n, Ns, tw);
    else wave_stage_ip<5, INV, NMAX>(a, f.n, Ns, tw);
    Ns *= R;
  }
}

// The blend with wavefronts owning lines: the W wavefronts of workgroup
// (row, j) form W / S groups of S, group q taking vector j * W / S + q and
// its wavefront p the terms t = p, p + S, ...; each term is an inverse row
// transform in the wavefront's own LDS line (no workgroup barrier between
// stages or terms), Re(A_t z_t) accumulated for the lane's columns
// x = lane + 64 i in registers.  With S > 1 the group's partial sums are
// added through LDS in wavefront order (S > 1 keeps every CU busy when B is
// small).  NMAX >= mx bounds the per-lane arrays.
template <int NMAX>
__global__ __launch_bounds__(256) void k_rows_inv_blend_w(SymGeo g, const float2 *__restrict__ z,
                                                         int T, int B, int S,
                                                         const float2 *__restrict__ A,
                                                         float scale, float *__restrict__ out) {
  constexpr int NACC = NMAX / 64;
  extern __shared__ float2 sm[];
  const int n = g.mx, nz = g.nz, nx = g.nx;
  const int W = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2 *tw = sm, *a = sm + n + w * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = g.fx.tw[i];
  __syncthreads();
  const int q = w / S, p = w - q * S;
  // the row's coefficient fields A are read by every vector group
  int row, grp;
  xcd_run(gridDim.x / nz, row, grp);
  const int v = grp * (W / S) + q;
  const bool live = v < B;  // uniform over the wavefront
  float acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0f;
  for (int t = p; live && t < T; t += S) {
    const float2 *zr = z + (((long long)v * T + t) * nz + row) * n;
    for (int base = lane; base < n; base += 8 * 64) {
      float2 tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + 64 * u;
        tmp[u] = i < n ? zr[i] : make_float2(0.0f, 0.0f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + 64 * u;
        if (i < n) a[i] = tmp[u];
      }
    }
    wave_sync();
    fft_wave_ip<true, NMAX>(a, g.fx, tw);
    const float2 *Ar = A + ((long long)t * nz + row) * nx;
#pragma unroll
    for (int i = 0; i < NACC; ++i) {
      const int x = lane + 64 * i;
      if (x < nx) {
        const float2 c = Ar[x], y = a[x];
        acc[i] = fmaf(c.x, y.x, fmaf(-c.y, y.y, acc[i]));
      }
    }
    wave_sync();  // the next term's loads overwrite the line
  }
  if (S > 1) {  // uniform over the workgroup
    float *part = reinterpret_cast<float *>(a);  // 2 n floats >= nx
#pragma unroll
    for (int i = 0; i < NACC; ++i) {
      const int x = lane + 64 * i;
      if (x < nx) part[x] = acc[i];
    }
    __syncthreads();
    if (p == 0) {
      for (int k = 1; k < S; ++k) {
        const float *pk = reinterpret_cast<const float *>(a + k * n);
#pragma unroll
        for (int i = 0; i < NACC; ++i) {
          const int x = lane + 64 * i;
          if (x < nx) acc[i] += pk[x];
        }
      }
    }
  }
  if (!live || p != 0) return;
  const float f = scale / ((float)g.mz * (float)g.mx);
  float *o = out + ((long long)v * nz + row) * nx;
#pragma unroll
  for (int i = 0; i < NACC; ++i) {
    const int x = lane + 64 * i;
    if (x < nx) o[x] = acc[i] * f;
  }
}

// The blend for rows of 960 = 15 x 64 points (the FFT grid of the 921 x 301
// model), with the line split so that most of the transform stays in
// registers.  With k = 64 k1 + k2 and n = n1 + 15 n2 the inverse DFT is
//   y[n1 + 15 n2] = sum_k2 w64^(n2 k2) w960^(n1 k2) sum_k1 x[64 k1 + k2] w15^(n1 k1)
// (w_L = e^(2 pi i / L)): lane k2 loads its 15 values straight from global
// memory (coalesced) and does the radix-15 DFT in registers; the 15 64-point
// DFTs over k2 = 8 a + b, n2 = c + 8 d are two radix-8 passes through LDS,
//   Z[c][b] = w64^(c b) sum_a V[8 a + b] w8^(c a),  y = sum_b w8^(d b) Z[c][b],
// lanes taking (n1, b) and then (n1, c) pairs.  Rows of the LDS line are
// BL_P = 68 slots apart and Z[c][b] sits at 8 c + (b ^ c): a pitch of 72
// would keep every 16-lane group of every pass on distinct banks, but 68
// fits four 4-wavefront workgroups in a CU's LDS instead of three (16
// wavefronts, at 126 VGPRs) for 2-way conflicts in half the accesses, and
// measures 4-5 % faster.  Three LDS passes per line instead of the Stockham
// form's five; the same workgroup and term-split structure as
// k_rows_inv_blend_w.  Lane (n1, c) ends with the outputs x = n1 + 15 (c + 8 d).
constexpr int BL_P = 68;
constexpr int SPLIT_LDS = 960 + 64;  // the two twiddle tables, in float2

// The twiddle tables of the split transform in LDS (every thread of the
// workgroup takes part; the caller synchronises): T2[n1][k2] = w960^(n1 k2),
// T3[c][b] = w64^(c b), conjugated for the inverse.
template <bool INV>
__device__ inline void split960_tables(const Fft1 &f, float2 *T2, float2 *T3) {
  for (int i = threadIdx.x; i < 960; i += blockDim.x) {
    const float2 t = f.tw[((i >> 6) * (i & 63)) % 960];
    T2[i] = make_float2(t.x, INV ? -t.y : t.y);
  }
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    const float2 t = f.tw[15 * (i >> 3) * (i & 7)];
    T3[i] = make_float2(t.x, INV ? -t.y : t.y);
  }
}

// One 960-point line transformed by one wavefront, split as above: u holds
// the lane's inputs x[64 k1 + lane], a is the wavefront's LDS line (15 rows
// BL_P apart).  emit(it, n1, c, y) receives, for each of the lane's (n1, c)
// pairs (pp = lane + 64 it < 120), the outputs y[d] = X[n1 + 15 (c + 8 d)].
// Ends with a wavefront fence, so the line may be rewritten at once.
template <bool INV, class Emit>
__device__ inline void split960(float2 (&u)[15], float2 *a, const float2 *T2, const float2 *T3,
                                Emit emit) {
  const int lane = threadIdx.x & 63;
  dft<15, INV>(u);
#pragma unroll
  for (int n1 = 0; n1 < 15; ++n1) a[n1 * BL_P + lane] = n1 ? cmul(u[n1], T2[n1 * 64 + lane]) : u[0];
  wave_sync();
  // the two halves of the pass touch disjoint rows (n1 < 8, n1 >= 8), so
  // each reads, fences and writes on its own with 8 values in registers
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int pp = lane + 64 * it, n1 = pp >> 3, b = pp & 7;
    float2 v8[8];
    if (pp < 120) {
#pragma unroll
      for (int k = 0; k < 8; ++k) v8[k] = a[n1 * BL_P + 8 * k + b];
    }
    wave_sync();
    if (pp < 120) {
      dft<8, INV>(v8);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        a[n1 * BL_P + 8 * c + (b ^ c)] = c ? cmul(v8[c], T3[c * 8 + b]) : v8[0];
    }
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int pp = lane + 64 * it, n1 = pp >> 3, c = pp & 7;
    if (pp < 120) {
      float2 v8[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v8[k] = a[n1 * BL_P + 8 * c + (k ^ c)];
      dft<8, INV>(v8);
      emit(it, n1, c, v8);
    }
  }
  wave_sync();
}

__global__ __launch_bounds__(256) void k_rows_inv_blend_960(SymGeo g, const float2 *__restrict__ z,
                                                           int T, int B, int S,
                                                           const float2 *__restrict__ A,
                                                           float scale, float *__restrict__ out) {
  extern __shared__ float2 sm[];
  constexpr int N = 960, LINE = 15 * BL_P;
  const int nz = g.nz, nx = g.nx;
  const int W = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2 *T2 = sm, *T3 = sm + N, *a = sm + SPLIT_LDS + w * LINE;
  split960_tables<true>(g.fx, T2, T3);
  __syncthreads();
  const int q = w / S, p = w - q * S;
  // the row's coefficient fields A are read by every vector group
  int row, grp;
  xcd_run(gridDim.x / nz, row, grp);
  const int v = grp * (W / S) + q;
  const bool live = v < B;  // uniform over the wavefront
  float acc[2][8];
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int d = 0; d < 8; ++d) acc[it][d] = 0.0f;
  for (int t = p; live && t < T; t += S) {
    const float2 *zr = z + (((long long)v * T + t) * nz + row) * N;
    float2 u[15];
#pragma unroll
    for (int k1 = 0; k1 < 15; ++k1) u[k1] = zr[64 * k1 + lane];
    const float2 *Ar = A + ((long long)t * nz + row) * nx;
    split960<true>(u, a, T2, T3, [&](int it, int n1, int c, const float2 (&y)[8]) {
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int x = n1 + 15 * (c + 8 * d);
        if (x < nx) {
          const float2 cf = Ar[x];
          acc[it][d] = fmaf(cf.x, y[d].x, fmaf(-cf.y, y[d].y, acc[it][d]));
        }
      }
    });
  }
  if (S > 1) {  // uniform over the workgroup
    float *part = reinterpret_cast<float *>(a);  // 2 LINE floats >= nx
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int pp = lane + 64 * it, n1 = pp >> 3, c = pp & 7;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int x = n1 + 15 * (c + 8 * d);
        if (pp < 120 && x < nx) part[x] = acc[it][d];
      }
    }
    __syncthreads();
    if (p == 0) {
      for (int k = 1; k < S; ++k) {
        const float *pk = reinterpret_cast<const float *>(a + k * LINE);
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int pp = lane + 64 * it, n1 = pp >> 3, c = pp & 7;
#pragma unroll
          for (int d = 0; d < 8; ++d) {
            const int x = n1 + 15 * (c + 8 * d);
            if (pp < 120 && x < nx) acc[it][d] += pk[x];
          }
        }
      }
    }
  }
  if (!live || p != 0) return;
  const float f = scale / ((float)g.mz * (float)N);
  float *o = out + ((long long)v * nz + row) * nx;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int pp = lane + 64 * it, n1 = pp >> 3, c = pp & 7;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int x = n1 + 15 * (c + 8 * d);
      if (pp < 120 && x < nx) o[x] = acc[it][d] * f;
    }
  }
}

// Forward row transforms of 960 points with the split transform of the
// blend (forward sign): one wavefront per row, four rows per workgroup, the
// real inputs loaded straight from global memory.  Rows in[row][cols] (zero
// beyond cols), row = the flat index over the batch; out[row][960].
__global__ __launch_bounds__(256) void k_rows_fwd_960(SymGeo g, const float *__restrict__ in,
                                                     int nrows, int cols,
                                                     float2 *__restrict__ out) {
  extern __shared__ float2 sm[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2 *T2 = sm, *T3 = sm + 960, *a = sm + SPLIT_LDS + w * 15 * BL_P;
  split960_tables<false>(g.fx, T2, T3);
  __syncthreads();
  const long long row = (long long)blockIdx.x * (blockDim.x >> 6) + w;
  if (row >= nrows) return;  // whole wavefront, after the only workgroup barrier
  const float *src = in + row * cols;
  float2 u[15];
#pragma unroll
  for (int k1 = 0; k1 < 15; ++k1) {
    const int i = 64 * k1 + lane;
    u[k1] = make_float2(i < cols ? src[i] : 0.0f, 0.0f);
  }
  float2 *dst = out + row * 960;
  split960<false>(u, a, T2, T3, [&](int, int n1, int c, const float2 (&y)[8]) {
#pragma unroll
    for (int d = 0; d < 8; ++d) dst[n1 + 15 * (c + 8 * d)] = y[d];
  });
}

// Inverse row transforms of z[0][t][row] and demodulation by the sample
// frequency: cols[t][row][x] = z_t e^{-i x.xi_t} / M (phase in FP64).  Grid
// (nz, T).
__global__ __launch_bounds__(NTH) void k_rows_inv_demod(SymGeo g, const float2 *__restrict__ z,
                                                        float2 *__restrict__ cols) {
  extern __shared__ float2 sm[];
  const int n = g.mx, nz = g.nz, nx = g.nx;
  float2 *a = sm, *b = sm + n;
  const float2 *tw = g.fx.tw;
  const int row = blockIdx.x, t = blockIdx.y;
  const float2 *zr = z + ((long long)t * nz + row) * n;
  staged<8>(n, [&](int i) { return zr[i]; }, [&](int i, float2 v) { a[i] = v; });
  __syncthreads();
  const float2 *res = fft_lines<true>(a, b, n, 1, g.fx, tw);
  const double inv_m = 1.0 / ((double)g.mz * g.mx);
  for (int x = threadIdx.x; x < nx; x += NTH) {
    const double ph = g.h * ((double)x * g.sx[t] + (double)row * g.sz[t]);
    double s, c;
    sincos(ph, &s, &c);
    const double re = res[x].x, im = res[x].y;
    cols[((long long)t * nz + row) * nx + x] =
        make_float2((float)((re * c + im * s) * inv_m), (float)((im * c - re * s) * inv_m));
  }
}

// ------------------------------------------------------------------- PDO

__global__ void k_pdo_probe(SymGeo g, float *__restrict__ vp) {
  const long long total = (long long)g.nz * g.nx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int iz = (int)(e / g.nx), ix = (int)(e - (long long)iz * g.nx);
    double s = 0.0;
    for (int k = 0; k < g.r / 2; ++k) s += 2.0 * cos(g.h * ((double)ix * g.sx[k] + (double)iz * g.sz[k]));
    vp[e] = (float)s;
  }
}

__device__ inline void reps(int p, int m, double step, double *v, int *cnt) {
  const int c = p <= m / 2 ? p : p - m;
  v[0] = c * step;
  *cnt = 1;
  if ((m & 1) == 0 && p == m / 2) {
    v[1] = -v[0];
    *cnt = 2;
  }
}

// Masks (nearest sample frequency, ties shared) and weights (rho / rho0 times
// the angular cardinal function) for k = 1..r/2, averaged over the
// representatives of each lattice point.  Either output may be null.
__global__ void k_pdo_tables(SymGeo g, float2 *__restrict__ masks, float2 *__restrict__ wts) {
  const long long plane = (long long)g.mz * g.mx;
  const int r = g.r, hr = r / 2;
  const double two_pi = 6.283185307179586476925;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < plane;
       e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e / g.mx), q = (int)(e - (long long)p * g.mx);
    double zr[2], xr[2];
    int nzr, nxr;
    reps(p, g.mz, two_pi / (g.mz * g.h), zr, &nzr);
    reps(q, g.mx, two_pi / (g.mx * g.h), xr, &nxr);
    double mk[SYM_RMAX / 2], wk[SYM_RMAX / 2];
    for (int k = 0; k < hr; ++k) mk[k] = wk[k] = 0.0;
    for (int a = 0; a < nzr; ++a) {
      for (int b = 0; b < nxr; ++b) {
        const double xz = zr[a], xx = xr[b];
        double d[SYM_RMAX];
        double dmin = 1e300;
        for (int k = 0; k < r; ++k) {
          const double sx = k < hr ? g.sx[k] : -g.sx[k - hr];
          const double sz = k < hr ? g.sz[k] : -g.sz[k - hr];
          d[k] = (xx - sx) * (xx - sx) + (xz - sz) * (xz - sz);
          dmin = fmin(dmin, d[k]);
        }
        const double lim = dmin + TIE * (xx * xx + xz * xz + g.rho0 * g.rho0);
        int cnt = 0;
        for (int k = 0; k < r; ++k) cnt += d[k] <= lim;
        const double rho = sqrt(xx * xx + xz * xz);
        const double th = atan2(xz, xx);
        for (int k = 0; k < hr; ++k) {
          if (d[k] <= lim) mk[k] += 1.0 / cnt;
          const double dth = th - two_pi * (k + 1) / r;
          double w = 1.0 + cos((r / 2) * dth);
          for (int m = 1; m < r / 2; ++m) w += 2.0 * cos(m * dth);
          wk[k] += rho / g.rho0 * w / r;
        }
      }
    }
    const double inv = 1.0 / (nzr * nxr);
    for (int k = 0; k < hr; ++k) {
      if (masks) masks[k * plane + e] = make_float2((float)(mk[k] * inv), 0.0f);
      if (wts) wts[k * plane + e] = make_float2((float)(wk[k] * inv), 0.0f);
    }
  }
}

// ------------------------------------------------------------------ PSF+

struct PsfLat {  // centre lattice of the PSF method
  int oz, ox, sz, sx, nzc, nxc, half, W, r;
};

// 1-D tent weights at index i: (c0, w0) and (c1, w1); c1 = c0 and w1 = 0 at
// the clamped ends.
__device__ inline void tent(int i, int o, int s, int n, int *c0, float *w0, int *c1, float *w1) {
  if (n == 1 || i <= o) {
    *c0 = *c1 = 0;
    *w0 = 1.0f;
    *w1 = 0.0f;
  } else if (i >= o + (n - 1) * s) {
    *c0 = *c1 = n - 1;
    *w0 = 1.0f;
    *w1 = 0.0f;
  } else {
    const int p = (i - o) / s;
    const float t = (float)(i - o - p * s) / (float)s;
    *c0 = p;
    *c1 = p + 1;
    *w0 = 1.0f - t;
    *w1 = t;
  }
}

// Real planes grid[j][mz][mx] holding kernel q_j at the wrapped offsets.
__global__ void k_pp_scatter(int mz, int mx, int half, int W, const float *__restrict__ q, int rank,
                             float *__restrict__ grid) {
  const long long plane = (long long)mz * mx, total = plane * rank;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e / plane);
    const long long o = e - j * plane;
    const int p = (int)(o / mx), c = (int)(o - (long long)p * mx);
    const int dz = p <= half ? p : (p >= mz - half ? p - mz : 1 << 20);
    const int dx = c <= half ? c : (c >= mx - half ? c - mx : 1 << 20);
    float v = 0.0f;
    if (dz <= half && dx <= half) v = q[(long long)j * W * W + (dz + half) * W + dx + half];
    grid[e] = v;
  }
}

// M_t = b_{2t} + i b_{2t+1}, b_j = conj(sum_d q_j(d) e^{-i d.xi}) = conj(Bq_j).
__global__ void k_pp_pack(long long plane, const float2 *__restrict__ Bq, int rank, int T,
                          float2 *__restrict__ M) {
  const long long total = plane * T;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / plane);
    const long long o = e - t * plane;
    const float2 b0 = Bq[(long long)(2 * t) * plane + o];
    float2 m = make_float2(b0.x, -b0.y);
    if (2 * t + 1 < rank) {
      const float2 b1 = Bq[(long long)(2 * t + 1) * plane + o];
      m.x += b1.y;  // i conj(b1) = (b1.y, b1.x)
      m.y += b1.x;
    }
    M[e] = m;
  }
}

// sigma_j = sqrt(M mu_j) from the Gram eigenvalues mu (descending), the
// kernel coefficients Qc[j][k] = U[k][j] / sigma_j (zero for dropped rows),
// info[1] = kept rows, info[2 + j] = sigma_j.
__global__ void k_pp_coefq(int rp, int rank, double M, const double *__restrict__ mu,
                           const double *__restrict__ U, float *__restrict__ Qc,
                           double *__restrict__ sigma, double *__restrict__ info) {
  const double top = mu[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rank * rp; e += gridDim.x * blockDim.x) {
    const int j = e / rp, k = e - j * rp;
    const bool keep = top > 0.0 && mu[j] > 1e-12 * top;
    const double s = keep ? sqrt(M * mu[j]) : 0.0;
    Qc[e] = keep ? (float)(U[(long long)k * rp + j] / s) : 0.0f;
    if (k == 0) {
      sigma[j] = s;
      info[2 + j] = s;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int kept = 0;
    for (int j = 0; j < rank; ++j) kept += (top > 0.0 && mu[j] > 1e-12 * top);
    info[1] = kept;
  }
}

// Bc[j][k] = sum_d q_j(d) e^{i d.xi_k} for k < r/2 (FP64 phases and sums).
// Grid (rank, r/2).
__global__ __launch_bounds__(NTH) void k_pp_bc(SymGeo g, int half, const float *__restrict__ q,
                                               double2 *__restrict__ Bc) {
  const int j = blockIdx.x, k = blockIdx.y, hr = gridDim.y, W = 2 * half + 1;
  double re = 0.0, im = 0.0;
  for (int e = threadIdx.x; e < W * W; e += NTH) {
    const int dz = e / W - half, dx = e % W - half;
    const double ph = g.h * ((double)dx * g.sx[k] + (double)dz * g.sz[k]);
    double s, c;
    sincos(ph, &s, &c);
    const double v = q[(long long)j * W * W + e];
    re += v * c;
    im += v * s;
  }
  __shared__ double rr[NTH], ii[NTH];
  rr[threadIdx.x] = re;
  ii[threadIdx.x] = im;
  __syncthreads();
  for (int w = NTH / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rr[threadIdx.x] += rr[threadIdx.x + w];
      ii[threadIdx.x] += ii[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) Bc[j * hr + k] = make_double2(rr[0], ii[0]);
}

// The Tikhonov normal equations: alpha = ||B[:, I_c]||^2 / ||B||^2 (= kept
// orthonormal rows), G = Re(Bc Bc^H) + alpha I over all r columns (the
// conjugate half doubles the real part), Ginv by Gauss-Jordan, and the
// per-point maps
//   Xr[k][l] = 2 sum_j Re Bc[j][k] Ginv[j][l],  Xi[k][l] = 2 sum_j Im Bc[j][k] Ginv[j][l],
//   Z[c][l]  = alpha sum_j U[c][j] sigma_j Ginv[j][l]
// so that a_l(x) = sum_k (Re C_k(x) Xr[k][l] + Im C_k(x) Xi[k][l])
//               + sum_c w_c(x) Z[c][l].
__global__ __launch_bounds__(NTH) void k_pp_solve(int rank, int hr, int rp,
                                                  const double2 *__restrict__ Bc,
                                                  const double *__restrict__ U,
                                                  const double *__restrict__ sigma,
                                                  float *__restrict__ Xr, float *__restrict__ Xi,
                                                  float *__restrict__ Z, double *__restrict__ info) {
  __shared__ double G[PP_RANK][2 * PP_RANK];
  __shared__ double alpha_s;
  if (threadIdx.x == 0) {
    double nb = 0.0;
    int kept = 0;
    for (int j = 0; j < rank; ++j) {
      kept += sigma[j] > 0.0;
      for (int k = 0; k < hr; ++k) nb += 2.0 * (Bc[j * hr + k].x * Bc[j * hr + k].x + Bc[j * hr + k].y * Bc[j * hr + k].y);
    }
    const double alpha = kept > 0 ? nb / kept : 0.0;
    alpha_s = alpha;
    info[0] = alpha;
    for (int j = 0; j < rank; ++j) {
      for (int l = 0; l < rank; ++l) {
        double s = 0.0;
        for (int k = 0; k < hr; ++k) s += Bc[j * hr + k].x * Bc[l * hr + k].x + Bc[j * hr + k].y * Bc[l * hr + k].y;
        G[j][l] = 2.0 * s + (j == l ? (alpha > 0.0 ? alpha : 1.0) : 0.0);
        G[j][rank + l] = j == l ? 1.0 : 0.0;
      }
    }
    // Gauss-Jordan with partial pivoting on [G | I]
    for (int c = 0; c < rank; ++c) {
      int piv = c;
      for (int i = c + 1; i < rank; ++i)
        if (fabs(G[i][c]) > fabs(G[piv][c])) piv = i;
      if (piv != c)
        for (int l = 0; l < 2 * rank; ++l) {
          const double t = G[c][l];
          G[c][l] = G[piv][l];
          G[piv][l] = t;
        }
      const double d = 1.0 / G[c][c];
      for (int l = 0; l < 2 * rank; ++l) G[c][l] *= d;
      for (int i = 0; i < rank; ++i) {
        if (i == c) continue;
        const double f = G[i][c];
        if (f != 0.0)
          for (int l = 0; l < 2 * rank; ++l) G[i][l] -= f * G[c][l];
      }
    }
  }
  __syncthreads();
  const double alpha = alpha_s;
  // with alpha = 0 (no basis energy at the samples) the coefficients are A0
  const double ya = alpha > 0.0 ? alpha : 1.0;
  for (int e = threadIdx.x; e < hr * rank; e += NTH) {
    const int k = e / rank, l = e - k * rank;
    double sr = 0.0, si = 0.0;
    if (alpha > 0.0)
      for (int j = 0; j < rank; ++j) {
        sr += Bc[j * hr + k].x * G[j][rank + l];
        si += Bc[j * hr + k].y * G[j][rank + l];
      }
    Xr[e] = (float)(2.0 * sr);
    Xi[e] = (float)(2.0 * si);
  }
  for (int e = threadIdx.x; e < rp * rank; e += NTH) {
    const int c = e / rank, l = e - c * rank;
    double s = 0.0;
    for (int j = 0; j < rank; ++j) s += U[(long long)c * rp + j] * sigma[j] * G[j][rank + l];
    Z[e] = (float)(ya * s);
  }
}

// a_l(x) for every model cell, packed A_t = a_{2t} - i a_{2t+1}.
__global__ __launch_bounds__(NTH) void k_pp_coef(int nz, int nx, PsfLat L, int rank, int hr,
                                                 const float2 *__restrict__ cols,
                                                 const float *__restrict__ Xr,
                                                 const float *__restrict__ Xi,
                                                 const float *__restrict__ Z,
                                                 float2 *__restrict__ A) {
  const long long plane = (long long)nz * nx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < plane;
       e += (long long)gridDim.x * blockDim.x) {
    const int iz = (int)(e / nx), ix = (int)(e - (long long)iz * nx);
    int pz0, pz1, qx0, qx1;
    float wz0, wz1, wx0, wx1;
    tent(iz, L.oz, L.sz, L.nzc, &pz0, &wz0, &pz1, &wz1);
    tent(ix, L.ox, L.sx, L.nxc, &qx0, &wx0, &qx1, &wx1);
    const int c00 = pz0 * L.nxc + qx0, c01 = pz0 * L.nxc + qx1;
    const int c10 = pz1 * L.nxc + qx0, c11 = pz1 * L.nxc + qx1;
    const float w00 = wz0 * wx0, w01 = wz0 * wx1, w10 = wz1 * wx0, w11 = wz1 * wx1;
    float a[PP_RANK];
#pragma unroll
    for (int l = 0; l < PP_RANK; ++l) a[l] = 0.0f;
    for (int k = 0; k < hr; ++k) {
      const float2 c = cols[k * plane + e];
#pragma unroll
      for (int l = 0; l < PP_RANK; ++l)
        if (l < rank) a[l] = fmaf(c.x, Xr[k * rank + l], fmaf(c.y, Xi[k * rank + l], a[l]));
    }
#pragma unroll
    for (int l = 0; l < PP_RANK; ++l) {
      if (l < rank) {
        float s = a[l];
        s = fmaf(w00, Z[c00 * rank + l], s);
        s = fmaf(w01, Z[c01 * rank + l], s);
        s = fmaf(w10, Z[c10 * rank + l], s);
        s = fmaf(w11, Z[c11 * rank + l], s);
        a[l] = s;
      }
    }
#pragma unroll
    for (int t = 0; t < PP_RANK / 2; ++t) {
      if (2 * t < rank)
        A[t * plane + e] = make_float2(a[2 * t], 2 * t + 1 < rank ? -a[2 * t + 1] : 0.0f);
    }
  }
}

unsigned nblk(long long n) { return (unsigned)std::min<long long>((n + NTH - 1) / NTH, 16384); }

}  // namespace
}  // namespace fwi

using namespace fwi;

struct fwi_symbol {
  fwi_symbol_grid gi{};
  SymGeo g{};
  std::vector<float2> host;  // twiddles of mx, then of mz
  size_t off_tz = 0;         // float2 offset of the mz table
  void *dev = nullptr;
  size_t zchunk = (size_t)4 << 30;  // bytes of partial transforms per vector chunk
  int split = 0;              // wavefronts per vector of the blend (0: by grid size)
  int r960 = 1;               // 1: the 15 x 64 blend for 960-point rows
};

namespace {

#define SY_TRY(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(FWI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

template <class T>
T *at_(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Stage radices of length n, largest first; `big` admits 15 and 9 (column
// passes only, see fft_lines).
bool factor(int n, Fft1 &f, bool big) {
  f.n = n;
  f.ns = 0;
  int m = n;
  const int all[7] = {8, 9, 15, 4, 2, 3, 5};
  for (int R : all) {
    if (!big && (R == 15 || R == 9)) continue;
    while (m % R == 0) {
      if (f.ns == FFT_MAXST) return false;
      f.radix[f.ns++] = R;
      m /= R;
    }
  }
  return m == 1;
}

int check_grid(const fwi_symbol_grid *g) {
  if (!g) return set_error(FWI_EINVAL, "symbol grid is null");
  if (g->nz < 1 || g->nx < 1 || g->nz > FFT_MAXN || g->nx > FFT_MAXN)
    return set_error(FWI_EINVAL, "symbol grid: nz, nx must be in [1, 2048]");
  if (g->mz < g->nz || g->mx < g->nx || g->mz > FFT_MAXN || g->mx > FFT_MAXN)
    return set_error(FWI_EINVAL, "symbol grid: need nz <= mz <= 2048 and nx <= mx <= 2048");
  Fft1 f;
  if (!factor(g->mz, f, true) || !factor(g->mx, f, false))
    return set_error(FWI_EINVAL, "symbol grid: mz and mx must have no prime factor above 5");
  if (!(g->h > 0.0)) return set_error(FWI_EINVAL, "symbol grid: h must be positive");
  if (g->r < 2 || g->r > SYM_RMAX || (g->r & 1))
    return set_error(FWI_EINVAL, "symbol grid: r must be even, in [2, 16]");
  if (!(g->rho0 > 0.0) || !std::isfinite(g->rho0))
    return set_error(FWI_EINVAL, "symbol grid: rho0 must be positive");
  return FWI_OK;
}

int check_bound(const fwi_symbol *s) {
  if (!s) return set_error(FWI_EINVAL, "symbol object is null");
  if (!s->dev) return set_error(FWI_EUNBOUND, "symbol object has no device block: call fwi_symbol_bind");
  return FWI_OK;
}

// Column band width of the column passes (LDS: twiddles + two bands).
int col_band(int mz) {  // log2 of the band width
  int C = (LDS_BUDGET / (int)sizeof(float2) - mz) / (2 * (mz + 1));
  C = std::max(1, std::min(16, C));
  int cs = 0;
  while ((2 << cs) <= C) ++cs;
  return cs;
}
// Workgroups of a column pass: the bands, padded to a multiple of the 8 XCDs.
unsigned band_grid(int mx, int C) { return (unsigned)(8 * (((mx + C - 1) / C + 7) / 8)); }
size_t col_lds(int mz, int cs) { return sizeof(float2) * (mz + 2 * ((size_t)1 << cs) * (mz + 1)); }
size_t row_lds(int mx) { return sizeof(float2) * 2 * (size_t)mx; }

// Wavefronts per workgroup of the blend: a line of
// mx values each plus the twiddles within the LDS budget (3 or 4 for mx <=
// 2048).
int blend_waves(int mx) { return std::min(4, (int)(LDS_BUDGET / sizeof(float2) - mx) / mx); }

// Wavefronts per vector of the blend: split the terms while the grid holds
// fewer than `target` wavefronts (S divides W, S <= T).
int blend_split(int W, int nz, int nb, int T, int target) {
  int S = 1;
  for (int c = 2; c <= W; ++c)
    if (W % c == 0 && c <= T && (long long)nz * nb * S < target) S = c;
  return S;
}

int blend_w(const fwi_symbol *s, const SymGeo &g, const float2 *z, int T, int nb,
            const float2 *A, float scale, float *out, hipStream_t st) {
  const int W = blend_waves(g.mx);
  const int S = s->split ? (W % s->split == 0 ? std::min(s->split, W) : 1)
                         : blend_split(W, g.nz, nb, T, 8192);
  const int vpw = W / S;
  const dim3 grid(g.nz * ((nb + vpw - 1) / vpw)), block(64 * W);
  const size_t lds = sizeof(float2) * (size_t)g.mx * (1 + W);
  if (g.mx == 960 && s->r960) {
    const size_t l960 = sizeof(float2) * (960 + 64 + (size_t)W * 15 * BL_P);
    hipLaunchKernelGGL(k_rows_inv_blend_960, grid, block, l960, st, g, z, T, nb, S, A, scale, out);
  } else if (g.mx <= 512)
    hipLaunchKernelGGL(k_rows_inv_blend_w<512>, grid, block, lds, st, g, z, T, nb, S, A, scale, out);
  else if (g.mx <= 1024)
    hipLaunchKernelGGL(k_rows_inv_blend_w<1024>, grid, block, lds, st, g, z, T, nb, S, A, scale, out);
  else
    hipLaunchKernelGGL(k_rows_inv_blend_w<2048>, grid, block, lds, st, g, z, T, nb, S, A, scale, out);
  return FWI_OK;
}

// Vectors per chunk of an apply: the partial transforms of one chunk stay
// within `zchunk` bytes (default 4 GiB: measured, smaller chunks that keep
// them in the last-level cache lose more to lower parallelism than they gain).
int apply_chunk(const fwi_symbol *s, int B, int T) {
  const size_t per = sizeof(float2) * (size_t)T * s->gi.nz * s->gi.mx;
  const int most = (int)std::max<size_t>(1, std::min<size_t>((size_t)B, s->zchunk / per));
  const int chunks = (B + most - 1) / most;
  return (B + chunks - 1) / chunks;  // balanced
}

struct ApplyLayout {
  size_t spec, rowt, z, total;
};
ApplyLayout apply_layout(const fwi_symbol *s, int B, int T) {
  const fwi_symbol_grid &g = s->gi;
  const int Bc = apply_chunk(s, B, T);
  ApplyLayout L{};
  size_t off = 0;
  L.spec = off; off += up256(sizeof(float2) * (size_t)Bc * g.mz * g.mx);
  L.rowt = off; off += up256(sizeof(float2) * (size_t)Bc * g.nz * g.mx);
  L.z = off; off += up256(sizeof(float2) * (size_t)Bc * T * g.nz * g.mx);
  L.total = off;
  return L;
}

// spec[b] = unnormalised forward 2-D DFT of the zero-padded real planes
// in[b][rows][cols] (rows <= mz, cols <= mx).
int forward(const fwi_symbol *s, const float *in, int rows, int cols, int B, float2 *rowt,
            float2 *spec, hipStream_t st) {
  const SymGeo &g = s->g;
  if (g.mx == 960 && s->r960) {
    const int nrows = rows * B;
    hipLaunchKernelGGL(k_rows_fwd_960, dim3((nrows + 3) / 4), dim3(256),
                       sizeof(float2) * (SPLIT_LDS + 4 * 15 * BL_P), st, g, in, nrows, cols, rowt);
  } else {
    hipLaunchKernelGGL(k_rows_fwd, dim3(rows, B), dim3(NTH), row_lds(g.mx), st, g, in, rows, cols,
                       rowt);
  }
  SY_TRY(hipGetLastError());
  const int cs = col_band(g.mz), C = 1 << cs;
  hipLaunchKernelGGL(k_cols_fwd, dim3(band_grid(g.mx, C), B), dim3(CNT), col_lds(g.mz, cs), st, g,
                     rowt, rows, cs, spec);
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

int inverse_cols(const fwi_symbol *s, const float2 *spec, const float2 *M, int T, int B, float2 *z,
                 hipStream_t st) {
  const SymGeo &g = s->g;
  const int cs = col_band(g.mz), C = 1 << cs;
  hipLaunchKernelGGL(k_cols_inv, dim3(band_grid(g.mx, C), T, B), dim3(CNT), col_lds(g.mz, cs), st, g,
                     spec, M, T, cs, z);
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

}  // namespace

extern "C" {

int fwi_symbol_check(const fwi_symbol_grid *g) { return check_grid(g); }

int fwi_symbol_set_option(fwi_symbol *s, int option, int value) {
  if (!s) return set_error(FWI_EINVAL, "null symbol");
  switch (option) {
    case FWI_SYM_OPT_CHUNK_MB:
      if (value < 1 || value > (1 << 20)) return set_error(FWI_EINVAL, "chunk must be in [1, 2^20] MiB");
      s->zchunk = (size_t)value << 20;
      return FWI_OK;
    case FWI_SYM_OPT_BLEND_SPLIT:
      if (value < 0 || value > 4) return set_error(FWI_EINVAL, "blend split must be in [0, 4]");
      s->split = value;
      return FWI_OK;
    case FWI_SYM_OPT_SPLIT_960:
      if (value < 0 || value > 1) return set_error(FWI_EINVAL, "960-point split must be 0 or 1");
      s->r960 = value;
      return FWI_OK;
    default:
      return set_error(FWI_EINVAL, "unknown symbol option");
  }
}

int fwi_symbol_get_option(const fwi_symbol *s, int option, int *value) {
  if (!s || !value) return set_error(FWI_EINVAL, "null argument");
  switch (option) {
    case FWI_SYM_OPT_CHUNK_MB: *value = (int)(s->zchunk >> 20); return FWI_OK;
    case FWI_SYM_OPT_BLEND_SPLIT: *value = s->split; return FWI_OK;
    case FWI_SYM_OPT_SPLIT_960: *value = s->r960; return FWI_OK;
    default: return set_error(FWI_EINVAL, "unknown symbol option");
  }
}

int fwi_symbol_create(const fwi_symbol_grid *g, fwi_symbol **out) {
  if (!out) return set_error(FWI_EINVAL, "null argument");
  *out = nullptr;
  if (int rc = check_grid(g)) return rc;
  fwi_symbol *s = new fwi_symbol;
  s->gi = *g;
  SymGeo &G = s->g;
  G.nz = g->nz;
  G.nx = g->nx;
  G.mz = g->mz;
  G.mx = g->mx;
  G.r = g->r;
  G.h = g->h;
  G.rho0 = g->rho0;
  factor(g->mz, G.fz, true);
  factor(g->mx, G.fx, false);
  for (int k = 0; k < g->r / 2; ++k) {
    const double th = 2.0 * M_PI * (k + 1) / g->r;
    G.sx[k] = g->rho0 * std::cos(th);
    G.sz[k] = g->rho0 * std::sin(th);
  }
  s->host.resize((size_t)g->mx + g->mz);
  for (int m = 0; m < g->mx; ++m) {
    const double a = -2.0 * M_PI * m / g->mx;
    s->host[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  s->off_tz = (size_t)g->mx;
  for (int m = 0; m < g->mz; ++m) {
    const double a = -2.0 * M_PI * m / g->mz;
    s->host[s->off_tz + m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  *out = s;
  return FWI_OK;
}

void fwi_symbol_destroy(fwi_symbol *s) { delete s; }

int fwi_symbol_device_bytes(const fwi_symbol *s, size_t *bytes) {
  if (!s || !bytes) return set_error(FWI_EINVAL, "null argument");
  *bytes = sizeof(float2) * s->host.size();
  return FWI_OK;
}

int fwi_symbol_bind(fwi_symbol *s, void *dev, size_t bytes, void *stream) {
  if (!s || !dev) return set_error(FWI_EINVAL, "null argument");
  if (bytes < sizeof(float2) * s->host.size()) return set_error(FWI_ENOMEM, "symbol device block too small");
  if (reinterpret_cast<uintptr_t>(dev) & 255)
    return set_error(FWI_EINVAL, "symbol device block must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SY_TRY(hipMemcpyAsync(dev, s->host.data(), sizeof(float2) * s->host.size(), hipMemcpyHostToDevice, st));
  SY_TRY(hipStreamSynchronize(st));
  s->dev = dev;
  s->g.fx.tw = static_cast<const float2 *>(dev);
  s->g.fz.tw = static_cast<const float2 *>(dev) + s->off_tz;
  return FWI_OK;
}

int fwi_symbol_workspace_size(const fwi_symbol *s, int B, int T, size_t *bytes) {
  if (!s || !bytes) return set_error(FWI_EINVAL, "null argument");
  if (B < 1 || B > 1024 || T < 1 || T > 64) return set_error(FWI_EINVAL, "B must be in [1, 1024], T in [1, 64]");
  *bytes = apply_layout(s, B, T).total;
  return FWI_OK;
}

int fwi_symbol_apply(fwi_symbol *s, int T, const float *A, const float *M, float scale,
                     const float *v, int B, float *out, void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_bound(s)) return rc;
  if (!A || !M || !v || !out || !ws) return set_error(FWI_EINVAL, "fwi_symbol_apply: null array");
  if (B < 1 || B > 1024 || T < 1 || T > 64) return set_error(FWI_EINVAL, "fwi_symbol_apply: B must be in [1, 1024], T in [1, 64]");
  if (v == out) return set_error(FWI_EINVAL, "fwi_symbol_apply: out must not alias v");
  const ApplyLayout L = apply_layout(s, B, T);
  if (ws_bytes < L.total) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(L.total));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const SymGeo &g = s->g;
  float2 *spec = at_<float2>(ws, L.spec), *rowt = at_<float2>(ws, L.rowt), *z = at_<float2>(ws, L.z);
  const int Bc = apply_chunk(s, B, T);
  const long long plane = (long long)g.nz * g.nx;
  for (int b0 = 0; b0 < B; b0 += Bc) {
    const int nb = std::min(Bc, B - b0);
    if (int rc = forward(s, v + b0 * plane, g.nz, g.nx, nb, rowt, spec, st)) return rc;
    if (int rc = inverse_cols(s, spec, reinterpret_cast<const float2 *>(M), T, nb, z, st)) return rc;
    if (int rc = blend_w(s, g, z, T, nb, reinterpret_cast<const float2 *>(A), scale,
                         out + b0 * plane, st))
      return rc;
    SY_TRY(hipGetLastError());
  }
  return FWI_OK;
}

int fwi_pdo_probe(fwi_symbol *s, float *vp, void *stream) {
  if (!s || !vp) return set_error(FWI_EINVAL, "fwi_pdo_probe: null argument");
  hipLaunchKernelGGL(k_pdo_probe, dim3(nblk((long long)s->g.nz * s->g.nx)), dim3(NTH), 0,
                     static_cast<hipStream_t>(stream), s->g, vp);
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

static int pdo_tables(fwi_symbol *s, float *masks, float *wts, void *stream) {
  hipLaunchKernelGGL(k_pdo_tables, dim3(nblk((long long)s->g.mz * s->g.mx)), dim3(NTH), 0,
                     static_cast<hipStream_t>(stream), s->g, reinterpret_cast<float2 *>(masks),
                     reinterpret_cast<float2 *>(wts));
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

int fwi_pdo_weights(fwi_symbol *s, float *M, void *stream) {
  if (!s || !M) return set_error(FWI_EINVAL, "fwi_pdo_weights: null argument");
  return pdo_tables(s, nullptr, M, stream);
}

int fwi_pdo_masks(fwi_symbol *s, float *masks, void *stream) {
  if (!s || !masks) return set_error(FWI_EINVAL, "fwi_pdo_masks: null argument");
  return pdo_tables(s, masks, nullptr, stream);
}

int fwi_pdo_workspace_size(const fwi_symbol *s, size_t *bytes) {
  if (!s || !bytes) return set_error(FWI_EINVAL, "null argument");
  const int hr = s->gi.r / 2;
  *bytes = apply_layout(s, 1, hr).total + up256(sizeof(float2) * (size_t)hr * s->gi.mz * s->gi.mx);
  return FWI_OK;
}

int fwi_pdo_columns(fwi_symbol *s, const float *hvp, float *cols, void *ws, size_t ws_bytes,
                    void *stream) {
  if (int rc = check_bound(s)) return rc;
  if (!hvp || !cols || !ws) return set_error(FWI_EINVAL, "fwi_pdo_columns: null array");
  size_t need = 0;
  fwi_pdo_workspace_size(s, &need);
  if (ws_bytes < need) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(need));
  const SymGeo &g = s->g;
  const int hr = g.r / 2;
  const ApplyLayout L = apply_layout(s, 1, hr);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2 *spec = at_<float2>(ws, L.spec), *rowt = at_<float2>(ws, L.rowt), *z = at_<float2>(ws, L.z);
  float2 *masks = at_<float2>(ws, L.total);
  if (int rc = pdo_tables(s, reinterpret_cast<float *>(masks), nullptr, stream)) return rc;
  if (int rc = forward(s, hvp, g.nz, g.nx, 1, rowt, spec, st)) return rc;
  if (int rc = inverse_cols(s, spec, masks, hr, 1, z, st)) return rc;
  hipLaunchKernelGGL(k_rows_inv_demod, dim3(g.nz, hr), dim3(NTH), row_lds(g.mx), st, g, z,
                     reinterpret_cast<float2 *>(cols));
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

}  // extern "C"

namespace {

struct PpLayout {
  size_t G, Z, w, Zs, part, sigma, Qc, q, grid, rowt, Bq, Bc, Xr, Xi, Zf, total;
};

PpLayout pp_layout(const fwi_symbol_grid &g, int rp, int W, int rank) {
  PpLayout L{};
  size_t off = 0;
  const size_t plane = (size_t)g.mz * g.mx;
  auto take = [&](size_t &f, size_t b) { f = off; off += up256(b); };
  take(L.G, sizeof(double) * rp * rp);
  take(L.Z, sizeof(double) * rp * rp);
  take(L.w, sizeof(double) * rp);
  take(L.Zs, sizeof(double) * rp * rp);
  take(L.part, sizeof(double) * (size_t)nchunks((long long)W * W) * rp * rp);
  take(L.sigma, sizeof(double) * rank);
  take(L.Qc, sizeof(float) * rank * rp);
  take(L.q, sizeof(float) * (size_t)rank * W * W);
  take(L.grid, sizeof(float) * rank * plane);
  take(L.rowt, sizeof(float2) * rank * plane);
  take(L.Bq, sizeof(float2) * rank * plane);
  take(L.Bc, sizeof(double2) * rank * (g.r / 2));
  take(L.Xr, sizeof(float) * rank * (g.r / 2));
  take(L.Xi, sizeof(float) * rank * (g.r / 2));
  take(L.Zf, sizeof(float) * (size_t)rp * rank);
  L.total = off;
  return L;
}

int pp_check(const fwi_symbol *s, const fwi_psf_grid *pg, int rank) {
  if (!s || !pg) return set_error(FWI_EINVAL, "null argument");
  if (int rc = fwi_psf_check(pg)) return rc;
  if (pg->nz != s->gi.nz || pg->nx != s->gi.nx)
    return set_error(FWI_EINVAL, "PSF grid and symbol grid describe different models");
  const int rp = pg->nzc * pg->nxc, W = 2 * pg->half + 1;
  if (rp > EIG_KMAX) return set_error(FWI_EINVAL, "PSF+: at most 512 PSFs");
  if (W > std::min(s->gi.mz, s->gi.mx)) return set_error(FWI_EINVAL, "PSF+: PSF window wider than the FFT grid");
  if (rank < 1 || rank > std::min(rp, PP_RANK)) return set_error(FWI_EINVAL, "PSF+: rank must be in [1, min(r_psf, 32)]");
  return FWI_OK;
}

}  // namespace

extern "C" {

int fwi_psfplus_workspace_size(const fwi_symbol *s, const fwi_psf_grid *pg, int rank,
                               size_t *bytes) {
  if (!bytes) return set_error(FWI_EINVAL, "null argument");
  if (int rc = pp_check(s, pg, rank)) return rc;
  *bytes = pp_layout(s->gi, pg->nzc * pg->nxc, 2 * pg->half + 1, rank).total;
  return FWI_OK;
}

int fwi_psfplus_build(fwi_symbol *s, const fwi_psf_grid *pg, const float *psf, const float *cols,
                      int rank, float *A, float *M, double *info, void *ws, size_t ws_bytes,
                      void *stream) {
  if (int rc = pp_check(s, pg, rank)) return rc;
  if (int rc = check_bound(s)) return rc;
  if (!psf || !cols || !A || !M || !info || !ws) return set_error(FWI_EINVAL, "fwi_psfplus_build: null array");
  const int rp = pg->nzc * pg->nxc, W = 2 * pg->half + 1, WW = W * W;
  const PpLayout L = pp_layout(s->gi, rp, W, rank);
  if (ws_bytes < L.total) return set_error(FWI_ENOMEM, "workspace too small: need " + std::to_string(L.total));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const SymGeo &g = s->g;
  const int hr = g.r / 2, T = (rank + 1) / 2;
  const long long plane = (long long)g.mz * g.mx;
  // Gram matrix of the PSF windows (FP64) and its eigenpairs
  {
    Gemm gm = plain(rp, rp, WW);
    gm.A = psf; gm.am = WW; gm.ak = 1;
    gm.B = psf; gm.bk = 1; gm.bn = WW;
    SY_TRY(gemm_long(gm, at_<double>(ws, L.part), at_<double>(ws, L.G), st));
  }
  SY_TRY(sym_eig(rp, at_<double>(ws, L.G), at_<double>(ws, L.Z), at_<double>(ws, L.w),
                 at_<double>(ws, L.Zs), st));
  hipLaunchKernelGGL(k_pp_coefq, dim3(nblk((long long)rank * rp)), dim3(NTH), 0, st, rp, rank,
                     (double)plane, at_<double>(ws, L.w), at_<double>(ws, L.Zs), at_<float>(ws, L.Qc),
                     at_<double>(ws, L.sigma), info);
  SY_TRY(hipGetLastError());
  // basis kernels q_j = sum_k U[k][j] p_k / sigma_j
  {
    Gemm gm = plain(rank, WW, rp);
    gm.A = at_<float>(ws, L.Qc); gm.am = rp; gm.ak = 1;
    gm.B = psf; gm.bk = WW; gm.bn = 1;
    gm.C = at_<float>(ws, L.q); gm.cm = WW; gm.cn = 1;
    SY_TRY(gemm(gm, 1, st));
  }
  // their symbols on the lattice, packed in pairs
  hipLaunchKernelGGL(k_pp_scatter, dim3(nblk(plane * rank)), dim3(NTH), 0, st, g.mz, g.mx,
                     pg->half, W, at_<float>(ws, L.q), rank, at_<float>(ws, L.grid));
  SY_TRY(hipGetLastError());
  if (int rc = forward(s, at_<float>(ws, L.grid), g.mz, g.mx, rank, at_<float2>(ws, L.rowt),
                       at_<float2>(ws, L.Bq), st))
    return rc;
  hipLaunchKernelGGL(k_pp_pack, dim3(nblk(plane * T)), dim3(NTH), 0, st, plane,
                     at_<float2>(ws, L.Bq), rank, T, reinterpret_cast<float2 *>(M));
  SY_TRY(hipGetLastError());
  // the basis at the sample frequencies, the normal equations, the coefficients
  hipLaunchKernelGGL(k_pp_bc, dim3(rank, hr), dim3(NTH), 0, st, g, pg->half, at_<float>(ws, L.q),
                     at_<double2>(ws, L.Bc));
  SY_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_pp_solve, dim3(1), dim3(NTH), 0, st, rank, hr, rp, at_<double2>(ws, L.Bc),
                     at_<double>(ws, L.Zs), at_<double>(ws, L.sigma), at_<float>(ws, L.Xr),
                     at_<float>(ws, L.Xi), at_<float>(ws, L.Zf), info);
  SY_TRY(hipGetLastError());
  PsfLat lat{pg->oz, pg->ox, pg->sz, pg->sx, pg->nzc, pg->nxc, pg->half, W, rp};
  hipLaunchKernelGGL(k_pp_coef, dim3(nblk((long long)g.nz * g.nx)), dim3(NTH), 0, st, g.nz, g.nx, lat,
                     rank, hr, reinterpret_cast<const float2 *>(cols), at_<float>(ws, L.Xr),
                     at_<float>(ws, L.Xi), at_<float>(ws, L.Zf), reinterpret_cast<float2 *>(A));
  SY_TRY(hipGetLastError());
  return FWI_OK;
}

}  // extern "C"

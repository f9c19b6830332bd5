// gfx950 kernels of the acoustic Gauss-Newton Hessian-vector product.
//
// Scheme (the paper's eq. (1) discretised; the paper does not fix the
// discretisation): u^{n+1} = 2a u^n - b u^{n-1} + c w^n, w^n = L u^n + f^n,
// with L the 8th-order Laplacian, a = 1/(1+kappa), b = (1-kappa)/(1+kappa),
// c = (dt m_pad)^2/(1+kappa).  The Born field obeys the same recurrence with
// source dc * w^n, dc = (2c/m_pad) * (P v).  The adjoint runs in the
// variable mu = c * lambda, for which the transposed recurrence becomes the
// forward one, mu^k = 2a mu^{k+1} - b mu^{k+2} + c (L mu^{k+1} + R^T r^k),
// and the zero-lag image is sum_n (2/m_pad) w^n mu^{n+1}.
//
// Every time step is one launch over (tile x shot) workgroups of 256 threads.
// A workgroup stages its 64 x 32 tile plus a 4-cell halo of the wavefield in
// LDS, each wavefront owns 8 consecutive rows of every column and keeps the
// column window in registers.  The stencil is memory bound (about 2 flop per
// byte against a vector ridge near 20), so no MFMA is involved.
#include "fwi_internal.h"

namespace fwi {

static_assert(TZ * 2 * HALO == NTHREADS, "side halo: one value per thread");
static_assert(LH % NWAVE == 0, "tile rows split evenly over wavefronts");

// Workgroup ids are dealt round-robin over the 8 XCDs.  Give each XCD one
// contiguous range of logical ids, so neighbouring tiles of one wavefield run
// on the same XCD and their halo re-reads hit its L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  constexpr int NXCD = 8;
  const int q = n / NXCD, rem = n % NXCD;
  const int x = bid % NXCD, slot = bid / NXCD;
  return (x < rem) ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
}

__device__ __forceinline__ float sponge_kappa(const Geo &g, int i, int j) {
  const int dxc = max(max(g.nb - j, 0), j - (g.nxp - 1 - g.nb));
  const int dzc = max(max(g.nb - i, 0), i - (g.nzp - 1 - g.nb));
  const float fx = dxc * g.inv_nb, fz = dzc * g.inv_nb;
  return g.kmax * (fx * fx + fz * fz);
}

// 2a and b of the damped leapfrog at padded cell (i, j).  The hardware
// reciprocal is exact at kappa = 0 (the whole interior); every kernel uses
// this one function, so forward and adjoint see identical coefficients.
__device__ __forceinline__ void sponge_ab(const Geo &g, int i, int j, float &a2, float &b) {
  const float kap = sponge_kappa(g, i, j);
  const float inv = __builtin_amdgcn_rcpf(1.0f + kap);
  a2 = 2.0f * inv;
  b = (1.0f - kap) * inv;
}

// One damped leapfrog update, a2 u - b u_prev + c w, in a fixed evaluation
// order.  The library is built without implicit FMA contraction, so every
// kernel that advances a wavefield (forward, forward+Born, segment recompute,
// adjoint) rounds identically and recomputed wavefields match the stored
// ones bit for bit.
__device__ __forceinline__ float leapfrog(float a2, float b, float u, float um, float c, float w) {
  return __builtin_fmaf(c, w, __builtin_fmaf(a2, u, -(b * um)));
}

// A tile (i0, j0) of one field with a HALO-wide border, as fetched by one
// thread before it is committed to LDS.  Values outside the padded grid are
// the zero boundary of the scheme.  Every load is issued unconditionally from
// a clamped (in-grid) address and masked afterwards, so all of a thread's
// loads are in flight together; fetch and commit are split so that other
// loads can join the same round trip.
struct TileRegs {
  float v[LH / NWAVE];
  float h;
};

__device__ __forceinline__ void fetch_tile(TileRegs &T, const float *__restrict__ f, int i0,
                                           int j0, const Geo &g, int tid) {
  const int lane = tid % TX, wv = tid / TX;
  const int j = j0 + lane;
  const int jc = min(j, g.nxp - 1);
  const bool jok = j < g.nxp;
#pragma unroll
  for (int q = 0; q < LH / NWAVE; ++q) {
    const int i = i0 - HALO + wv + q * NWAVE;
    const int ic = min(max(i, 0), g.nzp - 1);
    // multiply by a 0/1 mask instead of selecting: the load stays
    // unconditional (a select lets the compiler sink it into a branch)
    T.v[q] = f[ic * g.pitch + jc] * ((jok && i >= 0 && i < g.nzp) ? 1.0f : 0.0f);
  }
  const int r = tid / (2 * HALO), c = tid % (2 * HALO);
  const int col = c < HALO ? c - HALO : TX + c - HALO;
  const int i = i0 + r, jj = j0 + col;
  T.h = f[min(i, g.nzp - 1) * g.pitch + min(max(jj, 0), g.nxp - 1)] *
        ((i < g.nzp && jj >= 0 && jj < g.nxp) ? 1.0f : 0.0f);
}

__device__ __forceinline__ void commit_tile(float *__restrict__ L, const TileRegs &T, int tid) {
  const int lane = tid % TX, wv = tid / TX;
#pragma unroll
  for (int q = 0; q < LH / NWAVE; ++q) L[(wv + q * NWAVE) * LW + HALO + lane] = T.v[q];
  const int r = tid / (2 * HALO), c = tid % (2 * HALO);
  const int col = c < HALO ? c - HALO : TX + c - HALO;
  L[(r + HALO) * LW + HALO + col] = T.h;
}

// L applied at the RZ rows this thread owns; ctr receives the centre values.
// The weights sum to zero (C0 + 2(C1+..+C4) = 0), so L u is evaluated as
// sum_k C_k [(u_{+k} - u) + (u_{-k} - u)] over both axes: neighbour
// differences are nearly exact in FP32, which avoids the cancellation of the
// large centre term against the neighbour sum.
__device__ __forceinline__ void laplacian_rows(const float *__restrict__ L, const Geo &g,
                                               int lane, int wv, float (&lap)[RZ],
                                               float (&ctr)[RZ]) {
  float col[RZ + 2 * HALO];
#pragma unroll
  for (int q = 0; q < RZ + 2 * HALO; ++q) col[q] = L[(wv * RZ + q) * LW + HALO + lane];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const float *row = L + (wv * RZ + r + HALO) * LW + HALO + lane;
    const float u = col[r + 4];
    float acc = 0.0f;
#pragma unroll
    for (int k = HALO; k >= 1; --k) {
      const float sk = ((col[r + 4 - k] - u) + (col[r + 4 + k] - u)) +
                       ((row[-k] - u) + (row[k] - u));
      const float ck = k == 1 ? g.c1 : k == 2 ? g.c2 : k == 3 ? g.c3 : g.c4;
      acc = __builtin_fmaf(ck, sk, acc);
    }
    lap[r] = acc;
    ctr[r] = u;
  }
}

// Receiver gather of the values this workgroup just produced: route them
// through LDS so any thread can read any receiver node of the tile.
__device__ __forceinline__ void gather_receivers(float *__restrict__ L, const float (&val)[RZ],
                                                 const DevTables &t, int rp0, int rp1, int tid,
                                                 float *__restrict__ dst) {
  const int lane = tid % TX, wv = tid / TX;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RZ; ++r) L[(wv * RZ + r) * TX + lane] = val[r];
  __syncthreads();
  for (int e = rp0 + tid; e < rp1; e += NTHREADS) dst[t.rec_id[e]] = L[t.rec_local[e]];
}

// One forward time step (optionally with the B Born fields): reads u^n,
// u^{n-1}, writes u^{n+1} in place of u^{n-1}.
template <bool BORN>
__global__ __launch_bounds__(NTHREADS) void k_step(Geo g, DevTables t, StepArgs a) {
  __shared__ float L[LH * LW];
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  // order 0: shot-major (neighbouring tiles of one shot are adjacent ids);
  // order 1: tile-major (the shots of one tile are adjacent ids, so operands
  // shared by all shots, such as the Born coefficients, are reused from L2)
  const int s = a.order ? lid % g.ns : lid / g.ntiles;
  const int tile = a.order ? lid / g.ns : lid - s * g.ntiles;
  const int tzi = tile / g.tiles_x, txi = tile - tzi * g.tiles_x;
  const int i0 = tzi * TZ, j0 = txi * TX;
  const int tid = threadIdx.x, lane = tid % TX, wv = tid / TX;
  const int j = j0 + lane, ib = i0 + wv * RZ;
  const long long fs = g.fs;

  float *ubase = a.u + (long long)s * 2 * fs;
  const float *un = ubase + (a.n & 1) * fs;
  float *uo = ubase + ((a.n + 1) & 1) * fs;

  // element (ib + r, j) of every per-point array sits at idx[r]; rows and
  // columns outside the grid read a clamped element and store nothing
  const int jc = min(j, g.nxp - 1);
  const bool jok = j < g.nxp;
  int idx[RZ];
  float cc[RZ], unew[RZ], um[RZ];
  TileRegs T;
  fetch_tile(T, un, i0, j0, g, tid);
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    idx[r] = min(ib + r, g.nzp - 1) * g.pitch + jc;
    cc[r] = a.c[idx[r]];
    um[r] = uo[idx[r]];
  }
  commit_tile(L, T, tid);
  __syncthreads();
  float w[RZ], ctr[RZ];
  laplacian_rows(L, g, lane, wv, w, ctr);
  {
    const int si = t.src_ij[2 * s], sj = t.src_ij[2 * s + 1];
    if (sj == j) {
#pragma unroll
      for (int r = 0; r < RZ; ++r)
        if (ib + r == si) w[r] += a.src_amp;
    }
  }

  // rows outside the grid compute on clamped copies and store nothing
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    const int i = ib + r;
    const bool ok = jok && i < g.nzp;
    float a2, bb;
    sponge_ab(g, i, j, a2, bb);
    unew[r] = leapfrog(a2, bb, ctr[r], um[r], cc[r], w[r]);
    if (ok) {
      uo[idx[r]] = unew[r];
      if (a.w_out) a.w_out[s * fs + idx[r]] = w[r];
      if (a.ck) {
        a.ck[(2 * s + ((a.n + 1) & 1)) * fs + idx[r]] = unew[r];
        a.ck[(2 * s + (a.n & 1)) * fs + idx[r]] = ctr[r];
      }
    }
  }

  const int rp0 = t.tile_rec_ptr[tile], rp1 = t.tile_rec_ptr[tile + 1];
  if (a.d_out && rp1 > rp0)
    gather_receivers(L, unew, t, rp0, rp1, tid,
                     a.d_out + ((long long)s * g.nt + a.n + 1) * g.nr);

  if constexpr (BORN) {
    for (int b = 0; b < a.B; ++b) {
      float *dbase = a.du + ((long long)s * a.B + b) * 2 * fs;
      const float *dn = dbase + (a.n & 1) * fs;
      float *dout = dbase + ((a.n + 1) & 1) * fs;
      const float *dcb = a.dc + (long long)b * fs;
      float lap[RZ], dctr[RZ], dnew[RZ], dm[RZ], dcv[RZ];
      TileRegs D;
      fetch_tile(D, dn, i0, j0, g, tid);
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        dm[r] = dout[idx[r]];
        dcv[r] = dcb[idx[r]];
      }
      __syncthreads();
      commit_tile(L, D, tid);
      __syncthreads();
      laplacian_rows(L, g, lane, wv, lap, dctr);
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int i = ib + r;
        const bool ok = jok && i < g.nzp;
        float a2, bb;
        sponge_ab(g, i, j, a2, bb);
        dnew[r] = __builtin_fmaf(dcv[r], w[r], leapfrog(a2, bb, dctr[r], dm[r], cc[r], lap[r]));
        if (ok) dout[idx[r]] = dnew[r];
      }
      if (a.dd_out && rp1 > rp0)
        gather_receivers(L, dnew, t, rp0, rp1, tid,
                         a.dd_out + (((long long)b * g.ns + s) * g.nt + a.n + 1) * g.nr);
    }
  }
}

// One adjoint step for vector b over a group of shots: mu^k from mu^{k+1},
// mu^{k+2} (in place of mu^{k+2}), receiver injection c * R^T r^k, and the
// image term w^k * mu^{k+1} summed over the group's shots in registers, then
// added (times 2/m_pad) to the group's FP64 partial image.
__global__ __launch_bounds__(NTHREADS) void k_adjoint(Geo g, DevTables t, AdjArgs a) {
  __shared__ float L[LH * LW];
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  // order 0: field-major, tile fastest; order 1: tile-major with the vector
  // index fastest, so the forward wavefield w of a shot group (shared by all
  // vectors) is reused from L2 by consecutive workgroups
  int tile, b, grp;
  if (a.order) {
    b = lid % a.B;
    grp = (lid / a.B) % a.ngroups;
    tile = lid / (a.B * a.ngroups);
  } else {
    tile = lid % g.ntiles;
    const int rest = lid / g.ntiles;
    b = rest % a.B;
    grp = rest / a.B;
  }
  const int tzi = tile / g.tiles_x, txi = tile - tzi * g.tiles_x;
  const int i0 = tzi * TZ, j0 = txi * TX;
  const int tid = threadIdx.x, lane = tid % TX, wv = tid / TX;
  const int j = j0 + lane, ib = i0 + wv * RZ;
  const long long fs = g.fs;

  const int jc = min(j, g.nxp - 1);
  const bool jok = j < g.nxp;
  float cc[RZ], img[RZ];
  int idx[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    idx[r] = min(ib + r, g.nzp - 1) * g.pitch + jc;
    cc[r] = a.c[idx[r]];
    img[r] = 0.0f;
  }
  const int np0 = t.tile_node_ptr[tile], np1 = t.tile_node_ptr[tile + 1];
  const bool inject = (a.r != nullptr) && (np1 > np0);
  const int s0 = grp * a.group, s1 = min(g.ns, s0 + a.group);

  for (int s = s0; s < s1; ++s) {
    float *mb = a.mu + ((long long)b * g.ns + s) * 2 * fs;
    const float *m1 = mb + ((a.k + 1) & 1) * fs;
    float *m0 = mb + (a.k & 1) * fs;
    float lap[RZ], ctr[RZ], out[RZ], m2[RZ], wv_[RZ];
    const float *ws_ = a.w ? a.w + s * fs : nullptr;
    TileRegs T;
    fetch_tile(T, m1, i0, j0, g, tid);
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      m2[r] = m0[idx[r]];
      wv_[r] = ws_ ? ws_[idx[r]] : 0.0f;
    }
    if (s > s0) __syncthreads();
    commit_tile(L, T, tid);
    __syncthreads();
    laplacian_rows(L, g, lane, wv, lap, ctr);
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      float a2, bb;
      sponge_ab(g, ib + r, j, a2, bb);
      out[r] = leapfrog(a2, bb, ctr[r], m2[r], cc[r], lap[r]);
      img[r] = __builtin_fmaf(wv_[r], ctr[r], img[r]);
    }
    if (inject) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RZ; ++r) L[(wv * RZ + r) * TX + lane] = out[r];
      __syncthreads();
      const float *rs = a.r + (((long long)b * g.ns + s) * g.nt + a.k) * g.nr;
      for (int e = np0 + tid; e < np1; e += NTHREADS) {
        float acc = 0.0f;
        for (int q = t.node_rec_ptr[e]; q < t.node_rec_ptr[e + 1]; ++q) acc += rs[t.node_recs[q]];
        L[t.node_local[e]] += a.c[t.node_gidx[e]] * acc;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RZ; ++r) out[r] = L[(wv * RZ + r) * TX + lane];
    }
#pragma unroll
    for (int r = 0; r < RZ; ++r)
      if (jok && ib + r < g.nzp) m0[idx[r]] = out[r];
  }
  if (a.w) {
    double *ig = a.img + ((long long)grp * a.B + b) * fs;
    double old[RZ];
    float sm[RZ];
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      old[r] = ig[idx[r]];
      sm[r] = a.s2m[idx[r]];
    }
#pragma unroll
    for (int r = 0; r < RZ; ++r)
      if (jok && ib + r < g.nzp) ig[idx[r]] = old[r] + (double)sm[r] * (double)img[r];
  }
}

// Coefficients on the padded grid from the model (and Born perturbations).
__global__ void k_setup(Geo g, const float *__restrict__ m, const float *__restrict__ v, int B,
                        float *__restrict__ c, float *__restrict__ s2m, float *__restrict__ dc,
                        unsigned int *status) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.fs) return;
  const int i = (int)(p / g.pitch), j = (int)(p % g.pitch);
  const bool in = i < g.nzp && j < g.nxp;
  float cv = 0.0f, s2 = 0.0f, mv = 1.0f;
  long long mi = 0;
  if (in) {
    const int iz = min(max(i - g.nb, 0), g.nz - 1), ix = min(max(j - g.nb, 0), g.nx - 1);
    mi = (long long)iz * g.nx + ix;
    mv = m[mi];
    const bool bad = !(mv > 0.0f) || !isfinite(mv);
    if (bad) atomicOr(status, 1u);
    if (!bad && mv * g.dt * g.inv_dx > CFL_LIMIT) atomicOr(status, 2u);
    const float kap = sponge_kappa(g, i, j);
    const float vdt = g.dt * mv;
    cv = vdt * vdt / (1.0f + kap);
    s2 = 2.0f / mv;
  }
  c[p] = cv;
  if (s2m) s2m[p] = s2;
  if (dc) {
    const long long nm = (long long)g.nz * g.nx;
    for (int b = 0; b < B; ++b) dc[b * g.fs + p] = in ? s2 * cv * v[b * nm + mi] : 0.0f;
  }
}

__global__ void k_fill(float *__restrict__ p, long long n, float val) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = val;
}

__global__ void k_copy(float *__restrict__ dst, const float *__restrict__ src, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
    dst[q] = src[q];
}

__global__ void k_fill64(double *__restrict__ p, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = 0.0;
}

// Zero the n = 0 sample of `count` traces of length nt x nr.
__global__ void k_zero_t0(float *__restrict__ d, int count, int nt, int nr) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < (long long)count * nr;
       q += stride) {
    const long long tr = q / nr, rr = q % nr;
    d[tr * nt * nr + rr] = 0.0f;
  }
}

// r = d - dobs in place, per-block FP64 sums of r^2.
__global__ __launch_bounds__(256) void k_residual(float *__restrict__ d,
                                                  const float *__restrict__ dobs, long long n,
                                                  double *__restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const float x = d[q] - dobs[q];
    d[q] = x;
    acc += (double)x * (double)x;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// phi = scale * sum(part), summed in a fixed order by one workgroup.
__global__ __launch_bounds__(256) void k_phi(const double *__restrict__ part, int n, double scale,
                                             double *__restrict__ phi) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) acc += part[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *phi = scale * red[0];
}

// P^T and the sum over shot groups: out[b][iz][ix] = scale * sum of the
// partial images over every padded cell that copies model cell (iz, ix).
__global__ void k_fold(Geo g, const double *__restrict__ img, int G, int B, double scale,
                       float *__restrict__ out) {
  const long long nm = (long long)g.nz * g.nx;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nm * B; q += stride) {
  const int b = (int)(q / nm);
  const int rem = (int)(q % nm);
  const int iz = rem / g.nx, ix = rem % g.nx;
  const int ia = iz == 0 ? 0 : iz + g.nb, ie = iz == g.nz - 1 ? g.nzp - 1 : iz + g.nb;
  const int ja = ix == 0 ? 0 : ix + g.nb, je = ix == g.nx - 1 ? g.nxp - 1 : ix + g.nb;
  double acc = 0.0;
  for (int gg = 0; gg < G; ++gg) {
    const double *ig = img + ((long long)gg * B + b) * g.fs;
    for (int i = ia; i <= ie; ++i)
      for (int j = ja; j <= je; ++j) acc += ig[(long long)i * g.pitch + j];
  }
  out[q] = (float)(acc * scale);
  }
}

__global__ void k_check_finite(const float *__restrict__ p, long long n, unsigned int *status) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
    bad |= !isfinite(p[q]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, 4u);
}

// ------------------------------------------------------------ host launchers

static inline unsigned int blocks_for(long long n, int per) {
  long long b = (n + per - 1) / per;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned int)b;
}

hipError_t launch_step(const Geo &g, const DevTables &t, const StepArgs &a, bool born,
                       hipStream_t st) {
  const unsigned int grid = (unsigned int)(g.ntiles * g.ns);
  if (born)
    hipLaunchKernelGGL(k_step<true>, dim3(grid), dim3(NTHREADS), 0, st, g, t, a);
  else
    hipLaunchKernelGGL(k_step<false>, dim3(grid), dim3(NTHREADS), 0, st, g, t, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const Geo &g, const DevTables &t, const AdjArgs &a, hipStream_t st) {
  const unsigned int grid = (unsigned int)(g.ntiles * a.B * a.ngroups);
  hipLaunchKernelGGL(k_adjoint, dim3(grid), dim3(NTHREADS), 0, st, g, t, a);
  return hipGetLastError();
}

hipError_t launch_setup(const Geo &g, const float *m, const float *v, int B, float *c,
                        float *s2m, float *dc, unsigned int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3((unsigned int)((g.fs + 255) / 256)), dim3(256), 0, st, g, m,
                     v, B, c, s2m, dc, status);
  return hipGetLastError();
}

hipError_t launch_fill(float *p, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 1024)), dim3(256), 0, st, p, n, 0.0f);
  return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 1024)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fill64(double *p, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill64, dim3(blocks_for(n, 1024)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_t0(float *d, int count, int nt, int nr, hipStream_t st) {
  const long long n = (long long)count * nr;
  hipLaunchKernelGGL(k_zero_t0, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, count, nt, nr);
  return hipGetLastError();
}

hipError_t launch_residual(float *d, const float *dobs, long long n, double *part, int nparts,
                           double scale, double *phi, hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(nparts), dim3(256), 0, st, d, dobs, n, part);
  hipLaunchKernelGGL(k_phi, dim3(1), dim3(256), 0, st, part, nparts, scale, phi);
  return hipGetLastError();
}

hipError_t launch_fold(const Geo &g, const double *img, int G, int B, double scale, float *out,
                       hipStream_t st) {
  const long long n = (long long)g.nz * g.nx * B;
  hipLaunchKernelGGL(k_fold, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, img, G, B, scale,
                     out);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float *p, long long n, unsigned int *status,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 4096)), dim3(256), 0, st, p, n, status);
  return hipGetLastError();
}

}  // namespace fwi

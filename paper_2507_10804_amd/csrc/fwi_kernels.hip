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
// on the same XCD and their halo re-reads hit its L2 (one-step kernels; the
// two-step forward + Born kernel; the two-step adjoint runs in plain launch
// order).
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  constexpr int NXCD = 8;
  const int q = n / NXCD, rem = n % NXCD;
  const int x = bid % NXCD, slot = bid / NXCD;
  return (x < rem) ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
}

// Loads and stores at an element offset from a workgroup-uniform base, as
// raw buffer accesses: the base lives in a scalar buffer descriptor and each
// access needs one 32-bit byte offset in a vector register (plain pointers
// cost a 64-bit address per access).  The plan bounds every per-field byte
// offset below 2^31.  Descriptor word 3 is the gfx9-family raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float ldf(const float *base, unsigned e) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(rsrc(base), (int)(e << 2), 0, 0));
}
__device__ __forceinline__ void stf(float *base, unsigned e, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc(base), (int)(e << 2),
                                        0, 0);
}
// Wavefield store, non-temporal: the levels (and recorded fields and
// checkpoints) written here are read by a later launch, not by this one, so
// allocating them in L2 only evicts the halo lines that neighbouring tiles
// re-read.  The one-step forward recompute runs 28 % faster with it; the
// two-step kernels are unchanged.
__device__ __forceinline__ void stf_nt(float *base, unsigned e, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc(base), (int)(e << 2),
                                        0, 2 /* nt */);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double ldd(const double *base, unsigned e) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(rsrc(base), (int)(e << 3), 0, 0));
}
__device__ __forceinline__ void std_(double *base, unsigned e, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rsrc(base), (int)(e << 3),
                                        0, 0);
}

// Debug mode (plan option FWI_OPT_LDS_POISON): fill a workgroup's LDS
// arrays with NaN before anything is staged, so that a read of an entry no
// thread wrote -- a missing halo value or a missing barrier -- turns the
// outputs into NaN instead of silently reading a stale value.
__device__ __forceinline__ void poison_lds(float *L, int n, int nthreads) {
  for (int e = (int)threadIdx.x; e < n; e += nthreads) L[e] = __builtin_nanf("");
}

__device__ __forceinline__ float sponge_kappa(const Geo &g, int i, int j) {
  const int dxc = max(max(g.nb - j, 0), j - (g.nxp - 1 - g.nb));
  const int dzc = max(max(g.nb - i, 0), i - (g.nzp - 1 - g.nb));
  const float fx = dxc * g.inv_nb, fz = dzc * g.inv_nb;
  return g.kmax * (fx * fx + fz * fz);
}

// b = (1 - kappa) / (1 + kappa) of the damped leapfrog at padded cell (i, j).
// The hardware reciprocal is exact at kappa = 0 (the whole interior); every
// kernel uses this one function, so forward and adjoint see identical
// coefficients.
__device__ __forceinline__ float sponge_b(const Geo &g, int i, int j) {
  const float kap = sponge_kappa(g, i, j);
  return (1.0f - kap) * __builtin_amdgcn_rcpf(1.0f + kap);
}

// True when every cell of the tile whose top-left cell is (i0, j0) lies in
// the undamped interior, where a = b = 1 exactly (workgroup-uniform).
__device__ __forceinline__ bool tile_interior(const Geo &g, int i0, int j0, int tz, int tx) {
  return i0 >= g.nb && i0 + tz <= g.nzp - g.nb && j0 >= g.nb && j0 + tx <= g.nxp - g.nb;
}

// b, skipping the sponge arithmetic on interior tiles (same values).
__device__ __forceinline__ float coef_b(const Geo &g, bool interior, int i, int j) {
  return interior ? 1.0f : sponge_b(g, i, j);
}

// One damped leapfrog update, 2a u - b u_prev + c w with a = 1/(1+kappa),
// b = (1-kappa)/(1+kappa), evaluated as u + [b (u - u_prev) + c w]: the same
// number in exact arithmetic (2a - 1 - b = 0), but the bracket -- the time
// increment -- is formed at its own magnitude (u - u_prev is exact when
// consecutive levels are within a factor two), so the level is rounded once
// per step instead of twice; in an FP32 emulation of a 3000-step solve the
// receiver data error against FP64 drops from 1.1e-5 to 1.4e-6.  The order is
// fixed and the library is built without implicit FMA contraction, so every
// kernel that advances a wavefield (forward, forward+Born, segment
// recompute, adjoint) rounds identically and recomputed wavefields match the
// stored ones bit for bit.
__device__ __forceinline__ float leapfrog(float b, float u, float um, float c, float w) {
  return u + __builtin_fmaf(c, w, b * (u - um));
}
// The same with a Born source term dc * ws inside the increment.
__device__ __forceinline__ float leapfrog_src(float b, float u, float um, float c, float w,
                                              float dc, float ws) {
  return u + __builtin_fmaf(dc, ws, __builtin_fmaf(c, w, b * (u - um)));
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
    T.v[q] = ldf(f, (unsigned)(ic * g.pitch + jc)) * ((jok && i >= 0 && i < g.nzp) ? 1.0f : 0.0f);
  }
  const int r = tid / (2 * HALO), c = tid % (2 * HALO);
  const int col = c < HALO ? c - HALO : TX + c - HALO;
  const int i = i0 + r, jj = j0 + col;
  T.h = ldf(f, (unsigned)(min(i, g.nzp - 1) * g.pitch + min(max(jj, 0), g.nxp - 1))) *
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

typedef __attribute__((address_space(3))) const float lds_cf;

// Keeps an LDS address in a register of its own, so that the reads at small
// constant offsets from it take the read instruction's immediate offset
// instead of one address addition per read pair.
__device__ __forceinline__ lds_cf *lds_pin(lds_cf *p) {
  asm volatile("" : "+v"(p));
  return p;
}

// 8th-order Laplacian (over dx^2) at R consecutive points of one column, from
// a window staged in LDS with row pitch P: element o of L is the window's
// first row, HALO columns left of the points' column; the points sit on
// window rows HALO .. HALO+R-1.  L = sum_k C_k [(u_{i-k} - u) + (u_{i+k} - u)
// + (u_{j-k} - u) + (u_{j+k} - u)]; the z differences of neighbouring points
// are shared (u_{i-k} - u_i is minus the difference u_i - u_{i-k} of row
// i - k, exactly), which leaves every sum bitwise unchanged.
template <int R, int P>
__device__ __forceinline__ void lap_window(const float *__restrict__ L, int o, const Geo &g,
                                           float (&lap)[R], float (&ctr)[R]) {
  constexpr int W = R + 2 * HALO;  // window rows
  constexpr int NB = (W + 3) / 4;  // one pinned address per 4 rows (offsets <= 255 dwords)
  static_assert(3 * P + 2 * HALO <= 255, "read offsets must fit the ds_read2 offset field");
  lds_cf *base[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) base[b] = lds_pin((lds_cf *)L + o + 4 * b * P);
  float col[W];
#pragma unroll
  for (int q = 0; q < W; ++q) col[q] = base[q / 4][(q % 4) * P + HALO];
  // dz[k][q] = col[q + k] - col[q], made at row q and used again at row q + k
  float dz[HALO + 1][R + HALO];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = r + HALO;
    lds_cf *row = base[q / 4] + (q % 4) * P + HALO;
    const float u = col[q];
    float acc = 0.0f;
#pragma unroll
    for (int k = HALO; k >= 1; --k) {
      dz[k][q] = col[q + k] - u;
      if (r < k) dz[k][q - k] = u - col[q - k];
      const float sk = (dz[k][q] - dz[k][q - k]) + ((row[-k] - u) + (row[k] - u));
      const float ck = k == 1 ? g.c1 : k == 2 ? g.c2 : k == 3 ? g.c3 : g.c4;
      acc = __builtin_fmaf(ck, sk, acc);
    }
    lap[r] = acc;
    ctr[r] = u;
  }
}

// L applied at the RZ rows this thread owns; ctr receives the centre values.
// The weights sum to zero (C0 + 2(C1+..+C4) = 0), so L u is evaluated as
// sum_k C_k [(u_{+k} - u) + (u_{-k} - u)] over both axes: neighbour
// differences are nearly exact in FP32, which avoids the cancellation of the
// large centre term against the neighbour sum.
__device__ __forceinline__ void laplacian_rows(const float *__restrict__ L, const Geo &g,
                                               int lane, int wv, float (&lap)[RZ],
                                               float (&ctr)[RZ]) {
  lap_window<RZ, LW>(L, wv * RZ * LW + lane, g, lap, ctr);
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
  if (g.poison) {
    poison_lds(L, LH * LW, NTHREADS);
    __syncthreads();
  }
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  // order 0: shot-major (neighbouring tiles of one shot are adjacent ids);
  // order 1: tile-major (the shots of one tile are adjacent ids, so operands
  // shared by all shots, such as the Born coefficients, are reused from L2);
  // order 2: blocked -- a block of neighbouring tiles for every shot, block
  // after block, which keeps both the shared tiles and the halos in L2
  int s, tile;
  if (a.order == 2) {
    const int per = g.blk * g.ns;
    const int blk = lid / per, rem = lid - blk * per;
    s = rem / g.blk;
    const int p = blk * g.blk + (rem - s * g.blk);
    if (p >= g.ntiles) return;  // padding of the last block (whole workgroup)
    tile = t.tile_order[p];
  } else {
    s = a.order ? lid % g.ns : lid / g.ntiles;
    tile = a.order ? lid / g.ns : lid - s * g.ntiles;
  }
  const int tzi = tile / g.tiles_x, txi = tile - tzi * g.tiles_x;
  const int i0 = tzi * TZ, j0 = txi * TX;
  const int tid = threadIdx.x, lane = tid % TX, wv = tid / TX;
  const int j = j0 + lane, ib = i0 + wv * RZ;
  const long long fs = g.fs;
  const bool inner = tile_interior(g, i0, j0, TZ, TX);

  float *ubase = a.u + (long long)s * 2 * fs;
  const float *un = ubase + (a.n & 1) * fs;
  float *uo = ubase + ((a.n + 1) & 1) * fs;

  // element (ib + r, j) of every per-point array sits at idx[r]; rows and
  // columns outside the grid read a clamped element and store nothing
  const int jc = min(j, g.nxp - 1);
  const bool jok = j < g.nxp;
  unsigned idx[RZ];
  float cc[RZ], unew[RZ], um[RZ];
  TileRegs T;
  fetch_tile(T, un, i0, j0, g, tid);
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    idx[r] = (unsigned)(min(ib + r, g.nzp - 1) * g.pitch + jc);
    cc[r] = ldf(a.c, idx[r]);
    um[r] = ldf(uo, idx[r]);
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
    const float bb = coef_b(g, inner, i, j);
    unew[r] = leapfrog(bb, ctr[r], um[r], cc[r], w[r]);
    if (ok) {
      stf_nt(uo, idx[r], unew[r]);
      if (a.w_out) stf_nt(a.w_out + s * fs, idx[r], w[r]);
      if (a.ck) {
        stf_nt(a.ck + (2 * s + ((a.n + 1) & 1)) * fs, idx[r], unew[r]);
        stf_nt(a.ck + (2 * s + (a.n & 1)) * fs, idx[r], ctr[r]);
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
        dm[r] = ldf(dout, idx[r]);
        dcv[r] = ldf(dcb, idx[r]);
      }
      __syncthreads();
      commit_tile(L, D, tid);
      __syncthreads();
      laplacian_rows(L, g, lane, wv, lap, dctr);
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const int i = ib + r;
        const bool ok = jok && i < g.nzp;
        const float bb = coef_b(g, inner, i, j);
        dnew[r] = leapfrog_src(bb, dctr[r], dm[r], cc[r], lap[r], dcv[r], w[r]);
        if (ok) stf_nt(dout, idx[r], dnew[r]);
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
  if (g.poison) {
    poison_lds(L, LH * LW, NTHREADS);
    __syncthreads();
  }
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  // order 0: field-major, tile fastest; order 1: tile-major with the vector
  // index fastest, so the forward wavefield w of a shot group (shared by all
  // vectors) is reused from L2 by consecutive workgroups
  int tile, b, grp;
  if (a.order == 2) {
    const int nb = a.B * a.ngroups;
    const int per = g.blk * nb;
    const int blk = lid / per, rem = lid - blk * per;
    const int item = rem / g.blk;  // vector fastest within the batch items
    b = item % a.B;
    grp = item / a.B;
    const int p = blk * g.blk + (rem - item * g.blk);
    if (p >= g.ntiles) return;  // padding of the last block (whole workgroup)
    tile = t.tile_order[p];
  } else if (a.order) {
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
  const bool inner = tile_interior(g, i0, j0, TZ, TX);

  const int jc = min(j, g.nxp - 1);
  const bool jok = j < g.nxp;
  float cc[RZ], img[RZ];
  unsigned idx[RZ];
#pragma unroll
  for (int r = 0; r < RZ; ++r) {
    idx[r] = (unsigned)(min(ib + r, g.nzp - 1) * g.pitch + jc);
    cc[r] = ldf(a.c, idx[r]);
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
      m2[r] = ldf(m0, idx[r]);
      wv_[r] = ws_ ? ldf(ws_, idx[r]) : 0.0f;
    }
    if (s > s0) __syncthreads();
    commit_tile(L, T, tid);
    __syncthreads();
    laplacian_rows(L, g, lane, wv, lap, ctr);
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      const float bb = coef_b(g, inner, ib + r, j);
      out[r] = leapfrog(bb, ctr[r], m2[r], cc[r], lap[r]);
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
      if (jok && ib + r < g.nzp) stf(m0, idx[r], out[r]);
  }
  if (a.w) {
    double *ig = a.img + ((long long)grp * a.B + b) * fs;
    double old[RZ];
    float sm[RZ];
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
      old[r] = ldd(ig, idx[r]);
      sm[r] = ldf(a.s2m, idx[r]);
    }
#pragma unroll
    for (int r = 0; r < RZ; ++r)
      if (jok && ib + r < g.nzp) std_(ig, idx[r], old[r] + (double)sm[r] * (double)img[r]);
  }
}

// ----------------------------------------------------------------------
// Two time steps per launch (temporal blocking).  Per tile of TX2 x TZ2
// outputs: the input level is staged in LDS with a 2*HALO ring (IX x IZ), the
// intermediate level is computed on the tile plus a HALO ring (EX x EZ: lane
// = column, RA rows per wavefront) into LDS, and the second step produces the
// outputs (lanes HALO..HALO+TX2-1, RB rows per wavefront).  Each field is
// read twice and written twice per two steps, against three accesses per
// step for single steps.  Points outside the padded grid are zero, as in the
// one-step kernels, and every load is unconditional from a clamped address.

struct Tile2Regs {
  float v[IZ / NWAVE2];  // core 64 columns, 6 rows per wavefront
  float x;               // the 8 extra columns x 48 rows, one value per thread
};

static_assert(IZ % NWAVE2 == 0 && EZ % NWAVE2 == 0 && TZ2 % NWAVE2 == 0, "rows per wavefront");
static_assert(IZ * (IX - TX) <= NTHREADS2, "extra columns: at most one value per thread");

__device__ __forceinline__ float masked_load(const float *__restrict__ f, int i, int j,
                                             const Geo &g) {
  const int ic = min(max(i, 0), g.nzp - 1), jc = min(max(j, 0), g.nxp - 1);
  return ldf(f, (unsigned)(ic * g.pitch + jc)) *
         ((i >= 0 && i < g.nzp && j >= 0 && j < g.nxp) ? 1.0f : 0.0f);
}

// Input level on rows i0-2H..i0+TZ2+2H-1, columns j0-2H..j0+TX2+2H-1.
__device__ __forceinline__ void fetch_tile2(Tile2Regs &T, const float *__restrict__ f, int i0,
                                            int j0, const Geo &g, int tid) {
  const int lane = tid % TX, wv = tid / TX;
#pragma unroll
  for (int q = 0; q < IZ / NWAVE2; ++q)
    T.v[q] = masked_load(f, i0 - 2 * HALO + wv + q * NWAVE2, j0 - 2 * HALO + lane, g);
  const int c = tid % (IX - TX), r = min(tid / (IX - TX), IZ - 1);
  T.x = masked_load(f, i0 - 2 * HALO + r, j0 - 2 * HALO + TX + c, g);
}

__device__ __forceinline__ void commit_tile2(float *__restrict__ LI, const Tile2Regs &T,
                                             int tid) {
  const int lane = tid % TX, wv = tid / TX;
#pragma unroll
  for (int q = 0; q < IZ / NWAVE2; ++q) LI[(wv + q * NWAVE2) * IX + lane] = T.v[q];
  const int c = tid % (IX - TX), r = tid / (IX - TX);
  if (r < IZ) LI[r * IX + TX + c] = T.x;
}

// L at the RA intermediate points of this thread (E row wv*RA + r, column
// lane), from the staged input level; ctr = centre values.
__device__ __forceinline__ void lap_stepA(const float *__restrict__ LI, const Geo &g, int lane,
                                          int wv, float (&lap)[RA], float (&ctr)[RA]) {
  float col[RA + 2 * HALO];
#pragma unroll
  for (int q = 0; q < RA + 2 * HALO; ++q) col[q] = LI[(wv * RA + q) * IX + HALO + lane];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const float *row = LI + (wv * RA + r + HALO) * IX + HALO + lane;
    const float u = col[r + HALO];
    float acc = 0.0f;
#pragma unroll
    for (int k = HALO; k >= 1; --k) {
      const float sk = ((col[r + HALO - k] - u) + (col[r + HALO + k] - u)) +
                       ((row[-k] - u) + (row[k] - u));
      const float ck = k == 1 ? g.c1 : k == 2 ? g.c2 : k == 3 ? g.c3 : g.c4;
      acc = __builtin_fmaf(ck, sk, acc);
    }
    lap[r] = acc;
    ctr[r] = u;
  }
}

// L at the RB output points of this thread (E row wv*RB + r + HALO, column
// lb), from the intermediate level in LE.  lb is the lane clamped into the
// output columns so that every LDS address stays inside the row.
__device__ __forceinline__ void lap_stepB(const float *__restrict__ LE, const Geo &g, int lb,
                                          int wv, float (&lap)[RB], float (&ctr)[RB]) {
  float col[RB + 2 * HALO];
#pragma unroll
  for (int q = 0; q < RB + 2 * HALO; ++q) col[q] = LE[(wv * RB + q) * EX + lb];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const float *row = LE + (wv * RB + r + HALO) * EX + lb;
    const float u = col[r + HALO];
    float acc = 0.0f;
#pragma unroll
    for (int k = HALO; k >= 1; --k) {
      const float sk = ((col[r + HALO - k] - u) + (col[r + HALO + k] - u)) +
                       ((row[-k] - u) + (row[k] - u));
      const float ck = k == 1 ? g.c1 : k == 2 ? g.c2 : k == 3 ? g.c3 : g.c4;
      acc = __builtin_fmaf(ck, sk, acc);
    }
    lap[r] = acc;
    ctr[r] = u;
  }
}

// Values of the output points written into LE (at their E positions), then
// gathered at the tile's receivers.
__device__ __forceinline__ void gather2(float *__restrict__ LE, const float (&val)[RB],
                                        bool colT, int lane, int wv, const DevTables &t, int rp0,
                                        int rp1, int tid, float *__restrict__ dst) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RB; ++r)
    if (colT) LE[(wv * RB + r + HALO) * EX + lane] = val[r];
  __syncthreads();
  for (int e = rp0 + tid; e < rp1; e += NTHREADS2) dst[t.t2_rec_id[e]] = LE[t.t2_rec_local[e]];
}

template <bool BORN>
__global__ __launch_bounds__(NTHREADS2) void k_step2(Geo g, DevTables t, Step2Args a) {
  __shared__ float LI[IZ * IX];
  __shared__ float LE[EZ * EX];
  if (g.poison) {
    poison_lds(LI, IZ * IX, NTHREADS2);
    poison_lds(LE, EZ * EX, NTHREADS2);
    __syncthreads();
  }
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int s = lid / g.ntiles2, tile = lid - s * g.ntiles2;
  const int tzi = tile / g.tiles_x2, txi = tile - tzi * g.tiles_x2;
  const int i0 = tzi * TZ2, j0 = txi * TX2;
  const int tid = threadIdx.x, lane = tid % TX, wv = tid / TX;
  const long long fs = g.fs;
  const bool inner = tile_interior(g, i0 - HALO, j0 - HALO, EZ, EX);

  const int jE = j0 - HALO + lane;  // column of this lane (E and output)
  const bool colE = jE >= 0 && jE < g.nxp;
  const bool colT = lane >= HALO && lane < HALO + TX2 && colE;
  const int jc = min(max(jE, 0), g.nxp - 1);
  const int lb = min(max(lane, HALO), EX - 1 - HALO);
  const int iA = i0 - HALO + wv * RA;  // first intermediate row of this thread
  const int iB = i0 + wv * RB;         // first output row of this thread

  const float *un = a.uin + (2 * s + (a.n & 1)) * fs;
  const float *um = a.uin + (2 * s + ((a.n + 1) & 1)) * fs;
  float *o1 = a.uout + (2 * s + ((a.n + 1) & 1)) * fs;  // u^{n+1}
  float *o2 = a.uout + (2 * s + (a.n & 1)) * fs;        // u^{n+2}

  unsigned idxA[RA], idxB[RB];
  float cA[RA], cB[RB], umA[RA], unB[RB];
  Tile2Regs T;
  fetch_tile2(T, un, i0, j0, g, tid);
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    idxA[r] = (unsigned)(min(max(iA + r, 0), g.nzp - 1) * g.pitch + jc);
    cA[r] = ldf(a.c, idxA[r]);
    umA[r] = ldf(um, idxA[r]);
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    idxB[r] = (unsigned)(min(iB + r, g.nzp - 1) * g.pitch + jc);
    cB[r] = ldf(a.c, idxB[r]);
  }
  commit_tile2(LI, T, tid);
  __syncthreads();

  const int si = t.src_ij[2 * s], sj = t.src_ij[2 * s + 1];
  // step A: w^n and u^{n+1} on the extended region
  float wA[RA], ctrA[RA];
  lap_stepA(LI, g, lane, wv, wA, ctrA);
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const int i = iA + r;
    if (jE == sj && i == si) wA[r] += a.amp0;
    const float bb = coef_b(g, inner, i, jE);
    const float okE = (colE && i >= 0 && i < g.nzp) ? 1.0f : 0.0f;
    LE[(wv * RA + r) * EX + lane] = leapfrog(bb, ctrA[r], umA[r], cA[r], wA[r]) * okE;
    if (a.w_out0 && colT && i >= i0 && i < i0 + TZ2 && i < g.nzp)
      stf_nt(a.w_out0 + s * fs, idxA[r], wA[r]);
  }
  __syncthreads();
  const int rp0 = t.t2_rec_ptr[tile], rp1 = t.t2_rec_ptr[tile + 1];
  if (a.d_out)
    for (int e = rp0 + tid; e < rp1; e += NTHREADS2)
      a.d_out[((long long)s * g.nt + a.n + 1) * g.nr + t.t2_rec_id[e]] = LE[t.t2_rec_local[e]];

  // step B: w^{n+1} and u^{n+2} on the output tile
  float wB[RB], ctrB[RB], uB[RB];
  lap_stepB(LE, g, lb, wv, wB, ctrB);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int i = iB + r;
    if (jE == sj && i == si) wB[r] += a.amp1;
    const float bb = coef_b(g, inner, i, jE);
    const float unT = LI[(wv * RB + r + 2 * HALO) * IX + 2 * HALO + lb - HALO];
    uB[r] = leapfrog(bb, ctrB[r], unT, cB[r], wB[r]);
    unB[r] = unT;
    if (colT && i < g.nzp) {
      stf_nt(o1, idxB[r], ctrB[r]);
      stf_nt(o2, idxB[r], uB[r]);
      if (a.w_out1) stf_nt(a.w_out1 + s * fs, idxB[r], wB[r]);
      if (a.ck) {
        stf_nt(a.ck + (2 * s + ((a.n + 1) & 1)) * fs, idxB[r], ctrB[r]);
        stf_nt(a.ck + (2 * s + (a.n & 1)) * fs, idxB[r], uB[r]);
      }
    }
  }
  if (a.d_out && rp1 > rp0)
    gather2(LE, uB, colT, lane, wv, t, rp0, rp1, tid,
            a.d_out + ((long long)s * g.nt + a.n + 2) * g.nr);

  if constexpr (BORN) {
    for (int b = 0; b < a.B; ++b) {
      const long long fb = ((long long)s * a.B + b) * 2 * fs;
      const float *dn = a.duin + fb + (a.n & 1) * fs;
      const float *dm = a.duin + fb + ((a.n + 1) & 1) * fs;
      float *d1 = a.duout + fb + ((a.n + 1) & 1) * fs;
      float *d2 = a.duout + fb + (a.n & 1) * fs;
      const float *dcb = a.dc + (long long)b * fs;
      float dmA[RA], dcA[RA], dcB[RB];
      Tile2Regs D;
      fetch_tile2(D, dn, i0, j0, g, tid);
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        dmA[r] = ldf(dm, idxA[r]);
        dcA[r] = ldf(dcb, idxA[r]);
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) dcB[r] = ldf(dcb, idxB[r]);
      __syncthreads();
      commit_tile2(LI, D, tid);
      __syncthreads();
      float lA[RA], cdA[RA];
      lap_stepA(LI, g, lane, wv, lA, cdA);
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int i = iA + r;
        const float bb = coef_b(g, inner, i, jE);
        const float okE = (colE && i >= 0 && i < g.nzp) ? 1.0f : 0.0f;
        LE[(wv * RA + r) * EX + lane] =
            leapfrog_src(bb, cdA[r], dmA[r], cA[r], lA[r], dcA[r], wA[r]) * okE;
      }
      __syncthreads();
      if (a.dd_out)
        for (int e = rp0 + tid; e < rp1; e += NTHREADS2)
          a.dd_out[(((long long)b * g.ns + s) * g.nt + a.n + 1) * g.nr + t.t2_rec_id[e]] =
              LE[t.t2_rec_local[e]];
      float lB[RB], cdB[RB], dB[RB];
      lap_stepB(LE, g, lb, wv, lB, cdB);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int i = iB + r;
        const float bb = coef_b(g, inner, i, jE);
        const float dnT = LI[(wv * RB + r + 2 * HALO) * IX + 2 * HALO + lb - HALO];
        dB[r] = leapfrog_src(bb, cdB[r], dnT, cB[r], lB[r], dcB[r], wB[r]);
        if (colT && i < g.nzp) {
          stf_nt(d1, idxB[r], cdB[r]);
          stf_nt(d2, idxB[r], dB[r]);
        }
      }
      if (a.dd_out && rp1 > rp0)
        gather2(LE, dB, colT, lane, wv, t, rp0, rp1, tid,
                a.dd_out + (((long long)b * g.ns + s) * g.nt + a.n + 2) * g.nr);
    }
  }
}

// Two adjoint steps for a.nb vectors over a group of shots: mu^k on the
// extended region (with injection at every receiver node inside it), mu^{k-1}
// on the output tile (with injection at the nodes inside the tile), and the
// image terms w^k mu^{k+1} + w^{k-1} mu^k accumulated over the group's shots.
// The forward levels w^k, w^{k-1} of a shot are loaded once for all the
// workgroup's vectors; each vector's image accumulates in dynamic LDS, in
// entries private to the thread that owns the output point.
__global__ __launch_bounds__(NTHREADS2) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_adjoint2(Geo g, DevTables t, Adj2Args a) {
  extern __shared__ float LIMG[];  // [nb][TZ2][EX]
  __shared__ float LI[IZ * IX];
  __shared__ float LE[EZ * EX];
  if (g.poison) {
    poison_lds(LI, IZ * IX, NTHREADS2);
    poison_lds(LE, EZ * EX, NTHREADS2);
    poison_lds(LIMG, a.nb * TZ2 * EX, NTHREADS2);
    __syncthreads();
  }
  // Launch order, without the XCD remap: the tiles of a field are dealt
  // round-robin to the XCDs, so fewer halo re-reads hit an XCD's L2 (35 % more
  // L2-miss traffic on 921 x 301, 64 shots and 17 right-hand sides) but all
  // XCDs work on the same few fields, whose lines the other XCDs have just
  // fetched; the launch runs 0.5-1 % faster than in the remapped order.
  const int lid = blockIdx.x;
  const int tile = lid % g.ntiles2;
  const int rest = lid / g.ntiles2;
  const int nbg = (a.B + a.nb - 1) / a.nb;
  const int b0 = (rest % nbg) * a.nb, grp = rest / nbg;
  const int nbv = min(a.nb, a.B - b0);  // vectors of this workgroup
  const int tzi = tile / g.tiles_x2, txi = tile - tzi * g.tiles_x2;
  const int i0 = tzi * TZ2, j0 = txi * TX2;
  const int tid = threadIdx.x, lane = tid % TX, wv = tid / TX;
  const long long fs = g.fs;
  const bool inner = tile_interior(g, i0 - HALO, j0 - HALO, EZ, EX);

  const int jE = j0 - HALO + lane;
  const bool colE = jE >= 0 && jE < g.nxp;
  const bool colT = lane >= HALO && lane < HALO + TX2 && colE;
  const int jc = min(max(jE, 0), g.nxp - 1);
  const int lb = min(max(lane, HALO), EX - 1 - HALO);
  const int iA = i0 - HALO + wv * RA;
  const int iB = i0 + wv * RB;

  unsigned idxA[RA], idxB[RB];
  float cA[RA], cB[RB];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    idxA[r] = (unsigned)(min(max(iA + r, 0), g.nzp - 1) * g.pitch + jc);
    cA[r] = ldf(a.c, idxA[r]);
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    idxB[r] = (unsigned)(min(iB + r, g.nzp - 1) * g.pitch + jc);
    cB[r] = ldf(a.c, idxB[r]);
  }
  for (int q = 0; q < nbv; ++q)
#pragma unroll
    for (int r = 0; r < RB; ++r) LIMG[(q * TZ2 + wv * RB + r) * EX + lane] = 0.0f;
  const int np0 = t.t2_node_ptr[tile], np1 = t.t2_node_ptr[tile + 1];
  const bool inject = np1 > np0;
  const int s0 = grp * a.group, s1 = min(g.ns, s0 + a.group);

  for (int s = s0; s < s1; ++s) {
   float w0B[RB], w1B[RB];
#pragma unroll
   for (int r = 0; r < RB; ++r) {
     w0B[r] = a.w0 ? ldf(a.w0 + s * fs, idxB[r]) : 0.0f;
     w1B[r] = ldf(a.w1 + s * fs, idxB[r]);
   }
#pragma unroll 1
   for (int q = 0; q < nbv; ++q) {
    const int b = b0 + q;
    const long long fb = ((long long)b * g.ns + s) * 2 * fs;
    const float *m1 = a.muin + fb + ((a.k + 1) & 1) * fs;  // mu^{k+1}
    const float *m2 = a.muin + fb + (a.k & 1) * fs;        // mu^{k+2}
    float *o0 = a.muout + fb + (a.k & 1) * fs;             // mu^k
    float *om = a.muout + fb + ((a.k + 1) & 1) * fs;       // mu^{k-1}
    float m2A[RA];
    Tile2Regs T;
    fetch_tile2(T, m1, i0, j0, g, tid);
#pragma unroll
    for (int r = 0; r < RA; ++r) m2A[r] = ldf(m2, idxA[r]);
    if (s > s0 || q > 0) __syncthreads();
    commit_tile2(LI, T, tid);
    __syncthreads();
    // step A: mu^k on the extended region
    float lA[RA], cmA[RA];
    lap_stepA(LI, g, lane, wv, lA, cmA);
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int i = iA + r;
      const float bb = coef_b(g, inner, i, jE);
      const float okE = (colE && i >= 0 && i < g.nzp) ? 1.0f : 0.0f;
      LE[(wv * RA + r) * EX + lane] = leapfrog(bb, cmA[r], m2A[r], cA[r], lA[r]) * okE;
    }
    __syncthreads();
    const float *rs = a.r + (((long long)b * g.ns + s) * g.nt) * g.nr;
    if (inject) {
      const float *rk = rs + (long long)a.k * g.nr;
      for (int e = np0 + tid; e < np1; e += NTHREADS2) {
        float acc = 0.0f;
        for (int q = t.t2_node_rec_ptr[e]; q < t.t2_node_rec_ptr[e + 1]; ++q)
          acc += rk[t.t2_node_recs[q]];
        LE[t.t2_node_local[e]] += a.c[t.t2_node_gidx[e]] * acc;
      }
      __syncthreads();
    }
    // step B: mu^{k-1} on the output tile
    float lB[RB], cmB[RB], out[RB];
    lap_stepB(LE, g, lb, wv, lB, cmB);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = iB + r;
      const float bb = coef_b(g, inner, i, jE);
      const float m1T = LI[(wv * RB + r + 2 * HALO) * IX + 2 * HALO + lb - HALO];
      out[r] = leapfrog(bb, cmB[r], m1T, cB[r], lB[r]);
      float *acc = LIMG + (q * TZ2 + wv * RB + r) * EX + lane;
      *acc = __builtin_fmaf(w1B[r], cmB[r], __builtin_fmaf(w0B[r], m1T, *acc));
    }
    if (inject) {
      __syncthreads();
      if (lane == lb)  // output columns only: clamped lanes must not write
#pragma unroll
        for (int r = 0; r < RB; ++r) LE[(wv * RB + r + HALO) * EX + lb] = out[r];
      __syncthreads();
      const float *rk = rs + (long long)(a.k - 1) * g.nr;
      for (int e = np0 + tid; e < np1; e += NTHREADS2) {
        const int loc = t.t2_node_local[e];
        const int re = loc / EX, ce = loc - re * EX;
        if (re < HALO || re >= HALO + TZ2 || ce < HALO || ce >= HALO + TX2) continue;
        float acc = 0.0f;
        for (int q = t.t2_node_rec_ptr[e]; q < t.t2_node_rec_ptr[e + 1]; ++q)
          acc += rk[t.t2_node_recs[q]];
        LE[loc] += a.c[t.t2_node_gidx[e]] * acc;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RB; ++r) out[r] = LE[(wv * RB + r + HALO) * EX + lb];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (colT && iB + r < g.nzp) {
        stf_nt(o0, idxB[r], cmB[r]);
        stf_nt(om, idxB[r], out[r]);
      }
    }
   }
  }
  float sm[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sm[r] = ldf(a.s2m, idxB[r]);
  for (int q = 0; q < nbv; ++q) {
    double *ig = a.img + ((long long)grp * a.B + b0 + q) * fs;
    double old[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) old[r] = ldd(ig, idxB[r]);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const float im = LIMG[(q * TZ2 + wv * RB + r) * EX + lane];
      if (colT && iB + r < g.nzp) std_(ig, idxB[r], old[r] + (double)sm[r] * (double)im);
    }
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
// out[b] = scale * P^T sum_groups img[group][b0 + b], images [G][Bst][fs].
__global__ void k_fold(Geo g, const double *__restrict__ img, int G, int Bst, int b0, int B,
                       double scale, float *__restrict__ out) {
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
    const double *ig = img + ((long long)gg * Bst + b0 + b) * g.fs;
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

// A call's status word: cleared when the call starts; at its end its bits
// are OR-ed into the plan's word as well.
__global__ void k_status_open(unsigned int *status) { *status = 0u; }

__global__ void k_status_merge(const unsigned int *__restrict__ from, unsigned int *into) {
  const unsigned int v = *from;
  if (v) atomicOr(into, v);
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
  const unsigned int grid =
      (unsigned int)((a.order == 2 ? g.nblocks * g.blk : g.ntiles) * g.ns);
  if (born)
    hipLaunchKernelGGL(k_step<true>, dim3(grid), dim3(NTHREADS), 0, st, g, t, a);
  else
    hipLaunchKernelGGL(k_step<false>, dim3(grid), dim3(NTHREADS), 0, st, g, t, a);
  return hipGetLastError();
}

hipError_t launch_step2(const Geo &g, const DevTables &t, const Step2Args &a, bool born,
                        hipStream_t st) {
  const unsigned int grid = (unsigned int)(g.ntiles2 * g.ns);
  if (born)
    hipLaunchKernelGGL(k_step2<true>, dim3(grid), dim3(NTHREADS2), 0, st, g, t, a);
  else
    hipLaunchKernelGGL(k_step2<false>, dim3(grid), dim3(NTHREADS2), 0, st, g, t, a);
  return hipGetLastError();
}

hipError_t launch_adjoint2(const Geo &g, const DevTables &t, const Adj2Args &a, hipStream_t st) {
  const unsigned int grid = (unsigned int)(g.ntiles2 * ((a.B + a.nb - 1) / a.nb) * a.ngroups);
  const size_t lds = (size_t)a.nb * TZ2 * EX * sizeof(float);
  hipLaunchKernelGGL(k_adjoint2, dim3(grid), dim3(NTHREADS2), lds, st, g, t, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const Geo &g, const DevTables &t, const AdjArgs &a, hipStream_t st) {
  const unsigned int grid =
      (unsigned int)((a.order == 2 ? g.nblocks * g.blk : g.ntiles) * a.B * a.ngroups);
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

hipError_t launch_fold(const Geo &g, const double *img, int G, int Bst, int b0, int B,
                       double scale, float *out, hipStream_t st) {
  const long long n = (long long)g.nz * g.nx * B;
  hipLaunchKernelGGL(k_fold, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, img, G, Bst, b0, B,
                     scale, out);
  return hipGetLastError();
}

hipError_t launch_status_open(unsigned int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_status_open, dim3(1), dim3(1), 0, st, status);
  return hipGetLastError();
}

hipError_t launch_status_merge(const unsigned int *from, unsigned int *into, hipStream_t st) {
  hipLaunchKernelGGL(k_status_merge, dim3(1), dim3(1), 0, st, from, into);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float *p, long long n, unsigned int *status,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 4096)), dim3(256), 0, st, p, n, status);
  return hipGetLastError();
}

}  // namespace fwi

// Internal definitions shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace fwi {

// Records `msg` as the calling thread's last error (fwi_last_error) and
// returns `code`.
int set_error(int code, const std::string &msg);

// Tile of one workgroup: 64 columns (one wavefront wide) by TZ rows; each of
// the NWAVE wavefronts owns RZ consecutive rows of every column.
constexpr int TX = 64;
constexpr int NWAVE = 4;
constexpr int RZ = 8;
constexpr int TZ = NWAVE * RZ;
constexpr int HALO = 4;          // 8th-order stencil radius
constexpr int LW = TX + 2 * HALO;  // LDS row width
constexpr int LH = TZ + 2 * HALO;  // LDS rows
constexpr int NTHREADS = TX * NWAVE;

// Two-step (temporally blocked) tiles: TX2 x TZ2 outputs; the intermediate
// time level is computed on the tile plus a HALO ring (EX x EZ, one wave64
// row per tile row) and the input level is staged with a 2*HALO ring.
constexpr int TX2 = TX - 2 * HALO;      // 56 output columns
constexpr int TZ2 = TZ;                 // 32 output rows
constexpr int EX = TX2 + 2 * HALO;      // 64
constexpr int EZ = TZ2 + 2 * HALO;      // 40
constexpr int IX = TX2 + 4 * HALO;      // 72
constexpr int IZ = TZ2 + 4 * HALO;      // 48
constexpr int NWAVE2 = 8;               // wavefronts per two-step workgroup
constexpr int NTHREADS2 = TX * NWAVE2;  // 512
constexpr int RA = EZ / NWAVE2;         // 5 intermediate rows per wavefront
constexpr int RB = TZ2 / NWAVE2;        // 4 output rows per wavefront

// Largest Courant number max(m) dt/dx the scheme tolerates.
constexpr float CFL_LIMIT = 0.5546f;

// Geometry of the padded grid as the kernels see it.  Every per-point array
// (wavefields, coefficients, images) uses the same layout: element (i, j) of
// the padded grid at i*pitch + j, pitch a multiple of 64 floats and at least
// NXp, rows rounded up to whole tiles; `fs` is the element count of one
// such array.
struct Geo {
  int nz, nx, nb;
  int nzp, nxp, pitch;
  int tiles_x, tiles_z, ntiles;
  int ns, nt, nr;
  long long fs;
  float kmax, inv_nb;
  float c1, c2, c3, c4;  // C1..C4 of the stencil, divided by dx^2 (C0 = -2 sum)
  float dt, inv_dx;
  int blk;       // tiles per block in the blocked workgroup order
  int nblocks;   // ceil(ntiles / blk)
  int tiles_x2, tiles_z2, ntiles2;  // two-step tiling
  int poison;    // debug: fill LDS with NaN before use (FWI_OPT_LDS_POISON)
};

// Device block of a plan (offsets in int32 units from its base).
struct DevTables {
  const int *src_ij;        // ns x (i, j) padded coordinates
  const int *tile_rec_ptr;  // ntiles+1: receivers of tile t in [ptr[t], ptr[t+1])
  const int *rec_local;     // local index lz*TX + lx of each listed receiver
  const int *rec_id;        // receiver number of each listed receiver
  const int *tile_node_ptr; // ntiles+1: distinct receiver nodes of a tile
  const int *node_local;    // local index of each node
  const int *node_gidx;     // i*pitch + j of each node
  const int *node_rec_ptr;  // nnodes+1: receivers sitting on node k
  const int *node_recs;     // receiver numbers, grouped by node
  const int *tile_order;    // ntiles: tiles listed block by block (blocked order)
  // two-step tiling: receivers inside each output tile (E-local index
  // (i - i0 + HALO) * EX + (j - j0 + HALO)), and distinct receiver nodes
  // inside each tile's extended region, for injection
  const int *t2_rec_ptr, *t2_rec_local, *t2_rec_id;
  const int *t2_node_ptr, *t2_node_local, *t2_node_gidx, *t2_node_rec_ptr, *t2_node_recs;
  unsigned int *status;     // FWI_STATUS_* bits
};

// Arguments of one two-step forward / forward+Born launch (n even):
// reads (u^n, u^{n-1}) from `uin`, writes (u^{n+1}, u^{n+2}) to `uout`,
// both [ns][2][fs] with u^k in slot k & 1; Born fields likewise per vector.
struct Step2Args {
  const float *c;
  const float *dc;
  const float *uin;
  float *uout;
  const float *duin;   // [ns][B][2][fs]
  float *duout;
  float *w_out0;       // [ns][fs] receives w^n, or null
  float *w_out1;       // [ns][fs] receives w^{n+1}, or null
  float *d_out;        // [ns][nt][nr] receives R u^{n+1}, R u^{n+2}, or null
  float *dd_out;       // [B][ns][nt][nr], or null
  float *ck;           // [ns][2][fs]: receives (u^{n+1}, u^{n+2}), or null
  int n;
  int B;
  float amp0, amp1;    // s(n dt)/dx^2, s((n+1) dt)/dx^2
};

// Arguments of one two-step adjoint launch: (mu^{k+1}, mu^{k+2}) from `muin`
// to (mu^k, mu^{k-1}) in `muout`, image terms n = k (if w0) and n = k-1.
struct Adj2Args {
  const float *c;
  const float *s2m;
  const float *muin;   // [B][ns][2][fs]
  float *muout;
  const float *w0;     // [ns][fs] w^k, or null (k = nt-1: no image term)
  const float *w1;     // [ns][fs] w^{k-1}
  const float *r;      // [B][ns][nt][nr]
  double *img;         // [G][B][fs]
  int k;
  int B;
  int group;
  int ngroups;
  int nb;              // vectors per workgroup (share the loads of w), <= 4
};

// Arguments of one forward / forward+Born time step.
struct StepArgs {
  const float *c;     // [fs] (dt m_pad)^2 / (1 + kappa)
  const float *dc;    // [B][fs] Born coefficient perturbation, or null
  float *u;           // [ns][2][fs]: u^k lives in slot k & 1
  float *du;          // [ns][B][2][fs] Born wavefields, same slot rule
  float *w_out;       // [ns][fs]: receives w^n = L u^n + f^n, or null
  float *d_out;       // [ns][nt][nr]: receives R u^{n+1}, or null
  float *dd_out;      // [B][ns][nt][nr]: receives R du^{n+1}, or null
  float *ck;          // [ns][2][fs] checkpoint slot: u^{n+1}, u^n, or null
  int n;              // step: computes u^{n+1}
  int B;
  float src_amp;      // s(n dt) / dx^2
  int order;          // workgroup order: 0 shot-major, 1 tile-major, 2 blocked
};

// Arguments of one adjoint + imaging time step (mu = c * lambda form).
struct AdjArgs {
  const float *c;     // [fs]
  const float *s2m;   // [fs] 2 / m_pad
  float *mu;          // [B][ns][2][fs]: mu^k in slot k & 1
  const float *w;     // [ns][fs] w^k for this step, or null (no image term)
  const float *r;     // [B][ns][nt][nr] data injected at the receivers
  double *img;        // [G][B][fs] partial images, one per shot group
  int k;              // computes mu^k
  int B;
  int group;          // shots per workgroup
  int ngroups;
  int order;          // workgroup order: 0 vector-major, 1 tile-major, 2 blocked
};

// Dense products for the approximation layers (defined with the low-rank
// code): C(i, j) = alpha sum_p A(i, p) B(p, j) + beta C(i, j) over a batch,
// X(i, j) = X[b * xb + i * x1 + j * x2], FP32 operands read through LDS
// tiles, FP64 accumulation.  In split mode (part != null) the batch index
// runs over chunks of the inner dimension instead and each chunk writes its
// FP64 partial sum to part[chunk][M][N].
struct Gemm {
  int M, N, K;
  const float *A;
  long long ab, am, ak;
  const float *B;
  long long bb, bk, bn;
  float *C;
  long long cb, cm, cn;
  float alpha, beta;
  double *part;  // split mode: [nchunk][M][N]
  int kchunk;    // inner-dimension length per chunk (split mode)
};
constexpr int KCHUNK = 4096;  // inner-dimension chunk of the long products
Gemm plain(int M, int N, int K);  // alpha 1, beta 0, zero strides
hipError_t gemm(const Gemm &g, int batch, hipStream_t st);
int nchunks(long long K);
// out[M][N] (FP64) = A B over a long inner dimension, via FP64 partials.
hipError_t gemm_long(Gemm g, double *part, double *out, hipStream_t st);

// Eigenpairs of the symmetric k x k FP64 matrix A (overwritten; k <=
// EIG_KMAX) by parallel cyclic Jacobi: eigenvalues descending in w[k], the
// matching eigenvectors as the columns of Zs[k][k]; Z[k][k] is scratch.
constexpr int EIG_KMAX = 512;
hipError_t sym_eig(int k, double *A, double *Z, double *w, double *Zs, hipStream_t st);

}  // namespace fwi

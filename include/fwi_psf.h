/*
 * fwi_psf.h -- C ABI of the point-spread-function (PSF) approximation of the
 * misfit Hessian H_d on the model grid (MI355X / gfx950 library, the same
 * shared object as fwi.h; error codes and fwi_last_error() are shared).
 *
 * The method (Section 3.2, "Point spread function method"; Section 3.5, "PSF
 * method in PsiDO formulation"):
 *   - PSF k at sample point x_k is p_k(d) = (H_d e_{x_k})(x_k + d): the
 *     Hessian applied to a delta, read on a window d in [-half, half]^2.
 *     PSFs are local, so one Hessian product of a comb of well separated
 *     deltas yields many PSFs at once;
 *   - the PSFs are blended with interpolation weights w_k into an operator
 *     that applies in O(N * window) work.  In the PsiDO form of Section 3.5,
 *     H_d ~ sum_k D_{w_k} F^-1 D_{s_k} F with symbol rows s_k = conj(F p_k),
 *     which on the grid is
 *         (H~ v)(y) = sum_k w_k(y) sum_d p_k(d) v(y + d),          (ROWS)
 *     v taken as zero outside the model.  fwi_psf_apply evaluates exactly
 *     this sum in the space domain (the Fourier chain with zero padding gives
 *     the same numbers); it is the transpose of the product-convolution form
 *     sum_k p_k * (w_k v) of Section 3.2, and both approximate the
 *     self-adjoint H_d.
 *
 * Sample points and weights (the paper leaves the weights open, naming
 * radial basis functions as one choice): centres on a regular lattice,
 * rows oz + p*sz (p < nzc), columns ox + q*sx (q < nxc), k = p*nxc + q;
 * w_k(z, x) = t_p(z) t_q(x) with t the piecewise-linear tent functions of the
 * centre lattice, constant beyond the first and last centre, so that
 * sum_k w_k = 1, w_k >= 0 and w_k(x_j) = [k == j].
 *
 * Probing vectors: stride^2 combs; comb (p % stride)*stride + (q % stride)
 * holds the deltas of every centre (p, q) with those residues.  Windows of
 * one comb do not overlap when 2*half + 1 <= stride * min(sz, sx).
 *
 * All array arguments are DEVICE pointers to contiguous row-major FP32
 * arrays; calls validate synchronously, enqueue kernels on `stream` (a
 * hipStream_t, NULL = default) and return.  No device memory is allocated.
 */
#ifndef FWI_MI355X_PSF_H
#define FWI_MI355X_PSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nz, nx;    /* model grid: nz rows (depth) by nx columns (x fastest) */
  int32_t oz, ox;    /* row and column of the first centre (0 <= o < n) */
  int32_t sz, sx;    /* centre spacing in rows and in columns (>= 1) */
  int32_t nzc, nxc;  /* centres per column and per row; r = nzc * nxc PSFs;
                        the last centre must lie inside the grid */
  int32_t half;      /* PSF window half-width, 0..32; W = 2*half + 1 */
  int32_t stride;    /* combs per axis (>= 1): stride^2 probing vectors */
} fwi_psf_grid;

/* Validate a sampling description (FWI_OK or FWI_EINVAL with a message). */
int fwi_psf_check(const fwi_psf_grid *g);

/* PSFs from the Hessian products of the combs (Section 3.2).
 *   hv:  [stride^2][nz][nx]  H_d applied to each comb (fwi_gn_hvp output)
 *   psf: [r][W][W]           psf[k][half + dz][half + dx] =
 *                            hv[comb(k)][z_k + dz][x_k + dx], 0 outside the grid
 * Errors: FWI_EINVAL for a bad grid or a null pointer. */
int fwi_psf_extract(const fwi_psf_grid *g, const float *hv, float *psf, void *stream);

/* Apply the PSF approximation (ROWS form above) to B vectors.
 *   psf: [r][W][W]   (from fwi_psf_extract or any other source)
 *   v:   [B][nz][nx]
 *   out: [B][nz][nx] (must not alias v)
 * FP32 arithmetic with FP32 accumulation over the window; every output is
 * written by exactly one workgroup, in a fixed order (deterministic).
 * Errors: FWI_EINVAL for a bad grid, B outside [1, 65535] or a null
 * pointer; FWI_EHIP if the launch fails. */
int fwi_psf_apply(const fwi_psf_grid *g, const float *psf, const float *v, int B, float *out,
                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_MI355X_PSF_H */

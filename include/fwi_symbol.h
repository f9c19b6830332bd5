/*
 * fwi_symbol.h -- C ABI of the low-rank symbol approximations of the misfit
 * Hessian H_d: the pseudo-differential operator probing method (PDO,
 * Section 3.4 and Appendix A) and the low-rank symbol method PSF+ (Section
 * 3.6), with the fast apply both share (Section 3.3, eq. "lr-psido").  Same
 * shared object as fwi.h; error codes and fwi_last_error() are shared.
 *
 * Discrete setting.  A periodic FFT grid of mz x mx cells of spacing h holds
 * the nz x nx model grid in its first rows and columns (the rest is zero
 * padding; cell (iz, ix) is the point x = (ix h, iz h)).  Lattice
 * frequencies are xi = (2 pi q / (mx h), 2 pi p / (mz h)) for the centred
 * representatives p, q; on an even length the Nyquist index has two
 * representatives and every tabulated function of xi is their average.
 * Transform pair (the footnote of Section 3.3, sums for integrals):
 * v^(xi) = (1/M) sum_x e^{-i x.xi} v(x), v(x) = sum_xi e^{i x.xi} v^(xi),
 * M = mz mx.  The symbol of H is S[x, xi] = (H phi_xi)(x) / phi_xi(x),
 * phi_xi(x) = e^{i x.xi}.
 *
 * Low-rank symbol apply (eq. "lr-psido"):  for S ~ sum_t A_t(x) M_t(xi),
 *     out(x) = scale * Re sum_t A_t(x) sum_xi e^{i x.xi} M_t(xi) v^(xi)
 * on the model grid, v zero-padded: one forward 2-D FFT per vector and one
 * inverse 2-D FFT per term.  Real operators have conjugate-symmetric
 * symbols, which lets two real terms share one complex transform:
 *   - PDO: the columns at xi_k and -xi_k are conjugate, so the r columns
 *     become r/2 terms A_t = s_t, M_t = w_t with scale 2;
 *   - PSF+: real coefficients a_j and row-basis functions b_j with
 *     b_j(-xi) = conj b_j(xi) pair up as A_t = a_{2t} - i a_{2t+1},
 *     M_t = b_{2t} + i b_{2t+1}, scale 1.
 *
 * PDO (Section 3.4, Appendix A): sample frequencies xi_k = rho0 (cos
 * theta_k, sin theta_k), theta_k = 2 pi k / r, k = 1..r (r even).  Probe
 * v_p = sum_k phi_{xi_k} (eq. "pdo-vp").  Symbol columns (eq. "symbol") by
 * spectral separation of H v_p: every lattice frequency goes to its nearest
 * sample frequency (the angular sectors of width 2 pi / r around the
 * theta_k); a frequency equidistant from several samples within a relative
 * 1e-9 (the origin, lattice points on a sector boundary) is shared equally.
 * Weights (eq. "pdo-w"): w_k(xi) = (rho / rho0) w_k^circle(theta) with the
 * trigonometric interpolation cardinal functions on the r angles, the
 * Nyquist mode split evenly.
 *
 * PSF+ (Section 3.6): symbol rows S~[x_k, xi] = sum_d p_k(d) e^{i d.xi} of
 * the PSFs (fwi_psf.h); their SVD S~[I_r, :] = U Sigma V^H gives the row
 * basis B (leading `rank` rows of V^H, orthonormal) and A0 = W U Sigma (W the
 * PSF method's tent weights); the coefficients solve
 *     min_A ||A B[:, I_c] - S~[:, I_c]||_F^2 + alpha ||A - A0||_F^2,
 *     alpha = ||B[:, I_c]||_F^2 / ||B||_F^2   (eq. "psfplus"),
 * S~[:, I_c] the PDO columns.  Computed through the Gram matrix of the PSFs
 * (by Parseval, S~ S~^H = M P P^T for the PSF windows P, as long as a window
 * fits in the FFT grid), so B_j is the symbol of the real kernel
 * q_j = sum_k U[k, j] p_k / sigma_j and A is real; B[:, I_c] is summed
 * directly at the (off-lattice) sample frequencies.
 *
 * Conventions: all array arguments are DEVICE pointers to contiguous
 * row-major arrays; "complex" arrays hold interleaved FP32 (re, im) pairs.
 * A symbol object owns host tables (FFT twiddles) that fwi_symbol_bind
 * copies into a caller block; every call that needs scratch takes a caller
 * workspace (256-byte aligned).  Calls validate synchronously, enqueue on
 * `stream` (hipStream_t, NULL = default) and return.  No device memory is
 * allocated.  FP32 transforms (twiddles rounded from FP64); FP64 for the
 * phases, the separation decisions, the Gram and least-squares algebra.
 */
#ifndef FWI_MI355X_SYMBOL_H
#define FWI_MI355X_SYMBOL_H

#include <stddef.h>
#include <stdint.h>

#include "fwi.h"
#include "fwi_psf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nz, nx;  /* model grid, 1..2048 each */
  int32_t mz, mx;  /* FFT grid, mz >= nz, mx >= nx, <= 2048, factors 2, 3, 5 only */
  double h;        /* grid spacing (> 0) */
  int32_t r;       /* PDO sample directions: even, 2..16 */
  double rho0;     /* PDO sample radius (rad per unit length, > 0) */
} fwi_symbol_grid;

typedef struct fwi_symbol fwi_symbol;

/* Validate a grid (FWI_OK or FWI_EINVAL with a message). */
int fwi_symbol_check(const fwi_symbol_grid *g);
int fwi_symbol_create(const fwi_symbol_grid *g, fwi_symbol **out);
void fwi_symbol_destroy(fwi_symbol *s);
/* Tuning options of a symbol object (none changes what is computed; the
 * blend split changes the order of FP32 additions over the terms).  Defaults
 * are the fastest measured on MI355X. */
enum {
  FWI_SYM_OPT_CHUNK_MB = 0,    /* MiB of partial transforms per vector chunk of an
                                  apply, >= 1 (default 4096) */
  FWI_SYM_OPT_BLEND_SPLIT = 1, /* wavefronts sharing one vector's terms in the inverse
                                  row blend, 1..4 (must divide the wavefronts per
                                  workgroup, else 1); 0 (default): by grid size */
  FWI_SYM_OPT_SPLIT_960 = 2    /* 0/1: 960-point rows by the split 15 x 64 transform
                                  (default 1) */
};
/* FWI_EINVAL for an unknown option or a value out of range. */
int fwi_symbol_set_option(fwi_symbol *s, int option, int value);
int fwi_symbol_get_option(const fwi_symbol *s, int option, int *value);
/* Bytes of the device block (FFT twiddle tables). */
int fwi_symbol_device_bytes(const fwi_symbol *s, size_t *bytes);
/* Copy the tables into `dev` (256-byte aligned) and synchronise `stream`. */
int fwi_symbol_bind(fwi_symbol *s, void *dev, size_t bytes, void *stream);

/* Workspace of fwi_symbol_apply for B vectors and T terms, and of
 * fwi_pdo_columns (B = 1, T = r/2). */
int fwi_symbol_workspace_size(const fwi_symbol *s, int B, int T, size_t *bytes);

/* out[B][nz][nx] = scale * Re sum_t A_t . F^-1 (M_t . F v) (see above).
 *   A: [T][nz][nx] complex;  M: [T][mz][mx] complex (lattice order, index
 *   (p, q) at p*mx + q);  v: [B][nz][nx];  out must not alias v.
 * T in [1, 64], B in [1, 1024].  Deterministic (fixed summation order). */
int fwi_symbol_apply(fwi_symbol *s, int T, const float *A, const float *M, float scale,
                     const float *v, int B, float *out, void *ws, size_t ws_bytes, void *stream);

/* PDO probe v_p = 2 sum_{k=1}^{r/2} cos(x . xi_k) on the model grid
 * (phases in FP64): vp[nz][nx]. */
int fwi_pdo_probe(fwi_symbol *s, float *vp, void *stream);
/* PDO weight tables w_k for k = 1..r/2 as complex (w, 0): M[r/2][mz][mx]. */
int fwi_pdo_weights(fwi_symbol *s, float *M, void *stream);
/* Separation masks for k = 1..r/2 as complex (mask, 0): masks[r/2][mz][mx]
 * (what fwi_pdo_columns applies; exposed for inspection and tests). */
int fwi_pdo_masks(fwi_symbol *s, float *masks, void *stream);
/* Symbol columns s_k for k = 1..r/2 from hvp = H_d v_p (columns k + r/2 are
 * their conjugates): cols[r/2][nz][nx] complex.  ws: workspace of
 * fwi_symbol_workspace_size(s, 1, r/2) plus r/2 mz mx complex for the masks
 * (fwi_pdo_workspace_size). */
int fwi_pdo_workspace_size(const fwi_symbol *s, size_t *bytes);
int fwi_pdo_columns(fwi_symbol *s, const float *hvp, float *cols, void *ws, size_t ws_bytes,
                    void *stream);

/* PSF+ from r_psf PSFs (fwi_psf_extract layout [r_psf][W][W]; the PSF grid
 * must describe the same nz x nx model, r_psf <= 512, W <= min(mz, mx)) and
 * the r/2 PDO columns.  rank in [1, min(r_psf, 32)].  Outputs the apply
 * tables with T = ceil(rank / 2) terms (scale 1):
 *   A: [T][nz][nx] complex, M: [T][mz][mx] complex;
 *   info (device, FP64): [0] alpha, [1] number of basis rows kept (singular
 *   values below 1e-12 of the largest are dropped), [2 .. 2+rank) the
 *   singular values sigma_j of S~[I_r, :].
 * ws: fwi_psfplus_workspace_size bytes. */
int fwi_psfplus_workspace_size(const fwi_symbol *s, const fwi_psf_grid *pg, int rank,
                               size_t *bytes);
int fwi_psfplus_build(fwi_symbol *s, const fwi_psf_grid *pg, const float *psf, const float *cols,
                      int rank, float *A, float *M, double *info, void *ws, size_t ws_bytes,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_MI355X_SYMBOL_H */

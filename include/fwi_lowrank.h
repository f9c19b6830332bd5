/*
 * fwi_lowrank.h -- C ABI of the Matern prior and the low-rank (randomized)
 * approximation of the misfit Hessian (MI355X / gfx950 library, the same
 * shared object as fwi.h; error codes and fwi_last_error() are shared).
 *
 * Prior (Section 2): Gaussian with covariance (delta I - gamma Lap_h)^-2, so
 * the regularization Hessian is R = A^2, A = delta I - gamma Lap_h, with
 * Lap_h the 5-point Laplacian of spacing h on the nz x nx model grid and
 * mirrored (zero-flux) edges; delta, gamma > 0.  A is diagonalised by the
 * 2-D DCT-II, A = C^T diag(delta + gamma mu) C with
 * mu_pq = (4/h^2)(sin^2(pi p/(2 nz)) + sin^2(pi q/(2 nx))), which gives
 * R^-1 and A^-1 exactly.
 *
 * Low-rank approximation (Section 3.1): the r largest eigenpairs of the
 * pencil H_d v = lambda R v, V^T R V = I, by the double-pass randomized
 * method for Hermitian pencils, and the approximations built on them
 *   (H~_d + R) v = R v + R V L V^T R v,
 *   (H~_d + R)^-1 v = R^-1 v - V D V^T v,  D = L (L + I)^-1,
 *   zeta = (I - V S V^T R) A^-1 w,         S = I - (L + I)^-1/2
 * (zeta ~ N(0, (H~_d + R)^-1) for white w: the Laplace-approximation
 * proposal of Section 2.3).
 *
 * All arrays are DEVICE pointers to contiguous row-major arrays; vectors are
 * [B][nz][nx] FP32.  The library allocates no device memory: a prior owns
 * host tables that fwi_prior_bind copies into a caller block, and every call
 * takes a caller workspace.
 */
#ifndef FWI_MI355X_LOWRANK_H
#define FWI_MI355X_LOWRANK_H

#include <stddef.h>
#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fwi_prior fwi_prior;

/* Prior operations. */
enum {
  FWI_PRIOR_R = 0,     /* R v = A (A v) (stencil, no tables needed)  */
  FWI_PRIOR_RINV = 1,  /* R^-1 v                                       */
  FWI_PRIOR_AINV = 2   /* A^-1 v  (N(0, R^-1) draw from white v)       */
};

int fwi_prior_create(int32_t nz, int32_t nx, double h, double delta, double gamma,
                     fwi_prior **out);
void fwi_prior_destroy(fwi_prior *p);
/* Bytes of the prior's device block (DCT matrices and spectrum, FP32). */
int fwi_prior_device_bytes(const fwi_prior *p, size_t *bytes);
/* Copy the tables into `dev` (256-byte aligned, >= fwi_prior_device_bytes)
 * and synchronise `stream`. */
int fwi_prior_bind(fwi_prior *p, void *dev, size_t bytes, void *stream);
/* Workspace of fwi_prior_apply for B vectors. */
int fwi_prior_workspace_size(const fwi_prior *p, int B, size_t *bytes);
/* out[B] = op(v[B]); out must not alias v. */
int fwi_prior_apply(fwi_prior *p, int op, const float *v, int B, float *out, void *ws,
                    size_t ws_bytes, void *stream);

/* Low-rank approximation (double pass).  The caller runs the Hessian
 * products with fwi_gn_hvp:
 *   1. ybar = H_d omega for k random probes omega[k][nz][nx];
 *   2. fwi_lowrank_range: Y = R^-1 ybar, then twice: G = Y R Y^T (FP64),
 *      eigendecomposition of G, rows scaled by G's eigenvalues^-1/2, with
 *      the directions below tol times the largest dropped: Q[k][nz][nx] with
 *      Q R Q^T = I on its first *kept rows (the rest zero), RQ = R Q;
 *      *kept is written on the device;
 *   3. hq = H_d Q for the kept rows;
 *   4. fwi_lowrank_project: T = Q hq^T (kept x kept, FP64), T = U L U^T,
 *      lambda[r] = the r largest eigenvalues (descending, FP64, device),
 *      V[r][nz][nx] = U_r^T Q.
 * k <= 512; `k` in fwi_lowrank_project is the number of kept rows.  The
 * eigenproblems run in FP64 (parallel cyclic Jacobi, at most 60 sweeps).
 * ws: fwi_lowrank_workspace_size(p, k, B, r) bytes, 256-byte aligned. */
int fwi_lowrank_workspace_size(const fwi_prior *p, int k, int B, int r, size_t *bytes);
int fwi_lowrank_range(fwi_prior *p, int k, const float *ybar, double tol, float *Q, float *RQ,
                      int *kept, void *ws, size_t ws_bytes, void *stream);
int fwi_lowrank_project(fwi_prior *p, int k, const float *Q, const float *HQ, int r,
                        double *lambda, float *V, void *ws, size_t ws_bytes, void *stream);

/* Approximations from (lambda[r], V[r][nz][nx]) applied to B vectors:
 *   FWI_LOWRANK_HESSIAN: out = R v + R V L V^T R v      ((H~_d + R) v)
 *   FWI_LOWRANK_INVERSE: out = R^-1 v - V D V^T v       ((H~_d + R)^-1 v)
 *   FWI_LOWRANK_SAMPLE:  out = (I - V S V^T R) A^-1 v   (Laplace sample)
 * Projections onto V are FP64 sums over the grid.  out must not alias v. */
enum { FWI_LOWRANK_HESSIAN = 0, FWI_LOWRANK_INVERSE = 1, FWI_LOWRANK_SAMPLE = 2 };
int fwi_lowrank_apply(fwi_prior *p, int op, const double *lambda, const float *V, int r,
                      const float *v, int B, float *out, void *ws, size_t ws_bytes,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_MI355X_LOWRANK_H */

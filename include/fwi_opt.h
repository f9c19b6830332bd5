/*
 * fwi_opt.h -- C ABI of the vector algebra behind the MAP and sampling
 * drivers of Section 2 (MI355X / gfx950 library, the same shared object as
 * fwi.h; error codes and fwi_last_error() are shared).
 *
 * Section 2.1 solves min Phi(m) = phi_d(m) + 1/2 ||m - m_pr||^2_R by L-BFGS
 * with the initial inverse Hessian taken from a Hessian approximation; the
 * direction p = -H_k g comes from the two-loop recursion of L-BFGS (the
 * paper cites Nocedal and Wright, Section 7.2) over the stored pairs
 * s_i = m_{i+1} - m_i, y_i = g_{i+1} - g_i:
 *     loop 1, newest pair first:  alpha_i = rho_i s_i^T q;  q -= alpha_i y_i
 *     r = H0 q                    (any operator: the caller applies it)
 *     loop 2, oldest pair first:  beta = rho_i y_i^T r;    r += (alpha_i - beta) s_i
 * with rho_i = 1 / y_i^T s_i.  Section 2.3's gpCN sampler needs only the
 * update below and the dot product.
 *
 * Vectors are DEVICE arrays of n FP32 values; scalars marked "device" are
 * FP64 values in device memory, so a sequence of calls needs no host round
 * trip.  Dot products accumulate in FP64 with a fixed grid and a fixed
 * summation order (bitwise reproducible run to run).  Calls validate
 * synchronously, enqueue on `stream` (hipStream_t, NULL = default) and
 * return; none allocates device memory.  ws: fwi_vec_workspace_size bytes,
 * 256-byte aligned.  Errors: FWI_EINVAL (bad size or null pointer),
 * FWI_ENOMEM (workspace too small), FWI_EHIP (launch failure).
 */
#ifndef FWI_MI355X_OPT_H
#define FWI_MI355X_OPT_H

#include <stddef.h>
#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace of the calls below for vectors of n values (n in [1, 2^31)). */
int fwi_vec_workspace_size(int64_t n, size_t *bytes);

/* *out (device) = x^T y. */
int fwi_vec_dot(int64_t n, const float *x, const float *y, double *out, void *ws,
                size_t ws_bytes, void *stream);

/* y = a * s * x + b * y with s = *ad (device) when ad is not NULL, else 1.
 * Evaluated in FP64 per element, rounded once; x may equal y; with b = 0
 * y is only written (a copy or scaling into fresh memory). */
int fwi_vec_update(int64_t n, double a, const double *ad, const float *x, double b, float *y,
                   void *stream);

/* For a new pair (s, y): *rho = 1 / y^T s and *gamma = s^T y / y^T y
 * (device; gamma is the scaling of an identity H0, Nocedal and Wright eq.
 * 7.20).  The caller keeps the pair only if y^T s > 0. */
int fwi_lbfgs_pair(int64_t n, const float *s, const float *y, double *rho, double *gamma,
                   void *ws, size_t ws_bytes, void *stream);

/* The two loops over m stored pairs S[slot][n], Y[slot][n] with rho[slot]
 * and alpha[slot] (device), the slots visited in the order given by the
 * HOST array order[m] (newest first; loop 2 walks it backwards).  q and r
 * are updated in place.  m in [0, 64]; slots index S, Y, rho and alpha. */
int fwi_lbfgs_loop1(int64_t n, int m, const int *order, const float *S, const float *Y,
                    const double *rho, float *q, double *alpha, void *ws, size_t ws_bytes,
                    void *stream);
int fwi_lbfgs_loop2(int64_t n, int m, const int *order, const float *S, const float *Y,
                    const double *rho, const double *alpha, float *r, void *ws, size_t ws_bytes,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_MI355X_OPT_H */

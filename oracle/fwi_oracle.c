/*
 * Plain FP64 CPU oracle for the acoustic Gauss-Newton Hessian-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link or call
 * this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark use it.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes (paper Section 2, eq. (1) for the PDE with m the wave
 * speed; the data model and misfit of Section 2; the gradient eq. "grad" of
 * Section 2.1 with F the Born operator and F* migration; the misfit Hessian
 * of Section 3, applied matrix-free with one Born and one adjoint solve per
 * source):
 *
 *   forward   d_s = R u_s(m)                         for every shot s
 *   born      J v        (exact derivative of the discrete forward map)
 *   adjoint   J^T r      (its exact transpose)
 *   misfit    Phi = 1/2 inv_noise_var sum_s |d_s - dobs_s|^2,
 *             grad = inv_noise_var sum_s J_s^T (d_s - dobs_s)
 *   gn_hvp    H v = inv_noise_var sum_s J_s^T J_s v
 *
 * The paper leaves the discretisation open (Section 4.2 names finite
 * differences and fixes no scheme); the scheme below is the reading adopted
 * here:
 *   - padded grid NZp x NXp = (nz+2nb) x (nx+2nb), zero outside it;
 *   - L = 8th-order centred second differences in x and z (spacing dx);
 *   - sponge kappa = kappa_max((dx_pad/nb)^2 + (dz_pad/nb)^2), where dx_pad,
 *     dz_pad count cells into the pad; a = 1/(1+kappa),
 *     b = (1-kappa)/(1+kappa), c = (dt m_pad)^2/(1+kappa);
 *   - m_pad = P m replicates edge values into the pad; P^T folds them back;
 *   - source f^n = s(n dt)/dx^2 at the shot node; receivers sample nodes;
 *   - u^{-1} = u^0 = 0;  w^n = L u^n + f^n;
 *     u^{n+1} = 2a u^n - b u^{n-1} + c w^n,  n = 0..nt-2;  d^n = R u^n.
 *
 * Every shot keeps its whole forward history in memory (nt x NZp x NXp
 * doubles): no checkpointing, no blocking, no fusion.  Shots run in
 * parallel with OpenMP; per-shot results are summed in shot order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t nx, nz, nb, nt;
  int32_t ns, nr;
  int32_t nthreads; /* 0: OpenMP default */
  int32_t pad_;
  double dx, dt, kappa_max, inv_noise_var;
  const int32_t *src_zx; /* ns x (iz, ix) */
  const int32_t *rec_zx; /* nr x (iz, ix) */
  const double *wavelet; /* nt */
} orc_geom;

/* Standard centred 8th-order weights for the second derivative. */
static const double FD2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0,
                              -1.0 / 560.0};

#define NZP(g) ((g)->nz + 2 * (g)->nb)
#define NXP(g) ((g)->nx + 2 * (g)->nb)

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ---------------------------------------------------------------- grid ops */

/* (L u) on an nzp x nxp grid with zero values outside it. */
void orc_laplacian(int nzp, int nxp, double dx, const double *u, double *out) {
  for (int i = 0; i < nzp; ++i)
    for (int j = 0; j < nxp; ++j) {
      double s = 0.0;
      for (int k = -4; k <= 4; ++k) {
        double ck = FD2[k < 0 ? -k : k];
        double uz = (i + k >= 0 && i + k < nzp) ? u[(size_t)(i + k) * nxp + j] : 0.0;
        double ux = (j + k >= 0 && j + k < nxp) ? u[(size_t)i * nxp + j + k] : 0.0;
        s += ck * (uz + ux);
      }
      out[(size_t)i * nxp + j] = s / (dx * dx);
    }
}

/* m_pad = P m: every pad cell takes the value of the nearest model cell. */
static void pad_model(const orc_geom *g, const double *m, double *mp) {
  int nzp = NZP(g), nxp = NXP(g);
  for (int i = 0; i < nzp; ++i)
    for (int j = 0; j < nxp; ++j) {
      int iz = clampi(i - g->nb, 0, g->nz - 1), ix = clampi(j - g->nb, 0, g->nx - 1);
      mp[(size_t)i * nxp + j] = m[(size_t)iz * g->nx + ix];
    }
}

/* P^T: every padded cell's value is added to the model cell it copies. */
static void fold_pad(const orc_geom *g, const double *gp, double *gm) {
  int nzp = NZP(g), nxp = NXP(g);
  memset(gm, 0, sizeof(double) * (size_t)g->nz * g->nx);
  for (int i = 0; i < nzp; ++i)
    for (int j = 0; j < nxp; ++j) {
      int iz = clampi(i - g->nb, 0, g->nz - 1), ix = clampi(j - g->nb, 0, g->nx - 1);
      gm[(size_t)iz * g->nx + ix] += gp[(size_t)i * nxp + j];
    }
}

/* Sponge damping at padded cell (i, j). */
static double sponge_kappa(const orc_geom *g, int i, int j) {
  int nzp = NZP(g), nxp = NXP(g), nb = g->nb;
  if (nb <= 0) return 0.0;
  int dxc = 0, dzc = 0;
  if (nb - j > dxc) dxc = nb - j;
  if (j - (nxp - 1 - nb) > dxc) dxc = j - (nxp - 1 - nb);
  if (nb - i > dzc) dzc = nb - i;
  if (i - (nzp - 1 - nb) > dzc) dzc = i - (nzp - 1 - nb);
  double fx = (double)dxc / nb, fz = (double)dzc / nb;
  return g->kappa_max * (fx * fx + fz * fz);
}

typedef struct {
  double *a, *b, *c, *mp; /* each NZp*NXp */
} coefs;

static void make_coefs(const orc_geom *g, const double *m, coefs *k) {
  int nzp = NZP(g), nxp = NXP(g);
  size_t np = (size_t)nzp * nxp;
  k->a = malloc(np * sizeof(double));
  k->b = malloc(np * sizeof(double));
  k->c = malloc(np * sizeof(double));
  k->mp = malloc(np * sizeof(double));
  pad_model(g, m, k->mp);
  for (int i = 0; i < nzp; ++i)
    for (int j = 0; j < nxp; ++j) {
      size_t p = (size_t)i * nxp + j;
      double kap = sponge_kappa(g, i, j);
      double vdt = g->dt * k->mp[p];
      k->a[p] = 1.0 / (1.0 + kap);
      k->b[p] = (1.0 - kap) / (1.0 + kap);
      k->c[p] = vdt * vdt / (1.0 + kap);
    }
}

static void free_coefs(coefs *k) {
  free(k->a); free(k->b); free(k->c); free(k->mp);
}

static size_t src_node(const orc_geom *g, int s) {
  int i = g->src_zx[2 * s] + g->nb, j = g->src_zx[2 * s + 1] + g->nb;
  return (size_t)i * NXP(g) + j;
}

static size_t rec_node(const orc_geom *g, int r) {
  int i = g->rec_zx[2 * r] + g->nb, j = g->rec_zx[2 * r + 1] + g->nb;
  return (size_t)i * NXP(g) + j;
}

/* w^n = L u^n + f^n for shot s. */
static void forcing(const orc_geom *g, int s, int n, const double *u, double *w) {
  orc_laplacian(NZP(g), NXP(g), g->dx, u, w);
  w[src_node(g, s)] += g->wavelet[n] / (g->dx * g->dx);
}

/* --------------------------------------------------------------- per shot */

/* Forward solve for one shot.  hist (nt x Np) receives u^0..u^{nt-1}; d
 * (nt x nr) receives R u^n. */
static void forward_shot(const orc_geom *g, const coefs *k, int s, double *hist, double *d) {
  size_t np = (size_t)NZP(g) * NXP(g);
  double *w = malloc(np * sizeof(double));
  memset(hist, 0, np * sizeof(double)); /* u^0 = 0 */
  for (int n = 0; n + 1 < g->nt; ++n) {
    const double *un = hist + (size_t)n * np;
    const double *um = n > 0 ? hist + (size_t)(n - 1) * np : NULL; /* u^{-1} = 0 */
    double *up = hist + (size_t)(n + 1) * np;
    forcing(g, s, n, un, w);
    for (size_t p = 0; p < np; ++p)
      up[p] = 2.0 * k->a[p] * un[p] - (um ? k->b[p] * um[p] : 0.0) + k->c[p] * w[p];
  }
  for (int n = 0; n < g->nt; ++n)
    for (int r = 0; r < g->nr; ++r) d[(size_t)n * g->nr + r] = hist[(size_t)n * np + rec_node(g, r)];
  free(w);
}

/* Born solve for one shot, given the forward history: dd = J_s v. */
static void born_shot(const orc_geom *g, const coefs *k, int s, const double *hist,
                      const double *v, double *dd) {
  int nzp = NZP(g), nxp = NXP(g);
  size_t np = (size_t)nzp * nxp;
  double *vp = malloc(np * sizeof(double)), *dc = malloc(np * sizeof(double));
  double *w = malloc(np * sizeof(double)), *lq = malloc(np * sizeof(double));
  double *q0 = calloc(np, sizeof(double)), *q1 = calloc(np, sizeof(double));
  double *q2 = malloc(np * sizeof(double));
  pad_model(g, v, vp);
  /* c = dt^2 m^2 / (1+kappa)  =>  dc/dm_pad = 2 c / m_pad */
  for (size_t p = 0; p < np; ++p) dc[p] = 2.0 * k->c[p] / k->mp[p] * vp[p];
  for (int r = 0; r < g->nr; ++r) dd[r] = 0.0; /* delta u^0 = 0 */
  /* q0 = du^{n-1}, q1 = du^n, q2 = du^{n+1} */
  for (int n = 0; n + 1 < g->nt; ++n) {
    forcing(g, s, n, hist + (size_t)n * np, w);
    orc_laplacian(nzp, nxp, g->dx, q1, lq);
    for (size_t p = 0; p < np; ++p)
      q2[p] = 2.0 * k->a[p] * q1[p] - k->b[p] * q0[p] + k->c[p] * lq[p] + dc[p] * w[p];
    for (int r = 0; r < g->nr; ++r) dd[(size_t)(n + 1) * g->nr + r] = q2[rec_node(g, r)];
    double *t = q0; q0 = q1; q1 = q2; q2 = t;
  }
  free(vp); free(dc); free(w); free(lq); free(q0); free(q1); free(q2);
}

/* Adjoint solve and zero-lag imaging for one shot: gp (padded grid) = the
 * padded-grid image sum_n (2c/m_pad) w^n lambda^{n+1}, before P^T.
 *   lambda^{nt} = lambda^{nt+1} = 0,
 *   lambda^k = R^T r^k + 2a lambda^{k+1} + L(c lambda^{k+1}) - b lambda^{k+2},
 *   k = nt-1..1. */
static void adjoint_shot(const orc_geom *g, const coefs *k, int s, const double *hist,
                         const double *r, double *gp) {
  int nzp = NZP(g), nxp = NXP(g);
  size_t np = (size_t)nzp * nxp;
  double *l1 = calloc(np, sizeof(double)), *l2 = calloc(np, sizeof(double));
  double *l0 = malloc(np * sizeof(double)), *cl = malloc(np * sizeof(double));
  double *lc = malloc(np * sizeof(double)), *w = malloc(np * sizeof(double));
  memset(gp, 0, np * sizeof(double));
  /* l1 = lambda^{k+1}, l2 = lambda^{k+2}, l0 = lambda^k */
  for (int kk = g->nt - 1; kk >= 1; --kk) {
    for (size_t p = 0; p < np; ++p) cl[p] = k->c[p] * l1[p];
    orc_laplacian(nzp, nxp, g->dx, cl, lc);
    for (size_t p = 0; p < np; ++p) l0[p] = 2.0 * k->a[p] * l1[p] + lc[p] - k->b[p] * l2[p];
    for (int q = 0; q < g->nr; ++q) l0[rec_node(g, q)] += r[(size_t)kk * g->nr + q];
    /* image term n = kk-1 uses w^{kk-1} and lambda^{kk} */
    forcing(g, s, kk - 1, hist + (size_t)(kk - 1) * np, w);
    for (size_t p = 0; p < np; ++p) gp[p] += 2.0 * k->c[p] / k->mp[p] * w[p] * l0[p];
    double *t = l2; l2 = l1; l1 = l0; l0 = t;
  }
  free(l0); free(l1); free(l2); free(cl); free(lc); free(w);
}

/* ------------------------------------------------------------ public calls */

static void set_threads(const orc_geom *g) {
#ifdef _OPENMP
  if (g->nthreads > 0) omp_set_num_threads(g->nthreads);
#else
  (void)g;
#endif
}

static size_t hist_bytes(const orc_geom *g) {
  return (size_t)g->nt * NZP(g) * NXP(g) * sizeof(double);
}

/* d[ns][nt][nr] */
int orc_forward(const orc_geom *g, const double *m, double *d) {
  coefs k;
  make_coefs(g, m, &k);
  set_threads(g);
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
  for (int s = 0; s < g->ns; ++s) {
    double *hist = malloc(hist_bytes(g));
    if (!hist) { fail = 1; continue; }
    forward_shot(g, &k, s, hist, d + (size_t)s * g->nt * g->nr);
    free(hist);
  }
  free_coefs(&k);
  return fail ? -3 : 0;
}

/* v[nz][nx] -> dd[ns][nt][nr] */
int orc_born(const orc_geom *g, const double *m, const double *v, double *dd) {
  coefs k;
  make_coefs(g, m, &k);
  set_threads(g);
  int fail = 0;
  double *tmp = malloc((size_t)g->ns * g->nt * g->nr * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
  for (int s = 0; s < g->ns; ++s) {
    double *hist = malloc(hist_bytes(g));
    if (!hist) { fail = 1; continue; }
    forward_shot(g, &k, s, hist, tmp + (size_t)s * g->nt * g->nr);
    born_shot(g, &k, s, hist, v, dd + (size_t)s * g->nt * g->nr);
    free(hist);
  }
  free(tmp);
  free_coefs(&k);
  return fail ? -3 : 0;
}

/* r[ns][nt][nr] -> g[nz][nx] = sum_s J_s^T r_s (no noise weighting) */
static int adjoint_sum(const orc_geom *g, const coefs *k, const double *r, double *out,
                       const double *dobs, double *phi_shot) {
  size_t np = (size_t)NZP(g) * NXP(g);
  size_t nd = (size_t)g->nt * g->nr;
  double *gps = malloc((size_t)g->ns * np * sizeof(double));
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
  for (int s = 0; s < g->ns; ++s) {
    double *hist = malloc(hist_bytes(g));
    double *d = malloc(nd * sizeof(double));
    if (!hist || !d) { fail = 1; free(hist); free(d); continue; }
    forward_shot(g, k, s, hist, d);
    const double *rs;
    if (dobs) { /* residual d - dobs and its misfit */
      double acc = 0.0;
      for (size_t q = 0; q < nd; ++q) {
        d[q] -= dobs[(size_t)s * nd + q];
        acc += d[q] * d[q];
      }
      phi_shot[s] = 0.5 * acc;
      rs = d;
    } else {
      rs = r + (size_t)s * nd;
    }
    adjoint_shot(g, k, s, hist, rs, gps + (size_t)s * np);
    free(hist); free(d);
  }
  double *gp = calloc(np, sizeof(double));
  for (int s = 0; s < g->ns; ++s)
    for (size_t p = 0; p < np; ++p) gp[p] += gps[(size_t)s * np + p];
  fold_pad(g, gp, out);
  free(gp); free(gps);
  return fail ? -3 : 0;
}

int orc_adjoint(const orc_geom *g, const double *m, const double *r, double *out) {
  coefs k;
  make_coefs(g, m, &k);
  set_threads(g);
  int rc = adjoint_sum(g, &k, r, out, NULL, NULL);
  free_coefs(&k);
  return rc;
}

int orc_misfit_grad(const orc_geom *g, const double *m, const double *dobs, double *phi,
                    double *grad) {
  coefs k;
  make_coefs(g, m, &k);
  set_threads(g);
  double *ps = calloc((size_t)g->ns, sizeof(double));
  int rc = adjoint_sum(g, &k, NULL, grad, dobs, ps);
  double acc = 0.0;
  for (int s = 0; s < g->ns; ++s) acc += ps[s];
  *phi = g->inv_noise_var * acc;
  size_t nm = (size_t)g->nz * g->nx;
  for (size_t p = 0; p < nm; ++p) grad[p] *= g->inv_noise_var;
  free(ps);
  free_coefs(&k);
  return rc;
}

/* v[nz][nx] -> hv[nz][nx] = inv_noise_var sum_s J_s^T J_s v */
int orc_gn_hvp(const orc_geom *g, const double *m, const double *v, double *hv) {
  coefs k;
  make_coefs(g, m, &k);
  set_threads(g);
  size_t np = (size_t)NZP(g) * NXP(g);
  size_t nd = (size_t)g->nt * g->nr;
  double *gps = malloc((size_t)g->ns * np * sizeof(double));
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
  for (int s = 0; s < g->ns; ++s) {
    double *hist = malloc(hist_bytes(g));
    double *d = malloc(nd * sizeof(double)), *dd = malloc(nd * sizeof(double));
    if (!hist || !d || !dd) { fail = 1; free(hist); free(d); free(dd); continue; }
    forward_shot(g, &k, s, hist, d);
    born_shot(g, &k, s, hist, v, dd);
    adjoint_shot(g, &k, s, hist, dd, gps + (size_t)s * np);
    free(hist); free(d); free(dd);
  }
  double *gp = calloc(np, sizeof(double));
  for (int s = 0; s < g->ns; ++s)
    for (size_t p = 0; p < np; ++p) gp[p] += gps[(size_t)s * np + p];
  fold_pad(g, gp, hv);
  size_t nm = (size_t)g->nz * g->nx;
  for (size_t p = 0; p < nm; ++p) hv[p] *= g->inv_noise_var;
  free(gp); free(gps);
  free_coefs(&k);
  return fail ? -3 : 0;
}

/* Full forward wavefield history of one shot (for the Green's-function and
 * energy checks): hist[nt][NZp][NXp]. */
int orc_wavefield(const orc_geom *g, const double *m, int shot, double *hist) {
  coefs k;
  make_coefs(g, m, &k);
  double *d = malloc((size_t)g->nt * g->nr * sizeof(double) + 8);
  forward_shot(g, &k, shot, hist, d);
  free(d);
  free_coefs(&k);
  return 0;
}

/* The padded coefficient fields (for inspection by tests). */
int orc_coefficients(const orc_geom *g, const double *m, double *a, double *b, double *c,
                     double *mp) {
  coefs k;
  make_coefs(g, m, &k);
  size_t np = (size_t)NZP(g) * NXP(g);
  memcpy(a, k.a, np * sizeof(double));
  memcpy(b, k.b, np * sizeof(double));
  memcpy(c, k.c, np * sizeof(double));
  memcpy(mp, k.mp, np * sizeof(double));
  free_coefs(&k);
  return 0;
}

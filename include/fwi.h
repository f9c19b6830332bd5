/*
 * fwi.h -- C ABI of the MI355X (gfx950) library for matrix-free Gauss-Newton
 * Hessian-vector products of 2-D constant-density acoustic full-waveform
 * inversion.
 *
 * The operations follow the paper's statement of the problem:
 *   - eq. (1), Section 2: (1/m^2) u_tt - lap u = s(t) delta(x - x_s), with m
 *     the wave speed; the forward map f records u at the receivers;
 *   - Section 2: data model d = f(m) + eta, eta ~ N(0, sigma^2 I), and the
 *     data misfit 1/2 |f(m) - d|^2 weighted by 1/sigma^2;
 *   - eq. "grad", Section 2.1: the misfit gradient F* Gamma^-1 (f(m) - d),
 *     F = grad f the Born operator and F* its adjoint (migration);
 *   - Section 3: the misfit Hessian H_d applied matrix-free to vectors, one
 *     Born and one adjoint solve per source (plus the forward solve at a new
 *     model), as the Gauss-Newton normal operator F* Gamma^-1 F.
 *
 * Discretisation (the paper leaves it open): padded grid of (nz+2nb) rows by
 * (nx+2nb) columns with zero values outside it; 8th-order centred Laplacian;
 * second-order leapfrog in time; quadratic absorbing sponge in the nb pad
 * cells, kappa = kappa_max((cells into the pad in x / nb)^2 + (... in z / nb)^2);
 * velocity in the pad replicated from the nearest model cell (its derivative
 * folds back onto the edge cells); point source s(n dt)/dx^2 at the shot node;
 * receivers sample nodes; u^{-1} = u^0 = 0.  All results are exact
 * derivatives of this discrete forward map (discretise-then-differentiate).
 *
 * Memory and ownership.  The library never allocates device memory.  The
 * caller owns (1) the plan's device block, bound once with fwi_plan_bind(),
 * and (2) a workspace per call, sized by fwi_workspace_size(); all array
 * arguments of the compute calls are DEVICE pointers to contiguous row-major
 * FP32 arrays, except `phi`, a device double.  A plan copies the host
 * geometry it is given; it is not thread-safe: one plan per stream.
 *
 * Layouts (x is the fastest axis):
 *   model-space arrays m, v, g, hv:   [B][nz][nx]
 *   data-space arrays d, dd, r, dobs: [B][ns][nt][nr] (receiver fastest)
 *
 * Asynchrony.  Every compute call validates its arguments synchronously,
 * enqueues kernels on `stream` (a hipStream_t; NULL = the default stream) and
 * returns; outputs are valid once the stream has completed.  The enqueued
 * work contains kernel launches only (no memset, no host copies), so a call
 * can be captured into a hipGraph and replayed, provided the plan's device
 * block and the workspace stay where they are.
 *
 * Errors.  Return codes are FWI_OK or a negative FWI_E* value; nothing aborts
 * or throws across the ABI.  Argument and size errors are reported
 * synchronously with a message retrievable by fwi_last_error() (thread
 * local).  Data-dependent conditions found on the device (m <= 0 or not
 * finite, Courant number above the stability limit, non-finite output) are
 * recorded in the call's own status word, the first 4 bytes of its
 * workspace (cleared when the call starts, read by fwi_workspace_status()),
 * and OR-ed into the plan's status word (read and cleared by fwi_status()).
 * Calls that run concurrently on separate workspaces therefore keep separate
 * status words.
 */
#ifndef FWI_MI355X_H
#define FWI_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWI_ABI_VERSION 1

enum {
  FWI_OK = 0,
  FWI_EINVAL = -1,     /* bad argument, shape or position */
  FWI_EUNSTABLE = -2,  /* reserved: reported through the status word */
  FWI_ENOMEM = -3,     /* workspace or device block too small */
  FWI_EHIP = -4,       /* a HIP runtime call failed */
  FWI_ENUMERIC = -5,   /* reserved: reported through the status word */
  FWI_EUNBOUND = -6    /* plan has no device block yet (fwi_plan_bind) */
};

/* Bits of the device status word (fwi_status). */
enum {
  FWI_STATUS_BAD_MODEL = 1,   /* some m <= 0 or not finite */
  FWI_STATUS_CFL = 2,         /* max(m) dt / dx above 0.5546 */
  FWI_STATUS_NONFINITE = 4    /* an output held inf or nan */
};

/* Operations, for fwi_workspace_size. */
enum {
  FWI_OP_FORWARD = 0,
  FWI_OP_BORN = 1,
  FWI_OP_ADJOINT = 2,
  FWI_OP_MISFIT_GRAD = 3,
  FWI_OP_GN_HVP = 4,
  FWI_OP_MISFIT = 5,
  FWI_OP_GRAD_HVP = 6
};

typedef struct fwi_plan fwi_plan;

/* Host-side description of one problem.  All pointers are HOST pointers and
 * are copied by fwi_plan_create. */
typedef struct {
  int32_t nx, nz;          /* model grid: nz rows (depth) x nx columns, nx fastest */
  int32_t nb;              /* absorbing cells padded on each side (>= 0) */
  int32_t nt;              /* time samples n = 0..nt-1 (>= 2) */
  float dx;                /* grid spacing in metres (dz = dx) */
  float dt;                /* time step in seconds, fixed by the plan */
  float kappa_max;         /* peak sponge damping (>= 0, < 1/2) */
  int32_t ns;              /* shots */
  const int32_t *src_zx;   /* ns x (iz, ix) model cells */
  int32_t nr;              /* receivers, shared by all shots */
  const int32_t *rec_zx;   /* nr x (iz, ix) model cells */
  const float *wavelet;    /* nt samples s(n dt) */
  int32_t ckpt_every;      /* K: forward checkpoint interval in steps (>= 1); the
                              reverse sweep recomputes w^n (Section 2.1: the adjoint
                              needs the forward wavefield) segment by segment from
                              the checkpoints.  0: history mode -- the forward sweep
                              keeps every w^n, n = 0..nt-2, in the workspace and
                              nothing is recomputed (one field update per shot and
                              step fewer; the adjoint-bearing workspaces grow to
                              (nt-1) ns fields, see fwi_workspace_size) */
  double inv_noise_var;    /* 1/sigma^2 weighting of the misfit */
} fwi_geometry;

int fwi_abi_version(void);

/* Validate `g` and build the host plan (receiver/tile tables).  No HIP
 * call.  Returns FWI_EINVAL for a bad size, spacing, position or K. */
int fwi_plan_create(const fwi_geometry *g, fwi_plan **out);
void fwi_plan_destroy(fwi_plan *p);

/* Size in bytes of the plan's device block (tables, positions, status). */
int fwi_plan_device_bytes(const fwi_plan *p, size_t *bytes);

/* Upload the plan's tables into caller-owned device memory `dev` (at least
 * fwi_plan_device_bytes, 256-byte aligned) and keep the pointer.  Blocks
 * until the copy is done.  Must precede every compute call. */
int fwi_plan_bind(fwi_plan *p, void *dev, size_t bytes, void *stream);

/* Workspace bytes for operation `op` with `batch` vectors (1 for
 * FORWARD / MISFIT_GRAD).  Workspaces must be 256-byte aligned. */
int fwi_workspace_size(const fwi_plan *p, int op, int batch, size_t *bytes);

/* Tuning options of a plan: how the time loops are split into kernel
 * launches.  None changes what is computed; options marked (*) change the
 * order of FP32 additions in the images, so results can differ in the last
 * bits between settings (every setting is deterministic).  Defaults are the
 * fastest measured on MI355X for the workloads of this library.  Changing an
 * option can change fwi_workspace_size: query it again afterwards. */
enum {
  FWI_OPT_TWO_STEP_FORWARD = 0, /* 0/1: forward and recompute kernels advance two time
                                   steps per launch (default 0; needs an even K or
                                   history mode, as the two below) */
  FWI_OPT_TWO_STEP_BORN = 1,    /* 0/1: the same for forward + Born (default 1) */
  FWI_OPT_TWO_STEP_ADJOINT = 2, /* 0/1: the same for the adjoint (default 1) (*) */
  FWI_OPT_ADJ_VECTORS = 3,      /* right-hand sides per two-step adjoint workgroup,
                                   1..4; 0 (default): pairs (the last group ragged for
                                   odd counts), one group for 1 or 3 */
  FWI_OPT_ADJ_SHOT_GROUP = 4,   /* shots summed per adjoint workgroup; 0 (default):
                                   the largest power of two <= 16 that keeps >= 1536
                                   two-step (>= 4096 one-step) workgroups (*) */
  FWI_OPT_STEP_ORDER = 5,       /* workgroup order of the one-step forward kernels:  */
  FWI_OPT_BORN_ORDER = 6,       /*   0 shot-major (default), 1 tile-major, 2 blocked */
  FWI_OPT_ADJ_ORDER = 7,        /* the same for the one-step adjoint                  */
  FWI_OPT_BLOCK_X = 8,          /* tiles per block of the blocked order, 1..64 (default 2); */
  FWI_OPT_BLOCK_Z = 9,          /*   set before fwi_plan_bind                               */
  FWI_OPT_LDS_POISON = 10,      /* 0/1, debug (default 0): every stencil workgroup fills its
                                   LDS with NaN before staging, so a read of an entry no
                                   thread wrote (a missing halo value or barrier) makes the
                                   outputs NaN (status bit FWI_STATUS_NONFINITE) */
  FWI_OPT_COUNT = 11
};

/* Set option `option` to `value`.  FWI_EINVAL for an unknown option, a value
 * out of range, or a block size after fwi_plan_bind.  Takes effect from the
 * next compute call; not while a call on this plan is still being enqueued. */
int fwi_plan_set_option(fwi_plan *p, int option, int value);
int fwi_plan_get_option(const fwi_plan *p, int option, int *value);

/* Padded-grid geometry the kernels use (for tools and tests):
 * dims[0..5] = NZp, NXp, row pitch (floats), tile rows, tile columns, K
 * (nt - 1 in history mode). */
int fwi_plan_dims(const fwi_plan *p, int32_t dims[6]);

/* Forward map (Section 2): d[ns][nt][nr] = R u_s^n for every shot. */
int fwi_forward(fwi_plan *p, const float *m, float *d, void *ws, size_t ws_bytes,
                void *stream);

/* Born modelling (Section 2.1, F = grad f): dd[B][ns][nt][nr] = J v_b for the
 * B model perturbations v[B][nz][nx]. */
int fwi_born(fwi_plan *p, const float *m, const float *v, int B, float *dd, void *ws,
             size_t ws_bytes, void *stream);

/* Migration (Section 2.1, F*): g[B][nz][nx] = sum_s J_s^T r_{b,s} for the B
 * data vectors r[B][ns][nt][nr] (no noise weighting). */
int fwi_adjoint(fwi_plan *p, const float *m, const float *r, int B, float *g, void *ws,
                size_t ws_bytes, void *stream);

/* Forward map that also leaves in `ws` the coefficients and forward
 * checkpoints (every K steps) that fwi_adjoint_resume needs: d as
 * fwi_forward.  `ws` must be sized for FWI_OP_ADJOINT with the largest batch
 * the later adjoint calls will use. */
int fwi_forward_keep(fwi_plan *p, const float *m, float *d, void *ws, size_t ws_bytes,
                     void *stream);

/* Migration g[B][nz][nx] = sum_s J_s^T r_{b,s} (as fwi_adjoint) at the model
 * of the last fwi_forward_keep on this workspace, recomputing the forward
 * wavefield segment by segment from its checkpoints instead of solving the
 * forward again.  May be repeated; the checkpoints are left intact. */
int fwi_adjoint_resume(fwi_plan *p, const float *r, int B, float *g, void *ws,
                       size_t ws_bytes, void *stream);

/* Data misfit only (the quantity an MCMC proposal is accepted on, Section
 * 2.3): *phi (device double) = 1/2 inv_noise_var sum |d(m) - dobs|^2.  One
 * forward solve, no checkpoints. */
int fwi_misfit(fwi_plan *p, const float *m, const float *dobs, double *phi, void *ws,
               size_t ws_bytes, void *stream);

/* Data misfit and its gradient (Section 2.1, eq. grad, misfit half):
 * *phi (device double) = 1/2 inv_noise_var sum |d(m) - dobs|^2,
 * g[nz][nx] = inv_noise_var sum_s J_s^T (d_s(m) - dobs_s). */
int fwi_misfit_grad(fwi_plan *p, const float *m, const float *dobs, double *phi, float *g,
                    void *ws, size_t ws_bytes, void *stream);

/* Gauss-Newton misfit Hessian times B vectors (Section 3):
 * hv[B][nz][nx] = inv_noise_var sum_s J_s^T J_s v_b.  The forward solve and
 * its recomputation are shared by the whole batch. */
int fwi_gn_hvp(fwi_plan *p, const float *m, const float *v, int B, float *hv, void *ws,
               size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fwi_gn_hvp
 * with its workspace in a fixed array of FWI_NOALLOC_MAX_BYTES that the
 * library holds on every GPU it runs on (until the process ends), instead of
 * caller memory.  Same arguments, results and errors as fwi_gn_hvp, without
 * ws; FWI_ENOMEM (with a message) when fwi_workspace_size(FWI_OP_GN_HVP, B)
 * exceeds the array -- problems about the size of a 128 x 128 grid with 4
 * shots and 500 steps fit up to B = 5.  Calls no allocating routine.  All
 * calls on one GPU share that GPU's array: calls that overlap in time on one
 * GPU (other streams, other threads, other plans) race and must not be
 * issued.  The array keeps the last call's contents; every call clears what
 * it needs. */
#define FWI_NOALLOC_MAX_BYTES (64u << 20)
int fwi_gn_hvp_noalloc(fwi_plan *p, const float *m, const float *v, int B, float *hv,
                       void *stream);

/* Misfit, gradient and B Gauss-Newton products at one model, in one pass
 * (Section 3: a Hessian product reuses the forward wavefield of the gradient
 * at the same model, leaving two solves per source and vector).  Outputs are
 * those of fwi_misfit_grad (phi, g) and fwi_gn_hvp (hv) at m; one forward
 * solve with the B Born fields records both the data and J v_b, one
 * recompute serves the adjoint of the residual and of the B Born data
 * together.  Results agree with the separate calls up to the grouping of the
 * FP64 shot sums.  ws: fwi_workspace_size(FWI_OP_GRAD_HVP, B). */
int fwi_misfit_grad_hvp(fwi_plan *p, const float *m, const float *dobs, const float *v, int B,
                        double *phi, float *g, float *hv, void *ws, size_t ws_bytes,
                        void *stream);

/* Per-kernel timing telemetry.  While enabled, every launch of the three
 * stencil kernels is bracketed by a pair of HIP events recorded on the
 * call's stream (do not enable while the stream is being captured).
 * fwi_profile_read synchronises on the recorded events and returns, for one
 * kernel kind, the summed duration in milliseconds and the launch count since
 * the last reset.  Kinds: */
enum {
  FWI_KERNEL_STEP = 0,       /* forward (or recompute) time step */
  FWI_KERNEL_STEP_BORN = 1,  /* forward + B Born fields time step */
  FWI_KERNEL_ADJOINT = 2     /* adjoint + imaging time step */
};
int fwi_profile_enable(fwi_plan *p, int enable);
/* Time steps one launch of kernel `kind` advances under this plan: 2 where
 * the temporally blocked form is used (it needs an even K), else 1. */
int fwi_kernel_steps(const fwi_plan *p, int kind, int32_t *steps);
int fwi_profile_read(fwi_plan *p, int kind, double *total_ms, int64_t *launches);
int fwi_profile_reset(fwi_plan *p);

/* Synchronise `stream`, return the device status word in *status and clear
 * it. */
int fwi_status(fwi_plan *p, void *stream, uint32_t *status);

/* Synchronise `stream` and return in *status the status bits of the last
 * compute call that used workspace `ws` (device pointer) -- the bits of that
 * call alone, whatever other calls on the plan have flagged.  The word is
 * left as it is (the next call on `ws` clears it). */
int fwi_workspace_status(const fwi_plan *p, const void *ws, void *stream, uint32_t *status);

const char *fwi_strerror(int code);
const char *fwi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWI_MI355X_H */

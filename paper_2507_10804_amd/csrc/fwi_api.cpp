// Host side of the C ABI declared in include/fwi.h: plan construction
// (validation, receiver/tile tables), workspace planning and the time loops
// of each operation.  The library never allocates device memory: tables live
// in a caller-owned device block, scratch in a caller-owned workspace.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fwi.h"
#include "fwi_internal.h"

namespace fwi {
hipError_t launch_step(const Geo &g, const DevTables &t, const StepArgs &a, bool born,
                       hipStream_t st);
hipError_t launch_adjoint(const Geo &g, const DevTables &t, const AdjArgs &a, hipStream_t st);
hipError_t launch_step2(const Geo &g, const DevTables &t, const Step2Args &a, bool born,
                        hipStream_t st);
hipError_t launch_adjoint2(const Geo &g, const DevTables &t, const Adj2Args &a, hipStream_t st);
hipError_t launch_setup(const Geo &g, const float *m, const float *v, int B, float *c,
                        float *s2m, float *dc, unsigned int *status, hipStream_t st);
hipError_t launch_fill(float *p, long long n, hipStream_t st);
hipError_t launch_fill64(double *p, long long n, hipStream_t st);
hipError_t launch_copy(float *dst, const float *src, long long n, hipStream_t st);
hipError_t launch_zero_t0(float *d, int count, int nt, int nr, hipStream_t st);
hipError_t launch_residual(float *d, const float *dobs, long long n, double *part, int nparts,
                           double scale, double *phi, hipStream_t st);
hipError_t launch_fold(const Geo &g, const double *img, int G, int Bst, int b0, int B,
                       double scale, float *out,
                       hipStream_t st);
hipError_t launch_check_finite(const float *p, long long n, unsigned int *status,
                               hipStream_t st);
hipError_t launch_status_open(unsigned int *status, hipStream_t st);
hipError_t launch_status_merge(const unsigned int *from, unsigned int *into, hipStream_t st);
}  // namespace fwi

using namespace fwi;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

constexpr size_t ALIGN = 256;
constexpr int NPARTS = 1024;  // FP64 partial sums of the misfit

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

}  // namespace

int fwi::set_error(int code, const std::string &msg) { return fail(code, msg); }

struct fwi_plan {
  Geo geo{};
  int K = 1, nseg = 1;
  // ckpt_every == 0: the forward sweep keeps every w^n in the workspace (one
  // segment of nt - 1 levels), so the reverse sweep recomputes nothing
  bool hist = false;
  float dx = 0, dt = 0;
  double inv_noise_var = 1.0;
  std::vector<float> wavelet;
  // device block image, in int32 words, and offsets into it
  std::vector<int> blk;
  size_t off_status = 0, off_src = 0, off_trp = 0, off_rloc = 0, off_rid = 0, off_tnp = 0,
         off_nloc = 0, off_ngidx = 0, off_nrp = 0, off_nrec = 0, off_order = 0;
  size_t off2[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // two-step tables
  // requested options (fwi_plan_set_option), indexed by FWI_OPT_*
  int opt[FWI_OPT_COUNT] = {0, 1, 1, 0, 0, 0, 0, 0, 2, 2, 0};
  // advance two time steps per launch, per kernel family: the requested
  // option where K is even (the checkpoint levels must fall on launch
  // boundaries), else single steps
  bool ts_fwd = false, ts_born = true, ts_adj = true;
  // vectors per two-step adjoint workgroup (1..4; 0 = by batch, see adj_nb)
  int adj_pair = 0;
  void apply_options() {
    // with the whole history kept no checkpoint level has to fall on a launch
    // boundary, so two-step launches are allowed for any K
    const bool even = hist || K % 2 == 0;
    ts_fwd = even && opt[FWI_OPT_TWO_STEP_FORWARD];
    ts_born = even && opt[FWI_OPT_TWO_STEP_BORN];
    ts_adj = even && opt[FWI_OPT_TWO_STEP_ADJOINT];
    adj_pair = opt[FWI_OPT_ADJ_VECTORS];
    adj_group_override = opt[FWI_OPT_ADJ_SHOT_GROUP];
    step_order = opt[FWI_OPT_STEP_ORDER];
    born_order = opt[FWI_OPT_BORN_ORDER];
    adj_order = opt[FWI_OPT_ADJ_ORDER];
    geo.poison = opt[FWI_OPT_LDS_POISON];
  }
  int adj_nb(int B) const {
    if (adj_pair > 0) return std::min(adj_pair, B);
    // pairs, the last group ragged for odd counts (1 and 3 vectors: one group);
    // measured fastest for 16, 17 and 64 right-hand sides
    return (B % 2 == 0 || B >= 5) ? 2 : B;
  }
  void *dev = nullptr;
  DevTables tabs{};
  int adj_group_override = 0;
  int step_order = 0, born_order = 0, adj_order = 0;  // workgroup orders
  // telemetry: event pairs per kernel kind, from a reusable pool
  bool profiling = false;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks[3];
  ~fwi_plan() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

namespace {

// Byte layout of one operation's workspace.
struct Layout {
  size_t c = 0, s2m = 0, dc = 0, u = 0, du = 0, dd = 0, dres = 0, part = 0, ckpt = 0,
         wseg = 0, mu = 0, img = 0, total = 0;
  int G = 1, group = 1;
};

// Element offset of the second field set (two-step launches alternate sets).
size_t set_stride(const Geo &g, int per_shot) { return (size_t)2 * g.ns * per_shot * g.fs; }

int adjoint_group(const fwi_plan *p, int B) {
  if (p->adj_group_override > 0) return std::min(p->adj_group_override, p->geo.ns);
  // As many shots per workgroup as keep enough workgroups in flight (fewer
  // partial-image updates, and each shot reuses the workgroup's coefficient
  // and image tiles), at most 16.  Two-step kernel (512 threads, two per CU):
  // at least 1536 workgroups, three rounds of the 512 slots.  Measured on
  // 921 x 301 with 64 shots (198 tiles), per two-step launch: one vector group
  // (B = 1 or 2) takes 177 / 158 / 157 / 181 us with groups of 2 / 4 / 8 / 16
  // (16 leaves 792 workgroups); nine groups (B + 1 = 17) 2120 / 1977 / 1949 us
  // with 4 / 8 / 16; 32 groups (B = 64) 7821 / 7322 / 7110 us.  One-step
  // kernel (256 threads): at least 4096 workgroups.
  const int nbg = p->ts_adj ? (B + p->adj_nb(B) - 1) / p->adj_nb(B) : B;
  const long long base = (long long)(p->ts_adj ? p->geo.ntiles2 : p->geo.ntiles) * nbg;
  const long long need = p->ts_adj ? 1536 : 4096;
  int group = 1;
  while (group < 16 && group * 2 <= p->geo.ns &&
         base * ((p->geo.ns + group * 2 - 1) / (group * 2)) >= need)
    group *= 2;
  return group;
}

Layout layout(const fwi_plan *p, int op, int B) {
  const Geo &g = p->geo;
  const size_t F = (size_t)g.fs * sizeof(float);
  const size_t ndata = (size_t)g.ns * g.nt * g.nr * sizeof(float);
  const bool fused = op == FWI_OP_GRAD_HVP;
  const bool needs_dc = op == FWI_OP_BORN || op == FWI_OP_GN_HVP || fused;
  const bool needs_adj = op == FWI_OP_ADJOINT || op == FWI_OP_MISFIT_GRAD ||
                         op == FWI_OP_GN_HVP || fused;
  // adjoint right-hand sides: the residual (gradient) and/or B Born data
  const int Badj = op == FWI_OP_MISFIT_GRAD ? 1 : fused ? B + 1 : B;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  take(sizeof(unsigned int));  // the call's status word, at offset 0
  L.c = take(F);
  L.s2m = take(F);
  if (needs_dc) L.dc = take(F * B);
  // two-step launches read one field set and write the other
  const size_t usets = (p->ts_fwd || p->ts_born) ? 2 : 1;
  const size_t dsets = p->ts_born ? 2 : 1, msets = p->ts_adj ? 2 : 1;
  L.u = take(F * 2 * g.ns * usets);
  // the Born fields are dead once the forward sweep is over: the adjoint
  // fields of a Hessian product reuse their memory
  const bool alias_mu = op == FWI_OP_GN_HVP || fused;
  if (needs_dc)
    L.du = take(F * 2 * g.ns *
                std::max((size_t)B * dsets, alias_mu ? (size_t)Badj * msets : (size_t)0));
  if (op == FWI_OP_GN_HVP || fused) L.dd = take(ndata * Badj);
  if (op == FWI_OP_MISFIT_GRAD || op == FWI_OP_MISFIT) L.dres = take(ndata);
  if (op == FWI_OP_MISFIT_GRAD || op == FWI_OP_MISFIT || fused)
    L.part = take(NPARTS * sizeof(double));
  if (needs_adj) {
    L.group = adjoint_group(p, Badj);
    L.G = (g.ns + L.group - 1) / L.group;
    L.ckpt = p->hist ? 0 : take(F * 2 * g.ns * p->nseg);
    L.wseg = take(F * g.ns * p->K);
    L.mu = alias_mu ? L.du : take(F * 2 * g.ns * Badj * msets);
    L.img = take((size_t)g.fs * sizeof(double) * L.G * Badj);
  }
  L.total = o;
  return L;
}

template <class T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(FWI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Status word of the call that uses workspace `ws` (its first word).
unsigned int *ws_status(void *ws) { return static_cast<unsigned int *>(ws); }

int check_call(const fwi_plan *p, int op, int B, const void *ws, size_t ws_bytes) {
  if (!p) return fail(FWI_EINVAL, "plan is null");
  if (!p->dev) return fail(FWI_EUNBOUND, "plan has no device block: call fwi_plan_bind first");
  if (B < 1 || B > 4096) return fail(FWI_EINVAL, "batch must be in [1, 4096]");
  const size_t need = layout(p, op, B).total;
  if (!ws || ws_bytes < need)
    return fail(FWI_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN)
    return fail(FWI_EINVAL, "workspace must be 256-byte aligned");
  return FWI_OK;
}

float src_amp(const fwi_plan *p, int n) { return p->wavelet[n] / (p->dx * p->dx); }

hipError_t next_event(fwi_plan *p, hipEvent_t *e) {
  if (p->pool_used == p->pool.size()) {
    hipEvent_t ev;
    hipError_t rc = hipEventCreate(&ev);
    if (rc != hipSuccess) return rc;
    p->pool.push_back(ev);
  }
  *e = p->pool[p->pool_used++];
  return hipSuccess;
}

// Launch one stencil kernel, bracketed by events when profiling.
template <class F>
hipError_t timed(fwi_plan *p, int kind, hipStream_t st, F &&launch) {
  if (!p->profiling) return launch();
  hipEvent_t a, b;
  hipError_t rc = next_event(p, &a);
  if (rc == hipSuccess) rc = next_event(p, &b);
  if (rc == hipSuccess) rc = hipEventRecord(a, st);
  if (rc != hipSuccess) return rc;
  rc = launch();
  if (rc != hipSuccess) return rc;
  rc = hipEventRecord(b, st);
  if (rc == hipSuccess) p->marks[kind].emplace_back(a, b);
  return rc;
}

// Checkpoint slot that must receive u^{n}, u^{n-1} when level n starts a
// segment, or null.
float *ckpt_slot(const fwi_plan *p, float *ckpt, int n) {
  if (!ckpt || n % p->K) return nullptr;
  const int j = n / p->K;
  return j >= 1 && j < p->nseg ? ckpt + (size_t)j * 2 * p->geo.ns * p->geo.fs : nullptr;
}

// Forward sweep n = 0..nt-2 on the fields at ws+L.u (and Born fields):
// pairs of steps per launch while two remain, then single steps.  With
// `store_ckpt` it leaves what the reverse sweep needs: the checkpoints, or in
// history mode every w^n (n = 0..nt-2) in the segment buffer.
int forward_sweep(fwi_plan *p, const Layout &L, void *ws, int B, bool born, float *d_out,
                  float *dd_out, bool store_ckpt, hipStream_t st) {
  const Geo &g = p->geo;
  float *ckpt = store_ckpt && !p->hist ? at<float>(ws, L.ckpt) : nullptr;
  float *whist = store_ckpt && p->hist ? at<float>(ws, L.wseg) : nullptr;
  auto wlevel = [&](int n) { return whist ? whist + (size_t)n * g.ns * g.fs : nullptr; };
  float *u = at<float>(ws, L.u), *du = born ? at<float>(ws, L.du) : nullptr;
  const size_t us = set_stride(g, 1), dus = set_stride(g, B);
  int cur = 0, n = 0;
  if (born ? p->ts_born : p->ts_fwd) {
    Step2Args a{};
    a.c = at<float>(ws, L.c);
    a.dc = born ? at<float>(ws, L.dc) : nullptr;
    a.B = born ? B : 0;
    a.d_out = d_out;
    a.dd_out = dd_out;
    for (; n + 2 <= g.nt - 1; n += 2, cur ^= 1) {
      a.n = n;
      a.amp0 = src_amp(p, n);
      a.amp1 = src_amp(p, n + 1);
      a.uin = u + cur * us;
      a.uout = u + (cur ^ 1) * us;
      a.duin = born ? du + cur * dus : nullptr;
      a.duout = born ? du + (cur ^ 1) * dus : nullptr;
      a.ck = ckpt_slot(p, ckpt, n + 2);
      a.w_out0 = wlevel(n);
      a.w_out1 = wlevel(n + 1);
      HIP_TRY(timed(p, born ? FWI_KERNEL_STEP_BORN : FWI_KERNEL_STEP, st,
                    [&] { return launch_step2(g, p->tabs, a, born, st); }));
    }
  }
  StepArgs a{};
  a.c = at<float>(ws, L.c);
  a.dc = born ? at<float>(ws, L.dc) : nullptr;
  a.u = u + cur * us;
  a.du = born ? du + cur * dus : nullptr;
  a.B = born ? B : 0;
  a.d_out = d_out;
  a.dd_out = dd_out;
  a.order = born ? p->born_order : p->step_order;
  for (; n + 1 < g.nt; ++n) {
    a.n = n;
    a.src_amp = src_amp(p, n);
    a.ck = ckpt_slot(p, ckpt, n + 1);
    a.w_out = wlevel(n);
    HIP_TRY(timed(p, born ? FWI_KERNEL_STEP_BORN : FWI_KERNEL_STEP, st,
                  [&] { return launch_step(g, p->tabs, a, born, st); }));
  }
  return FWI_OK;
}

// Reverse sweep: segment-wise recompute of w^n from the checkpoints (skipped in
// history mode: the forward sweep left every level), then the adjoint steps
// k = nt-1..0 with injection of r[B][ns][nt][nr].  Leaves the partial images
// in ws+L.img.
int reverse_sweep(fwi_plan *p, const Layout &L, void *ws, int B, const float *r,
                  hipStream_t st) {
  const Geo &g = p->geo;
  const size_t msets = p->ts_adj ? 2 : 1;
  const size_t us = set_stride(g, 1), ms = set_stride(g, B);
  float *u = at<float>(ws, L.u), *mu = at<float>(ws, L.mu);
  HIP_TRY(launch_fill(mu, (long long)(ms * msets), st));
  HIP_TRY(launch_fill64(at<double>(ws, L.img), (long long)g.fs * L.G * B, st));
  float *ckpt = p->hist ? nullptr : at<float>(ws, L.ckpt);
  float *wseg = at<float>(ws, L.wseg);
  auto wbuf = [&](int n, int n0) { return wseg + (size_t)(n - n0) * g.ns * g.fs; };
  int mcur = 0;  // field set holding the adjoint state
  for (int j = p->nseg - 1; j >= 0; --j) {
    const int n0 = j * p->K;
    const int n1 = std::min((j + 1) * p->K, g.nt - 1);
    // recompute on a copy so the checkpoints survive (the adjoint can be
    // repeated after one forward, see fwi_adjoint_resume)
    int ucur = 0, n = p->hist ? n1 : n0;
    if (!p->hist) HIP_TRY(launch_copy(u, ckpt + (size_t)j * 2 * g.ns * g.fs, (long long)us, st));
    if (p->ts_fwd) {
      Step2Args f{};
      f.c = at<float>(ws, L.c);
      for (; n + 2 <= n1; n += 2, ucur ^= 1) {
        f.n = n;
        f.amp0 = src_amp(p, n);
        f.amp1 = src_amp(p, n + 1);
        f.uin = u + ucur * us;
        f.uout = u + (ucur ^ 1) * us;
        f.w_out0 = wbuf(n, n0);
        f.w_out1 = wbuf(n + 1, n0);
        HIP_TRY(timed(p, FWI_KERNEL_STEP, st,
                      [&] { return launch_step2(g, p->tabs, f, false, st); }));
      }
    }
    if (n < n1) {
      StepArgs f{};
      f.c = at<float>(ws, L.c);
      f.u = u + ucur * us;
      f.order = p->step_order;
      for (; n < n1; ++n) {
        f.n = n;
        f.src_amp = src_amp(p, n);
        f.w_out = wbuf(n, n0);
        HIP_TRY(timed(p, FWI_KERNEL_STEP, st,
                      [&] { return launch_step(g, p->tabs, f, false, st); }));
      }
    }
    int k = (j == p->nseg - 1) ? g.nt - 1 : n1 - 1;
    if (p->ts_adj) {
      Adj2Args a{};
      a.c = at<float>(ws, L.c);
      a.s2m = at<float>(ws, L.s2m);
      a.r = r;
      a.img = at<double>(ws, L.img);
      a.B = B;
      a.group = L.group;
      a.ngroups = L.G;
      a.nb = p->adj_nb(B);
      for (; k - 1 >= n0; k -= 2, mcur ^= 1) {
        a.k = k;
        a.muin = mu + mcur * ms;
        a.muout = mu + (mcur ^ 1) * ms;
        a.w0 = (k <= g.nt - 2) ? wbuf(k, n0) : nullptr;
        a.w1 = wbuf(k - 1, n0);
        HIP_TRY(timed(p, FWI_KERNEL_ADJOINT, st,
                      [&] { return launch_adjoint2(g, p->tabs, a, st); }));
      }
    }
    if (k >= n0) {
      AdjArgs a{};
      a.c = at<float>(ws, L.c);
      a.s2m = at<float>(ws, L.s2m);
      a.mu = mu + mcur * ms;
      a.r = r;
      a.img = at<double>(ws, L.img);
      a.B = B;
      a.group = L.group;
      a.ngroups = L.G;
      a.order = p->adj_order;
      for (; k >= n0; --k) {
        a.k = k;
        a.w = (k <= g.nt - 2) ? wbuf(k, n0) : nullptr;
        HIP_TRY(timed(p, FWI_KERNEL_ADJOINT, st,
                      [&] { return launch_adjoint(g, p->tabs, a, st); }));
      }
    }
  }
  return FWI_OK;
}

int prologue(fwi_plan *p, const Layout &L, void *ws, const float *m, const float *v, int B,
             bool born, bool adj, hipStream_t st) {
  const Geo &g = p->geo;
  HIP_TRY(launch_setup(g, m, v, B, at<float>(ws, L.c), at<float>(ws, L.s2m),
                       born ? at<float>(ws, L.dc) : nullptr, ws_status(ws), st));
  HIP_TRY(launch_fill(at<float>(ws, L.u), (long long)set_stride(g, 1), st));
  if (born) HIP_TRY(launch_fill(at<float>(ws, L.du), (long long)set_stride(g, B), st));
  if (adj && !p->hist) HIP_TRY(launch_fill(at<float>(ws, L.ckpt), (long long)g.fs * 2 * g.ns, st));
  return FWI_OK;
}

// Blocked workgroup order of the one-step kernels: rectangles of
// FWI_OPT_BLOCK_X x FWI_OPT_BLOCK_Z tiles, row by row, written into the
// plan's device-block image.
void build_order(fwi_plan *p) {
  Geo &g = p->geo;
  const int bx = p->opt[FWI_OPT_BLOCK_X], bz = p->opt[FWI_OPT_BLOCK_Z];
  int *order = p->blk.data() + p->off_order;
  int q = 0;
  for (int z0 = 0; z0 < g.tiles_z; z0 += bz)
    for (int x0 = 0; x0 < g.tiles_x; x0 += bx)
      for (int z = z0; z < std::min(z0 + bz, g.tiles_z); ++z)
        for (int x = x0; x < std::min(x0 + bx, g.tiles_x); ++x) order[q++] = z * g.tiles_x + x;
  g.blk = bx * bz;
  g.nblocks = (g.ntiles + g.blk - 1) / g.blk;
}

}  // namespace

extern "C" {

int fwi_abi_version(void) { return FWI_ABI_VERSION; }

int fwi_plan_set_option(fwi_plan *p, int option, int value) {
  if (!p) return fail(FWI_EINVAL, "null plan");
  if (option < 0 || option >= FWI_OPT_COUNT) return fail(FWI_EINVAL, "unknown option");
  int lo = 0, hi = 0;
  switch (option) {
    case FWI_OPT_TWO_STEP_FORWARD:
    case FWI_OPT_TWO_STEP_BORN:
    case FWI_OPT_TWO_STEP_ADJOINT:
    case FWI_OPT_LDS_POISON: hi = 1; break;
    case FWI_OPT_ADJ_VECTORS: hi = 4; break;
    case FWI_OPT_ADJ_SHOT_GROUP: hi = 65536; break;
    case FWI_OPT_STEP_ORDER:
    case FWI_OPT_BORN_ORDER:
    case FWI_OPT_ADJ_ORDER: hi = 2; break;
    default: lo = 1; hi = 64; break;  // block sizes
  }
  if (value < lo || value > hi)
    return fail(FWI_EINVAL, "option " + std::to_string(option) + " takes values in [" +
                                std::to_string(lo) + ", " + std::to_string(hi) + "]");
  if ((option == FWI_OPT_BLOCK_X || option == FWI_OPT_BLOCK_Z) && p->dev)
    return fail(FWI_EINVAL, "block sizes must be set before fwi_plan_bind");
  p->opt[option] = value;
  p->apply_options();
  if (option == FWI_OPT_BLOCK_X || option == FWI_OPT_BLOCK_Z) build_order(p);
  return FWI_OK;
}

int fwi_plan_get_option(const fwi_plan *p, int option, int *value) {
  if (!p || !value) return fail(FWI_EINVAL, "null argument");
  if (option < 0 || option >= FWI_OPT_COUNT) return fail(FWI_EINVAL, "unknown option");
  *value = p->opt[option];
  return FWI_OK;
}

const char *fwi_strerror(int code) {
  switch (code) {
    case FWI_OK: return "ok";
    case FWI_EINVAL: return "invalid argument";
    case FWI_EUNSTABLE: return "unstable time step";
    case FWI_ENOMEM: return "workspace or device block too small";
    case FWI_EHIP: return "HIP runtime error";
    case FWI_ENUMERIC: return "non-finite result";
    case FWI_EUNBOUND: return "plan not bound to a device block";
    default: return "unknown error";
  }
}

const char *fwi_last_error(void) { return g_last_error.c_str(); }

int fwi_plan_create(const fwi_geometry *gi, fwi_plan **out) {
  if (!gi || !out) return fail(FWI_EINVAL, "null argument");
  *out = nullptr;
  const fwi_geometry &G = *gi;
  if (G.nx < 1 || G.nz < 1) return fail(FWI_EINVAL, "nx and nz must be >= 1");
  if (G.nb < 0 || G.nb > 1000) return fail(FWI_EINVAL, "nb must be in [0, 1000]");
  if (G.nt < 2) return fail(FWI_EINVAL, "nt must be >= 2");
  if (G.ns < 1 || G.nr < 1) return fail(FWI_EINVAL, "need at least one shot and one receiver");
  if (!(G.dx > 0.f) || !(G.dt > 0.f) || !std::isfinite(G.dx) || !std::isfinite(G.dt))
    return fail(FWI_EINVAL, "dx and dt must be positive");
  if (!(G.kappa_max >= 0.f) || !(G.kappa_max < 0.5f))
    return fail(FWI_EINVAL, "kappa_max must be in [0, 0.5)");
  if (G.ckpt_every < 0) return fail(FWI_EINVAL, "ckpt_every must be >= 0");
  if (!G.src_zx || !G.rec_zx || !G.wavelet) return fail(FWI_EINVAL, "null geometry array");
  if (!(G.inv_noise_var >= 0.0) || !std::isfinite(G.inv_noise_var))
    return fail(FWI_EINVAL, "inv_noise_var must be finite and >= 0");
  const long long nzp = (long long)G.nz + 2 * G.nb, nxp = (long long)G.nx + 2 * G.nb;
  if (nzp > 65536 || nxp > 65536) return fail(FWI_EINVAL, "padded grid too large");
  for (int s = 0; s < G.ns; ++s) {
    const int iz = G.src_zx[2 * s], ix = G.src_zx[2 * s + 1];
    if (iz < 0 || iz >= G.nz || ix < 0 || ix >= G.nx)
      return fail(FWI_EINVAL, "source " + std::to_string(s) + " outside the model grid");
  }
  for (int r = 0; r < G.nr; ++r) {
    const int iz = G.rec_zx[2 * r], ix = G.rec_zx[2 * r + 1];
    if (iz < 0 || iz >= G.nz || ix < 0 || ix >= G.nx)
      return fail(FWI_EINVAL, "receiver " + std::to_string(r) + " outside the model grid");
  }
  for (int n = 0; n < G.nt; ++n)
    if (!std::isfinite(G.wavelet[n])) return fail(FWI_EINVAL, "wavelet not finite");

  fwi_plan *p = new fwi_plan();
  Geo &g = p->geo;
  g.nz = G.nz;
  g.nx = G.nx;
  g.nb = G.nb;
  g.nzp = (int)nzp;
  g.nxp = (int)nxp;
  g.pitch = (int)((nxp + TX - 1) / TX * TX);
  g.tiles_x = g.pitch / TX;
  g.tiles_z = (int)((nzp + TZ - 1) / TZ);
  g.ntiles = g.tiles_x * g.tiles_z;
  g.ns = G.ns;
  g.nt = G.nt;
  g.nr = G.nr;
  g.fs = (long long)g.tiles_z * TZ * g.pitch;
  g.kmax = G.kappa_max;
  g.inv_nb = G.nb > 0 ? 1.0f / (float)G.nb : 0.0f;
  const double h2 = (double)G.dx * (double)G.dx;
  // centred 8th-order second-difference weights (the centre weight -205/72
  // is implied: the kernels difference neighbours against the centre)
  g.c1 = (float)((8.0 / 5.0) / h2);
  g.c2 = (float)((-1.0 / 5.0) / h2);
  g.c3 = (float)((8.0 / 315.0) / h2);
  g.c4 = (float)((-1.0 / 560.0) / h2);
  g.dt = G.dt;
  g.inv_dx = 1.0f / G.dx;
  p->dx = G.dx;
  p->dt = G.dt;
  p->hist = G.ckpt_every == 0;
  p->K = p->hist ? G.nt - 1 : std::min(G.ckpt_every, G.nt - 1);
  p->nseg = (G.nt - 1 + p->K - 1) / p->K;
  p->inv_noise_var = G.inv_noise_var;
  p->wavelet.assign(G.wavelet, G.wavelet + G.nt);

  // receiver tables: sort receivers by (tile, local index, number)
  std::vector<std::tuple<int, int, int, long long>> recs;  // tile, local, id, gidx
  for (int r = 0; r < G.nr; ++r) {
    const int i = G.rec_zx[2 * r] + G.nb, j = G.rec_zx[2 * r + 1] + G.nb;
    const int tile = (i / TZ) * g.tiles_x + j / TX;
    const int local = (i % TZ) * TX + j % TX;
    recs.emplace_back(tile, local, r, (long long)i * g.pitch + j);
  }
  std::sort(recs.begin(), recs.end());
  std::vector<int> trp(g.ntiles + 1, 0), rloc, rid, tnp(g.ntiles + 1, 0), nloc, ngidx, nrp,
      nrec;
  for (auto &e : recs) {
    trp[std::get<0>(e) + 1]++;
    rloc.push_back(std::get<1>(e));
    rid.push_back(std::get<2>(e));
  }
  for (int t = 0; t < g.ntiles; ++t) trp[t + 1] += trp[t];
  for (size_t q = 0; q < recs.size(); ++q) {
    const bool fresh = q == 0 || std::get<0>(recs[q]) != std::get<0>(recs[q - 1]) ||
                       std::get<1>(recs[q]) != std::get<1>(recs[q - 1]);
    if (fresh) {
      tnp[std::get<0>(recs[q]) + 1]++;
      nloc.push_back(std::get<1>(recs[q]));
      ngidx.push_back((int)std::get<3>(recs[q]));
      nrp.push_back((int)nrec.size());
    }
    nrec.push_back(std::get<2>(recs[q]));
  }
  nrp.push_back((int)nrec.size());
  for (int t = 0; t < g.ntiles; ++t) tnp[t + 1] += tnp[t];
  if ((long long)g.fs * (long long)sizeof(double) > 2147483647LL) {
    delete p;
    return fail(FWI_EINVAL, "padded field too large for 32-bit byte offsets");
  }

  // device block image
  auto &b = p->blk;
  auto put = [&](const std::vector<int> &v) {
    const size_t at = b.size();
    b.insert(b.end(), v.begin(), v.end());
    b.resize((b.size() + 63) / 64 * 64, 0);
    return at;
  };
  p->off_status = put(std::vector<int>(1, 0));
  std::vector<int> src(2 * G.ns);
  for (int s = 0; s < G.ns; ++s) {
    src[2 * s] = G.src_zx[2 * s] + G.nb;
    src[2 * s + 1] = G.src_zx[2 * s + 1] + G.nb;
  }
  p->off_src = put(src);
  p->off_trp = put(trp);
  p->off_rloc = put(rloc);
  p->off_rid = put(rid);
  p->off_tnp = put(tnp);
  p->off_nloc = put(nloc);
  p->off_ngidx = put(ngidx);
  p->off_nrp = put(nrp);
  p->off_nrec = put(nrec);
  // blocked workgroup order (rebuilt by fwi_plan_set_option before binding)
  p->off_order = put(std::vector<int>(g.ntiles, 0));
  build_order(p);

  // two-step tiling and its receiver tables
  g.tiles_x2 = (int)((nxp + TX2 - 1) / TX2);
  g.tiles_z2 = (int)((nzp + TZ2 - 1) / TZ2);
  g.ntiles2 = g.tiles_x2 * g.tiles_z2;
  {
    std::vector<int> rp(g.ntiles2 + 1, 0), rloc2, rid2, np2(g.ntiles2 + 1, 0), nloc2, ngid2,
        nrp2, nrec2;
    // distinct receiver nodes and the receivers on each
    std::vector<std::tuple<int, int, int>> byn;  // i, j, receiver
    for (int r = 0; r < G.nr; ++r)
      byn.emplace_back(G.rec_zx[2 * r] + G.nb, G.rec_zx[2 * r + 1] + G.nb, r);
    std::sort(byn.begin(), byn.end());
    for (int t2 = 0; t2 < g.ntiles2; ++t2) {
      const int i0 = (t2 / g.tiles_x2) * TZ2, j0 = (t2 % g.tiles_x2) * TX2;
      for (size_t q = 0; q < byn.size(); ++q) {
        const int i = std::get<0>(byn[q]), j = std::get<1>(byn[q]);
        const int le = (i - i0 + HALO) * EX + (j - j0 + HALO);
        if (i >= i0 && i < i0 + TZ2 && j >= j0 && j < j0 + TX2) {
          rloc2.push_back(le);
          rid2.push_back(std::get<2>(byn[q]));
          rp[t2 + 1]++;
        }
        const bool fresh = q == 0 || std::get<0>(byn[q - 1]) != i || std::get<1>(byn[q - 1]) != j;
        if (fresh && i >= i0 - HALO && i < i0 + TZ2 + HALO && j >= j0 - HALO &&
            j < j0 + TX2 + HALO) {
          nloc2.push_back(le);
          ngid2.push_back(i * g.pitch + j);
          nrp2.push_back((int)nrec2.size());
          for (size_t q2 = q; q2 < byn.size() && std::get<0>(byn[q2]) == i &&
                              std::get<1>(byn[q2]) == j;
               ++q2)
            nrec2.push_back(std::get<2>(byn[q2]));
          np2[t2 + 1]++;
        }
      }
    }
    nrp2.push_back((int)nrec2.size());
    for (int t2 = 0; t2 < g.ntiles2; ++t2) {
      rp[t2 + 1] += rp[t2];
      np2[t2 + 1] += np2[t2];
    }
    p->off2[0] = put(rp);
    p->off2[1] = put(rloc2);
    p->off2[2] = put(rid2);
    p->off2[3] = put(np2);
    p->off2[4] = put(nloc2);
    p->off2[5] = put(ngid2);
    p->off2[6] = put(nrp2);
    p->off2[7] = put(nrec2);
  }
  p->apply_options();
  *out = p;
  return FWI_OK;
}

void fwi_plan_destroy(fwi_plan *p) { delete p; }

int fwi_plan_device_bytes(const fwi_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(FWI_EINVAL, "null argument");
  *bytes = p->blk.size() * sizeof(int);
  return FWI_OK;
}

int fwi_plan_dims(const fwi_plan *p, int32_t dims[6]) {
  if (!p || !dims) return fail(FWI_EINVAL, "null argument");
  dims[0] = p->geo.nzp;
  dims[1] = p->geo.nxp;
  dims[2] = p->geo.pitch;
  dims[3] = p->geo.tiles_z;
  dims[4] = p->geo.tiles_x;
  dims[5] = p->K;
  return FWI_OK;
}

int fwi_plan_bind(fwi_plan *p, void *dev, size_t bytes, void *stream) {
  if (!p || !dev) return fail(FWI_EINVAL, "null argument");
  if (bytes < p->blk.size() * sizeof(int))
    return fail(FWI_ENOMEM, "device block too small");
  if (reinterpret_cast<uintptr_t>(dev) % ALIGN)
    return fail(FWI_EINVAL, "device block must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(dev, p->blk.data(), p->blk.size() * sizeof(int), hipMemcpyHostToDevice,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  p->dev = dev;
  int *base = static_cast<int *>(dev);
  DevTables &t = p->tabs;
  t.status = reinterpret_cast<unsigned int *>(base + p->off_status);
  t.src_ij = base + p->off_src;
  t.tile_rec_ptr = base + p->off_trp;
  t.rec_local = base + p->off_rloc;
  t.rec_id = base + p->off_rid;
  t.tile_node_ptr = base + p->off_tnp;
  t.node_local = base + p->off_nloc;
  t.node_gidx = base + p->off_ngidx;
  t.node_rec_ptr = base + p->off_nrp;
  t.node_recs = base + p->off_nrec;
  t.tile_order = base + p->off_order;
  t.t2_rec_ptr = base + p->off2[0];
  t.t2_rec_local = base + p->off2[1];
  t.t2_rec_id = base + p->off2[2];
  t.t2_node_ptr = base + p->off2[3];
  t.t2_node_local = base + p->off2[4];
  t.t2_node_gidx = base + p->off2[5];
  t.t2_node_rec_ptr = base + p->off2[6];
  t.t2_node_recs = base + p->off2[7];
  return FWI_OK;
}

int fwi_workspace_size(const fwi_plan *p, int op, int batch, size_t *bytes) {
  if (!p || !bytes) return fail(FWI_EINVAL, "null argument");
  if (op < FWI_OP_FORWARD || op > FWI_OP_GRAD_HVP) return fail(FWI_EINVAL, "unknown op");
  if (batch < 1 || batch > 4096) return fail(FWI_EINVAL, "batch must be in [1, 4096]");
  *bytes = layout(p, op, batch).total;
  return FWI_OK;
}

int fwi_forward(fwi_plan *p, const float *m, float *d, void *ws, size_t ws_bytes,
                void *stream) {
  if (int rc = check_call(p, FWI_OP_FORWARD, 1, ws, ws_bytes)) return rc;
  if (!m || !d) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_FORWARD, 1);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  if (int rc = prologue(p, L, ws, m, nullptr, 0, false, false, st)) return rc;
  HIP_TRY(launch_zero_t0(d, g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, 1, false, d, nullptr, false, st)) return rc;
  HIP_TRY(launch_check_finite(d, (long long)g.ns * g.nt * g.nr, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_born(fwi_plan *p, const float *m, const float *v, int B, float *dd, void *ws,
             size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_BORN, B, ws, ws_bytes)) return rc;
  if (!m || !v || !dd) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_BORN, B);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  if (int rc = prologue(p, L, ws, m, v, B, true, false, st)) return rc;
  HIP_TRY(launch_zero_t0(dd, B * g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, B, true, nullptr, dd, false, st)) return rc;
  HIP_TRY(launch_check_finite(dd, (long long)B * g.ns * g.nt * g.nr, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_adjoint(fwi_plan *p, const float *m, const float *r, int B, float *gout, void *ws,
                size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_ADJOINT, B, ws, ws_bytes)) return rc;
  if (!m || !r || !gout) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_ADJOINT, B);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  if (int rc = prologue(p, L, ws, m, nullptr, 0, false, true, st)) return rc;
  if (int rc = forward_sweep(p, L, ws, 1, false, nullptr, nullptr, true, st)) return rc;
  if (int rc = reverse_sweep(p, L, ws, B, r, st)) return rc;
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, B, 0, B, 1.0, gout, st));
  HIP_TRY(launch_check_finite(gout, (long long)B * g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_forward_keep(fwi_plan *p, const float *m, float *d, void *ws, size_t ws_bytes,
                     void *stream) {
  if (int rc = check_call(p, FWI_OP_ADJOINT, 1, ws, ws_bytes)) return rc;
  if (!m || !d) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_ADJOINT, 1);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  if (int rc = prologue(p, L, ws, m, nullptr, 0, false, true, st)) return rc;
  HIP_TRY(launch_zero_t0(d, g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, 1, false, d, nullptr, true, st)) return rc;
  HIP_TRY(launch_check_finite(d, (long long)g.ns * g.nt * g.nr, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_adjoint_resume(fwi_plan *p, const float *r, int B, float *gout, void *ws,
                       size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_ADJOINT, B, ws, ws_bytes)) return rc;
  if (!r || !gout) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_ADJOINT, B);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  if (int rc = reverse_sweep(p, L, ws, B, r, st)) return rc;
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, B, 0, B, 1.0, gout, st));
  HIP_TRY(launch_check_finite(gout, (long long)B * g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_misfit(fwi_plan *p, const float *m, const float *dobs, double *phi, void *ws,
               size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_MISFIT, 1, ws, ws_bytes)) return rc;
  if (!m || !dobs || !phi) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_MISFIT, 1);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  float *dres = at<float>(ws, L.dres);
  if (int rc = prologue(p, L, ws, m, nullptr, 0, false, false, st)) return rc;
  HIP_TRY(launch_zero_t0(dres, g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, 1, false, dres, nullptr, false, st)) return rc;
  HIP_TRY(launch_residual(dres, dobs, (long long)g.ns * g.nt * g.nr, at<double>(ws, L.part),
                          NPARTS, 0.5 * p->inv_noise_var, phi, st));
  HIP_TRY(launch_check_finite(dres, (long long)g.ns * g.nt * g.nr, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_misfit_grad(fwi_plan *p, const float *m, const float *dobs, double *phi, float *gout,
                    void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_MISFIT_GRAD, 1, ws, ws_bytes)) return rc;
  if (!m || !dobs || !phi || !gout) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_MISFIT_GRAD, 1);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  float *dres = at<float>(ws, L.dres);
  if (int rc = prologue(p, L, ws, m, nullptr, 0, false, true, st)) return rc;
  HIP_TRY(launch_zero_t0(dres, g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, 1, false, dres, nullptr, true, st)) return rc;
  HIP_TRY(launch_residual(dres, dobs, (long long)g.ns * g.nt * g.nr, at<double>(ws, L.part),
                          NPARTS, 0.5 * p->inv_noise_var, phi, st));
  if (int rc = reverse_sweep(p, L, ws, 1, dres, st)) return rc;
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, 1, 0, 1, p->inv_noise_var, gout, st));
  HIP_TRY(launch_check_finite(gout, (long long)g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_gn_hvp(fwi_plan *p, const float *m, const float *v, int B, float *hv, void *ws,
               size_t ws_bytes, void *stream) {
  if (int rc = check_call(p, FWI_OP_GN_HVP, B, ws, ws_bytes)) return rc;
  if (!m || !v || !hv) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_GN_HVP, B);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  float *dd = at<float>(ws, L.dd);
  if (int rc = prologue(p, L, ws, m, v, B, true, true, st)) return rc;
  HIP_TRY(launch_zero_t0(dd, B * g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, B, true, nullptr, dd, true, st)) return rc;
  if (int rc = reverse_sweep(p, L, ws, B, dd, st)) return rc;
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, B, 0, B, p->inv_noise_var, hv, st));
  HIP_TRY(launch_check_finite(hv, (long long)B * g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_misfit_grad_hvp(fwi_plan *p, const float *m, const float *dobs, const float *v, int B,
                        double *phi, float *gout, float *hv, void *ws, size_t ws_bytes,
                        void *stream) {
  if (int rc = check_call(p, FWI_OP_GRAD_HVP, B, ws, ws_bytes)) return rc;
  if (!m || !dobs || !v || !phi || !gout || !hv) return fail(FWI_EINVAL, "null array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(p, FWI_OP_GRAD_HVP, B);
  HIP_TRY(launch_status_open(ws_status(ws), st));
  const Geo &g = p->geo;
  const long long nd = (long long)g.ns * g.nt * g.nr;
  float *dd = at<float>(ws, L.dd);  // [B+1][ns][nt][nr]: d - dobs, then J v_b
  if (int rc = prologue(p, L, ws, m, v, B, true, true, st)) return rc;
  HIP_TRY(launch_zero_t0(dd, (B + 1) * g.ns, g.nt, g.nr, st));
  if (int rc = forward_sweep(p, L, ws, B, true, dd, dd + nd, true, st)) return rc;
  HIP_TRY(launch_residual(dd, dobs, nd, at<double>(ws, L.part), NPARTS, 0.5 * p->inv_noise_var,
                          phi, st));
  if (int rc = reverse_sweep(p, L, ws, B + 1, dd, st)) return rc;
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, B + 1, 0, 1, p->inv_noise_var, gout, st));
  HIP_TRY(launch_fold(g, at<double>(ws, L.img), L.G, B + 1, 1, B, p->inv_noise_var, hv, st));
  HIP_TRY(launch_check_finite(gout, (long long)g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_check_finite(hv, (long long)B * g.nz * g.nx, ws_status(ws), st));
  HIP_TRY(launch_status_merge(ws_status(ws), p->tabs.status, st));
  return FWI_OK;
}

int fwi_profile_enable(fwi_plan *p, int enable) {
  if (!p) return fail(FWI_EINVAL, "null plan");
  p->profiling = enable != 0;
  return FWI_OK;
}

int fwi_kernel_steps(const fwi_plan *p, int kind, int32_t *steps) {
  if (!p || !steps) return fail(FWI_EINVAL, "null argument");
  if (kind < 0 || kind > 2) return fail(FWI_EINVAL, "unknown kernel kind");
  const bool two = kind == FWI_KERNEL_STEP ? p->ts_fwd
                   : kind == FWI_KERNEL_STEP_BORN ? p->ts_born
                                                  : p->ts_adj;
  *steps = two ? 2 : 1;
  return FWI_OK;
}

int fwi_profile_reset(fwi_plan *p) {
  if (!p) return fail(FWI_EINVAL, "null plan");
  for (auto &m : p->marks) m.clear();
  p->pool_used = 0;
  return FWI_OK;
}

int fwi_profile_read(fwi_plan *p, int kind, double *total_ms, int64_t *launches) {
  if (!p || !total_ms || !launches) return fail(FWI_EINVAL, "null argument");
  if (kind < 0 || kind > 2) return fail(FWI_EINVAL, "unknown kernel kind");
  double acc = 0.0;
  for (auto &pr : p->marks[kind]) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    acc += ms;
  }
  *total_ms = acc;
  *launches = (int64_t)p->marks[kind].size();
  return FWI_OK;
}

int fwi_workspace_status(const fwi_plan *p, const void *ws, void *stream, uint32_t *status) {
  if (!p || !ws || !status) return fail(FWI_EINVAL, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned int v = 0;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost));
  *status = v;
  return FWI_OK;
}

int fwi_status(fwi_plan *p, void *stream, uint32_t *status) {
  if (!p || !status) return fail(FWI_EINVAL, "null argument");
  if (!p->dev) return fail(FWI_EUNBOUND, "plan has no device block");
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned int v = 0, zero = 0;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(&v, p->tabs.status, sizeof(v), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p->tabs.status, &zero, sizeof(zero), hipMemcpyHostToDevice));
  *status = v;
  return FWI_OK;
}

}  // extern "C"

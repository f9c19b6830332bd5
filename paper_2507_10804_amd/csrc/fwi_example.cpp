// fwi_example -- a complete caller of libfwi_mi355x.so through include/fwi.h
// alone (no Python, no torch): it builds a small problem on the host, owns
// every device buffer, and computes Gauss-Newton Hessian-vector products
// (Section 3: H_d v = F* Gamma^-1 F v, summed over shots).
//
//   fwi_example OUTDIR
//
// The problem: a 61 x 83 grid (dx = 10 m) with a velocity that grows with
// depth from 1800 to 2400 m/s plus a 300 m/s Gaussian anomaly, 3 shots and 27
// receivers one cell below the top edge, 12 sponge cells, 240 time steps of a
// 15 Hz Ricker wavelet, checkpoints every 40 steps, and B = 2 smooth
// perturbations.  It writes what it used and what it got to OUTDIR as raw
// little-endian arrays, so that the products can be checked elsewhere:
//   geometry.txt   nx nz nb nt dx dt kappa_max ns nr ckpt_every inv_noise_var
//                  (floats printed with 9 significant digits: exact for FP32)
//   src.i32 [ns][2]   rec.i32 [nr][2]   wavelet.f32 [nt]
//   m.f32 [nz][nx]    v.f32 [B][nz][nx] hv.f32 [B][nz][nx]
// It also shows the error path: a workspace one byte short is refused with
// FWI_ENOMEM and a message.  Exit status 0 on success, 1 on any failure.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "fwi.h"

namespace {

bool hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "fwi_example: %s: %s\n", what, hipGetErrorString(e));
  return false;
}

bool fwi_ok(int rc, const char *what) {
  if (rc == FWI_OK) return true;
  std::fprintf(stderr, "fwi_example: %s: %s (%s)\n", what, fwi_strerror(rc), fwi_last_error());
  return false;
}

template <typename T>
bool write_raw(const std::string &path, const std::vector<T> &a) {
  FILE *f = std::fopen(path.c_str(), "wb");
  if (!f) return false;
  const size_t n = std::fwrite(a.data(), sizeof(T), a.size(), f);
  return std::fclose(f) == 0 && n == a.size();
}

// Device buffers the example owns; freed on every exit path.
struct DeviceBuffers {
  std::vector<void *> ptrs;
  void *get(size_t bytes, const char *what) {
    void *p = nullptr;
    if (!hip_ok(hipMalloc(&p, bytes), what)) return nullptr;
    ptrs.push_back(p);
    return p;
  }
  ~DeviceBuffers() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

int run(const std::string &out) {
  const int nz = 61, nx = 83, nb = 12, nt = 240, ns = 3, K = 40, B = 2;
  const float dx = 10.0f, vmax = 2700.0f, f0 = 15.0f;
  const float dt = 0.45f * dx / vmax;  // Courant number 0.45 at the fastest cell
  // sponge peak 3 C ln(1e3) / (2 nb), the usual choice for a quadratic profile
  const float kappa_max = static_cast<float>(3.0 * 0.45 * std::log(1.0e3) / (2.0 * nb));

  std::vector<int32_t> src, rec;
  for (int s = 0; s < ns; ++s) src.insert(src.end(), {1, (2 * s + 1) * nx / (2 * ns)});
  for (int ix = 2; ix < nx - 2; ix += 3) rec.insert(rec.end(), {1, ix});
  const int nr = static_cast<int>(rec.size()) / 2;

  std::vector<float> wavelet(nt);
  for (int n = 0; n < nt; ++n) {
    const double t = n * static_cast<double>(dt) - 1.5 / f0;
    const double a = (M_PI * f0 * t) * (M_PI * f0 * t);
    wavelet[n] = static_cast<float>((1.0 - 2.0 * a) * std::exp(-a));
  }

  std::vector<float> m(static_cast<size_t>(nz) * nx), v(static_cast<size_t>(B) * nz * nx);
  for (int iz = 0; iz < nz; ++iz)
    for (int ix = 0; ix < nx; ++ix) {
      const double z = iz * dx, x = ix * dx, zc = 0.55 * nz * dx, xc = 0.45 * nx * dx;
      const double bump = 300.0 * std::exp(-((z - zc) * (z - zc) + (x - xc) * (x - xc)) / (2.0 * 80.0 * 80.0));
      m[static_cast<size_t>(iz) * nx + ix] = static_cast<float>(1800.0 + 600.0 * iz / (nz - 1) + bump);
      for (int b = 0; b < B; ++b) {
        const double kz = M_PI * (b + 1) / (nz - 1), kx = M_PI * (b + 2) / (nx - 1);
        v[(static_cast<size_t>(b) * nz + iz) * nx + ix] =
            static_cast<float>(std::sin(kz * iz) * std::cos(kx * ix + 0.3 * b));
      }
    }

  fwi_geometry g{};
  g.nx = nx; g.nz = nz; g.nb = nb; g.nt = nt; g.dx = dx; g.dt = dt; g.kappa_max = kappa_max;
  g.ns = ns; g.src_zx = src.data(); g.nr = nr; g.rec_zx = rec.data(); g.wavelet = wavelet.data();
  g.ckpt_every = K; g.inv_noise_var = 1.0;

  if (fwi_abi_version() != FWI_ABI_VERSION) {
    std::fprintf(stderr, "fwi_example: library ABI %d, header %d\n", fwi_abi_version(), FWI_ABI_VERSION);
    return 1;
  }
  fwi_plan *plan = nullptr;
  if (!fwi_ok(fwi_plan_create(&g, &plan), "fwi_plan_create")) return 1;
  struct PlanGuard { fwi_plan *p; ~PlanGuard() { fwi_plan_destroy(p); } } guard{plan};

  hipStream_t stream = nullptr;
  if (!hip_ok(hipStreamCreate(&stream), "hipStreamCreate")) return 1;
  struct StreamGuard { hipStream_t s; ~StreamGuard() { (void)hipStreamDestroy(s); } } sguard{stream};

  DeviceBuffers dev;
  size_t plan_bytes = 0, ws_bytes = 0;
  if (!fwi_ok(fwi_plan_device_bytes(plan, &plan_bytes), "fwi_plan_device_bytes")) return 1;
  void *plan_mem = dev.get(plan_bytes, "hipMalloc(plan block)");
  if (!plan_mem || !fwi_ok(fwi_plan_bind(plan, plan_mem, plan_bytes, stream), "fwi_plan_bind")) return 1;
  if (!fwi_ok(fwi_workspace_size(plan, FWI_OP_GN_HVP, B, &ws_bytes), "fwi_workspace_size")) return 1;
  void *ws = dev.get(ws_bytes, "hipMalloc(workspace)");
  float *dm = static_cast<float *>(dev.get(m.size() * sizeof(float), "hipMalloc(m)"));
  float *dv = static_cast<float *>(dev.get(v.size() * sizeof(float), "hipMalloc(v)"));
  float *dhv = static_cast<float *>(dev.get(v.size() * sizeof(float), "hipMalloc(hv)"));
  if (!ws || !dm || !dv || !dhv) return 1;
  if (!hip_ok(hipMemcpy(dm, m.data(), m.size() * sizeof(float), hipMemcpyHostToDevice), "copy m") ||
      !hip_ok(hipMemcpy(dv, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice), "copy v"))
    return 1;

  // The error path: a workspace one byte short is refused before any launch.
  const int short_rc = fwi_gn_hvp(plan, dm, dv, B, dhv, ws, ws_bytes - 1, stream);
  if (short_rc != FWI_ENOMEM) {
    std::fprintf(stderr, "fwi_example: a short workspace returned %d, expected FWI_ENOMEM\n", short_rc);
    return 1;
  }
  std::printf("short workspace refused: %s (%s)\n", fwi_strerror(short_rc), fwi_last_error());

  if (!fwi_ok(fwi_gn_hvp(plan, dm, dv, B, dhv, ws, ws_bytes, stream), "fwi_gn_hvp")) return 1;
  uint32_t status = 0;
  if (!fwi_ok(fwi_status(plan, stream, &status), "fwi_status")) return 1;
  std::vector<float> hv(v.size());
  if (!hip_ok(hipMemcpy(hv.data(), dhv, hv.size() * sizeof(float), hipMemcpyDeviceToHost), "copy hv"))
    return 1;
  if (status != 0) {
    std::fprintf(stderr, "fwi_example: device status word %u\n", status);
    return 1;
  }

  FILE *f = std::fopen((out + "/geometry.txt").c_str(), "w");
  if (!f) {
    std::fprintf(stderr, "fwi_example: cannot write to %s\n", out.c_str());
    return 1;
  }
  std::fprintf(f, "%d %d %d %d %.9g %.9g %.9g %d %d %d %.17g\n", nx, nz, nb, nt, dx, dt, kappa_max, ns,
               nr, K, g.inv_noise_var);
  std::fclose(f);
  if (!write_raw(out + "/src.i32", src) || !write_raw(out + "/rec.i32", rec) ||
      !write_raw(out + "/wavelet.f32", wavelet) || !write_raw(out + "/m.f32", m) ||
      !write_raw(out + "/v.f32", v) || !write_raw(out + "/hv.f32", hv)) {
    std::fprintf(stderr, "fwi_example: writing the arrays to %s failed\n", out.c_str());
    return 1;
  }
  double n2[B] = {};
  for (int b = 0; b < B; ++b)
    for (size_t i = 0; i < m.size(); ++i) n2[b] += static_cast<double>(hv[b * m.size() + i]) * hv[b * m.size() + i];
  std::printf("gn_hvp %dx%d, %d shots, nt=%d, B=%d: |hv_0| = %.6e, |hv_1| = %.6e, status %u\n", nz, nx, ns,
              nt, B, std::sqrt(n2[0]), std::sqrt(n2[1]), status);
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s OUTDIR\n", argv[0]);
    return 1;
  }
  return run(argv[1]);
}

"""The C-ABI example program (a caller that uses include/fwi.h and the HIP
runtime alone, no Python binding or torch) run as a subprocess on the GPU: its
Gauss-Newton products (Section 3) against the FP64 oracle on the very inputs it
wrote out.  Tolerance: relative L2 1e-5 per vector, as for the binding's
products of the same size."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2507_10804_amd import synth
from paper_2507_10804_amd.csrc import build as hip_build
from tests._cases import rel

pytestmark = pytest.mark.gpu


def _read(d, name, dtype, shape):
    a = np.fromfile(os.path.join(d, name), dtype=dtype)
    assert a.size == int(np.prod(shape)), name
    return a.reshape(shape)


def test_c_example_products_match_the_oracle(tmp_path):
    print("fwi_example: 61x83, 3 shots, nt=240, B=2", flush=True)
    assert os.path.exists(hip_build.EXAMPLE), "fwi_example is not built (run build())"
    out = subprocess.run([hip_build.EXAMPLE, str(tmp_path)], capture_output=True, text=True,
                         timeout=120)
    sys.stdout.write(out.stdout)
    assert out.returncode == 0, out.stderr
    assert "short workspace refused: workspace or device block too small" in out.stdout
    f = open(os.path.join(tmp_path, "geometry.txt")).read().split()
    nx, nz, nb, nt = map(int, f[:4])
    dx, dt, kap = (float(np.float32(x)) for x in f[4:7])
    ns, nr, K = map(int, f[7:10])
    g = synth.Geometry(nx=nx, nz=nz, dx=dx, dt=dt, nt=nt, nb=nb, kappa_max=kap,
                       src_zx=_read(tmp_path, "src.i32", np.int32, (ns, 2)),
                       rec_zx=_read(tmp_path, "rec.i32", np.int32, (nr, 2)),
                       wavelet=_read(tmp_path, "wavelet.f32", np.float32, (nt,)).astype(np.float64),
                       ckpt_every=K, inv_noise_var=float(f[10]))
    m = _read(tmp_path, "m.f32", np.float32, (nz, nx)).astype(np.float64)
    v = _read(tmp_path, "v.f32", np.float32, (2, nz, nx)).astype(np.float64)
    hv = _read(tmp_path, "hv.f32", np.float32, (2, nz, nx)).astype(np.float64)
    ref = oracle.gn_hvp(g, m, v)
    errs = [rel(hv[b], ref[b]) for b in range(2)]
    print(f"fwi_example vs oracle: rel-L2 {errs[0]:.2e} {errs[1]:.2e}", flush=True)
    assert max(errs) < 1e-5, errs

"""Small seeded problem instances shared by the tests."""
import numpy as np

from paper_2507_10804_amd import synth


def tiny(nx=48, nz=40, ns=3, nr=12, nt=250, nb=10, f0=15.0, seed=0, ckpt_every=50):
    """Heterogeneous model (two Gaussian anomalies on 2000 m/s), surface shots
    and receivers, sponge on; a few million point updates per solve."""
    m = synth.gaussian_anomaly_model(nx, nz, seed=seed, width=60.0, min_sep=120.0)
    rec_ix = np.linspace(2, nx - 3, nr).round().astype(np.int64)
    g = synth.make_geometry(nx, nz, nt=nt, ns=ns, rec_ix=rec_ix, f0=f0,
                            v_nominal=2300.0, nb=nb, ckpt_every=ckpt_every)
    return g, m


def dense_case():
    """16x16 model, 4 sponge cells, 2 shots, 8 receivers, 120 steps."""
    nx = nz = 16
    m = 2000.0 + 150.0 * synth.smooth_random((nz, nx), seed=3, sigma=3.0) / 0.2
    m = np.clip(m, 1700.0, 2300.0)
    rec_ix = np.array([1, 3, 5, 7, 9, 11, 13, 14])
    g = synth.make_geometry(nx, nz, nt=120, ns=2, rec_ix=rec_ix, f0=25.0,
                            v_nominal=2300.0, nb=4)
    return g, m


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))

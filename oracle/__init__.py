"""FP64 CPU oracle for the acoustic Gauss-Newton Hessian-vector product.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the HIP library (see ``fwi_oracle.c`` for the scheme and
the paper passages each function follows).

Pins (what fixes the oracle other than itself) live in ``tests/test_oracle_*.py``:
polynomial exactness of the Laplacian, the analytic 2-D Green's function
and its convergence order, discrete reciprocity, the adjoint dot-product
identity, finite-difference derivative checks, Hessian symmetry / PSD /
zero-residual identity, and brute-force dense Jacobians on tiny grids.  The
absorbing sponge is a chosen convention (the paper fixes no boundary
treatment); it is pinned to the normal-incidence reflection of the
continuous damped wave equation off the same layer (a frequency-domain ODE
solve), to the additivity of the two axes' damping in the corners, and to
energy decay.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwi_oracle.c")
_LIB = os.path.join(_HERE, "_fwi_oracle.so")
_lib = None


SANITIZED_LIB = os.path.join(_HERE, "_build", "asan", "_fwi_oracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc -O2 (IEEE FP64, no fast-math).  With
    `sanitize`, a checking build (clang, AddressSanitizer + UndefinedBehavior
    Sanitizer, same arithmetic flags) goes to _build/asan/ instead."""
    if sanitize:
        os.makedirs(os.path.dirname(SANITIZED_LIB), exist_ok=True)
        tmp = SANITIZED_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([CLANG, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-shared-libasan", _SRC, "-o",
                               tmp, "-lm"])
        os.replace(tmp, SANITIZED_LIB)
        return SANITIZED_LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def use_library(path: str) -> None:
    """Load the oracle from `path` (e.g. the sanitizer build) instead."""
    global _LIB, _lib
    _LIB, _lib = path, None


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("ns", ctypes.c_int32), ("nr", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("kappa_max", ctypes.c_double), ("inv_noise_var", ctypes.c_double),
                ("src_zx", ctypes.c_void_p), ("rec_zx", ctypes.c_void_p),
                ("wavelet", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        G = ctypes.POINTER(_Geom)
        for name, args in [("orc_forward", [G, P, P]), ("orc_born", [G, P, P, P]),
                           ("orc_adjoint", [G, P, P, P]),
                           ("orc_misfit_grad", [G, P, P, P, P]),
                           ("orc_gn_hvp", [G, P, P, P]),
                           ("orc_wavefield", [G, P, ctypes.c_int, P]),
                           ("orc_coefficients", [G, P, P, P, P, P])]:
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.orc_laplacian.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P]
        lib.orc_laplacian.restype = None
        _lib = lib
    return _lib


class _Ctx:
    """Keeps the numpy buffers behind a geometry struct alive."""

    def __init__(self, geom, nthreads=0):
        self.src = np.ascontiguousarray(geom.src_zx, dtype=np.int32)
        self.rec = np.ascontiguousarray(geom.rec_zx, dtype=np.int32)
        self.wav = np.ascontiguousarray(geom.wavelet[: geom.nt], dtype=np.float64)
        self.g = _Geom(nx=geom.nx, nz=geom.nz, nb=geom.nb, nt=geom.nt, ns=self.src.shape[0],
                       nr=self.rec.shape[0], nthreads=int(nthreads), pad_=0,
                       dx=geom.dx, dt=geom.dt, kappa_max=geom.kappa_max,
                       inv_noise_var=geom.inv_noise_var,
                       src_zx=self.src.ctypes.data, rec_zx=self.rec.ctypes.data,
                       wavelet=self.wav.ctypes.data)
        self.ptr = ctypes.byref(self.g)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise MemoryError(f"oracle {name} failed with code {rc}")


def forward(geom, m, nthreads=0):
    """d[ns][nt][nr] = R u_s(m)."""
    c = _Ctx(geom, nthreads)
    m = _f64(m)
    d = np.zeros((geom.ns, geom.nt, geom.nr))
    _check(_load().orc_forward(c.ptr, m.ctypes.data, d.ctypes.data), "forward")
    return d


def born(geom, m, v, nthreads=0):
    """J v: dd[ns][nt][nr]."""
    c = _Ctx(geom, nthreads)
    m, v = _f64(m), _f64(v)
    dd = np.zeros((geom.ns, geom.nt, geom.nr))
    _check(_load().orc_born(c.ptr, m.ctypes.data, v.ctypes.data, dd.ctypes.data), "born")
    return dd


def adjoint(geom, m, r, nthreads=0):
    """J^T r summed over shots (no noise weighting): g[nz][nx]."""
    c = _Ctx(geom, nthreads)
    m, r = _f64(m), _f64(r)
    assert r.shape == (geom.ns, geom.nt, geom.nr)
    g = np.zeros((geom.nz, geom.nx))
    _check(_load().orc_adjoint(c.ptr, m.ctypes.data, r.ctypes.data, g.ctypes.data), "adjoint")
    return g


def misfit_grad(geom, m, dobs, nthreads=0):
    """(Phi, grad) of the data misfit."""
    c = _Ctx(geom, nthreads)
    m, dobs = _f64(m), _f64(dobs)
    assert dobs.shape == (geom.ns, geom.nt, geom.nr)
    g = np.zeros((geom.nz, geom.nx))
    phi = np.zeros(1)
    _check(_load().orc_misfit_grad(c.ptr, m.ctypes.data, dobs.ctypes.data, phi.ctypes.data,
                                   g.ctypes.data), "misfit_grad")
    return float(phi[0]), g


def gn_hvp(geom, m, v, nthreads=0):
    """Gauss-Newton H v for one vector v[nz][nx] (or a batch v[B][nz][nx])."""
    m, v = _f64(m), _f64(v)
    if v.ndim == 3:
        return np.stack([gn_hvp(geom, m, vb, nthreads) for vb in v])
    c = _Ctx(geom, nthreads)
    hv = np.zeros((geom.nz, geom.nx))
    _check(_load().orc_gn_hvp(c.ptr, m.ctypes.data, v.ctypes.data, hv.ctypes.data), "gn_hvp")
    return hv


def wavefield(geom, m, shot=0):
    """u^n on the padded grid for n = 0..nt-1, one shot."""
    c = _Ctx(geom)
    m = _f64(m)
    nzp, nxp = geom.nz + 2 * geom.nb, geom.nx + 2 * geom.nb
    h = np.zeros((geom.nt, nzp, nxp))
    _load().orc_wavefield(c.ptr, m.ctypes.data, int(shot), h.ctypes.data)
    return h


def coefficients(geom, m):
    """(a, b, c, m_pad) on the padded grid."""
    c = _Ctx(geom)
    m = _f64(m)
    nzp, nxp = geom.nz + 2 * geom.nb, geom.nx + 2 * geom.nb
    out = [np.zeros((nzp, nxp)) for _ in range(4)]
    _load().orc_coefficients(c.ptr, m.ctypes.data, *[o.ctypes.data for o in out])
    return tuple(out)


def laplacian(u, dx):
    """8th-order Laplacian of a 2-D array (zero outside it)."""
    u = _f64(u)
    out = np.zeros_like(u)
    _load().orc_laplacian(u.shape[0], u.shape[1], float(dx), u.ctypes.data, out.ctypes.data)
    return out

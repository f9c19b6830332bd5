"""FP64 oracle of the point-spread-function (PSF) Hessian approximation.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by the tests,
the smoke check and the CPU-baseline leg of the benchmark; shares no code
with the HIP library.  Plain NumPy/SciPy, float64, written from Sections 3.2
("Point spread function method"), 3.3 (the PDO/symbol formulation) and 3.5
("PSF method in PsiDO formulation").

Objects (sampling description in ``synth.PsfGrid``):

* PSF k at centre x_k is p_k(d) = (H e_{x_k})(x_k + d) for d in the window
  [-half, half]^2 (Section 3.2, the PSF definition), read off the Hessian
  product of the comb that holds x_k; cells outside the model are zero.
* Interpolation weights w_k: tensor products of 1-D piecewise-linear "tent"
  functions on the centre rows and columns, constant beyond the first and
  last centre, so that sum_k w_k = 1 everywhere, w_k >= 0 and
  w_k(x_j) = [k == j].  (The paper names radial basis functions as one
  choice and leaves the weights open; tents are the reading used here.)
* Product-convolution form (Section 3.2, the product-convolution equation):
      (A v)(y) = sum_k sum_d p_k(d) w_k(y - d) v(y - d)      -- apply_pc
* Symbol-row form (Section 3.5: the same approximation rewritten with the
  Fourier transform and the self-adjointness of H):
      (B v)(y) = sum_k w_k(y) sum_d p_k(d) v(y + d)          -- apply_rows
  which is sum_k D_{w_k} F^-1 D_{s_k} F v with symbol row
  s_k = conj(F p_k) (up to the (2 pi)^2 of the continuous convention);
  ``apply_psido`` evaluates exactly that chain with zero-padded FFTs.
  B is the transpose of A; for a self-adjoint H both approximate H.

The per-k sums run over the support box of w_k only (w_k is zero elsewhere);
nothing else is reordered or fused.

Pins (tests/test_oracle_psf.py): partition of unity and the centre property
of the weights; exact reproduction of a translation-invariant operator from
its extracted PSFs; the centre columns (A) and rows (B) of the approximation
equal the extracted PSFs; A = B^T by dense matrices; the FFT chain equals the
spatial symbol-row form; brute-force loops on tiny grids.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import convolve2d, correlate2d


def tent_1d(n: int, first: int, spacing: int, count: int) -> np.ndarray:
    """[count][n] piecewise-linear nodal functions on the centres
    first + j*spacing of a line of n cells, extended as constants beyond the
    first and last centre."""
    z = np.arange(n, dtype=np.float64)
    c = first + spacing * np.arange(count, dtype=np.float64)
    out = np.zeros((count, n))
    if count == 1:
        out[0] = 1.0
        return out
    for j in range(count):
        w = np.maximum(0.0, 1.0 - np.abs(z - c[j]) / spacing)
        if j == 0:
            w[z <= c[0]] = 1.0
        if j == count - 1:
            w[z >= c[-1]] = 1.0
        out[j] = w
    return out


def weights(g) -> np.ndarray:
    """[r][nz][nx] interpolation weights w_k = tent_p(z) tent_q(x), k = p*nxc + q."""
    hz = tent_1d(g.nz, g.oz, g.sz, g.nzc)
    hx = tent_1d(g.nx, g.ox, g.sx, g.nxc)
    return np.einsum("pz,qx->pqzx", hz, hx).reshape(g.r, g.nz, g.nx)


def _support(w1: np.ndarray):
    nz = np.nonzero(w1)[0]
    return int(nz[0]), int(nz[-1]) + 1


def comb_of(g, k: int) -> int:
    p, q = divmod(k, g.nxc)
    return (p % g.stride) * g.stride + q % g.stride


def extract(g, hv_combs: np.ndarray) -> np.ndarray:
    """[r][W][W] PSF windows from the Hessian products of the combs."""
    h, W = g.half, g.width
    out = np.zeros((g.r, W, W))
    for k, (iz, ix) in enumerate(g.centres()):
        src = hv_combs[comb_of(g, k)]
        z0, z1 = max(iz - h, 0), min(iz + h + 1, g.nz)
        x0, x1 = max(ix - h, 0), min(ix + h + 1, g.nx)
        out[k, z0 - iz + h:z1 - iz + h, x0 - ix + h:x1 - ix + h] = src[z0:z1, x0:x1]
    return out


def apply_pc(g, psf: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Product-convolution form: sum_k p_k * (w_k v), linear convolution with
    the PSF centred on its window, zero outside the model."""
    h = g.half
    hz = tent_1d(g.nz, g.oz, g.sz, g.nzc)
    hx = tent_1d(g.nx, g.ox, g.sx, g.nxc)
    out = np.zeros((g.nz + 2 * h, g.nx + 2 * h))  # full-convolution frame
    for k in range(g.r):
        p, q = divmod(k, g.nxc)
        z0, z1 = _support(hz[p])
        x0, x1 = _support(hx[q])
        u = np.outer(hz[p, z0:z1], hx[q, x0:x1]) * v[z0:z1, x0:x1]
        full = convolve2d(u, psf[k], mode="full")  # rows z0-h .. z1+h-1
        out[z0:z1 + 2 * h, x0:x1 + 2 * h] += full
    return out[h:h + g.nz, h:h + g.nx]


def apply_rows(g, psf: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Symbol-row form: sum_k w_k(y) sum_d p_k(d) v(y + d), zero outside."""
    h = g.half
    hz = tent_1d(g.nz, g.oz, g.sz, g.nzc)
    hx = tent_1d(g.nx, g.ox, g.sx, g.nxc)
    vp = np.zeros((g.nz + 2 * h, g.nx + 2 * h))
    vp[h:h + g.nz, h:h + g.nx] = v
    out = np.zeros((g.nz, g.nx))
    for k in range(g.r):
        p, q = divmod(k, g.nxc)
        z0, z1 = _support(hz[p])
        x0, x1 = _support(hx[q])
        win = vp[z0:z1 + 2 * h, x0:x1 + 2 * h]
        corr = correlate2d(win, psf[k], mode="valid")  # (z1-z0, x1-x0)
        out[z0:z1, x0:x1] += np.outer(hz[p, z0:z1], hx[q, x0:x1]) * corr
    return out


def symbol_rows(g, psf: np.ndarray, shape) -> np.ndarray:
    """[r][shape] complex symbol rows conj(F p_k) on an FFT grid of `shape`,
    with the PSF's centre at index (0, 0) (Section 3.5)."""
    h = g.half
    out = np.empty((g.r,) + tuple(shape), dtype=np.complex128)
    for k in range(g.r):
        e = np.zeros(shape)
        e[:g.width, :g.width] = psf[k]
        e = np.roll(e, (-h, -h), axis=(0, 1))
        out[k] = np.conj(np.fft.fft2(e))
    return out


def apply_psido(g, psf: np.ndarray, v: np.ndarray) -> np.ndarray:
    """sum_k D_{w_k} F^-1 D_{s_k} F v on a zero-padded FFT grid large enough
    that the circular products equal linear ones on the model."""
    shape = (g.nz + 2 * g.half, g.nx + 2 * g.half)
    s = symbol_rows(g, psf, shape)
    w = weights(g)
    vp = np.zeros(shape)
    vp[:g.nz, :g.nx] = v
    V = np.fft.fft2(vp)
    out = np.zeros((g.nz, g.nx))
    for k in range(g.r):
        out += w[k] * np.real(np.fft.ifft2(s[k] * V))[:g.nz, :g.nx]
    return out


def apply_pc_at(g, psf: np.ndarray, v: np.ndarray, points) -> np.ndarray:
    """Product-convolution form at individual output cells (iz, ix), summed
    term by term from its definition."""
    w = weights(g)
    h = g.half
    d = np.arange(-h, h + 1)
    res = []
    for iz, ix in points:
        zz, xx = iz - d[:, None], ix - d[None, :]  # input cells y - d
        ok = (zz >= 0) & (zz < g.nz) & (xx >= 0) & (xx < g.nx)
        zc, xc = np.clip(zz, 0, g.nz - 1), np.clip(xx, 0, g.nx - 1)
        vin = np.where(ok, v[zc, xc], 0.0)
        res.append(sum(float(np.sum(psf[k] * w[k][zc, xc] * vin)) for k in range(g.r)))
    return np.array(res)


def apply_rows_at(g, psf: np.ndarray, v: np.ndarray, points) -> np.ndarray:
    """Symbol-row form at individual output cells, from its definition."""
    w = weights(g)
    h = g.half
    d = np.arange(-h, h + 1)
    res = []
    for iz, ix in points:
        zz, xx = iz + d[:, None], ix + d[None, :]
        ok = (zz >= 0) & (zz < g.nz) & (xx >= 0) & (xx < g.nx)
        vin = np.where(ok, v[np.clip(zz, 0, g.nz - 1), np.clip(xx, 0, g.nx - 1)], 0.0)
        res.append(sum(w[k, iz, ix] * float(np.sum(psf[k] * vin)) for k in range(g.r)))
    return np.array(res)

"""Pins of the PSF oracle (oracle/psf.py) against facts fixed by the
mathematics of Sections 3.2-3.5, not by the oracle itself:

* tent weights: partition of unity, non-negativity, the centre property,
  exact reproduction of linear functions between the first and last centre;
* a translation-invariant operator (every PSF equal) is reproduced exactly:
  the product-convolution form equals the plain convolution and the
  symbol-row form the plain correlation, both summed here by brute force;
* extraction from comb products of a convolution operator returns the kernel;
* the product-convolution form maps a delta at a centre to that centre's PSF
  (its columns at the centres are the PSFs); the symbol-row form's rows at
  the centres are the PSFs;
* the symbol-row form is the transpose of the product-convolution form
  (dense matrices on a tiny grid);
* the Fourier chain sum_k D_w F^-1 D_s F equals the spatial symbol-row form;
* for H = D_a C (a smooth, C a convolution) the approximation error falls
  as the square of the centre spacing (second-order tent interpolation).
"""
import numpy as np
import pytest

from oracle import psf as P
from paper_2507_10804_amd import synth


def small_grid(nz=37, nx=45, s=8, half=5, o=3, stride=2):
    nzc = (nz - 1 - o) // s + 1
    nxc = (nx - 1 - o) // s + 1
    return synth.PsfGrid(nz, nx, o, o, s, s, nzc, nxc, half, stride)


def brute_conv(p, v):
    """(p * v)(y) = sum_x p(y - x) v(x), p centred on its window."""
    h = p.shape[0] // 2
    nz, nx = v.shape
    out = np.zeros_like(v)
    for iz in range(nz):
        for ix in range(nx):
            acc = 0.0
            for dz in range(-h, h + 1):
                for dx in range(-h, h + 1):
                    z, x = iz - dz, ix - dx
                    if 0 <= z < nz and 0 <= x < nx:
                        acc += p[dz + h, dx + h] * v[z, x]
            out[iz, ix] = acc
    return out


def brute_corr(p, v):
    return brute_conv(p[::-1, ::-1], v)


def test_tent_weights():
    for n, first, s, c in [(50, 3, 8, 6), (40, 0, 13, 4), (17, 5, 4, 1), (33, 7, 9, 3)]:
        t = P.tent_1d(n, first, s, c)
        assert np.allclose(t.sum(axis=0), 1.0, atol=1e-15)
        assert (t >= 0).all()
        for j in range(c):
            assert t[j, first + j * s] == 1.0
        if c > 1:  # linear functions interpolated exactly between first and last centre
            z = np.arange(n, dtype=float)
            centres = first + s * np.arange(c)
            lin = 2.5 * centres - 7.0
            rec = lin @ t
            inside = (z >= centres[0]) & (z <= centres[-1])
            assert np.allclose(rec[inside], 2.5 * z[inside] - 7.0, atol=1e-12)
    g = small_grid()
    w = P.weights(g)
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-15)
    for k, (iz, ix) in enumerate(g.centres()):
        col = w[:, iz, ix]
        assert col[k] == 1.0 and np.count_nonzero(col) == 1


def test_stationary_operator_reproduced_exactly():
    g = small_grid(nz=23, nx=27, s=6, half=3, o=2)
    rng = np.random.default_rng(0)
    p = rng.standard_normal((g.width, g.width))
    v = rng.standard_normal((g.nz, g.nx))
    psf = np.broadcast_to(p, (g.r, g.width, g.width)).copy()
    assert np.allclose(P.apply_pc(g, psf, v), brute_conv(p, v), atol=1e-12)
    assert np.allclose(P.apply_rows(g, psf, v), brute_corr(p, v), atol=1e-12)


def test_extraction_of_a_convolution():
    g = small_grid(nz=40, nx=44, s=7, half=6, o=3)
    assert g.stride * g.sz >= g.width
    rng = np.random.default_rng(1)
    p = rng.standard_normal((g.width, g.width))
    hv = np.stack([brute_conv(p, c) for c in synth.psf_combs(g)])
    psf = P.extract(g, hv)
    h = g.half
    for k, (iz, ix) in enumerate(g.centres()):
        inside = h <= iz < g.nz - h and h <= ix < g.nx - h
        if inside:
            assert np.array_equal(psf[k], p)
        else:  # truncated by the model edge, equal where the window is inside
            dz = np.arange(-h, h + 1)
            ok = ((iz + dz >= 0) & (iz + dz < g.nz))[:, None] & \
                 ((ix + dz >= 0) & (ix + dz < g.nx))[None, :]
            assert np.array_equal(psf[k][ok], p[ok]) and (psf[k][~ok] == 0).all()


def test_centre_columns_and_rows_are_the_psfs():
    g = small_grid()
    rng = np.random.default_rng(2)
    psf = rng.standard_normal((g.r, g.width, g.width))
    h = g.half
    v = rng.standard_normal((g.nz, g.nx))
    rows = P.apply_rows(g, psf, v)
    for k, (iz, ix) in enumerate(g.centres()):
        e = np.zeros((g.nz, g.nx))
        e[iz, ix] = 1.0
        col = P.apply_pc(g, psf, e)
        expect = np.zeros((g.nz + 2 * h, g.nx + 2 * h))
        expect[iz:iz + g.width, ix:ix + g.width] = psf[k]
        assert np.allclose(col, expect[h:h + g.nz, h:h + g.nx], atol=1e-14)
        # row at the centre: sum_d p_k(d) v(x_k + d)
        vp = np.zeros((g.nz + 2 * h, g.nx + 2 * h))
        vp[h:h + g.nz, h:h + g.nx] = v
        assert rows[iz, ix] == pytest.approx(
            float(np.sum(psf[k] * vp[iz:iz + g.width, ix:ix + g.width])), abs=1e-12)


def dense(fn, g, psf):
    n = g.nz * g.nx
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = fn(g, psf, e.reshape(g.nz, g.nx)).ravel()
    return M


def test_rows_form_is_transpose_of_product_convolution():
    g = small_grid(nz=13, nx=15, s=5, half=2, o=1)
    psf = np.random.default_rng(3).standard_normal((g.r, g.width, g.width))
    A = dense(P.apply_pc, g, psf)
    B = dense(P.apply_rows, g, psf)
    assert np.allclose(A, B.T, atol=1e-13)
    # and each form at single points, summed from its definition
    v = np.random.default_rng(4).standard_normal((g.nz, g.nx))
    pts = [(0, 0), (6, 7), (12, 14), (3, 11)]
    assert np.allclose(P.apply_pc_at(g, psf, v, pts), [(A @ v.ravel())[i * g.nx + j] for i, j in pts])
    assert np.allclose(P.apply_rows_at(g, psf, v, pts), [(B @ v.ravel())[i * g.nx + j] for i, j in pts])


def test_fourier_chain_equals_spatial_rows():
    g = small_grid()
    rng = np.random.default_rng(5)
    psf = rng.standard_normal((g.r, g.width, g.width))
    v = rng.standard_normal((g.nz, g.nx))
    a = P.apply_psido(g, psf, v)
    b = P.apply_rows(g, psf, v)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13


def test_interpolation_error_is_second_order():
    """H = D_a C: PSF k is a(x_k + d) p(d); the approximation replaces a(y)
    by its tent interpolant in the centre variable, so the error on a smooth
    a falls ~4x per halving of the spacing (both forms)."""
    nz = nx = 97
    h = 3
    dz = np.arange(-h, h + 1)
    p = np.exp(-(dz[:, None] ** 2 + dz[None, :] ** 2) / 4.0)
    z = np.arange(nz, dtype=float)
    a = 1.0 + 0.5 * np.sin(2 * np.pi * z / 120.0)[:, None] * np.cos(2 * np.pi * z / 150.0)[None, :]
    v = synth.smooth_random((nz, nx), seed=6, sigma=2.0)
    H = a * brute_conv(p, v)  # the exact operator
    HT = brute_conv(p[::-1, ::-1], a * v)  # its transpose, C^T D_a
    errs_a, errs_b = [], []
    for s in (16, 8, 4):
        o = 0
        nzc = (nz - 1 - o) // s + 1
        g = synth.PsfGrid(nz, nx, o, o, s, s, nzc, nzc, h, 2)
        psf = np.stack([a[np.clip(iz + dz, 0, nz - 1)][:, np.clip(ix + dz, 0, nx - 1)] * p
                        for iz, ix in g.centres()])
        inner = (slice(20, 77), slice(20, 77))
        errs_a.append(np.linalg.norm((P.apply_pc(g, psf, v) - H)[inner]) / np.linalg.norm(H[inner]))
        errs_b.append(np.linalg.norm((P.apply_rows(g, psf, v) - HT)[inner]) / np.linalg.norm(HT[inner]))
    for e in (errs_a, errs_b):
        r1, r2 = e[0] / e[1], e[1] / e[2]
        assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, e

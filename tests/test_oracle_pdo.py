"""Pins of the PDO / PSF+ oracle (oracle/pdo.py) against facts fixed by the
definitions of Sections 3.3-3.6 and Appendix A, each independent of the code
under test:

* the low-rank symbol apply at full rank, fed with the brute-force symbol
  S[x, xi] = (H phi_xi)(x) / phi_xi(x) of a dense operator, reproduces H v;
* the angular interpolation weights are cardinal, sum to one and reproduce
  trigonometric polynomials up to the Nyquist mode;
* the separation masks partition the lattice, are symmetric under
  xi -> -xi, and agree with an angle-sector assignment away from the sector
  boundaries;
* for samples on the lattice, symbol columns come back exactly, and for a
  symbol c(x) rho (alpha + beta cos 2 theta) the whole PDO approximation is
  exact;
* for any field the columns re-synthesise it (sum_k phi_k s_k = H v_p) and
  come in conjugate pairs;
* PSF+ on a separable symbol c(x) sigma(xi) has the closed-form coefficient
  (c + W c(x_k)) / 2 (derived by hand from the least-squares problem with
  alpha = ||B[:, I_c]||^2 / ||B||^2), checked through a direct correlation;
* PSF+ at full rank, with the columns taken from the PSF approximation
  itself, returns the PSF approximation (oracle.psf.apply_rows, a spatial
  code path).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import pdo as D
from oracle import psf as P
from paper_2507_10804_amd import synth


def band_limited(G, rng, kmax, complex_=False):
    """Field on the whole grid with lattice modes |p|, |q| <= kmax only."""
    spec = np.zeros((G.mz, G.mx), dtype=np.complex128)
    for p in range(-kmax, kmax + 1):
        for q in range(-kmax, kmax + 1):
            if p * p + q * q <= kmax * kmax:
                spec[p % G.mz, q % G.mx] = rng.standard_normal() + 1j * rng.standard_normal()
    f = np.fft.ifft2(spec) * G.mz * G.mx / (G.mz * G.mx)
    f = f / np.abs(f).max()
    return f if complex_ else f.real


def test_full_rank_apply_reproduces_dense_operator():
    G = synth.SymbolGrid(6, 5, 6, 5, 1.3, 8, 1.0)
    rng = np.random.default_rng(0)
    M = G.mz * G.mx
    H = rng.standard_normal((M, M))
    S = D.full_symbol(G, H)  # [x][p][q]
    a = S.reshape(M, M).T.reshape(M, G.nz, G.nx)  # a_xi(x) = S[x, xi]
    b = np.eye(M).reshape(M, G.mz, G.mx).astype(np.complex128)
    v = rng.standard_normal((G.nz, G.nx))
    got = D.symbol_apply(G, a, b, v)
    assert np.allclose(got.ravel(), H @ v.ravel(), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("r", [4, 6, 8])
def test_circle_weights_interpolate(r):
    t = D.thetas(r)
    W = D.circle_weights(r, t)
    assert np.allclose(W, np.eye(r), atol=1e-13)
    th = np.random.default_rng(1).uniform(-7, 7, 200)
    w = D.circle_weights(r, th)
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-13)
    # trigonometric polynomial of degree < r/2 plus the cos Nyquist mode
    f = lambda x: 0.3 + np.cos(x) - 0.5 * np.sin(x) + 0.7 * np.cos((r // 2) * x) + (
        0.2 * np.cos(2 * x) - 0.4 * np.sin(2 * x) if r // 2 > 2 else 0.0)
    assert np.allclose(f(t) @ w, f(th), atol=1e-12)


def test_masks_partition_symmetry_and_sectors():
    G = synth.SymbolGrid(10, 9, 12, 10, 1.0, 8, 2.0)
    m = D.masks(G)
    assert np.allclose(m.sum(axis=0), 1.0, atol=1e-14)
    neg = lambda a: np.roll(np.flip(a, axis=(-2, -1)), (1, 1), axis=(-2, -1))  # xi -> -xi
    for k in range(G.r):
        assert np.allclose(m[(k + G.r // 2) % G.r], neg(m[k]), atol=1e-14)
    # angle sectors (an independent rule) away from boundaries and Nyquist
    zc, _ = D._axis(G.mz, G.h)
    xc, _ = D._axis(G.mx, G.h)
    width = 2 * np.pi / G.r
    checked = 0
    for p in range(G.mz):
        for q in range(G.mx):
            if (p, q) == (0, 0) or p == G.mz // 2 or q == G.mx // 2:
                continue
            ang = np.arctan2(zc[p], xc[q]) % (2 * np.pi)
            j = int(np.floor(ang / width + 0.5)) % G.r
            off = abs(ang / width + 0.5 - np.round(ang / width + 0.5))
            if off < 1e-6:
                continue
            k = (j - 1) % G.r  # theta_k = 2 pi k / r stored at index k - 1
            assert m[k, p, q] == 1.0
            checked += 1
    assert checked > 80
    assert np.allclose(m[:, 0, 0], 1.0 / G.r)


def test_columns_exact_for_lattice_samples():
    n = 24
    G = synth.SymbolGrid(n, n, n, n, 1.0, 4, 2 * np.pi * 6 / n)
    rng = np.random.default_rng(2)
    x, z = D.coords(G)
    c1 = band_limited(G, rng, 2, complex_=True)
    c2 = band_limited(G, rng, 2, complex_=True)
    cs = [c1, c2, np.conj(c1), np.conj(c2)]
    xs = D.samples(G)
    hvp = sum(np.exp(1j * (x * a + z * b)) * c for (a, b), c in zip(xs, cs))
    assert np.abs(hvp.imag).max() < 1e-12
    cols = D.columns(G, hvp.real)
    for k in range(4):
        assert np.allclose(cols[k], cs[k], atol=1e-12)


def _separable(G, rng, alpha=1.0, beta=0.4):
    c = 1.5 + 0.5 * band_limited(G, rng, 2)
    sig = D.on_lattice(G, lambda xx, zz: np.hypot(xx, zz) * (
        alpha + beta * np.cos(2 * np.arctan2(zz, xx))))
    H = lambda v: c * D.synth_from(G, sig * D.hat(G, v)).real
    return c, H


def test_pdo_exact_for_separable_symbol():
    n = 24
    G = synth.SymbolGrid(n, n, n, n, 1.0, 4, 2 * np.pi * 6 / n)
    rng = np.random.default_rng(3)
    c, H = _separable(G, rng)
    cols = D.columns(G, H(D.probe(G)))
    for k, (a, b) in enumerate(D.samples(G)):
        th = np.arctan2(b, a)
        assert np.allclose(cols[k], c * G.rho0 * (1.0 + 0.4 * np.cos(2 * th)), atol=1e-11)
    v = rng.standard_normal((n, n))
    assert np.allclose(D.pdo_apply(G, cols, v), H(v), atol=1e-10)
    # a wrong weight (no radial extension) breaks it
    bad = D.symbol_apply(G, cols, np.ones((4, n, n), complex) * D.on_lattice(
        G, lambda xx, zz: 0 * xx + 0.25), v)
    assert not np.allclose(bad, H(v), atol=1e-3)


def test_columns_resynthesise_and_pair():
    G = synth.symbol_grid(20, 28, 5.0, 7, r=8, rho0=0.37)
    rng = np.random.default_rng(4)
    g = rng.standard_normal((G.nz, G.nx))
    cols = D.columns(G, g)
    x, z = D.coords(G)
    back = sum(np.exp(1j * (x * a + z * b)) * cols[k] for k, (a, b) in enumerate(D.samples(G)))
    assert np.allclose(back, g, atol=1e-12)
    for k in range(4):
        assert np.allclose(cols[k + 4], np.conj(cols[k]), atol=1e-12)
    v = D.probe(G)
    x, z = D.coords(G)
    alt = sum(2 * np.cos(x * a + z * b) for a, b in D.samples(G)[:4])
    assert np.allclose(v, alt, atol=1e-12)


def test_psf_plus_closed_form_on_separable_symbol():
    nz, nx, h = 30, 40, 2.0
    pg = synth.psf_grid(nz, nx, spacing=8, half=3)
    G = synth.symbol_grid(nz, nx, h, pg.half, r=8, rho0=0.9)
    rng = np.random.default_rng(5)
    kap = rng.standard_normal((7, 7))
    kap = kap + kap[::-1, ::-1]  # even kernel: real symbol
    zz, xx = np.mgrid[0:nz, 0:nx]
    cfield = 1.0 + 0.3 * np.sin(zz / 5.0) * np.cos(xx / 7.0) + 0.01 * xx
    ck = np.array([cfield[iz, ix] for iz, ix in pg.centres()])
    psf = ck[:, None, None] * kap[None]
    sig_c = np.array([np.sum(kap * np.exp(1j * h * (np.arange(-3, 4)[:, None] * b +
                                                   np.arange(-3, 4)[None, :] * a)))
                      for a, b in D.samples(G)])
    cols = cfield[None] * sig_c[:, None, None]
    A, B, alpha = D.psf_plus(G, pg, psf, cols, rank=1)
    v = rng.standard_normal((nz, nx))
    got = D.psf_plus_apply(G, A, B, v)
    c_interp = np.einsum("kzx,k->zx", P.weights(pg), ck)
    expect = 0.5 * (cfield + c_interp) * correlate2d(v, kap, mode="same")
    assert np.allclose(got, expect, atol=1e-10 * np.abs(expect).max())
    assert alpha > 0


def test_psf_plus_full_rank_with_psf_columns_is_psf():
    nz, nx, h = 16, 18, 1.0
    pg = synth.psf_grid(nz, nx, spacing=8, half=3)
    assert pg.r == 4
    G = synth.symbol_grid(nz, nx, h, pg.half, r=8, rho0=1.1)
    rng = np.random.default_rng(6)
    psf = rng.standard_normal((pg.r, pg.width, pg.width))
    W = P.weights(pg)
    Sc = D.rows_at(G, pg, psf, D.samples(G))  # [r_psf][r]
    cols = np.einsum("kzx,kc->czx", W, Sc)
    A, B, _ = D.psf_plus(G, pg, psf, cols, rank=pg.r)
    v = rng.standard_normal((nz, nx))
    got = D.psf_plus_apply(G, A, B, v)
    assert np.allclose(got, P.apply_rows(pg, psf, v), atol=1e-10)
    # a truncated basis with the same columns no longer reproduces it
    A2, B2, _ = D.psf_plus(G, pg, psf, cols, rank=2)
    assert not np.allclose(D.psf_plus_apply(G, A2, B2, v), P.apply_rows(pg, psf, v), atol=1e-3)


def test_psf_plus_closed_form_rank_two():
    """Rows c_k sigma1 + e_k sigma2 with an even kernel kappa1 and an odd
    kernel kappa2: sigma1 and sigma2 are orthogonal on the lattice and over
    the +-xi_k sample pairs, so in the basis (sigma1/|sigma1|,
    sigma2/|sigma2|) B[:, I_c] B[:, I_c]^H = diag(n1^2, n2^2) and the
    Tikhonov solution is coefficientwise
        (n_j^2 t_j + alpha t_j^I) / (n_j^2 + alpha),  alpha = (n1^2 + n2^2)/2,
    t the true coefficient field and t^I its tent interpolant (the product
    A B does not depend on the orthonormal basis the SVD picks).  Norms by
    Parseval: |sigma|^2 = M sum_d kappa(d)^2."""
    nz, nx, h = 26, 34, 3.0
    pg = synth.psf_grid(nz, nx, spacing=8, half=3)
    G = synth.symbol_grid(nz, nx, h, pg.half, r=8, rho0=0.45)
    rng = np.random.default_rng(7)
    k1 = rng.standard_normal((7, 7))
    k1 = k1 + k1[::-1, ::-1]
    k2 = rng.standard_normal((7, 7))
    k2 = k2 - k2[::-1, ::-1]
    zz, xx = np.mgrid[0:nz, 0:nx]
    c = 1.0 + 0.4 * np.cos(zz / 4.0 + xx / 9.0)
    e = 0.5 * np.sin(xx / 6.0) - 0.02 * zz
    cen = pg.centres()
    ck = np.array([c[i, j] for i, j in cen])
    ek = np.array([e[i, j] for i, j in cen])
    psf = ck[:, None, None] * k1 + ek[:, None, None] * k2
    d = np.arange(-3, 4) * h
    sig = lambda kap, a, b: np.sum(kap * np.exp(1j * (d[:, None] * b + d[None, :] * a)))
    s1 = np.array([sig(k1, a, b) for a, b in D.samples(G)])
    s2 = np.array([sig(k2, a, b) for a, b in D.samples(G)])
    cols = c[None] * s1[:, None, None] + e[None] * s2[:, None, None]
    A, B, alpha = D.psf_plus(G, pg, psf, cols, rank=2)
    M = G.mz * G.mx
    n1 = np.sum(np.abs(s1) ** 2) / (M * np.sum(k1 ** 2))
    n2 = np.sum(np.abs(s2) ** 2) / (M * np.sum(k2 ** 2))
    assert alpha == pytest.approx(0.5 * (n1 + n2), rel=1e-10)
    Wt = P.weights(pg)
    cI = np.einsum("kzx,k->zx", Wt, ck)
    eI = np.einsum("kzx,k->zx", Wt, ek)
    a1 = (n1 * c + alpha * cI) / (n1 + alpha)
    a2 = (n2 * e + alpha * eI) / (n2 + alpha)
    v = rng.standard_normal((nz, nx))
    expect = a1 * correlate2d(v, k1, mode="same") + a2 * correlate2d(v, k2, mode="same")
    got = D.psf_plus_apply(G, A, B, v)
    assert np.allclose(got, expect, atol=1e-10 * np.abs(expect).max())

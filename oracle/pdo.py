"""FP64 oracle of the pseudo-differential operator probing method (PDO,
Section 3.4 and Appendix A), of the low-rank symbol method PSF+ (Section
3.6), and of the low-rank symbol apply both share (Section 3.3, eq.
"lr-psido").

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by the tests
and the benchmark's CPU-baseline leg; shares no code with the HIP library.
Plain NumPy, float64 / complex128; ``numpy.fft`` and ``numpy.linalg`` serve as
library steps.

Discrete setting (``synth.SymbolGrid``):

* a periodic FFT grid of mz x mx cells of spacing h; the model grid is its
  first nz rows and nx columns, the rest is zero padding.  A cell (iz, ix) is
  the point x = (ix h, iz h) (first component horizontal).
* Lattice frequencies xi = (2 pi q / (mx h), 2 pi p / (mz h)) for the centred
  representatives p, q.  On an even length the Nyquist index has two
  representatives (+m/2 and -m/2); every function of xi evaluated on the
  lattice below is the average over the representatives of the point, which
  keeps it symmetric under xi -> -xi.
* The transform pair of the footnote of Section 3.3, with sums for the
  integrals: v^(xi) = (1/M) sum_x e^{-i x.xi} v(x), v(x) = sum_xi e^{i x.xi}
  v^(xi), M = mz mx.  The discrete symbol of an operator H on the grid is
  S[x, xi] = (H phi_xi)(x) / phi_xi(x), phi_xi(x) = e^{i x.xi}, so that
  (H v)(x) = sum_xi e^{i x.xi} S[x, xi] v^(xi) exactly (eq. "psido").
* Low-rank symbol apply (eqs. "lr_symbol" and "lr-psido"): for
  S ~ sum_k a_k(x) b_k(xi),
      (H~ v)(x) = Re sum_k a_k(x) sum_xi e^{i x.xi} b_k(xi) v^(xi)
  on the model grid, v zero-padded.  (The real part: a real operator's
  symbol satisfies S[x, -xi] = conj S[x, xi], and for such a symbol the sum is
  real; the rounding residue of the imaginary part is discarded.)

PDO (Section 3.4, Appendix A):

* sample frequencies xi_k = rho0 (cos theta_k, sin theta_k), theta_k =
  2 pi k / r, k = 1..r (r even; the paper uses r = 8, rho0 ~ 2 pi f_max /
  c_max read as an angular wavenumber);
* probe v_p = sum_k phi_{xi_k} (eq. "pdo-vp"), real because the angles come in
  pairs theta, theta + pi;
* spectral separation: the spectrum of H v_p is split among the samples by
  nearest sample frequency (the Voronoi cells of the xi_k, i.e. angular
  sectors of width 2 pi / r centred on the theta_k); a frequency equidistant
  from several samples (the origin, and cell boundaries that fall on lattice
  points) is shared equally among them.  Symbol column k is
  s_k = (F^-1 of the k-th part) / phi_{xi_k} (eq. "symbol").
* weights (eq. "pdo-w"): w_k(xi) = (rho / rho0) w_k^circle(theta), with the
  angular FFT (trigonometric) interpolation cardinal functions
  w_k^circle(theta) = (1/r) [1 + 2 sum_{m=1}^{r/2-1} cos(m (theta - theta_k))
  + cos((r/2)(theta - theta_k))] (the Nyquist mode split evenly, so the
  weights are real);
* the PDO approximation is the low-rank symbol (s_k, w_k) (eq. "pdo-symbol").

PSF+ (Section 3.6), from the PSFs of ``oracle.psf`` and the PDO columns:

1. symbol rows S~[x_k, xi] = sum_d p_k(d) e^{i d.xi} on the lattice (the
   discrete form of (2 pi)^2 conj(p^_k)); S_psf = W S~[I_r, :] with the
   tent weights W of the PSF method;
2. SVD S~[I_r, :] = U Sigma V^H; B = the leading `rank` rows of V^H
   (orthonormal), A0 = W U_rank Sigma_rank;
3. min_A ||A B[:, I_c] - S~[:, I_c]||_F^2 + alpha ||A - A0||_F^2 with
   alpha = ||B[:, I_c]||_F^2 / ||B||_F^2 (eq. "psfplus"), solved as the
   stacked least-squares problem [B[:, I_c]^T; sqrt(alpha) I] a(x) =
   [S~[x, I_c]; sqrt(alpha) A0[x, :]] for every model cell x.  The sampled
   frequencies are off the lattice, so B[:, I_c] is evaluated from the row
   definition: B[:, xi] = Sigma^-1 U^H S~[I_r, xi] with S~[x_k, xi_c] summed
   directly.

Pins (tests/test_oracle_pdo.py): the full-rank apply reproduces a dense
operator from its brute-force symbol; interpolation, partition and symmetry
properties of the weights and masks; exact recovery of symbol columns and of
the whole PDO operator for lattice-aligned samples and a symbol of the form
c(x) rho (alpha + beta cos 2 theta); the sum of the columns rebuilds H v_p;
conjugate pairing of the columns; a closed form of the PSF+ solution for a
separable symbol; PSF+ at full rank with columns taken from the PSF
approximation equals the PSF method's own symbol-row form.
"""
from __future__ import annotations

import numpy as np

from oracle import psf as P


# --------------------------------------------------------------------------
# lattice and transforms
# --------------------------------------------------------------------------

def _axis(m: int, h: float):
    """The two representatives (equal except at an even length's Nyquist
    index) of the lattice frequencies along one axis."""
    k = np.arange(m)
    c = np.where(k <= m // 2, k, k - m).astype(np.float64)
    alt = c.copy()
    if m % 2 == 0:
        alt[m // 2] = -(m // 2)
    s = 2.0 * np.pi / (m * h)
    return c * s, alt * s


def on_lattice(G, f):
    """[mz][mx] values of f(xi_x, xi_z) averaged over the representatives of
    each lattice point; f takes broadcastable arrays."""
    zc, za = _axis(G.mz, G.h)
    xc, xa = _axis(G.mx, G.h)
    acc = 0.0
    for z in (zc, za):
        for x in (xc, xa):
            acc = acc + f(x[None, :], z[:, None])
    return acc / 4.0


def coords(G):
    """Model-grid coordinates (x[nz][nx], z[nz][nx])."""
    z = (np.arange(G.nz) * G.h)[:, None] * np.ones((1, G.nx))
    x = np.ones((G.nz, 1)) * (np.arange(G.nx) * G.h)[None, :]
    return x, z


def pad(G, v):
    out = np.zeros(np.shape(v)[:-2] + (G.mz, G.mx), dtype=np.result_type(v, np.float64))
    out[..., :G.nz, :G.nx] = v
    return out


def hat(G, v):
    """v^ = (1/M) sum_x e^{-i x.xi} v(x) of a zero-padded model-grid field."""
    return np.fft.fft2(pad(G, v)) / (G.mz * G.mx)


def synth_from(G, vhat):
    """sum_xi e^{i x.xi} vhat(xi), on the model grid."""
    return (np.fft.ifft2(vhat) * (G.mz * G.mx))[..., :G.nz, :G.nx]


def symbol_apply(G, a, b, v):
    """(H~ v)(x) = Re sum_k a_k(x) sum_xi e^{i x.xi} b_k(xi) v^(xi); a[K][nz][nx],
    b[K][mz][mx] (complex), v[nz][nx] real."""
    vh = hat(G, v)
    out = np.zeros((G.nz, G.nx), dtype=np.complex128)
    for k in range(len(a)):
        out += a[k] * synth_from(G, b[k] * vh)
    return out.real


def full_symbol(G, H):
    """S[x, xi] of a dense operator H on the whole periodic grid (nz = mz,
    nx = mx), columns indexed like numpy's FFT output: [M][mz][mx]."""
    assert (G.nz, G.nx) == (G.mz, G.mx)
    x, z = coords(G)
    zc, _ = _axis(G.mz, G.h)
    xc, _ = _axis(G.mx, G.h)
    S = np.empty((G.mz * G.mx, G.mz, G.mx), dtype=np.complex128)
    for p in range(G.mz):
        for q in range(G.mx):
            phi = np.exp(1j * (x * xc[q] + z * zc[p]))
            S[:, p, q] = (H @ phi.ravel()) / phi.ravel()
    return S


# --------------------------------------------------------------------------
# PDO
# --------------------------------------------------------------------------

def thetas(r: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(1, r + 1) / r


def samples(G) -> np.ndarray:
    """[r][2] sample frequencies (xi_x, xi_z) on the circle of radius rho0."""
    t = thetas(G.r)
    return G.rho0 * np.stack([np.cos(t), np.sin(t)], axis=1)


def probe(G) -> np.ndarray:
    """v_p = sum_k e^{i x.xi_k} on the model grid (real up to rounding)."""
    x, z = coords(G)
    v = np.zeros((G.nz, G.nx), dtype=np.complex128)
    for xk, zk in samples(G):
        v += np.exp(1j * (x * xk + z * zk))
    return v.real


TIE = 1e-9  # relative tolerance under which two distances count as equal


def masks(G) -> np.ndarray:
    """[r][mz][mx] spectral separation: share of each lattice frequency
    assigned to sample k (nearest sample frequency, ties shared equally)."""
    xs = samples(G)
    out = []
    for k in range(G.r):
        def f(xx, zz, k=k):
            d = np.stack([(xx - a) ** 2 + (zz - b) ** 2 for a, b in xs])
            scale = xx * xx + zz * zz + G.rho0 * G.rho0
            near = d <= d.min(axis=0) + TIE * scale
            return near[k] / near.sum(axis=0)
        out.append(on_lattice(G, f))
    return np.stack(out)


def columns(G, hvp) -> np.ndarray:
    """[r][nz][nx] complex symbol columns s(., xi_k) from H v_p."""
    gh = hat(G, hvp)
    x, z = coords(G)
    m = masks(G)
    out = []
    for k, (xk, zk) in enumerate(samples(G)):
        part = synth_from(G, m[k] * gh)
        out.append(part / np.exp(1j * (x * xk + z * zk)))
    return np.stack(out)


def circle_weights(r: int, theta) -> np.ndarray:
    """[r][...] trigonometric interpolation cardinal functions on the nodes
    theta_k = 2 pi k / r."""
    theta = np.asarray(theta, dtype=np.float64)
    out = []
    for tk in thetas(r):
        d = theta - tk
        w = np.ones_like(d)
        for m in range(1, r // 2):
            w = w + 2.0 * np.cos(m * d)
        w = w + np.cos((r // 2) * d)
        out.append(w / r)
    return np.stack(out)


def weights(G) -> np.ndarray:
    """[r][mz][mx] w_k(xi) = (rho / rho0) w_k^circle(theta)."""
    out = []
    for k in range(G.r):
        def f(xx, zz, k=k):
            rho = np.sqrt(xx * xx + zz * zz)
            return rho / G.rho0 * circle_weights(G.r, np.arctan2(zz, xx))[k]
        out.append(on_lattice(G, f))
    return np.stack(out)


def pdo_apply(G, cols, v):
    """PDO approximation of H applied to v: the low-rank symbol (s_k, w_k)."""
    return symbol_apply(G, cols, weights(G).astype(np.complex128), v)


# --------------------------------------------------------------------------
# PSF+
# --------------------------------------------------------------------------

def psf_rows(G, pg, psf) -> np.ndarray:
    """[r_psf][mz][mx] symbol rows sum_d p_k(d) e^{i d.xi} on the lattice."""
    assert pg.width <= min(G.mz, G.mx)
    return P.symbol_rows(pg, psf, (G.mz, G.mx))


def rows_at(G, pg, psf, xis) -> np.ndarray:
    """[r_psf][len(xis)] symbol rows at arbitrary frequencies, summed directly."""
    d = np.arange(-pg.half, pg.half + 1) * G.h
    out = np.empty((pg.r, len(xis)), dtype=np.complex128)
    for c, (xx, zz) in enumerate(xis):
        e = np.exp(1j * (d[:, None] * zz + d[None, :] * xx))  # [dz][dx]
        out[:, c] = np.einsum("kzx,zx->k", psf, e)
    return out


def psf_plus(G, pg, psf, cols, rank):
    """Coefficients A[rank][nz][nx] and row basis B[rank][mz][mx] of the PSF+
    low-rank symbol A B."""
    rows = psf_rows(G, pg, psf).reshape(pg.r, -1)
    U, s, Vh = np.linalg.svd(rows, full_matrices=False)
    U, s = U[:, :rank], s[:rank]
    B = Vh[:rank]
    W = P.weights(pg).reshape(pg.r, -1).T  # [N][r_psf]
    A0 = W @ (U * s)  # [N][rank]
    Bc = (U.conj().T @ rows_at(G, pg, psf, samples(G))) / s[:, None]  # [rank][r]
    alpha = np.sum(np.abs(Bc) ** 2) / np.sum(np.abs(B) ** 2)
    C = cols.reshape(G.r, -1)  # [r][N]: row c is S~[:, xi_c]
    K = np.vstack([Bc.T, np.sqrt(alpha) * np.eye(rank)])
    rhs = np.vstack([C, np.sqrt(alpha) * A0.T])
    X = np.linalg.lstsq(K, rhs, rcond=None)[0]  # [rank][N] = A^T
    return X.reshape(rank, G.nz, G.nx), B.reshape(rank, G.mz, G.mx), alpha


def psf_plus_apply(G, A, B, v):
    return symbol_apply(G, A, B, v)

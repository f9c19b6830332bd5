"""Pins of the low-rank oracle (oracle/lowrank.py) against facts fixed by
the mathematics of Sections 2 and 3.1:

* the mirrored-edge 5-point Laplacian has the closed-form DCT-II eigenpairs
  -(4/h^2)(sin^2(pi p / 2 nz) + sin^2(pi q / 2 nx));
* R on the cosine modes is (delta + gamma (4/h^2)(sin^2 + sin^2))^2, and
  R^-1 R = I;
* when the probes outnumber the rank of H_d, the randomized double pass
  returns the pencil's leading eigenpairs exactly (against scipy.linalg.eigh
  on the dense pencil), R-orthonormal, with H V = R V L (the null directions
  of the probe images are dropped);
* at full rank the three formulas of Section 3.1 are exact: (H~_d + R) v,
  (H~_d + R)^-1 v (Woodbury), and the covariance of the samples,
  M M^T = (H_d + R)^-1 for the linear map M: w -> zeta.
"""
import numpy as np
import pytest
from scipy.linalg import eigh

from oracle import lowrank as LR
from paper_2507_10804_amd import synth


def small_prior(nz=6, nx=7, h=10.0):
    return synth.matern_prior(nz, nx, h, corr_length=30.0, std=2.0)


def dense(op, n, shape):
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = np.asarray(op(e.reshape(shape))).ravel()
    return M


def test_laplacian_dct_eigenpairs():
    nz, nx, h = 9, 13, 7.0
    L = LR.laplacian(nz, nx, h)
    i = np.arange(nz)[:, None] + 0.5
    j = np.arange(nx)[None, :] + 0.5
    for p, q in [(0, 0), (1, 0), (0, 5), (4, 7), (8, 12)]:
        phi = np.cos(np.pi * p * i / nz) * np.cos(np.pi * q * j / nx)
        mu = -(4.0 / h**2) * (np.sin(np.pi * p / (2 * nz)) ** 2 + np.sin(np.pi * q / (2 * nx)) ** 2)
        assert np.allclose(L @ phi.ravel(), mu * phi.ravel(), atol=1e-12)
    assert np.allclose((L - L.T).toarray(), 0.0)


def test_prior_on_dct_modes():
    """R phi_pq = (delta + gamma (4/h^2)(sin^2 + sin^2))^2 phi_pq: the Matern
    precision (delta I - gamma Lap)^2 on the cosine modes."""
    P = synth.matern_prior(11, 17, 8.0, corr_length=60.0, std=3.0)
    pr = LR.Prior(P)
    i = np.arange(P.nz)[:, None] + 0.5
    j = np.arange(P.nx)[None, :] + 0.5
    for p, q in [(0, 0), (2, 3), (10, 16), (5, 0)]:
        phi = np.cos(np.pi * p * i / P.nz) * np.cos(np.pi * q * j / P.nx)
        mu = (4.0 / P.h**2) * (np.sin(np.pi * p / (2 * P.nz)) ** 2 +
                               np.sin(np.pi * q / (2 * P.nx)) ** 2)
        expect = (P.delta + P.gamma * mu) ** 2 * phi
        assert np.allclose(pr.apply(phi), expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())
        assert np.allclose(pr.solve(expect), phi, rtol=1e-8, atol=1e-10)


def test_prior_solve_inverts_apply():
    pr = LR.Prior(synth.matern_prior(20, 31, 10.0, corr_length=100.0, std=50.0))
    x = np.random.default_rng(0).standard_normal((3, 20, 31))
    assert np.allclose(pr.solve(pr.apply(x)), x, rtol=1e-9, atol=1e-9 * np.abs(x).max())
    y = pr.apply(pr.solve(x))
    assert np.linalg.norm(y - x) / np.linalg.norm(x) < 1e-9


def _pencil(rank, seed=1):
    """H = U diag(d) U^T, U random orthogonal, `rank` eigenvalues from 1e-3
    down to 1e-5 (a conditioning the double precision Gram matrices of the
    algorithm resolve at full rank), the rest zero."""
    P = small_prior()
    pr = LR.Prior(P)
    n = P.nz * P.nx
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.zeros(n)
    d[:rank] = 1e-3 * np.geomspace(1.0, 1e-2, rank)
    H = (U * d) @ U.T
    return P, pr, n, 0.5 * (H + H.T)


def test_double_pass_exact_on_low_rank_pencil():
    P, pr, n, H = _pencil(rank=8)
    R = dense(pr.apply, n, (P.nz, P.nx))
    hv = lambda X: (H @ X.reshape(X.shape[0], -1).T).T.reshape(X.shape)
    omega = synth.gaussian_probes(P.nz, P.nx, 12, seed=3)
    lam, V = LR.double_pass(hv, pr, omega, r=8)
    ref = eigh(H, R, eigvals_only=True)[::-1][:8]
    assert np.allclose(lam, ref, rtol=1e-8)
    Vf = V.reshape(8, -1)
    assert np.allclose(Vf @ R @ Vf.T, np.eye(8), atol=1e-9)
    assert np.allclose(H @ Vf.T, R @ Vf.T * lam, rtol=1e-7, atol=1e-9 * np.abs(H).max())


def test_full_rank_formulas_are_exact():
    P, pr, n, H = _pencil(rank=42, seed=2)
    R = dense(pr.apply, n, (P.nz, P.nx))
    hv = lambda X: (H @ X.reshape(X.shape[0], -1).T).T.reshape(X.shape)
    omega = synth.gaussian_probes(P.nz, P.nx, n, seed=4)
    lam, V = LR.double_pass(hv, pr, omega, r=n)
    shape = (P.nz, P.nx)
    Hs = dense(lambda v: LR.hessian_apply(pr, lam, V, v), n, shape)
    assert np.allclose(Hs, H + R, rtol=1e-7, atol=1e-9 * np.abs(H + R).max())
    Hi = dense(lambda v: LR.inverse_apply(pr, lam, V, v), n, shape)
    assert np.allclose(Hi, np.linalg.inv(H + R), rtol=1e-6, atol=1e-8 * np.abs(Hi).max())
    M = dense(lambda w: LR.sample(pr, lam, V, w), n, shape)
    C = M @ M.T
    assert np.allclose(C, np.linalg.inv(H + R), rtol=1e-6, atol=1e-8 * np.abs(C).max())


def test_truncated_formulas_exact_at_the_rank_of_h():
    P, pr, n, H = _pencil(rank=6, seed=5)
    R = dense(pr.apply, n, (P.nz, P.nx))
    hv = lambda X: (H @ X.reshape(X.shape[0], -1).T).T.reshape(X.shape)
    omega = synth.gaussian_probes(P.nz, P.nx, 10, seed=6)
    lam, V = LR.double_pass(hv, pr, omega, r=6)
    v = np.random.default_rng(7).standard_normal((P.nz, P.nx))
    got = LR.inverse_apply(pr, lam, V, v).ravel()
    assert np.allclose(got, np.linalg.solve(H + R, v.ravel()), rtol=1e-6,
                       atol=1e-8 * np.abs(got).max())
    got = LR.hessian_apply(pr, lam, V, v).ravel()
    assert np.allclose(got, (H + R) @ v.ravel(), rtol=1e-7, atol=1e-9 * np.abs(got).max())

"""FP64 oracle of the low-rank Hessian approximation (Section 3.1) under the
Matern prior of Section 2.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by the tests
and the benchmark's CPU-baseline leg; shares no code with the HIP library.

* Prior precision R = A^2, A = delta I - gamma Lap_h, Lap_h the 5-point
  Laplacian on the nz x nx model grid with mirrored ghost cells (zero flux at
  every edge), h the grid spacing.  A is a sparse SPD matrix; R^-1 is two
  sparse LU solves with A.
* The generalized eigenproblem H_d v = lambda R v (Section 3.1, eq. "eig")
  by the double-pass randomized algorithm for Hermitian pencils (Saibaba,
  Lee and Kitanidis 2016, the method of the hIPPYlib framework the paper
  cites): Y = R^-1 H_d Omega; an R-orthonormal basis Q of range(Y) by two
  rounds of Gram-matrix diagonalisation in the R inner product (dropping
  numerically null directions); T = Q^T H_d Q; T = U L U^T; V = Q U,
  keeping the r largest eigenvalues.  V^T R V = I.
* The approximations built on it (Section 3.1):
    (H~_d + R) v      = R v + R V L V^T R v
    (H~_d + R)^-1 v   = R^-1 v - V D V^T v,   D = L (L + I)^-1
    zeta              = (I - V S V^T R) z,     S = I - (L + I)^-1/2,
  with z ~ N(0, R^-1), i.e. z = A^-1 w for white w.

Pins (tests/test_oracle_lowrank.py): the Laplacian's closed-form DCT
eigenpairs; R^-1 R = I; exact recovery of the pencil's eigenpairs when the
probes span the range of H_d (against scipy.linalg.eigh on the dense pencil);
R-orthonormality; the Woodbury identities of the three formulas on dense
matrices at full rank; the sample covariance identity.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import eigh


def laplacian(nz: int, nx: int, h: float) -> sp.csr_matrix:
    """5-point Laplacian, row-major (x fastest), mirrored ghosts at the edges."""

    def lap1(n):
        main = -2.0 * np.ones(n)
        if n > 1:
            main[0] = main[-1] = -1.0
        else:
            main[0] = 0.0
        off = np.ones(n - 1)
        return sp.diags([off, main, off], [-1, 0, 1], format="csr")

    return (sp.kron(lap1(nz), sp.identity(nx)) + sp.kron(sp.identity(nz), lap1(nx))) / (h * h)


class Prior:
    def __init__(self, pr):
        self.pr = pr
        n = pr.nz * pr.nx
        self.A = (pr.delta * sp.identity(n) - pr.gamma * laplacian(pr.nz, pr.nx, pr.h)).tocsc()
        self._lu = spla.splu(self.A)

    def _flat(self, v):
        return np.asarray(v, dtype=np.float64).reshape(-1, self.pr.nz * self.pr.nx)

    def apply(self, v):
        """R v for v[..., nz, nx]."""
        x = self._flat(v)
        return (self.A @ (self.A @ x.T)).T.reshape(np.shape(v))

    def solve(self, b):
        """R^-1 b."""
        x = self._flat(b)
        y = np.stack([self._lu.solve(self._lu.solve(c)) for c in x])
        return y.reshape(np.shape(b))

    def sqrt_inv(self, w):
        """A^-1 w: a draw from N(0, R^-1) for white w."""
        x = self._flat(w)
        return np.stack([self._lu.solve(c) for c in x]).reshape(np.shape(w))


def r_orthonormalize(Y, RY, tol=1e-10):
    """Rows Q spanning the rows of Y with Q R Q^T = I: twice, the Gram matrix
    G = Y R Y^T is diagonalised, directions with eigenvalue below tol times
    the largest are dropped and the rest scaled to unit R-norm.  Returns
    (Q, R Q); Q may have fewer rows than Y when Y is rank deficient."""
    Q, RQ = Y, RY
    for _ in range(2):
        G = Q @ RQ.T
        G = 0.5 * (G + G.T)
        sig, W = eigh(G)
        keep = sig > tol * sig.max()
        T = W[:, keep].T / np.sqrt(sig[keep])[:, None]
        Q, RQ = T @ Q, T @ RQ
    return Q, RQ


def double_pass(hv, prior: Prior, omega, r, tol=1e-10):
    """r largest eigenpairs of H_d v = lambda R v.  hv maps [k][nz][nx] to
    H_d applied to each; omega[k][nz][nx] are the random probes (k > r).
    Returns (lambda[r] descending, V[r][nz][nx])."""
    shape = omega.shape
    k = shape[0]
    n = shape[1] * shape[2]
    Ybar = np.asarray(hv(omega), dtype=np.float64).reshape(k, n)
    Y = prior.solve(Ybar.reshape(shape)).reshape(k, n)
    Q, _ = r_orthonormalize(Y, Ybar, tol)  # R Y = Ybar
    kq = Q.shape[0]
    HQ = np.asarray(hv(Q.reshape((kq,) + shape[1:])), dtype=np.float64).reshape(kq, n)
    T = Q @ HQ.T
    T = 0.5 * (T + T.T)
    lam, U = eigh(T)
    order = np.argsort(lam)[::-1][:r]
    lam, U = lam[order], U[:, order]
    V = U.T @ Q
    return lam, V.reshape((len(lam),) + shape[1:])


def hessian_apply(prior: Prior, lam, V, v):
    """(H~_d + R) v = R v + R V L V^T R v."""
    Vf = V.reshape(len(lam), -1)
    Rv = prior.apply(v).reshape(-1)
    RV = prior.apply(V).reshape(len(lam), -1)
    return (Rv + RV.T @ (lam * (Vf @ Rv))).reshape(np.shape(v))


def inverse_apply(prior: Prior, lam, V, v):
    """(H~_d + R)^-1 v = R^-1 v - V D V^T v."""
    Vf = V.reshape(len(lam), -1)
    d = lam / (lam + 1.0)
    vf = np.asarray(v, dtype=np.float64).reshape(-1)
    return (prior.solve(v).reshape(-1) - Vf.T @ (d * (Vf @ vf))).reshape(np.shape(v))


def sample(prior: Prior, lam, V, w):
    """zeta = (I - V S V^T R) z with z = A^-1 w."""
    Vf = V.reshape(len(lam), -1)
    s = 1.0 - 1.0 / np.sqrt(lam + 1.0)
    z = prior.sqrt_inv(w).reshape(-1)
    Rz = prior.apply(z.reshape(np.shape(w))).reshape(-1)
    return (z - Vf.T @ (s * (Vf @ Rz))).reshape(np.shape(w))

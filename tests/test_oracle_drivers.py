"""Pins of the L-BFGS and gpCN oracle (oracle/drivers.py):

* the two-loop recursion equals the explicit BFGS inverse-Hessian update
  H+ = (I - rho s y^T) H (I - rho y s^T) + rho s s^T applied pair by pair to
  a dense H0 (Nocedal and Wright, eqs. 6.17 and 7.19);
* with the exact inverse Hessian as H0, L-BFGS solves a quadratic in one
  unit step; with the scaled identity it decreases Phi monotonically and
  converges to the minimiser;
* grad Phi (data misfit plus Matern prior) against central differences on a
  16 x 16 wave problem;
* gpCN: the first proposal follows eq. "gpcn" in closed form; with an exact
  Laplace approximation (Phi quadratic with Hessian H~) Delta is constant and
  every proposal is accepted; a planted Delta jump is accepted exactly when
  u < exp(-jump).
"""
import math

import numpy as np
import pytest

from oracle import drivers as Dr
from oracle import lowrank as LR
from paper_2507_10804_amd import synth


def _spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def test_two_loop_equals_explicit_bfgs_update():
    n = 12
    rng = np.random.default_rng(0)
    A = _spd(n, 1)
    H0 = _spd(n, 2, cond=5.0)
    S = [rng.standard_normal(n) for _ in range(4)]
    Y = [A @ s for s in S]
    H = H0.copy()
    I = np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    g = rng.standard_normal(n)
    assert np.allclose(Dr.two_loop(g, S, Y, lambda q: H0 @ q), H @ g, rtol=1e-10, atol=1e-12)


def test_lbfgs_exact_h0_solves_quadratic_in_one_step():
    n = 15
    A = _spd(n, 3)
    b = np.random.default_rng(4).standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    Ainv = np.linalg.inv(A)
    out = Dr.lbfgs(fg, np.zeros(n), 1, h0=lambda q: Ainv @ q)
    assert out["t"] == [1.0] and out["backtracks"] == [0]
    assert np.allclose(out["m"][1], np.linalg.solve(A, b), rtol=1e-10)


def test_lbfgs_scaled_operator_h0_recovers_the_unit_step():
    """H0 = c A^-1 with c = 1000 on a quadratic: the first step (along the
    Newton direction, c times too long) backtracks; its pair gives
    gamma = s^T y / y^T H0 y = 1/c and the second direction is the Newton
    step: unit step, no backtracking, onto the minimiser."""
    n = 12
    A = _spd(n, 5)
    b = np.random.default_rng(6).standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    Ainv = np.linalg.inv(A)
    out = Dr.lbfgs(fg, np.zeros(n), 2, h0=lambda q: 1000.0 * (Ainv @ q))
    assert out["backtracks"][0] > 0
    assert out["t"][1] == 1.0 and out["backtracks"][1] == 0
    assert np.allclose(out["m"][2], np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)


def test_lbfgs_identity_operator_equals_scaled_identity():
    """H0 given as the identity operator is scaled by s^T y / y^T y of the
    newest pair, which is the built-in scaled identity (eq. 7.20): the two
    runs take the same steps on a quadratic with condition number 50.  An
    operator applied unscaled takes shorter accepted steps and fails."""
    n = 20
    rng = np.random.default_rng(7)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.geomspace(1.0, 50.0, n)) @ Q.T
    b = rng.standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    ref = Dr.lbfgs(fg, np.zeros(n), 6)
    op = Dr.lbfgs(fg, np.zeros(n), 6, h0=lambda q: q.copy())
    assert op["t"] == ref["t"] and op["backtracks"] == ref["backtracks"]
    for a, c in zip(op["m"], ref["m"]):
        assert np.allclose(a, c, rtol=1e-12, atol=1e-14)


def test_lbfgs_scaled_identity_converges_monotonically():
    n = 10
    A = _spd(n, 5, cond=20.0)
    b = np.random.default_rng(6).standard_normal(n)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    out = Dr.lbfgs(fg, np.zeros(n), 30, mem=5)
    assert all(f1 <= f0 + 1e-13 for f0, f1 in zip(out["phi"], out["phi"][1:]))
    assert np.linalg.norm(out["m"][-1] - np.linalg.solve(A, b)) < 1e-6


def test_objective_gradient_central_differences():
    import oracle

    nx = nz = 16
    m = 2000.0 + 100.0 * synth.smooth_random((nz, nx), seed=3, sigma=3.0)
    g = synth.make_geometry(nx, nz, nt=120, ns=2, rec_ix=np.array([1, 4, 7, 10, 13]), f0=25.0,
                            v_nominal=2300.0, nb=4)
    m_true = m + 30.0 * synth.smooth_random((nz, nx), seed=4, sigma=2.0)
    dobs = oracle.forward(g, m_true)
    pr = LR.Prior(synth.matern_prior(nz, nx, g.dx, 40.0, 50.0))
    m_pr = np.full((nz, nx), 2000.0)
    f, grad = Dr.objective(g, pr, m_pr, dobs, m)
    v = synth.smooth_random((nz, nx), seed=5, sigma=2.0)
    eps = 0.05
    fp, _ = Dr.objective(g, pr, m_pr, dobs, m + eps * v)
    fm, _ = Dr.objective(g, pr, m_pr, dobs, m - eps * v)
    fd = (fp - fm) / (2 * eps)
    assert fd == pytest.approx(float(np.sum(grad * v)), rel=1e-5)


def test_gpcn_exact_laplace_accepts_everything():
    n = 8
    H = _spd(n, 7, cond=10.0)
    m_map = np.random.default_rng(8).standard_normal(n)
    L = np.linalg.cholesky(np.linalg.inv(H))
    phi = lambda m: 3.0 + 0.5 * (m - m_map) @ H @ (m - m_map)
    rng = np.random.default_rng(9)
    w = rng.standard_normal((20, n))
    u = rng.uniform(size=20)
    m0 = m_map + rng.standard_normal(n)
    states, acc, deltas = Dr.gpcn(phi, m_map, m0, 0.3, lambda wk: L @ wk, lambda x: H @ x, w, u)
    assert all(acc)
    assert np.allclose(deltas, 3.0)
    assert np.allclose(states[1], m_map + math.sqrt(1 - 0.09) * (m0 - m_map) + 0.3 * (L @ w[0]))


def test_gpcn_acceptance_rule():
    """Phi = Delta jump on one side of a hyperplane: the first proposal (made
    to land there) is accepted exactly when u < exp(-jump)."""
    n = 4
    m_map = np.zeros(n)
    jump = 0.7
    phi = lambda m: 0.5 * m @ m + (jump if m[0] > 0.5 else 0.0)
    m0 = np.zeros(n)
    w = np.array([[10.0, 0.0, 0.0, 0.0]])
    for uk, expect in ((math.exp(-jump) - 1e-6, True), (math.exp(-jump) + 1e-6, False)):
        _, acc, _ = Dr.gpcn(phi, m_map, m0, 0.2, lambda wk: wk, lambda x: x, w, [uk])
        assert acc == [expect]


@pytest.mark.parametrize("c1", [1e-4, 0.5])
def test_lbfgs_backtracking_takes_the_largest_armijo_step(c1):
    """f = a x^2 / 2 from x = 1 with H0 = I: the first step is the largest
    t = 2^-k with f(1 - t a) <= f(1) - c1 t a^2, found by brute force."""
    a = 10.0
    fg = lambda x: (0.5 * a * float(x @ x), a * x)
    out = Dr.lbfgs(fg, np.ones(1), 1, h0=lambda q: q, c1=c1)
    k = next(k for k in range(40) if 0.5 * a * (1 - a * 0.5 ** k) ** 2 <= 0.5 * a - c1 * 0.5 ** k * a * a)
    assert out["t"] == [0.5 ** k] and out["backtracks"] == [k]


def test_lbfgs_failed_line_search_keeps_the_iterate():
    """An objective that is finite only within 1e-9 of the start (every trial
    step down to t = 2^-20 lands where the wave solve would be unstable):
    no trial passes, so the iterate, Phi and the gradient stay, the step is
    recorded as failed with t = 0, and the iteration stops instead of moving
    to a point whose Phi is not finite."""
    m0 = np.array([1.0, -2.0, 0.5])

    def fg(m):
        if np.linalg.norm(m - m0) > 1e-9:
            return math.inf, np.full(3, np.nan)
        return 0.5 * float(m @ m), m.copy()

    out = Dr.lbfgs(fg, m0, 5, max_backtrack=20)
    assert out["failed"]
    assert out["t"] == [0.0] and out["backtracks"] == [20]
    assert out["evals"] == 1 + 21
    assert np.array_equal(out["m"][-1], m0) and out["phi"] == [out["phi"][0]] * 2
    assert all(math.isfinite(f) for f in out["phi"])
    # a finite objective in reach is unaffected: plain convergence on a quadratic
    ok = Dr.lbfgs(lambda m: (0.5 * float(m @ m), m.copy()), m0, 3)
    assert not ok["failed"] and ok["phi"][-1] < 1e-20

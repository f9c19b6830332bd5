"""FP64 oracle of the MAP and sampling drivers of Section 2: L-BFGS on the
negative log-posterior with an initial inverse Hessian built from a Hessian
approximation (Section 2.1), and MCMC by generalized preconditioned
Crank-Nicolson (gpCN, Section 2.3) with the Laplace approximation of Section
2.2 as proposal.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by the tests
and the benchmark's CPU-baseline leg; shares no code with the HIP library.

* Objective (Section 2.1): Phi(m) = phi_d(m) + 1/2 (m - m_pr)^T R (m - m_pr),
  phi_d the weighted data misfit of the wave-equation model (``oracle``'s C
  solver) and R the Matern prior precision (``oracle.lowrank.Prior``);
  grad Phi = grad phi_d + R (m - m_pr) (eq. "grad").
* L-BFGS (the paper cites Nocedal and Wright, Section 7.2): direction
  p = -H_k g by the two-loop recursion over the last `mem` pairs
  (s_i, y_i), rho_i = 1 / y_i^T s_i, with the initial inverse Hessian H0
  applied between the loops.  H0 is one of
    - "identity": gamma_k I, gamma_k = s^T y / y^T y of the newest pair
      (Nocedal and Wright's eq. 7.20), 1 before the first pair;
    - any linear operator M, e.g. the prior R^-1 or (H~_d + R)^-1 of a
      Hessian approximation (the paper's preconditioning), scaled the same
      way: gamma_k M, gamma_k = s^T y / y^T M y of the newest pair, 1 before
      the first pair (eq. 7.20 with M in place of the identity).  A truncated
      approximation leaves the data Hessian out of most directions, where M
      alone would take steps orders of magnitude too long; the scaling
      brings the first trial step to the curvature seen along the last step.
  Step length by backtracking from t = 1 (halving) until the Armijo
  condition Phi(m + t p) <= Phi(m) + c1 t g^T p holds, c1 = 1e-4 (a trial
  whose Phi is not finite -- an unstable wave solve -- fails it); the pair
  is stored only if s^T y > 0.  If no trial of the max_backtrack halvings
  passes, no step is taken: the iterate, Phi and gradient stay, the step is
  recorded as failed (t = 0) and the iteration stops, since the same
  direction would be tried again.  (The paper does not state its line
  search; this is the reading.)
* gpCN (Section 2.3, eq. "gpcn"): m' = m_map + sqrt(1 - beta^2)(m_k - m_map)
  + beta zeta with zeta ~ N(0, Gamma~_post), accepted when u_k < min(1,
  exp(Delta(m_k) - Delta(m'))), Delta(m) = Phi(m) - 1/2 ||m - m_map||^2
  weighted by Gamma~_post^-1 = H~ (the approximate Hessian); a proposal
  with a non-finite Delta is rejected.  The white noise behind zeta and the
  uniforms u_k are inputs.

Pins (tests/test_oracle_drivers.py): the two-loop recursion equals the
explicit BFGS inverse-Hessian update; L-BFGS with the exact inverse Hessian
as H0 solves a quadratic in one unit step, and with H0 a multiple c of it the
second step is the unit step to the minimiser (gamma = 1/c); with the scaled
identity it
converges on a quadratic and decreases Phi monotonically; grad Phi against
central differences on a small wave problem; gpCN accepts every proposal
when the Laplace approximation is exact, and its proposal and acceptance
follow the closed forms.
"""
from __future__ import annotations

import math

import numpy as np


def objective(geom, prior, m_pr, dobs, m):
    """(Phi(m), grad Phi(m)) with the C oracle's misfit and gradient."""
    import oracle

    phi_d, g_d = oracle.misfit_grad(geom, m, dobs)
    dm = np.asarray(m, np.float64) - m_pr
    Rdm = prior.apply(dm)
    return phi_d + 0.5 * float(np.sum(dm * Rdm)), g_d + Rdm


def two_loop(g, S, Y, h0):
    """H_k g by the two-loop recursion; S, Y lists ordered oldest to newest,
    h0 a callable applying the initial inverse Hessian."""
    q = np.array(g, dtype=np.float64)
    rho = [1.0 / float(np.sum(y * s)) for s, y in zip(S, Y)]
    alpha = [0.0] * len(S)
    for i in reversed(range(len(S))):
        alpha[i] = rho[i] * float(np.sum(S[i] * q))
        q = q - alpha[i] * Y[i]
    r = h0(q)
    for i in range(len(S)):
        beta = rho[i] * float(np.sum(Y[i] * r))
        r = r + S[i] * (alpha[i] - beta)
    return r


def lbfgs(fg, m0, iters, h0=None, mem=5, c1=1e-4, max_backtrack=20):
    """Run `iters` L-BFGS iterations of fg: m -> (Phi, grad).  h0 None is the
    scaled identity.  Returns a dict with the iterates, Phi values, step
    lengths, backtracking counts and objective evaluations."""
    m = np.array(m0, dtype=np.float64)
    f, g = fg(m)
    S, Y = [], []
    out = {"m": [m.copy()], "phi": [f], "t": [], "backtracks": [], "evals": 1, "failed": False}
    for _ in range(iters):
        if h0 is None:
            gam = float(np.sum(S[-1] * Y[-1]) / np.sum(Y[-1] * Y[-1])) if S else 1.0
            H0 = lambda q, gam=gam: gam * q
        else:
            gam = 1.0
            if S:
                yhy = float(np.sum(Y[-1] * h0(Y[-1])))
                if yhy > 0.0 and math.isfinite(yhy):  # H0 positive definite: always
                    gam = float(np.sum(S[-1] * Y[-1])) / yhy
            H0 = lambda q, gam=gam: gam * h0(q)
        p = -two_loop(g, S, Y, H0)
        gp = float(np.sum(g * p))
        t, nb = 1.0, 0
        while True:
            mn = m + t * p
            fn, gn = fg(mn)
            out["evals"] += 1
            if math.isfinite(fn) and fn <= f + c1 * t * gp:
                break
            if nb == max_backtrack:
                t = 0.0  # no acceptable step
                break
            t *= 0.5
            nb += 1
        if t == 0.0:
            out["m"].append(m.copy())
            out["phi"].append(f)
            out["t"].append(0.0)
            out["backtracks"].append(nb)
            out["failed"] = True
            break
        s, y = mn - m, gn - g
        if float(np.sum(s * y)) > 0.0:
            S.append(s)
            Y.append(y)
            if len(S) > mem:
                S.pop(0)
                Y.pop(0)
        m, f, g = mn, fn, gn
        out["m"].append(m.copy())
        out["phi"].append(f)
        out["t"].append(t)
        out["backtracks"].append(nb)
    return out


def gpcn(phi, m_map, m0, beta, sample, hess, w, u):
    """gpCN chain: phi(m) -> Phi; sample(w_k) -> zeta ~ N(0, Gamma~_post);
    hess(x) -> H~ x.  Returns (states, accepted flags, Delta values)."""
    m_map = np.asarray(m_map, np.float64)

    def delta(m):
        d = m - m_map
        return phi(m) - 0.5 * float(np.sum(d * hess(d)))

    m = np.array(m0, dtype=np.float64)
    dm = delta(m)
    states, acc, deltas = [m.copy()], [], [dm]
    c = math.sqrt(1.0 - beta * beta)
    for wk, uk in zip(w, u):
        prop = m_map + c * (m - m_map) + beta * sample(wk)
        dp = delta(prop)
        a = min(1.0, math.exp(min(dm - dp, 0.0))) if math.isfinite(dp) else 0.0
        if uk < a:
            m, dm = prop, dp
            acc.append(True)
        else:
            acc.append(False)
        states.append(m.copy())
        deltas.append(dm)
    return states, acc, deltas

"""MAP and sampling drivers of Section 2 on the GPU.

* :class:`Posterior`: Phi(m) = phi_d(m) + 1/2 (m - m_pr)^T R (m - m_pr) and
  its gradient (Section 2.1, eq. "grad"): the misfit and its gradient from
  the wave-equation plan, the Matern prior R from :mod:`.lowrank`.
* :class:`Lbfgs`: L-BFGS with the two-loop recursion of ``include/fwi_opt.h``
  and an initial inverse Hessian H0 that is either the scaled identity or any
  operator M -- the prior R^-1, or (H~_d + R)^-1 of a Hessian approximation
  (the paper's preconditioning) -- scaled by gamma = s^T y / y^T M y of the
  newest pair (Nocedal and Wright's eq. 7.20 with M for the identity; 1
  before the first pair), so that a truncated approximation, which leaves
  the data Hessian out of most directions, does not set trial steps orders
  of magnitude too long.  Backtracking from t = 1 by halving until
  the Armijo condition Phi(m + t p) <= Phi(m) + c1 t g^T p holds (c1 =
  1e-4); a pair is stored only if s^T y > 0.
* :func:`gpcn`: generalized preconditioned Crank-Nicolson MCMC (Section 2.3,
  eq. "gpcn") with the Laplace approximation as proposal; the white noise
  and the uniforms are inputs.

Every vector operation runs in the library's kernels (dot products, updates,
the two loops, the misfit and gradient solves, the prior and the low-rank
operators).  Python sequences the calls and takes the scalar decisions --
the Armijo test, the pair test and the acceptance test -- in FP64 on values
read back from the device.
"""
from __future__ import annotations

import ctypes
import math

from . import fwi
from . import lowrank as glr


def _p(x):
    return ctypes.c_void_p(x.data_ptr())


class Vec:
    """Dot products and updates of FP32 device vectors of n values."""

    def __init__(self, n, device):
        import torch

        self.torch = torch
        self.lib = fwi.load_library()
        self.n = int(n)
        self.device = device
        nb = ctypes.c_size_t()
        fwi._check(self.lib.fwi_vec_workspace_size(self.n, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.nws = nb.value
        self._out = torch.empty(1, dtype=torch.float64, device=device)

    def st(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _chk(self, x):
        if x.numel() != self.n or not x.is_contiguous() or x.dtype != self.torch.float32:
            raise ValueError("vectors must be contiguous float32 with n values")
        return x

    def dot(self, x, y) -> float:
        fwi._check(self.lib.fwi_vec_dot(self.n, _p(self._chk(x)), _p(self._chk(y)), _p(self._out),
                                        _p(self.ws), self.nws, self.st()))
        return float(self._out.item())

    def update(self, a, x, b, y, ad=None):
        """y = a (*ad) x + b y."""
        fwi._check(self.lib.fwi_vec_update(self.n, float(a), None if ad is None else _p(ad),
                                           _p(self._chk(x)), float(b), _p(self._chk(y)),
                                           self.st()))
        return y

    def lincomb(self, a, x, b, y, out=None):
        """out = a x + b y (out may be new)."""
        out = self.torch.empty_like(x) if out is None else out
        self.update(a, x, 0.0, out)
        return self.update(b, y, 1.0, out)


class Posterior:
    """Negative log-posterior of Section 2 on the device."""

    def __init__(self, plan: "fwi.Plan", prior: "glr.Prior", m_pr, dobs):
        self.plan, self.prior = plan, prior
        self.m_pr = m_pr.contiguous()
        self.dobs = dobs.contiguous()
        self.vec = Vec(m_pr.numel(), m_pr.device)
        self.evals = 0

    def _prior_term(self, m):
        dm = self.vec.lincomb(1.0, m, -1.0, self.m_pr)
        Rdm = self.prior.apply(glr.PRIOR_R, dm)
        return 0.5 * self.vec.dot(dm, Rdm), Rdm

    def value(self, m) -> float:
        """Phi(m); +inf when the plan flags the model (outside the stability
        limit, non-positive or not finite) or the result is not finite."""
        phi_d = self.plan.misfit(m, self.dobs)
        self.evals += 1
        if self.plan.status():
            return math.inf
        pt, _ = self._prior_term(m)
        f = float(phi_d.item()) + pt
        return f if math.isfinite(f) else math.inf

    def value_grad(self, m):
        phi_d, g = self.plan.misfit_grad(m, self.dobs)
        self.evals += 1
        if self.plan.status():
            return math.inf, g
        pt, Rdm = self._prior_term(m)
        self.vec.update(1.0, Rdm, 1.0, g)
        f = float(phi_d.item()) + pt
        return (f if math.isfinite(f) else math.inf), g


class Lbfgs:
    """L-BFGS on a :class:`Posterior` from m0; h0 None is the scaled
    identity, otherwise a callable q -> H0 q returning a new tensor."""

    def __init__(self, post: Posterior, m0, h0=None, mem=5, c1=1e-4, max_backtrack=20):
        t = post.vec.torch
        self.post, self.vec, self.h0 = post, post.vec, h0
        self.mem, self.c1, self.max_backtrack = int(mem), float(c1), int(max_backtrack)
        if not 1 <= self.mem <= 63:
            raise ValueError("mem must be in [1, 63]")
        self.m = m0.clone().contiguous()
        self.f, self.g = post.value_grad(self.m)
        shape = (self.mem + 1,) + tuple(m0.shape)  # one spare slot for a candidate pair
        dev = m0.device
        self.S = t.empty(shape, dtype=t.float32, device=dev)
        self.Y = t.empty(shape, dtype=t.float32, device=dev)
        self.rho = t.zeros(self.mem + 1, dtype=t.float64, device=dev)
        self.alpha = t.zeros(self.mem + 1, dtype=t.float64, device=dev)
        self.gamma = t.ones(1, dtype=t.float64, device=dev)
        self.slots = []  # oldest .. newest
        self.failed = False  # a line search found no acceptable step
        self.history = {"phi": [self.f], "t": [], "backtracks": []}

    def direction(self):
        lib, v = self.vec.lib, self.vec
        q = v.lincomb(1.0, self.g, 0.0, self.g)
        order = list(reversed(self.slots))
        arr = (ctypes.c_int * max(1, len(order)))(*order)
        fwi._check(lib.fwi_lbfgs_loop1(v.n, len(order), arr, _p(self.S), _p(self.Y), _p(self.rho),
                                       _p(q), _p(self.alpha), _p(v.ws), v.nws, v.st()))
        if self.h0 is None:
            r = v.torch.empty_like(q)
            v.update(1.0, q, 0.0, r, ad=self.gamma)
        else:
            gam = 1.0
            if self.slots:
                s, y = self.S[self.slots[-1]], self.Y[self.slots[-1]]
                yhy = v.dot(y, self.h0(y).contiguous())
                if yhy > 0.0 and math.isfinite(yhy):  # H0 positive definite: always
                    gam = v.dot(s, y) / yhy
            r = self.h0(q).contiguous()
            v.update(gam, r, 0.0, r)
        fwi._check(lib.fwi_lbfgs_loop2(v.n, len(order), arr, _p(self.S), _p(self.Y), _p(self.rho),
                                       _p(self.alpha), _p(r), _p(v.ws), v.nws, v.st()))
        return v.update(-1.0, r, 0.0, r)

    def step(self):
        v = self.vec
        p = self.direction()
        gp = v.dot(self.g, p)
        t, nb = 1.0, 0
        while True:
            mn = v.lincomb(1.0, self.m, t, p)
            fn, gn = self.post.value_grad(mn)
            if math.isfinite(fn) and fn <= self.f + self.c1 * t * gp:
                break
            if nb == self.max_backtrack:
                # no acceptable step: the iterate, Phi and gradient stay
                self.failed = True
                self.history["phi"].append(self.f)
                self.history["t"].append(0.0)
                self.history["backtracks"].append(nb)
                return {"phi": self.f, "t": 0.0, "backtracks": nb, "failed": True}
            t *= 0.5
            nb += 1
        slot = next(i for i in range(self.mem + 1) if i not in self.slots)
        s, y = self.S[slot], self.Y[slot]
        v.lincomb(1.0, mn, -1.0, self.m, out=s)
        v.lincomb(1.0, gn, -1.0, self.g, out=y)
        if v.dot(s, y) > 0.0:
            fwi._check(v.lib.fwi_lbfgs_pair(v.n, _p(s), _p(y), _p(self.rho[slot:]),
                                            _p(self.gamma), _p(v.ws), v.nws, v.st()))
            if len(self.slots) == self.mem:
                self.slots.pop(0)
            self.slots.append(slot)
        self.m, self.f, self.g = mn, fn, gn
        self.history["phi"].append(fn)
        self.history["t"].append(t)
        self.history["backtracks"].append(nb)
        return {"phi": fn, "t": t, "backtracks": nb, "failed": False}

    def run(self, iters):
        """Up to `iters` steps; stops after a failed line search (the same
        direction would be tried again)."""
        for _ in range(iters):
            if self.step()["failed"]:
                break
        return self.history


def gpcn(post: Posterior, m_map, m0, beta, sample, hess, w, u):
    """gpCN chain (Section 2.3): sample(w_k) -> zeta ~ N(0, Gamma~_post),
    hess(x) -> H~ x (device tensors); w[k] white-noise fields, u[k] uniforms.
    Returns (states, accepted flags, Delta values)."""
    v = post.vec
    c = math.sqrt(1.0 - beta * beta)

    def delta(m):
        f = post.value(m)
        if not math.isfinite(f):
            return math.inf
        d = v.lincomb(1.0, m, -1.0, m_map)
        return f - 0.5 * v.dot(d, hess(d).contiguous())

    m = m0.clone().contiguous()
    dm = delta(m)
    states, acc, deltas = [m.clone()], [], [dm]
    for k in range(len(u)):
        zeta = sample(w[k]).contiguous()
        prop = v.lincomb(c, m, 1.0 - c, m_map)
        v.update(beta, zeta, 1.0, prop)
        dp = delta(prop)
        a = min(1.0, math.exp(min(dm - dp, 0.0))) if math.isfinite(dp) else 0.0
        if float(u[k]) < a:
            m, dm = prop, dp
            acc.append(True)
        else:
            acc.append(False)
        states.append(m.clone())
        deltas.append(dm)
    return states, acc, deltas

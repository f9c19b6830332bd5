"""Matern prior and low-rank approximation of the misfit Hessian (Sections 2
and 3.1): thin binding of ``include/fwi_lowrank.h``.

:class:`Prior` holds the prior's device tables and applies R, R^-1 and
A^-1.  :class:`LowRank` runs the double-pass randomized method for the
pencil H_d v = lambda R v: the two batches of Hessian products go through
:meth:`fwi.Plan.gn_hvp`, the R-orthonormal range, the projected eigenproblem
and the three approximations of Section 3.1 through the library.  Python
only sequences the calls and reads back the number of kept directions.
"""
from __future__ import annotations

import ctypes

from . import fwi

PRIOR_R, PRIOR_RINV, PRIOR_AINV = 0, 1, 2
HESSIAN, INVERSE, SAMPLE = 0, 1, 2


def _p(x):
    return ctypes.c_void_p(x.data_ptr())


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Prior:
    """R = (delta I - gamma Lap_h)^2 on the model grid (synth.Prior)."""

    def __init__(self, pr, device=None):
        import torch

        self.torch = torch
        self.pr = pr
        self.lib = fwi.load_library()
        self.device = torch.device(device if device is not None else "cuda")
        h = ctypes.c_void_p()
        fwi._check(self.lib.fwi_prior_create(pr.nz, pr.nx, float(pr.h), float(pr.delta),
                                             float(pr.gamma), ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        fwi._check(self.lib.fwi_prior_device_bytes(h, ctypes.byref(nb)))
        self._blk = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        fwi._check(self.lib.fwi_prior_bind(h, _p(self._blk), nb.value,
                                           _stream(torch, self.device)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.fwi_prior_destroy(h)
            self._h = None

    def _vec(self, v):
        t = self.torch
        if not isinstance(v, t.Tensor) or v.device.type != "cuda" or v.dtype != t.float32:
            raise TypeError("vectors must be float32 CUDA tensors")
        v = v.contiguous()
        if tuple(v.shape[-2:]) != (self.pr.nz, self.pr.nx):
            raise ValueError(f"vectors have shape {tuple(v.shape)}, expected (..., "
                             f"{self.pr.nz}, {self.pr.nx})")
        return v

    def apply(self, op, v):
        v = self._vec(v)
        single = v.dim() == 2
        v = v.reshape(-1, self.pr.nz, self.pr.nx)
        B = v.shape[0]
        out = self.torch.empty_like(v)
        n = ctypes.c_size_t()
        fwi._check(self.lib.fwi_prior_workspace_size(self._h, B, ctypes.byref(n)))
        ws = self.torch.empty(n.value, dtype=self.torch.uint8, device=self.device)
        fwi._check(self.lib.fwi_prior_apply(self._h, int(op), _p(v), B, _p(out), _p(ws),
                                            n.value, _stream(self.torch, self.device)))
        return out[0] if single else out


class LowRank:
    """r leading eigenpairs of H_d v = lambda R v at model m from k probes."""

    def __init__(self, plan: "fwi.Plan", m, prior: Prior, omega, r: int, tol: float = 1e-7):
        t = prior.torch
        lib = prior.lib
        self.prior = prior
        k = omega.shape[0]
        if not 1 <= r < k:
            raise ValueError("need 1 <= r < k")
        nz, nx = prior.pr.nz, prior.pr.nx
        dev = prior.device
        st = _stream(t, dev)
        n = ctypes.c_size_t()
        fwi._check(lib.fwi_lowrank_workspace_size(prior._h, k, 1, r, ctypes.byref(n)))
        ws = t.empty(n.value, dtype=t.uint8, device=dev)
        ev = [t.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        ybar = plan.gn_hvp(m, omega)                      # pass 1: H_d omega
        ev[1].record()
        plan.release_workspaces()  # a k-vector product workspace is ~1 GB per vector
        Q = t.empty((k, nz, nx), dtype=t.float32, device=dev)
        RQ = t.empty_like(Q)
        kept = t.zeros((), dtype=t.int32, device=dev)
        fwi._check(lib.fwi_lowrank_range(prior._h, k, _p(ybar), float(tol), _p(Q), _p(RQ),
                                         _p(kept), _p(ws), n.value, st))
        ev[2].record()
        del ybar
        self.kept = int(kept.item())
        if self.kept < r:
            raise RuntimeError(f"only {self.kept} independent directions for rank {r}")
        Qk = Q[:self.kept].contiguous()
        hq = plan.gn_hvp(m, Qk)                           # pass 2: H_d Q
        ev[3].record()
        plan.release_workspaces()
        self.lam = t.empty(r, dtype=t.float64, device=dev)
        self.V = t.empty((r, nz, nx), dtype=t.float32, device=dev)
        fwi._check(lib.fwi_lowrank_project(prior._h, self.kept, _p(Qk), _p(hq), r,
                                           _p(self.lam), _p(self.V), _p(ws), n.value, st))
        ev[4].record()
        ev[4].synchronize()
        #: milliseconds of the four phases (device events on the current stream)
        self.timing_ms = {"hessian_pass1": ev[0].elapsed_time(ev[1]),
                          "range": ev[1].elapsed_time(ev[2]),
                          "hessian_pass2": ev[2].elapsed_time(ev[3]),
                          "project": ev[3].elapsed_time(ev[4])}
        self.r = r

    @classmethod
    def from_pairs(cls, prior: Prior, lam, V):
        """An approximation from given eigenpairs (lam FP64, V[r][nz][nx] FP32)."""
        self = cls.__new__(cls)
        self.prior, self.lam, self.V = prior, lam.contiguous(), V.contiguous()
        self.r = int(lam.shape[0])
        self.kept = self.r
        return self

    def apply(self, op, v):
        pr, t = self.prior, self.prior.torch
        v = pr._vec(v)
        single = v.dim() == 2
        v = v.reshape(-1, pr.pr.nz, pr.pr.nx)
        B = v.shape[0]
        out = t.empty_like(v)
        n = ctypes.c_size_t()
        fwi._check(pr.lib.fwi_lowrank_workspace_size(pr._h, self.r, B, self.r, ctypes.byref(n)))
        ws = t.empty(n.value, dtype=t.uint8, device=pr.device)
        fwi._check(pr.lib.fwi_lowrank_apply(pr._h, int(op), _p(self.lam), _p(self.V), self.r,
                                            _p(v), B, _p(out), _p(ws), n.value,
                                            _stream(t, pr.device)))
        return out[0] if single else out

    def hessian(self, v):
        return self.apply(HESSIAN, v)

    def inverse(self, v):
        return self.apply(INVERSE, v)

    def sample(self, w):
        return self.apply(SAMPLE, w)

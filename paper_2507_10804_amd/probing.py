"""Batched probing: many Gauss-Newton Hessian-vector products at one model.

The point-spread-function and pseudo-differential-probing approximations of
the paper (Sections 3.2 and 3.4; Section 4.1.1 spends 4 products on 36 PSFs
and 1 product on 8 symbol columns) and randomized low-rank corrections
(Section 3.1) all consume batches of H_d v at a fixed model.  A
:class:`ProbeSession` runs B products per call, sharing the forward solve and
its recompute across the batch, and captures the whole call -- the two time
loops of several thousand kernel launches -- once into a HIP graph that is
replayed for every later batch.

The library enqueues kernel launches only (no memset, no host copies), so the
call is capture-safe; the workspace, model and batch buffers are allocated
before capture and stay fixed.  The session owns its workspace (not the
plan's cache), so the captured graph keeps pointing at live memory whatever
the plan does with its own cached workspaces.
"""
from __future__ import annotations

import torch

from . import fwi


class ProbeSession:
    def __init__(self, plan: "fwi.Plan", m: torch.Tensor, batch: int, use_graph: bool = True):
        g = plan.geom
        self.plan = plan
        self.batch = int(batch)
        dev = plan.device
        self.m = torch.empty((g.nz, g.nx), dtype=torch.float32, device=dev)
        self.m.copy_(m)
        self.v = torch.zeros((self.batch, g.nz, g.nx), dtype=torch.float32, device=dev)
        self.hv = torch.empty((self.batch, g.nz, g.nx), dtype=torch.float32, device=dev)
        self.graph = None
        # allocated before capture and held for the session's lifetime
        self.ws = plan.new_workspace(fwi.FWI_OP_GN_HVP, self.batch)
        if use_graph:
            side = torch.cuda.Stream(device=dev)
            side.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(side):  # eager run on a side stream first
                plan.gn_hvp(self.m, self.v, out=self.hv, ws=self.ws)
            torch.cuda.current_stream(dev).wait_stream(side)
            torch.cuda.synchronize(dev)
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                plan.gn_hvp(self.m, self.v, out=self.hv, ws=self.ws)
            torch.cuda.synchronize(dev)

    def run(self, v: torch.Tensor) -> torch.Tensor:
        """H_d v for v[batch][nz][nx] (fewer rows are zero-padded).  Returns a
        view of the session's output buffer, valid until the next call."""
        n = v.shape[0]
        if n > self.batch:
            raise ValueError(f"batch of {n} exceeds the session's {self.batch}")
        self.v[:n].copy_(v)
        if n < self.batch:
            self.v[n:].zero_()
        if self.graph is not None:
            self.graph.replay()
        else:
            self.plan.gn_hvp(self.m, self.v, out=self.hv, ws=self.ws)
        return self.hv[:n]

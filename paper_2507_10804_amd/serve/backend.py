"""Execution backends for the request server.

``GpuBackend`` runs requests through the HIP library, one stream per server
slot, on datasets (plan, observed data, resident models) kept in HBM.  Every
job allocates its own workspace on its slot's stream, so concurrent jobs never
share scratch memory; its size -- forward checkpoints plus segment buffers
plus batch fields -- is what the server reserves against the memory budget.
A job's status bits live in its own workspace, so a flagged proposal fails
its own request only (never a neighbour's running on another slot).
"""
from __future__ import annotations

import threading

import numpy as np

from .. import fwi
from .server import RequestError

_OPS = {"misfit": fwi.FWI_OP_MISFIT, "forward": fwi.FWI_OP_FORWARD, "hvp": fwi.FWI_OP_GN_HVP}


class Dataset:
    def __init__(self, plan, dobs, models):
        self.plan = plan
        self.dobs = dobs
        self.models = models


class FlaggedModel(RequestError):
    """The library flagged the request's model or output (non-positive or
    non-finite speed, Courant number above the stability limit, non-finite
    result): the result would be meaningless and is not returned."""


def _raise_flagged(plan, ws, what):
    bits = plan.workspace_status(ws)
    if bits:
        names = [n for b, n in ((fwi.STATUS_BAD_MODEL, "model not positive and finite"),
                                (fwi.STATUS_CFL, "Courant number above the stability limit"),
                                (fwi.STATUS_NONFINITE, "non-finite output")) if bits & b]
        raise FlaggedModel(f"{what}: " + ", ".join(names))


class GpuBackend:
    def __init__(self, slots: int = 4, device: str = "cuda:0", budget_fraction: float = 0.8,
                 max_batch: int = 16):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.datasets: dict[str, Dataset] = {}
        self.budget_fraction = budget_fraction
        self._max_batch = int(max_batch)
        self._lock = threading.Lock()

    # -------------------------------------------------------------- residency
    def add_dataset(self, key, geom, dobs=None, models=None):
        """Keep a plan, its observed data and named models resident in HBM."""
        t = self.torch
        plan = fwi.Plan(geom, device=self.device)
        f32 = lambda a: a if isinstance(a, t.Tensor) else t.as_tensor(
            np.asarray(a, np.float32), device=self.device)
        ms = {k: f32(v).contiguous() for k, v in (models or {}).items()}
        d = f32(dobs).contiguous() if dobs is not None else None
        self.datasets[key] = Dataset(plan, d, ms)
        t.cuda.synchronize(self.device)
        return plan

    def mem_budget(self) -> int:
        free, _total = self.torch.cuda.mem_get_info(self.device)
        return int(self.budget_fraction * free)

    def max_batch(self, req) -> int:
        return self._max_batch

    # ------------------------------------------------------------------ jobs
    def prepare(self, req):
        """Called at submit time: remember where device inputs were produced so
        the slot stream can wait for them."""
        t = self.torch
        for x in (req.m, req.v):
            if isinstance(x, t.Tensor) and x.is_cuda:
                ev = t.cuda.Event()
                ev.record(t.cuda.current_stream(self.device))
                req.ready_event = ev
                break

    def job_bytes(self, reqs) -> int:
        r0 = reqs[0]
        ds = self.datasets[r0.dataset]
        g = ds.plan.geom
        B = sum(r.nvec for r in reqs)
        ws = ds.plan.workspace_bytes(_OPS[r0.kind], B if r0.kind == "hvp" else 1)
        if r0.kind == "hvp":
            out = 2 * B * g.nz * g.nx * 4
        elif r0.kind == "forward":
            out = g.ns * g.nt * g.nr * 4
        else:
            out = 8
        return ws + out

    def run(self, slot, reqs):
        t = self.torch
        r0 = reqs[0]
        ds = self.datasets[r0.dataset]
        plan, g = ds.plan, ds.plan.geom
        st = self.streams[slot]
        for r in reqs:
            if r.ready_event is not None:
                st.wait_event(r.ready_event)
        with t.cuda.stream(st):
            if r0.kind == "hvp":
                m = ds.models[r0.model]
                vs = [r.v.reshape(-1, g.nz, g.nx) for r in reqs]
                V = vs[0] if len(vs) == 1 else t.cat(vs, 0)
                B = V.shape[0]
                ws = t.empty(plan.workspace_bytes(fwi.FWI_OP_GN_HVP, B), dtype=t.uint8,
                             device=self.device)
                hv = plan.gn_hvp(m, V.contiguous(), ws=ws)
                st.synchronize()
                _raise_flagged(plan, ws, "Hessian-vector product")
                out, k = [], 0
                for r, v in zip(reqs, vs):
                    n = v.shape[0]
                    out.append(hv[k:k + n] if r.v.dim() == 3 else hv[k])
                    k += n
                return out
            if len(reqs) != 1:
                raise ValueError("only Hessian-vector requests are merged")
            if r0.kind == "misfit":
                ws = t.empty(plan.workspace_bytes(fwi.FWI_OP_MISFIT), dtype=t.uint8,
                             device=self.device)
                phi = plan.misfit(r0.m, ds.dobs, ws=ws)
                st.synchronize()
                _raise_flagged(plan, ws, "misfit")
                return [float(phi)]
            if r0.kind == "forward":
                ws = t.empty(plan.workspace_bytes(fwi.FWI_OP_FORWARD), dtype=t.uint8,
                             device=self.device)
                d = plan.forward(r0.m, ws=ws)
                st.synchronize()
                _raise_flagged(plan, ws, "forward")
                return [d]
            raise ValueError(f"unknown request kind {r0.kind!r}")

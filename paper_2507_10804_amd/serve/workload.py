"""Synthetic serving workload: closed-loop MCMC-style chains and probe
batches on three grids with resident models.

Grids (seeded layered-faulted models, dx = 10 m, 20 sponge cells):
256 x 128 with 16 shots and 2000 steps, 512 x 192 with 32 shots and 3000
steps, 921 x 301 with 64 shots and 4000 steps.  Each grid keeps four resident
models (the smoothed truth at four smoothing widths) and observed data of the
truth.  A chain alternates exponential think times with one request:
a misfit evaluation of a proposal (a resident model plus a seeded smooth
perturbation), a single Hessian-vector product at a resident model, or --
for one request in ten -- a probe batch of 4 smoothed Rademacher vectors.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from .. import synth
from .server import Request

GRIDS = {
    "g256": dict(nx=256, nz=128, ns=16, nt=2000),
    "g512": dict(nx=512, nz=192, ns=32, nt=3000),
    "g921": dict(nx=921, nz=301, ns=64, nt=4000),
}
SMOOTHING = (6.0, 8.0, 10.0, 12.0)


def grid_geometry(key, nt=None):
    c = GRIDS[key]
    nx, nz = c["nx"], c["nz"]
    return synth.make_geometry(nx, nz, nt=nt or c["nt"], ns=c["ns"], rec_ix=2 * np.arange(nx // 2),
                               f0=8.0, v_nominal=5500.0, ckpt_every=50)


def load_datasets(backend, keys=tuple(GRIDS), nt_override=None):
    """Register the resident datasets; the observed data are the forward data
    of the true model computed on the device (setup, untimed)."""
    import torch

    banks = {}
    for i, key in enumerate(keys):
        g = grid_geometry(key, nt_override)
        m_true = synth.layered_faulted_model(g.nx, g.nz, seed=i)
        water = int(round(300.0 / 10.0))
        models = {f"m{j}": synth.smoothed_start(m_true, s, water_rows=water)
                  for j, s in enumerate(SMOOTHING)}
        plan = backend.add_dataset(key, g, dobs=None, models=models)
        d = plan.forward(torch.as_tensor(m_true.astype(np.float32), device=backend.device))
        torch.cuda.synchronize(backend.device)
        backend.datasets[key].dobs = d
        bank = synth.smooth_random_batch(g.nz, g.nx, seeds=range(1000, 1004), sigma=8.0)
        banks[key] = torch.as_tensor((20.0 * bank / np.abs(bank).max()).astype(np.float32),
                                     device=backend.device)
    return banks


class Progress:
    """Completed-request counter that reports every `every` completions."""

    def __init__(self, every=32, log=None):
        self.every, self.log = every, log
        self.n = 0
        self.lock = threading.Lock()
        self.t0 = time.monotonic()

    def tick(self):
        with self.lock:
            self.n += 1
            if self.log and self.n % self.every == 0:
                self.log(f"  {self.n} requests done, {time.monotonic() - self.t0:.0f} s")


class Chain:
    """One closed-loop client: think, submit, wait, repeat."""

    def __init__(self, idx, server, backend, banks, mean_think, keys, seed=0, probe_every=10,
                 progress=None):
        self.idx = idx
        self.server = server
        self.backend = backend
        self.banks = banks
        self.mean_think = mean_think
        self.keys = list(keys)
        self.rng = np.random.default_rng(seed * 1009 + idx)
        self.probe_every = probe_every
        self.records = []
        self.stop = False
        self.progress = progress

    def make_request(self, n):
        import torch

        key = self.keys[self.rng.integers(len(self.keys))]
        ds = self.backend.datasets[key]
        g = ds.plan.geom
        model = f"m{self.rng.integers(len(SMOOTHING))}"
        if self.probe_every and n % self.probe_every == self.probe_every - 1:
            seeds = self.rng.integers(0, 2 ** 31, size=4)
            v = synth.rademacher_smoothed(g.nz, g.nx, seeds=seeds, sigma=5.0)
            return Request("hvp", key, model=model,
                           v=torch.as_tensor(v.astype(np.float32), device=self.backend.device))
        if self.rng.random() < 0.5:
            coef = float(self.rng.standard_normal())
            k = int(self.rng.integers(self.banks[key].shape[0]))
            m = ds.models[model] + coef * self.banks[key][k]
            return Request("misfit", key, m=m)
        seed = int(self.rng.integers(0, 2 ** 31))
        v = synth.smooth_random((g.nz, g.nx), seed=seed, sigma=5.0)
        return Request("hvp", key, model=model,
                       v=torch.as_tensor(v.astype(np.float32), device=self.backend.device))

    def run(self, n_requests):
        for n in range(n_requests):
            if self.stop:
                return
            time.sleep(self.rng.exponential(self.mean_think))
            req = self.make_request(n)
            fut = self.server.submit(req)
            try:
                fut.result()
                ok = True
            except Exception:
                ok = False
            r = fut.request
            self.records.append((r.kind, r.nvec, r.t_submit, r.t_start, r.t_end, r.batch, ok,
                                 r.dataset))
            if self.progress:
                self.progress.tick()


def run_closed_loop(server, backend, banks, chains=32, rate=50.0, requests_per_chain=20,
                    keys=tuple(GRIDS), seed=0, warmup_s=0.0, log=None):
    """32 chains with exponential think times (aggregate offered rate `rate`
    when service were instantaneous); returns per-request records."""
    mean_think = chains / rate
    prog = Progress(log=log)
    cs = [Chain(i, server, backend, banks, mean_think, keys, seed, progress=prog)
          for i in range(chains)]
    th = [threading.Thread(target=c.run, args=(requests_per_chain,), daemon=True) for c in cs]
    t0 = time.monotonic()
    for t in th:
        t.start()
    for t in th:
        t.join()
    t1 = time.monotonic()
    recs = [r for c in cs for r in c.records]
    return recs, t0 + warmup_s, t1


def summarize(recs, t0, t1):
    """p50/p99 latency and throughput over requests submitted after t0."""
    rs = [r for r in recs if r[2] >= t0]
    if not rs:
        return {}
    lat = np.array([r[4] - r[2] for r in rs]) * 1e3
    hv = [r for r in rs if r[0] == "hvp" and r[6]]
    window = max(max(r[4] for r in rs) - t0, 1e-9)
    out = {"requests": len(rs), "ok": int(sum(r[6] for r in rs)), "window_s": window,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "req_per_s": len(rs) / window, "hv_per_s": sum(r[1] for r in hv) / window,
           "mean_batch": float(np.mean([r[5] for r in hv])) if hv else 0.0}
    if hv:
        hl = np.array([r[4] - r[2] for r in hv]) * 1e3
        out["hv_p50_ms"] = float(np.percentile(hl, 50))
        out["hv_p99_ms"] = float(np.percentile(hl, 99))
    return out

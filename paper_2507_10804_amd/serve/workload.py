"""Synthetic serving workload: closed-loop MCMC-style chains on mixed grids,
shot counts and record lengths, with resident models.

Every request draws, independently and uniformly (seeded per chain):
* a grid: 256 x 128, 512 x 192 or 921 x 301 (seeded layered-faulted models,
  dx = 10 m, 20 sponge cells, receivers every 2 cells at 10 m depth);
* a shot count ns in {16, 32, 64} (surface shots in equal strips);
* a record length nt in {2000, 3000, 4000} steps (dt fixed by the 5500 m/s
  nominal speed at Courant number 0.4, Ricker 8 Hz, K = 50);
* a kind, 1:1: "misfit" -- the data misfit Phi(m') of a gpCN proposal m'
  (Section 2.3: every proposal needs Phi at the proposed model, one forward
  solve), m' a resident model plus a seeded smooth perturbation -- or "hvp",
  one Gauss-Newton product at a resident model on a seeded smooth vector;
* one of four resident models of that grid (the smoothed truth at four
  smoothing widths).
Observed data are the forward data of each grid's true model for every
(ns, nt), computed on the device at setup.  A chain has at most one
request outstanding; exponential think times give the offered rate.
"""
from __future__ import annotations

import json
import threading
import time

import numpy as np

from .. import synth
from .server import Request

GRIDS = {"g256": (256, 128), "g512": (512, 192), "g921": (921, 301)}
SHOTS = (16, 32, 64)
NTS = (2000, 3000, 4000)
SMOOTHING = (6.0, 8.0, 10.0, 12.0)


def dataset_key(grid, ns, nt):
    return f"{grid}_s{ns}_t{nt}"


def grid_geometry(grid, ns, nt):
    nx, nz = GRIDS[grid]
    return synth.make_geometry(nx, nz, nt=nt, ns=ns, rec_ix=2 * np.arange(nx // 2), f0=8.0,
                               v_nominal=5500.0, ckpt_every=50)


def load_datasets(backend, grids=tuple(GRIDS), shots=SHOTS, nts=NTS):
    """Register one resident dataset per (grid, ns, nt): its plan and the
    observed data of the grid's true model; the four models of a grid are
    shared by its datasets.  Returns a bank of proposal perturbations per
    grid (device tensors)."""
    import torch

    banks = {}
    for i, grid in enumerate(grids):
        nx, nz = GRIDS[grid]
        m_true = synth.layered_faulted_model(nx, nz, seed=i)
        water = int(round(300.0 / 10.0))
        models = None
        mt = torch.as_tensor(m_true.astype(np.float32), device=backend.device)
        for ns in shots:
            for nt in nts:
                g = grid_geometry(grid, ns, nt)
                if models is None:
                    plan = backend.add_dataset(
                        dataset_key(grid, ns, nt), g, dobs=None,
                        models={f"m{j}": synth.smoothed_start(m_true, s, water_rows=water)
                                for j, s in enumerate(SMOOTHING)})
                    models = backend.datasets[dataset_key(grid, ns, nt)].models
                else:
                    plan = backend.add_dataset(dataset_key(grid, ns, nt), g, dobs=None,
                                               models=models)
                ws = plan.new_workspace(0)
                d = plan.forward(mt, ws=ws)
                torch.cuda.synchronize(backend.device)
                del ws
                backend.datasets[dataset_key(grid, ns, nt)].dobs = d
        bank = synth.smooth_random_batch(nz, nx, seeds=range(1000, 1004), sigma=8.0)
        banks[grid] = torch.as_tensor((20.0 * bank / np.abs(bank).max()).astype(np.float32),
                                      device=backend.device)
    return banks


def draw_request(rng, backend, banks, grids=tuple(GRIDS), shots=SHOTS, nts=NTS):
    """One request of the trace (see the module docstring); returns the
    Request and its description for the log."""
    import torch

    grid = grids[int(rng.integers(len(grids)))]
    ns = shots[int(rng.integers(len(shots)))]
    nt = nts[int(rng.integers(len(nts)))]
    kind = "misfit" if rng.random() < 0.5 else "hvp"
    model = f"m{int(rng.integers(len(SMOOTHING)))}"
    key = dataset_key(grid, ns, nt)
    ds = backend.datasets[key]
    g = ds.plan.geom
    if kind == "misfit":
        coef = float(rng.standard_normal())
        k = int(rng.integers(banks[grid].shape[0]))
        req = Request("misfit", key, m=ds.models[model] + coef * banks[grid][k])
    else:
        seed = int(rng.integers(0, 2 ** 31))
        v = synth.smooth_random((g.nz, g.nx), seed=seed, sigma=5.0)
        req = Request("hvp", key, model=model,
                      v=torch.as_tensor(v.astype(np.float32), device=backend.device))
    return req, {"grid": grid, "shots": ns, "nt": nt, "kind": kind, "model": model}


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

    def __init__(self, idx, server, backend, banks, mean_think, seed=0, progress=None,
                 draw=None):
        self.idx = idx
        self.server = server
        self.backend = backend
        self.banks = banks
        self.mean_think = mean_think
        self.rng = np.random.default_rng(seed * 1009 + idx)
        self.records = []
        self.stop = False
        self.progress = progress
        self.draw = draw or (lambda rng: draw_request(rng, backend, banks))

    def run(self, n_requests):
        for n in range(n_requests):
            if self.stop:
                return
            time.sleep(self.rng.exponential(self.mean_think))
            req, desc = self.draw(self.rng)
            fut = self.server.submit(req)
            err = None
            try:
                fut.result()
            except Exception as exc:  # recorded, the chain goes on
                err = f"{type(exc).__name__}: {exc}"
            r = fut.request
            self.records.append(dict(desc, chain=self.idx, seq=n, rid=r.rid, nvec=r.nvec,
                                     t_submit=r.t_submit, t_start=r.t_start, t_end=r.t_end,
                                     batch=r.batch, ok=err is None, error=err))
            if self.progress:
                self.progress.tick()


def run_closed_loop(server, backend, banks, chains=32, rate=50.0, requests_per_chain=20,
                    seed=0, warmup_s=0.0, log=None, draw=None):
    """`chains` closed-loop chains with exponential think times (aggregate
    offered rate `rate` if service were instantaneous); returns the
    per-request records and the measured window (t0, t1)."""
    mean_think = chains / rate
    prog = Progress(log=log)
    cs = [Chain(i, server, backend, banks, mean_think, seed, progress=prog, draw=draw)
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


def write_log(recs, path, t_origin, path_mode="w"):
    """Per-request JSONL: grid, shots, nt, kind, queue, device and total times
    (ms), merged batch size and outcome, one line per request."""
    with open(path, path_mode) as f:
        for r in sorted(recs, key=lambda r: r["t_submit"]):
            f.write(json.dumps({
                "rid": r["rid"], "chain": r["chain"], "seq": r["seq"], "grid": r["grid"],
                "shots": r["shots"], "nt": r["nt"], "kind": r["kind"], "model": r["model"],
                "submit_s": r["t_submit"] - t_origin,
                "queue_ms": 1e3 * (r["t_start"] - r["t_submit"]) if r["t_start"] else None,
                "device_ms": 1e3 * (r["t_end"] - r["t_start"]) if r["t_start"] else None,
                "latency_ms": 1e3 * (r["t_end"] - r["t_submit"]) if r["t_end"] else None,
                "batch": r["batch"], "ok": r["ok"], "error": r["error"]}) + "\n")


def summarize(recs, t0, t1):
    """p50/p99 latency and throughput over requests submitted after t0."""
    rs = [r for r in recs if r["t_submit"] >= t0]
    if not rs:
        return {}
    lat = np.array([r["t_end"] - r["t_submit"] for r in rs]) * 1e3
    hv = [r for r in rs if r["kind"] == "hvp" and r["ok"]]
    mf = [r for r in rs if r["kind"] == "misfit" and r["ok"]]
    window = max(max(r["t_end"] for r in rs) - t0, 1e-9)
    out = {"requests": len(rs), "ok": int(sum(r["ok"] for r in rs)), "window_s": window,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "req_per_s": len(rs) / window, "hv_per_s": sum(r["nvec"] for r in hv) / window,
           "misfit_per_s": len(mf) / window,
           "mean_hv_batch": float(np.mean([r["batch"] for r in hv])) if hv else 0.0}
    for name, sel in (("hv", hv), ("misfit", mf)):
        if sel:
            lt = np.array([r["t_end"] - r["t_submit"] for r in sel]) * 1e3
            out[f"{name}_p50_ms"] = float(np.percentile(lt, 50))
            out[f"{name}_p99_ms"] = float(np.percentile(lt, 99))
    return out

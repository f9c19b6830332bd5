#!/usr/bin/env python
"""Throughput of the matrix-free Gauss-Newton Hessian-vector product on one
MI355X.

Workload (one "step"): on the seeded 921 x 301 layered-faulted model
(dx = 10 m, 20 sponge cells per side), 64 surface shots, 461 receivers, Ricker
8 Hz, 4000 time steps, forward checkpoints every 50 steps: one misfit gradient
at the smoothed model plus one batched call of 16 Gauss-Newton Hessian-vector
products on seeded smooth random vectors.  Inputs are resident in HBM before
the timed region; the observed data are the forward data of the true model.

Prints one JSON line: Hv/s (value), per-step time, Gpt-updates/s, the
headline HBM fraction, the roofline of the dominant kernel (HIP-event times of
every launch in the timed region), and the FP64 oracle timed on the host on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GN Hessian-vector products/s + Gpt-updates/s (%HBM peak); p50/p99 Hv latency"
KERNEL_NAMES = (0, 1, 2)  # forward, forward+Born, adjoint (see fwi.Plan.kernel_name)
KERNEL_SRC = os.path.join(ROOT, "paper_2507_10804_amd", "csrc", "fwi_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_kernels_921x301_64shots_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes(g, B, nseg, K, fused=True, hist=False):
    """Compulsory HBM bytes of one step (misfit, gradient and B products at
    one model: one fused pass, or a gradient call plus a B-vector Hv call),
    per kernel kind: every array element a launch must read or write, once.
    With `hist` (history mode, ckpt_every = 0) the forward sweeps store w^n
    at every step instead of checkpoints, and nothing is recomputed.

    Np = padded grid points.  Per launch:
      forward step      4 Np (3 ns + 1)       u^n, u^{n-1}, c -> u^{n+1}
        + 4 ns nr         receiver gather (when data are recorded)
        + 8 ns Np         checkpoint pair (every K-th step)
        + 4 ns Np         w^n store (segment recompute)
      forward+Born step 4 Np (3 ns + 1) + 4 Np B (3 ns + 1) + 4 B ns nr
        + 8 ns Np         checkpoint pair (every K-th step)
      adjoint step      12 Np B ns (mu^{k+1}, mu^{k+2} -> mu^k) + 4 B ns nr
        + 4 Np ns + 8 Np + 16 Np B   w^k, c, 2/m and one FP64 image per
                                     vector (steps with an image term)
    """
    nzp, nxp = g.nz + 2 * g.nb, g.nx + 2 * g.nb
    Np = nzp * nxp
    ns, nr, nt = g.ns, g.nr, g.nt
    ck_steps = 0 if hist else nseg - 1

    def adj(b):
        return nt * (12 * Np * b * ns + 4 * b * ns * nr) + (nt - 1) * (4 * Np * ns + 8 * Np + 16 * Np * b)

    keep = (nt - 1) * 4 * ns * Np if hist else 0  # w^n stores of the forward sweep
    fwd = (nt - 1) * (4 * Np * (3 * ns + 1) + 4 * ns * nr) + ck_steps * 8 * ns * Np
    rec = (nt - 1) * (4 * Np * (3 * ns + 1) + 4 * ns * Np)
    born = ((nt - 1) * (4 * Np * (3 * ns + 1) + 4 * Np * B * (3 * ns + 1) + 4 * B * ns * nr)
            + ck_steps * 8 * ns * Np)
    if hist:
        if fused:
            return {0: 0, 1: born + keep + (nt - 1) * 4 * ns * nr, 2: adj(B + 1)}
        return {0: fwd + keep, 1: born + keep, 2: adj(1) + adj(B)}

    if fused:
        # one pass: forward+Born (gathering d and J v) + one recompute + adjoint(B + 1)
        return {0: rec, 1: born + (nt - 1) * 4 * ns * nr, 2: adj(B + 1)}
    # gradient: forward (gathering d) + recompute + adjoint(B=1)
    # Hv call : forward+Born + recompute + adjoint(B)
    return {0: fwd + 2 * rec, 1: born, 2: adj(1) + adj(B)}


UPDATE_BYTES = 16  # read u^n, u^{n-1}, c, write u^{n+1}: FP32, per field update


def field_updates(g, B, fused=True, hist=False):
    """Field updates (one grid point of one wavefield advanced one step) of
    one step, per kernel kind, on the padded grid: the unit of the headline
    16 bytes per update.  Fused: a recompute of the forward field (kind 0),
    forward + B Born fields (kind 1) and B + 1 adjoint fields (kind 2) over
    nt - 1 steps.  Separate calls: the gradient's forward, two recomputes,
    the Hv call's forward + B Born, and 1 + B adjoint fields.  History mode
    (`hist`) has no recomputes."""
    Np = (g.nz + 2 * g.nb) * (g.nx + 2 * g.nb)
    per = g.ns * Np * (g.nt - 1)
    if fused:
        return {0: 0 if hist else per, 1: (1 + B) * per, 2: (B + 1) * per}
    return {0: (1 if hist else 3) * per, 1: (1 + B) * per, 2: (1 + B) * per}


def read_traffic(kind_name):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel source sha256\[:16\]:\s*([0-9a-f]{16})", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(re.escape(kind_name) + r"\s*\|\s*([0-9.eE+]+)\s*\|", text)
    return float(m.group(1)) if m else None


def cpu_baseline(g, m, v, threads, nt_sample):
    """The FP64 oracle, as it stands, on `threads` shots of the full grid for
    nt_sample steps, one Gauss-Newton product at a fresh model (forward,
    Born, adjoint: shots run in parallel, one per thread); scaled to Hv/s of
    the whole 64-shot x 4000-step workload by the fraction of shot-steps
    done.  The GPU line's value is B products per fused pass (one forward,
    B Born and B + 1 adjoint solves), so per product the GPU runs about two
    solves per shot against the oracle's three here."""
    import oracle

    oracle.build(force=False)
    threads = max(1, min(threads, g.ns))  # one shot per thread
    gs = g.with_shots(np.arange(threads)).with_nt(nt_sample)
    t0 = time.perf_counter()
    oracle.gn_hvp(gs, m, v, nthreads=threads)
    dt = time.perf_counter() - t0
    frac = (threads * (nt_sample - 1)) / (g.ns * (g.nt - 1))
    # the same on one core (one shot, 60 % of the steps): the per-core rate
    g1 = g.with_shots([0]).with_nt(max(2, int(0.6 * nt_sample)))
    t1 = time.perf_counter()
    oracle.gn_hvp(g1, m, v, nthreads=1)
    dt1 = time.perf_counter() - t1
    frac1 = (g1.nt - 1) / (g.ns * (g.nt - 1))
    cpu = host_cpu()
    return {"value": frac / dt, "unit": "Hv/s", "cores": threads, "kind": "oracle",
            "sample": f"one GN Hv at a fresh model on {threads} of {g.ns} shots (one per "
                      f"thread), full 921x301 grid, {nt_sample} of {g.nt} steps, {dt:.1f} s "
                      f"wall; scaled by shot-steps",
            "per_core_value": frac1 / dt1,
            "per_core_sample": f"one shot, {g1.nt} steps, 1 thread, {dt1:.1f} s wall; "
                               f"scaled by shot-steps",
            "host": cpu}


def small_case_timings(threads):
    """The 128x128 / 4-shot / 500-step problem: Phi + gradient and one Hv by
    the FP64 oracle (shots in parallel on `threads` threads, and on one) and
    by the GPU (median of 5 calls, HIP events on the call's stream)."""
    import oracle
    import torch
    from paper_2507_10804_amd import fwi, synth

    g, m_true, m_eval = synth.config_small()
    v = synth.smooth_random((g.nz, g.nx), seed=1, sigma=5.0)
    dobs = oracle.forward(g, m_true)
    out = {"workload": "128x128, 4 shots, 32 receivers, Ricker 10 Hz, nt=500"}
    for name, nth in (("oracle_threads", threads), ("oracle_1_thread", 1)):
        t0 = time.perf_counter()
        oracle.misfit_grad(g, m_eval, dobs, nthreads=nth)
        t1 = time.perf_counter()
        oracle.gn_hvp(g, m_eval, v, nthreads=nth)
        t2 = time.perf_counter()
        out[name] = {"threads": nth, "misfit_grad_s": t1 - t0, "gn_hvp_s": t2 - t1}
    plan = fwi.Plan(g)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device="cuda:0")
    md, dd, vd = f32(m_eval), f32(dobs), f32(v)
    st = torch.cuda.current_stream()
    for name, fn in (("misfit_grad", lambda: plan.misfit_grad(md, dd)),
                     ("gn_hvp", lambda: plan.gn_hvp(md, vd))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[f"gpu_{name}_ms"] = float(np.median(ts))
    return out


COPY_VARIANTS = {0: "plain, one pass", 1: "non-temporal, one pass",
                 2: "plain x4, one pass", 3: "non-temporal x4, one pass",
                 4: "plain, 2048 WGs", 5: "non-temporal, 2048 WGs",
                 6: "plain x4, 2048 WGs", 7: "non-temporal x4, 2048 WGs",
                 8: "plain, 8192 WGs", 9: "non-temporal, 8192 WGs",
                 10: "plain x4, 8192 WGs", 11: "non-temporal x4, 8192 WGs"}


def copy_rates(nbytes=2 << 30, reps=10, variants=tuple(COPY_VARIANTS)):
    """GB/s (read + write) of the library's STREAM-style copy (fwi_calib_copy,
    16-byte accesses) of `nbytes`, per launch variant, HIP-event timed on the
    stream the copies are enqueued on."""
    import ctypes

    import torch
    from paper_2507_10804_amd import fwi

    lib = fwi.load_library()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    out = {}
    for var in variants:
        call = lambda: fwi._check(lib.fwi_calib_copy(ctypes.c_void_p(dst.data_ptr()),
                                                      ctypes.c_void_p(src.data_ptr()),
                                                      nbytes, var, sp))
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            call()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[var] = 2 * nbytes / (ms * 1e-3) / 1e9
    assert bool((dst == 1.0).all())
    return out


def calibrate_copy(variant=None, reps=10, nbytes=2 << 30):
    """The copy of known size: with --copy-variant, one variant `reps` times
    (for counter runs: each dispatch reads and writes `nbytes`); without, a
    sweep of every variant.  One JSON line."""
    if variant is not None:
        r = copy_rates(nbytes, reps, (variant,))
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "variant": variant, "form": COPY_VARIANTS[variant],
                          "dispatches": reps + 1, "gbs": r[variant]}), flush=True)
        return
    r = copy_rates(nbytes, reps)
    best = max(r, key=r.get)
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "gbs": {COPY_VARIANTS[k]: round(v, 1) for k, v in r.items()},
                      "best": COPY_VARIANTS[best], "best_gbs": r[best],
                      "best_frac_of_peak": r[best] / HBM_PEAK_GBS}), flush=True)


def host_cpu():
    """Cores the process may use, what the OS reports, and the CPU model."""
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": affinity, "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def serve_bench(args):
    """Serving row: the same seeded closed-loop trace of 32 chains -- misfit
    (gpCN proposal) and single Hessian-vector requests 1:1, each on a grid,
    shot count and record length drawn independently, four resident models
    per grid -- through the plain one-at-a-time path and through the
    continuous-batching server; per-request JSONL logs and one JSON line."""
    import torch
    from paper_2507_10804_amd.serve import Server
    from paper_2507_10804_amd.serve.backend import GpuBackend
    from paper_2507_10804_amd.serve import workload as wl

    be = GpuBackend(slots=args.slots, max_batch=16)
    t_setup = time.monotonic()
    banks = wl.load_datasets(be)
    log(f"serving: {len(be.datasets)} datasets resident after {time.monotonic() - t_setup:.0f} s, "
        f"budget {be.mem_budget() / 1e9:.0f} GB")
    out = {"metric": "serving: Hv/s and p50/p99 latency, plain path vs continuous batching",
           "unit": "Hv/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "32 closed-loop chains, offered 50 req/s; per request "
                                  "independently: grid 256x128, 512x192 or 921x301, shots "
                                  "16/32/64, nt 2000/3000/4000, misfit (gpCN proposal) or "
                                  "one GN Hv 1:1, one of 4 resident models per grid",
                      "requests_per_chain": args.requests_per_chain, "slots": args.slots,
                      "warmup_s": args.serve_warmup}}
    os.makedirs(args.serve_log_dir, exist_ok=True)
    for name, slots, coalesce in (("plain", 1, False), ("serving", args.slots, True)):
        with Server(be, slots=slots, coalesce=coalesce, max_batch=16) as srv:
            t0 = time.monotonic()
            recs, tw, t1 = wl.run_closed_loop(srv, be, banks, chains=32, rate=50.0,
                                              requests_per_chain=args.requests_per_chain,
                                              seed=args.seed, warmup_s=args.serve_warmup,
                                              log=log)
        torch.cuda.synchronize()
        path = os.path.join(args.serve_log_dir, f"serve_requests_{name}.jsonl")
        wl.write_log(recs, path, t0)
        res = wl.summarize(recs, tw, t1)
        res["wall_s"] = t1 - t0
        res["log"] = path
        log(f"{name}: {json.dumps(res)}")
        out[name] = res
    out["value"] = out["serving"]["hv_per_s"]
    out["vs_plain_hv_per_s"] = out["serving"]["hv_per_s"] / max(out["plain"]["hv_per_s"], 1e-12)
    print(json.dumps(out), flush=True)


def _kernel_table(plan, steps, alg=None):
    kern = {}
    for kind in KERNEL_NAMES:
        ms, n = plan.profile_read(kind)
        if not n:
            continue
        name = plan.kernel_name(kind)
        kern[name] = {"steps_per_launch": plan.kernel_steps(kind),
                      "launches_per_step": n / steps, "avg_us": 1e3 * ms / n,
                      "total_ms_per_step": ms / steps}
        if alg is not None:
            per = alg[kind] / (n / steps)
            kern[name]["alg_bytes_per_launch"] = per
            kern[name]["achieved_gbs"] = per / (1e-3 * ms / n) / 1e9
    return kern


def hvp_field_updates(g, batches):
    """Field updates of Gauss-Newton product calls with the given batch
    sizes, per kernel kind: the forward recompute, the forward + B Born
    fields, and B adjoint fields, each advanced nt - 1 steps."""
    per = g.ns * (g.nz + 2 * g.nb) * (g.nx + 2 * g.nb) * (g.nt - 1)
    return {0: per * len(batches), 1: per * sum(1 + b for b in batches),
            2: per * sum(batches)}


def _headline_unit(kern, plan, upd):
    """Requote a kernel table built on compulsory bytes in the headline unit,
    16 B per field update, keeping the compulsory figures beside it."""
    for kind in KERNEL_NAMES:
        kt = kern.get(plan.kernel_name(kind))
        if not kt or "achieved_gbs" not in kt:
            continue
        u = upd[kind] / kt["launches_per_step"]
        kt["compulsory_bytes_per_launch"] = kt.pop("alg_bytes_per_launch")
        kt["compulsory_gbs"] = kt.pop("achieved_gbs")
        kt["field_updates_per_launch"] = u
        kt["alg_bytes_per_launch"] = UPDATE_BYTES * u
        kt["achieved_gbs"] = UPDATE_BYTES * u / (kt["avg_us"] * 1e-6) / 1e9
    return kern


def probing_bench(args):
    """Batched probing row: 64 Gauss-Newton products per launch at the
    smoothed layered model (921x301, 64 shots, 4000 steps) on impulse combs
    (a delta every 40 cells, offsets without replacement) and smoothed +-1
    Rademacher probes, the whole call captured once in a HIP graph and
    replayed; the same calls eagerly for comparison."""
    import torch
    from paper_2507_10804_amd import fwi, probing, synth

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    B = 64
    combs = synth.impulse_combs(g.nz, g.nx, count=B, spacing=40, seed=100)
    rad = synth.rademacher_smoothed(g.nz, g.nx, seeds=range(200, 200 + B), sigma=5.0)
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    me = f32(m_eval)
    t0 = time.perf_counter()
    sess = probing.ProbeSession(plan, me, batch=B, use_graph=True)
    t_capture = time.perf_counter() - t0
    log(f"probing: graph captured in {t_capture:.1f} s (includes one eager warm-up call)")
    out = {"metric": "GN Hessian-vector products/s, batched probing (64 per launch)",
           "unit": "Hv/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301, {g.ns} shots, nt={g.nt}, "
                                  "64 impulse combs + 64 smoothed Rademacher probes per "
                                  "launch, HIP-graph replay", "batch": B},
           "graph_capture_s": t_capture}
    for mode in ("graph", "eager"):
        times = []
        for name, V in (("combs", combs), ("rademacher", rad)):
            Vd = f32(V)
            torch.cuda.synchronize()
            plan.profile(mode == "eager")
            plan.profile_reset()
            t1 = time.perf_counter()
            if mode == "graph":
                sess.run(Vd)
            else:
                plan.gn_hvp(me, Vd, out=sess.hv)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            log(f"{mode} {name}: {times[-1]:.2f} s")
            if mode == "eager" and name == "rademacher":
                nseg = (g.nt - 1 + plan.K - 1) // plan.K
                alg = algorithmic_bytes_hvp(g, B, nseg)
                out["kernels"] = _headline_unit(_kernel_table(plan, 1, alg), plan,
                                                hvp_field_updates(g, [B]))
            plan.profile(False)
        out[mode] = {"s_per_launch": float(np.mean(times)), "hv_per_s": B / float(np.mean(times))}
    out["value"] = out["graph"]["hv_per_s"]
    k = max(out["kernels"], key=lambda n: out["kernels"][n]["total_ms_per_step"])
    kk = out["kernels"][k]
    out["roofline"] = {"bound": "hbm", "kernel": k, "achieved": kk["achieved_gbs"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": kk["achieved_gbs"] / HBM_PEAK_GBS, "traffic": None,
                       "unit_bytes_per_field_update": UPDATE_BYTES,
                       "compulsory_gbs": kk["compulsory_gbs"],
                       "compulsory_frac": kk["compulsory_gbs"] / HBM_PEAK_GBS,
                       "avg_launch_us": kk["avg_us"]}
    print(json.dumps(out), flush=True)


FP32_VALU_PEAK_TFLOPS = 157.3


def psf_algorithmic_flops(pg):
    """FLOPs of one symbol-row apply of one vector by its definition: for
    every PSF k, every output y with w_k(y) > 0 and every tap d, one
    multiply-add (2 FLOPs).  The tent support of centre j on an axis of n
    cells spans the open interval to its neighbours, or to the edge for the
    first and last centre."""

    def support(n, first, s, count):
        if count == 1:
            return [n]
        c = [first + j * s for j in range(count)]
        out = [c[1]]
        out += [c[j + 1] - c[j - 1] - 1 for j in range(1, count - 1)]
        out.append(n - 1 - c[-2])
        return out

    sz = support(pg.nz, pg.oz, pg.sz, pg.nzc)
    sx = support(pg.nx, pg.ox, pg.sx, pg.nxc)
    return 2.0 * sum(sz) * sum(sx) * pg.width * pg.width


def psf_bench(args):
    """PSF approximation row (Sections 3.2, 3.5) on the 921x301 / 64-shot /
    4000-step workload at the smoothed model: 4 comb Hessian products (one
    batched call) give the PSFs of a 9 x 29 lattice (spacing 32, windows
    63 x 63), extracted on the device; the approximation is then applied to
    batches of smooth vectors and compared with true products."""
    import torch
    from oracle import psf as P
    from paper_2507_10804_amd import fwi, synth
    from paper_2507_10804_amd import psf as gpsf

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    pg = synth.psf_grid(g.nz, g.nx)
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    me = f32(m_eval)
    B = args.batch
    V = f32(synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, B + 1)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = gpsf.PsfOperator(plan, me, pg)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    log(f"psf: {pg.r} PSFs from {pg.ncombs} comb products in {t_build:.1f} s")
    out_buf = torch.empty_like(V)
    for _ in range(args.warmup + 1):
        op(V, out=out_buf)
    torch.cuda.synchronize()
    reps = max(5, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        op(V, out=out_buf)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    log(f"psf: apply of {B} vectors {ms:.3f} ms")
    flops = psf_algorithmic_flops(pg) * B
    achieved = flops / (ms * 1e-3) / 1e12
    # quality on the true operator (information, not parity): four smooth vectors
    hv = plan.gn_hvp(me, V[:4])
    approx = op(V[:4])
    q = [float((approx[i] - hv[i]).norm() / hv[i].norm()) for i in range(4)]
    torch.cuda.synchronize()
    plan.release_workspaces()
    out = {"metric": "PSF-approximate H_d v applies/s", "unit": "applies/s",
           "value": B / (ms * 1e-3), "n_gpus": 1, "steps": reps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301 at the smoothed model, {g.ns} shots, "
                                  f"nt={g.nt}; PSF lattice {pg.nzc}x{pg.nxc} (spacing {pg.sz}, "
                                  f"window {pg.width}x{pg.width}) from {pg.ncombs} comb products; "
                                  f"apply to {B} smooth vectors per call", "batch": B,
                      "psfs": pg.r, "window": pg.width},
           "build_s": t_build,
           "psf_rel_error_vs_true_hv": q,
           "roofline": {"bound": "alu", "kernel": "k_psf_rows", "achieved": achieved,
                        "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                        "alg_flops_per_launch": flops, "avg_launch_us": ms * 1e3}}
    if not args.no_cpu_baseline:
        vh = V[0].double().cpu().numpy()
        ph = op.psf.double().cpu().numpy()
        t1 = time.perf_counter()
        P.apply_rows(pg, ph, vh)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "applies/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one vector through the FP64 oracle's symbol-row "
                                         f"apply on the full grid, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def lowrank_bench(args):
    """Low-rank row (Section 3.1) on the 921x301 / 64-shot / 4000-step
    workload at the smoothed model: the r = 100 leading eigenpairs of
    H_d v = lambda R v (Matern prior, correlation length 500 m, pointwise
    standard deviation 200 m/s) from k = r + 10 Gaussian probes by the double
    pass (2k Hessian products), then the approximations of Section 3.1
    applied to batches of 16 vectors."""
    import torch
    from paper_2507_10804_amd import fwi, synth
    from paper_2507_10804_amd import lowrank as glr

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    r = args.rank
    k = r + 10
    P = synth.matern_prior(g.nz, g.nx, g.dx, 500.0, 200.0)
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    me = f32(m_eval)
    omega = f32(synth.gaussian_probes(g.nz, g.nx, k, seed=300))
    gp = glr.Prior(P, device=dev)
    plan.profile(True)
    plan.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lr = glr.LowRank(plan, me, gp, omega, r)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    nseg = (g.nt - 1 + plan.K - 1) // plan.K
    a1, a2 = algorithmic_bytes_hvp(g, k, nseg), algorithmic_bytes_hvp(g, lr.kept, nseg)
    kern = _headline_unit(_kernel_table(plan, 1, {kind: a1[kind] + a2[kind] for kind in a1}),
                          plan, hvp_field_updates(g, [k, lr.kept]))
    plan.profile(False)
    plan.release_workspaces()
    del omega
    lam = lr.lam.cpu().numpy()
    log(f"lowrank: kept {lr.kept} of {k}, build {t_build:.1f} s, {lr.timing_ms}")
    V16 = f32(synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, 17)))
    apply_ms = {}
    for name, fn in (("hessian", lr.hessian), ("inverse", lr.inverse), ("sample", lr.sample)):
        fn(V16)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn(V16)
        e1.record()
        torch.cuda.synchronize()
        apply_ms[name] = e0.elapsed_time(e1) / 5
    n_hv = k + lr.kept
    dom = max(kern, key=lambda n: kern[n]["total_ms_per_step"])
    out = {"metric": "rank-100 low-rank approximation of H_d (generalized eigenpairs): build time",
           "unit": "s", "value": t_build, "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": t_build * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (FP64 algebra)", "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301 at the smoothed model, {g.ns} shots, "
                                  f"nt={g.nt}; Matern prior rho=500 m sigma=200 m/s; "
                                  f"r={r}, k={k} Gaussian probes, double pass",
                      "rank": r, "probes": k, "kept": lr.kept},
           "hessian_products": n_hv, "hv_per_s_in_build": n_hv / t_build,
           "phase_ms": lr.timing_ms,
           "algebra_ms": lr.timing_ms["range"] + lr.timing_ms["project"],
           "apply_ms_per_16_vectors": apply_ms,
           "eigenvalues": {"first": float(lam[0]), "tenth": float(lam[9]),
                           "last": float(lam[-1])},
           "kernels": {n: {kk: vv for kk, vv in v.items()} for n, v in kern.items()},
           "roofline": _roofline_from(kern, dom, "the two batches of Hessian products "
                                                 "dominate; algorithmic bytes per launch of "
                                                 "those two calls")}
    if not args.no_cpu_baseline:
        base = cpu_baseline(g, m_eval, synth.smooth_random((g.nz, g.nx), seed=1),
                            min(16, len(os.sched_getaffinity(0))), args.cpu_nt)
        out["cpu_baseline"] = {"value": n_hv / base["value"], "unit": "s", "cores": base["cores"],
                               "kind": "oracle",
                               "sample": base["sample"] + f"; build time = {n_hv} products at "
                                                          "that rate (algebra not counted)"}
    print(json.dumps(out), flush=True)


def symbol_apply_bytes(G, B, T):
    """Algorithmic HBM bytes of one low-rank symbol apply of B vectors with T
    terms: every pass reads its inputs and writes its outputs once (forward
    rows: v -> row spectra of the nz data rows; forward columns: -> the
    mz x mx spectrum; inverse columns: spectrum and T tables -> T partial
    transforms of the nz model rows; inverse rows: those and the T
    coefficient fields -> out).  complex64 = 8 bytes, float32 = 4."""
    nz, nx, mz, mx = G.nz, G.nx, G.mz, G.mx
    return (4 * B * nz * nx + 8 * B * nz * mx            # rows forward
            + 8 * B * nz * mx + 8 * B * mz * mx          # columns forward
            + 8 * B * mz * mx + 8 * T * mz * mx + 8 * B * T * nz * mx   # columns inverse
            + 8 * B * T * nz * mx + 8 * T * nz * nx + 4 * B * nz * nx)  # rows inverse


def symbol_bench(args):
    """PDO and PSF+ rows (Sections 3.4, 3.6, Appendix A) on the 921x301 /
    64-shot / 4000-step workload at the smoothed model: one batched Hessian
    product of the sinusoid probe (r = 8 directions at rho0 = 2 pi f_max /
    c_max, f_max = 2.5 f0) and the 4 PSF combs; symbol columns, PSF
    extraction (9 x 29 lattice, 63 x 63 windows) and the PSF+ tables of rank
    `--symbol-rank` on the device; then both approximations applied to
    batches of smooth vectors through the FFT chain (360 x 960 FFT grid)."""
    import torch
    from oracle import pdo as D
    from paper_2507_10804_amd import fwi, synth
    from paper_2507_10804_amd import psf as gpsf
    from paper_2507_10804_amd import symbol as S

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    pg = synth.psf_grid(g.nz, g.nx)
    G = synth.symbol_grid(g.nz, g.nx, g.dx, pg.half, r=8,
                          rho0=synth.probe_radius(2.5 * g.f0, float(m_eval.max())))
    rank = args.symbol_rank
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    me = f32(m_eval)
    sym = S.Symbol(G, device=dev)
    probes = torch.cat([sym.pdo_probe()[None], f32(synth.psf_combs(pg))])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hv = plan.gn_hvp(me, probes)
    torch.cuda.synchronize()
    t_hv = time.perf_counter() - t0
    plan.release_workspaces()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    pdo_op, cols = S.pdo(sym, hv[0])
    ev[1].record()
    psf = gpsf.extract(pg, hv[1:].contiguous())
    ev[2].record()
    pp_op, info = S.psf_plus(sym, pg, psf, cols, rank)
    ev[3].record()
    torch.cuda.synchronize()
    build_ms = {"pdo_columns": ev[0].elapsed_time(ev[1]), "psf_extract": ev[1].elapsed_time(ev[2]),
                "psf_plus_tables": ev[2].elapsed_time(ev[3])}
    info_h = info.cpu().numpy()
    log(f"symbol: 5 Hessian products {t_hv:.1f} s; build {build_ms}; alpha {info_h[0]:.3e}")
    B = args.batch
    V = f32(synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, B + 1)))
    out_buf = torch.empty_like(V)
    res = {}
    reps = max(10, args.steps)
    for name, op in (("pdo", pdo_op), ("psf_plus", pp_op)):
        for bb in (1, B):
            for _ in range(args.warmup + 1):
                op(V[:bb], out=out_buf[:bb])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op(V[:bb], out=out_buf[:bb])
            e1.record()
            torch.cuda.synchronize()
            res[(name, bb)] = e0.elapsed_time(e1) / reps
            log(f"symbol: {name} apply, {bb} vectors: {res[(name, bb)]:.3f} ms")
    # quality against true products (information, not parity)
    hv4 = plan.gn_hvp(me, V[:4])
    plan.release_workspaces()
    psf_approx = gpsf.apply(pg, psf, V[:4])
    q = {}
    for name, a in (("psf", psf_approx), ("pdo", pdo_op(V[:4])), ("psf_plus", pp_op(V[:4]))):
        q[name] = [float((a[i] - hv4[i]).norm() / hv4[i].norm()) for i in range(4)]
    T = pp_op.terms
    ms = res[("psf_plus", B)]
    nbytes = symbol_apply_bytes(G, B, T)
    achieved = nbytes / (ms * 1e-3) / 1e9
    out = {"metric": "PSF+-approximate H_d v applies/s", "unit": "applies/s",
           "value": B / (ms * 1e-3), "n_gpus": 1, "steps": reps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (FP64 algebra)", "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301 at the smoothed model, {g.ns} shots, "
                                  f"nt={g.nt}; PDO r=8 at rho0={G.rho0:.4g} rad/m; PSF lattice "
                                  f"{pg.nzc}x{pg.nxc} window {pg.width}; PSF+ rank {rank}; FFT "
                                  f"grid {G.mz}x{G.mx}; apply to {B} smooth vectors per call",
                      "batch": B, "rank": rank, "terms": T, "fft_grid": [G.mz, G.mx]},
           "hessian_products_s": t_hv, "build_ms": build_ms,
           "alpha": float(info_h[0]), "kept": int(info_h[1]),
           "apply_ms": {f"{n}_B{b}": v for (n, b), v in res.items()},
           "rel_error_vs_true_hv": q,
           "roofline": {"bound": "hbm", "kernel": "fwi_symbol_apply (4 launches)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "alg_bytes_per_call": nbytes, "avg_call_us": ms * 1e3}}
    if not args.no_cpu_baseline:
        A_h = pp_op.A.cpu().numpy().astype(np.complex128)
        M_h = pp_op.M.cpu().numpy().astype(np.complex128)
        v_h = V[0].double().cpu().numpy()
        t1 = time.perf_counter()
        D.symbol_apply(G, A_h, M_h, v_h)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "applies/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one vector through the FP64 oracle's low-rank symbol "
                                         f"apply with the same {T} tables, {dt:.2f} s"}
    print(json.dumps(out), flush=True)


def map_bench(args):
    """Driver row (Sections 2.1, 2.3) on the 921x301 / 64-shot / 4000-step
    workload: data from the true layered-faulted model, the Matern prior
    (rho = 500 m, sigma = 200 m/s) centred at the smoothed model.  A rank-20
    low-rank approximation (30 probes, double pass) at the smoothed model
    gives H0 = (H~_d + R)^-1 for `--steps` L-BFGS iterations (the paper's
    preconditioning) and the Laplace approximation for `--steps` + 2 gpCN
    steps (beta = 0.2) from the last iterate."""
    import torch
    from paper_2507_10804_amd import drivers as D
    from paper_2507_10804_amd import fwi, synth
    from paper_2507_10804_amd import lowrank as glr

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    P = synth.matern_prior(g.nz, g.nx, g.dx, 500.0, 200.0)
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    dobs = plan.forward(f32(m_true))
    plan.release_workspaces()
    gp = glr.Prior(P, device=dev)
    me = f32(m_eval)
    r, k = 20, 30
    t1 = time.perf_counter()
    lr = glr.LowRank(plan, me, gp, f32(synth.gaussian_probes(g.nz, g.nx, k, seed=400)), r)
    torch.cuda.synchronize()
    t_lr = time.perf_counter() - t1
    plan.release_workspaces()
    post = D.Posterior(plan, gp, me, dobs)
    plan.profile(True)
    plan.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    opt = D.Lbfgs(post, me, h0=lr.inverse)
    hist = opt.run(args.steps)
    torch.cuda.synchronize()
    t_lbfgs = time.perf_counter() - t0
    evals = post.evals
    nseg = (g.nt - 1 + plan.K - 1) // plan.K
    kern = _kernel_table(plan, evals, algorithmic_bytes_grad(g, nseg))
    plan.profile(False)
    log(f"map: low-rank r={r} in {t_lr:.1f} s; {args.steps} L-BFGS iterations, {evals} "
        f"evaluations, {t_lbfgs:.1f} s; Phi {hist['phi'][0]:.4e} -> {hist['phi'][-1]:.4e}; "
        f"t {hist['t']}")
    plan.release_workspaces()
    nsteps = args.steps + 2
    rng = np.random.default_rng(args.seed + 7)
    w = f32(rng.standard_normal((nsteps, g.nz, g.nx)))
    u = rng.uniform(size=nsteps)
    t2 = time.perf_counter()
    st, acc, de = D.gpcn(post, opt.m, opt.m, 0.2, lr.sample, lr.hessian, w, u)
    torch.cuda.synchronize()
    t_gpcn = time.perf_counter() - t2
    plan.release_workspaces()
    log(f"map: gpCN {nsteps} steps {t_gpcn:.1f} s, accepted {sum(acc)}")
    dom = max(kern, key=lambda n: kern[n]["total_ms_per_step"])
    out = {"metric": "L-BFGS iterations/s (H0 = low-rank (H~_d + R)^-1, full misfit+gradient "
                     "per evaluation)",
           "unit": "iterations/s", "value": args.steps / t_lbfgs, "n_gpus": 1,
           "steps": args.steps, "warmup": 0, "ms_per_step": t_lbfgs * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (FP64 reductions)", "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301, {g.ns} shots, nt={g.nt}; Matern "
                                  f"prior rho=500 m sigma=200 m/s at the smoothed model; L-BFGS "
                                  f"mem 5, H0 = gamma (H~_d + R)^-1 of a rank-{r} approximation (gamma = "
                                  "s^T y / y^T H0 y of the newest pair), Armijo "
                                  f"backtracking; gpCN beta 0.2 with the same Laplace "
                                  f"approximation",
                      "iterations": args.steps},
           "objective_evaluations": evals, "evaluations_per_s": evals / t_lbfgs,
           "phi": hist["phi"], "step_lengths": hist["t"],
           "lowrank_build_s": t_lr, "gpcn_steps_per_s": nsteps / t_gpcn,
           "gpcn_accepted": int(sum(acc)), "gpcn_steps": nsteps,
           "kernels": kern,
           "roofline": _roofline_from(kern, dom, "the misfit + gradient solves dominate; "
                                                 "algorithmic bytes per launch of one "
                                                 "evaluation (forward with checkpoints, "
                                                 "recompute, one adjoint)")}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import drivers as Dr
        from oracle import lowrank as LR

        oracle.build(force=False)
        threads = min(16, len(os.sched_getaffinity(0)))
        gs = g.with_shots(np.arange(threads)).with_nt(args.cpu_nt)
        ds = oracle.forward(gs, m_true)
        t3 = time.perf_counter()
        Dr.objective(gs, LR.Prior(P), np.asarray(m_eval, np.float64), ds, m_eval)
        dt = time.perf_counter() - t3
        frac = (threads * (args.cpu_nt - 1)) / (g.ns * (g.nt - 1))
        per_iter = evals / args.steps
        out["cpu_baseline"] = {"value": frac / dt / per_iter, "unit": "iterations/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"one objective + gradient on {threads} of {g.ns} "
                                         f"shots, {args.cpu_nt} of {g.nt} steps, {dt:.1f} s; "
                                         f"scaled by shot-steps and by the GPU run's "
                                         f"{per_iter:.1f} evaluations per iteration"}
    print(json.dumps(out), flush=True)


def algorithmic_bytes_grad(g, nseg):
    """Algorithmic bytes of one misfit + gradient call per kernel kind:
    forward (gathering the data, storing checkpoints) and the segment
    recompute on the forward kernel, one adjoint (see algorithmic_bytes)."""
    full = algorithmic_bytes(g, 0, nseg, None, fused=False)
    nzp, nxp = g.nz + 2 * g.nb, g.nx + 2 * g.nb
    rec = (g.nt - 1) * (4 * nzp * nxp * (3 * g.ns + 1) + 4 * g.ns * nzp * nxp)
    adj1 = g.nt * (12 * nzp * nxp * g.ns + 4 * g.ns * g.nr) + (g.nt - 1) * (
        4 * nzp * nxp * g.ns + 8 * nzp * nxp + 16 * nzp * nxp)
    return {0: full[0] - rec, 2: adj1}


def _roofline_from(kern, dom, note):
    k = kern[dom]
    ach = k.get("achieved_gbs")
    out = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": None if ach is None else ach / HBM_PEAK_GBS, "traffic": None,
           "alg_bytes_per_launch": k.get("alg_bytes_per_launch"), "avg_launch_us": k["avg_us"],
           "note": note}
    if "compulsory_gbs" in k:
        out["unit_bytes_per_field_update"] = UPDATE_BYTES
        out["compulsory_gbs"] = k["compulsory_gbs"]
        out["compulsory_frac"] = k["compulsory_gbs"] / HBM_PEAK_GBS
    return out


def algorithmic_bytes_hvp(g, B, nseg):
    """Algorithmic bytes of one B-vector Hessian-vector call alone (forward
    + Born, recompute, adjoint), per kernel kind (see algorithmic_bytes)."""
    nzp, nxp = g.nz + 2 * g.nb, g.nx + 2 * g.nb
    Np = nzp * nxp
    ns, nr, nt = g.ns, g.nr, g.nt
    rec = (nt - 1) * (4 * Np * (3 * ns + 1) + 4 * ns * Np)
    born = ((nt - 1) * (4 * Np * (3 * ns + 1) + 4 * Np * B * (3 * ns + 1) + 4 * B * ns * nr)
            + (nseg - 1) * 8 * ns * Np)
    adj = nt * (12 * Np * B * ns + 4 * B * ns * nr) + (nt - 1) * (4 * Np * ns + 8 * Np + 16 * Np * B)
    return {0: rec, 1: born, 2: adj}


def autograd_bench(args):
    """Differentiation row: misfit and gradient, migration, and one
    Gauss-Newton product through the torch.autograd.Function on the
    921x301 / 64-shot / 4000-step workload, against the direct ABI calls."""
    import torch
    from paper_2507_10804_amd import autograd as ag
    from paper_2507_10804_amd import fwi, synth

    g, m_true, m_eval = synth.config_layered(nt=args.nt)
    dev = torch.device("cuda:0")
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    mt, me = f32(m_true), f32(m_eval)
    v = f32(synth.smooth_random((g.nz, g.nx), seed=1, sigma=5.0))
    dobs = plan.forward(mt)
    torch.cuda.synchronize()

    def timeit(fn, reps=args.steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def ag_grad():
        m = me.clone().requires_grad_(True)
        d = ag.forward(m, plan)
        (0.5 * ((d - dobs) ** 2).sum()).backward()
        return m.grad

    def ag_misfit():
        m = me.clone().requires_grad_(True)
        ag.misfit(m, dobs, plan).backward()
        return m.grad

    res = {
        "direct misfit_grad": timeit(lambda: plan.misfit_grad(me, dobs)),
        "autograd Misfit + backward": timeit(ag_misfit),
        "autograd FwiForward + backward (checkpoint resume)": timeit(ag_grad),
        "direct gn_hvp B=1": timeit(lambda: plan.gn_hvp(me, v)),
        "autograd jvp then vjp": timeit(lambda: ag.gn_hvp_autograd(me, v, plan)),
    }
    for k, t in res.items():
        log(f"{k}: {t * 1e3:.0f} ms")
    out = {"metric": "autograd layer: seconds per gradient / Gauss-Newton product vs direct",
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"layered-faulted 921x301, {g.ns} shots, nt={g.nt}, K=50"},
           "seconds": res,
           "value": res["autograd FwiForward + backward (checkpoint resume)"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-nt", type=int, default=1000)
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-launch HIP events (rocprofv3 runs)")
    ap.add_argument("--copy-variant", type=int, default=None,
                    help="with --calibrate-copy: time one copy variant only")
    ap.add_argument("--copy-reps", type=int, default=10)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only time a plain device-to-device copy of 2 GiB (the "
                         "reference kernel for HBM counters and attainable bandwidth)")
    ap.add_argument("--mode", choices=["hvp", "serve", "probing", "autograd", "psf", "lowrank",
                                       "symbol", "map"], default="hvp")
    ap.add_argument("--rank", type=int, default=100)
    ap.add_argument("--symbol-rank", type=int, default=16)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--requests-per-chain", type=int, default=6)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-log-dir", default=os.path.join(ROOT, "serve_logs"))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ckpt-every", type=int, default=50,
                    help="checkpoint interval K of the default mode; 0 keeps the whole forward "
                         "history instead (needs (nt - 1) x shots fields of workspace)")
    ap.add_argument("--separate", action="store_true",
                    help="time the step as fwi_misfit_grad + fwi_gn_hvp instead of the fused "
                         "fwi_misfit_grad_hvp")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the Hessian-vector product shards over shots "
              "with one all-reduce of the images, which is not implemented here; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "serve":
        serve_bench(args)
        return
    if args.mode == "probing":
        probing_bench(args)
        return
    if args.mode == "psf":
        return psf_bench(args)
    if args.mode == "lowrank":
        return lowrank_bench(args)
    if args.mode == "symbol":
        return symbol_bench(args)
    if args.mode == "map":
        return map_bench(args)
    if args.mode == "autograd":
        autograd_bench(args)
        return
    if args.calibrate_copy:
        calibrate_copy(args.copy_variant, args.copy_reps)
        return

    import torch
    from paper_2507_10804_amd import fwi, synth

    g, m_true, m_eval = synth.config_layered(ns=args.shots, nt=args.nt,
                                             ckpt_every=args.ckpt_every)
    hist = args.ckpt_every == 0
    B = args.batch
    vs = synth.smooth_random_batch(g.nz, g.nx, seeds=range(1, B + 1))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = fwi.Plan(g, device=dev)
    f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=dev)
    mt, me, vd = f32(m_true), f32(m_eval), f32(vs)
    log(f"workload: 921x301 padded {plan.nzp}x{plan.nxp}, {g.ns} shots, {g.nr} receivers, "
        f"nt={g.nt}, K={'history' if hist else plan.K}, B={B}")
    dobs = plan.forward(mt)  # synthetic observed data (untimed)
    hv = torch.empty((B, g.nz, g.nx), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    ws_gb = (plan.workspace_bytes(fwi.FWI_OP_GN_HVP, B) +
             plan.workspace_bytes(fwi.FWI_OP_MISFIT_GRAD)) / 1e9

    fused = not args.separate
    if fused:
        ws_gb = plan.workspace_bytes(fwi.FWI_OP_GRAD_HVP, B) / 1e9
    free_gb = torch.cuda.mem_get_info(dev)[0] / 1e9
    if ws_gb > free_gb:
        print(f"bench.py: the step needs {ws_gb:.1f} GB of workspace and {free_gb:.1f} GB are free"
              + (" (history mode keeps every forward level: use fewer shots or steps, or a "
                 "checkpoint interval)" if hist else ""), file=sys.stderr)
        sys.exit(2)

    def step():
        if fused:
            return plan.misfit_grad_hvp(me, dobs, vd, out=hv)[:2]
        phi, grad = plan.misfit_grad(me, dobs)
        plan.gn_hvp(me, vd, out=hv)
        return phi, grad

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    if plan.status():
        raise RuntimeError("device status flags set after warm-up")

    if not args.no_profile:
        plan.profile(True)
        plan.profile_reset()
    st = torch.cuda.current_stream(dev)
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(st)
        if fused:
            plan.misfit_grad_hvp(me, dobs, vd, out=hv)
            e1.record(st)
        else:
            phi, grad = plan.misfit_grad(me, dobs)
            e1.record(st)
            plan.gn_hvp(me, vd, out=hv)
        e2.record(st)
        ev.append((e0, e1, e2))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for i in range(args.steps):
        log(f"timed step {i + 1}/{args.steps}: {ev[i][0].elapsed_time(ev[i][2]):.1f} ms")
    if plan.status():
        raise RuntimeError("device status flags set in the timed region")

    ms_step = wall * 1e3 / args.steps
    call_lat = np.array([e[0].elapsed_time(e[2]) for e in ev])
    hv_lat = np.array([e[1].elapsed_time(e[2]) for e in ev])
    grad_lat = np.array([e[0].elapsed_time(e[1]) for e in ev])
    nzp, nxp = g.nz + 2 * g.nb, g.nx + 2 * g.nb
    solve_updates = g.ns * nzp * nxp * (g.nt - 1)
    # credited solves (recomputes are not): fused = forward + B Born + (B + 1) adjoint;
    # separate = gradient (forward + adjoint) + Hv (forward + B Born + B adjoint)
    solves = 2 + 2 * B if fused else 2 + 1 + 2 * B
    gpts = solves * solve_updates / (ms_step * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": B / (ms_step * 1e-3),
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"layered-faulted 921x301 dx=10m, {g.ns} shots, {g.nr} receivers, "
                               f"Ricker 8 Hz, nt={g.nt}, "
                               f"{'whole forward history kept' if hist else f'K={plan.K}'}: "
                               f"misfit, gradient and "
                               f"{B} GN Hv at one model per step"
                               + (", one fused pass (shared forward solve and recompute)"
                                  if fused else ", as two calls"),
                   "call": "fwi_misfit_grad_hvp" if fused else "fwi_misfit_grad + fwi_gn_hvp",
                   "grid": [g.nz, g.nx], "padded": [nzp, nxp], "shots": g.ns,
                   "receivers": g.nr, "nt": g.nt, "batch": B, "ckpt_every": 0 if hist else plan.K,
                   "workspace_gb": round(ws_gb, 2)},
        "gpt_updates_per_s": gpts,
        "hbm_headline_frac": gpts * 1e9 * 16 / (HBM_PEAK_GBS * 1e9),
    }
    if fused:
        out["call_latency_ms"] = {"p50": float(np.percentile(call_lat, 50)),
                                  "p99": float(np.percentile(call_lat, 99)), "batch": B}
    else:
        out["hv_call_latency_ms"] = {"p50": float(np.percentile(hv_lat, 50)),
                                     "p99": float(np.percentile(hv_lat, 99)), "batch": B}
        out["grad_latency_ms"] = float(np.median(grad_lat))

    if not args.no_profile:
        nseg = (g.nt - 1 + plan.K - 1) // plan.K
        comp = algorithmic_bytes(g, B, nseg, plan.K, fused=fused, hist=hist)
        upd = field_updates(g, B, fused=fused, hist=hist)
        kern = {}
        for kind in KERNEL_NAMES:
            name = plan.kernel_name(kind)
            ms, n = plan.profile_read(kind)
            n_step = n / args.steps
            avg_s = 1e-3 * ms / max(n, 1)
            u_launch = upd[kind] / n_step if n_step else 0.0
            c_launch = comp[kind] / n_step if n_step else 0.0
            kern[name] = {"kind": ["forward", "forward+Born", "adjoint"][kind],
                          "steps_per_launch": plan.kernel_steps(kind),
                          "launches_per_step": n_step, "avg_us": 1e6 * avg_s,
                          "total_ms_per_step": ms / args.steps,
                          "field_updates_per_launch": u_launch,
                          "alg_bytes_per_launch": UPDATE_BYTES * u_launch,
                          "achieved_gbs": UPDATE_BYTES * u_launch / avg_s / 1e9 if n else 0.0,
                          "compulsory_bytes_per_launch": c_launch,
                          "compulsory_gbs": c_launch / avg_s / 1e9 if n else 0.0}
        plan.profile(False)
        dom = max(kern, key=lambda k: kern[k]["total_ms_per_step"])
        k = kern[dom]
        # the committed counter runs are of the default workload's launches
        # (921x301, 64 shots, B = 16, one fused pass); other shapes get none
        same = (g.nz, g.nx, g.ns, B, fused, hist) == (301, 921, 64, 16, True, False)
        traffic = read_traffic(dom) if same else None
        copy = copy_rates(reps=5)
        attain = max(copy.values())
        out["roofline"] = {
            "bound": "hbm", "kernel": dom,
            "achieved": k["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": k["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": k["alg_bytes_per_launch"],
            "unit_bytes_per_field_update": UPDATE_BYTES,
            "avg_launch_us": k["avg_us"],
            "counter_gbs": traffic / (1e-6 * k["avg_us"]) / 1e9 if traffic else None,
            "counter_frac": traffic / (1e-6 * k["avg_us"]) / 1e9 / HBM_PEAK_GBS if traffic else None,
            "compulsory_bytes_per_launch": k["compulsory_bytes_per_launch"],
            "compulsory_gbs": k["compulsory_gbs"],
            "compulsory_frac": k["compulsory_gbs"] / HBM_PEAK_GBS,
            "attainable_copy_gbs": attain,
            "attainable_copy_frac": attain / HBM_PEAK_GBS}
        out["kernels"] = kern

    if not args.no_cpu_baseline:
        # the process's CPU share: the cores it may run on, capped by the
        # OpenMP thread count the host sets for it
        cpu = host_cpu()
        threads = cpu["affinity"]
        if cpu["omp_num_threads"]:
            threads = min(threads, int(cpu["omp_num_threads"]))
        del hv, dobs
        plan.release_workspaces()
        out["cpu_baseline"] = cpu_baseline(g, m_eval, vs[0], threads, args.cpu_nt)
        out["cpu_baseline"]["small_case"] = small_case_timings(threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Scheduling logic of the request server on the CPU, with a simulated
backend (sleep-based service times, closed-form results): routing of
results, merging, memory admission, rejection, cancellation, deadlines,
failure isolation, ordering and overlap."""
import threading
import time

import numpy as np
import pytest
import torch

from paper_2507_10804_amd.serve import (AdmissionError, Cancelled, DeadlineExceeded, Request,
                                        Server)


class FakeBackend:
    """Service time proportional to the request; result = closed form."""

    def __init__(self, per_req=0.02, per_vec=0.005, budget=10_000, bytes_per=100):
        self.per_req, self.per_vec = per_req, per_vec
        self.budget, self.bytes_per = budget, bytes_per
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.batches = []
        self.reserved_trace = []

    def mem_budget(self):
        return self.budget

    def max_batch(self, req):
        return 8

    def prepare(self, req):
        pass

    def job_bytes(self, reqs):
        big = max((r.tag or {}).get("bytes", self.bytes_per) for r in reqs)
        return big + self.bytes_per * (len(reqs) - 1)

    def run(self, slot, reqs):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.batches.append(len(reqs))
        try:
            nvec = sum(r.nvec for r in reqs)
            extra = max((r.tag or {}).get("sleep", 0.0) for r in reqs)
            time.sleep(self.per_req + self.per_vec * nvec + extra)
            for r in reqs:
                if (r.tag or {}).get("poison"):
                    raise RuntimeError(f"request {r.rid} is poison")
            out = []
            for r in reqs:
                if r.kind == "hvp":
                    out.append(2.0 * r.v + float(r.model[1:]))
                else:
                    out.append(float(r.m.sum()))
            return out
        finally:
            with self.lock:
                self.running -= 1


def hv_req(model="m1", seed=0, tag=None):
    v = torch.as_tensor(np.random.default_rng(seed).standard_normal((3, 4)))
    return Request("hvp", "d", model=model, v=v, tag=tag)


def mf_req(seed=0, tag=None):
    m = torch.as_tensor(np.random.default_rng(seed).standard_normal((3, 4)))
    return Request("misfit", "d", m=m, tag=tag)


def expected(r):
    if r.kind == "hvp":
        return 2.0 * r.v + float(r.model[1:])
    return float(r.m.sum())


def check(fut):
    res = fut.result(timeout=10)
    exp = expected(fut.request)
    if isinstance(exp, float):
        assert res == exp
    else:
        assert torch.equal(res, exp)


def test_results_routed_alone_and_in_mix():
    be = FakeBackend()
    with Server(be, slots=3, coalesce=True) as srv:
        futs = [srv.submit(hv_req(f"m{i % 3}", seed=i) if i % 2 else mf_req(seed=i))
                for i in range(40)]
        for f in futs:
            check(f)
    with Server(FakeBackend(), slots=1, coalesce=False) as srv:
        for i in range(6):
            check(srv.submit(hv_req("m2", seed=i)))


def test_merging_at_same_model():
    be = FakeBackend(per_req=0.05)
    with Server(be, slots=1, coalesce=True, max_batch=8) as srv:
        blocker = srv.submit(mf_req(seed=99))
        time.sleep(0.01)  # the blocker occupies the only slot
        futs = [srv.submit(hv_req("m1", seed=i)) for i in range(6)]
        futs += [srv.submit(hv_req("m2", seed=10 + i)) for i in range(3)]
        for f in futs + [blocker]:
            check(f)
    assert max(be.batches) >= 6  # the six m1 requests ran as one batch
    assert all(f.request.batch >= 3 for f in futs)


def test_probe_batch_counts_vectors():
    be = FakeBackend()
    with Server(be, slots=1, coalesce=True, max_batch=8) as srv:
        blocker = srv.submit(mf_req())
        time.sleep(0.01)
        v5 = torch.zeros((5, 3, 4))
        big = srv.submit(Request("hvp", "d", model="m1", v=v5))
        small = [srv.submit(hv_req("m1", seed=i)) for i in range(4)]
        for f in [blocker, big] + small:
            check(f)
    assert max(be.batches) <= 4  # 5 + 3 singles = 8 vectors at most per call


def test_memory_admission_never_exceeds_budget():
    be = FakeBackend(budget=350, bytes_per=100)
    srv = Server(be, slots=4, coalesce=False)
    peak = [0]
    stop = threading.Event()

    def watch():
        while not stop.is_set():
            peak[0] = max(peak[0], srv._reserved)
            time.sleep(0.001)

    t = threading.Thread(target=watch)
    t.start()
    futs = [srv.submit(mf_req(seed=i)) for i in range(20)]
    for f in futs:
        check(f)
    stop.set()
    t.join()
    srv.shutdown()
    assert peak[0] <= 350
    assert be.max_running <= 3  # 3 x 100 bytes fit, a fourth does not


def test_oversized_request_rejected():
    be = FakeBackend(budget=500)
    with Server(be, slots=2) as srv:
        big = srv.submit(mf_req(tag={"bytes": 10_000}))
        ok = srv.submit(mf_req(seed=3))
        with pytest.raises(AdmissionError):
            big.result(timeout=5)
        check(ok)


def test_cancellation_and_deadline():
    be = FakeBackend(per_req=0.1)
    with Server(be, slots=1) as srv:
        running = srv.submit(mf_req(seed=1))
        time.sleep(0.02)
        cancel_me = srv.submit(mf_req(seed=2))
        late = Request("misfit", "d", m=torch.zeros(3, 4), deadline=time.monotonic() + 0.01)
        late_f = srv.submit(late)
        assert cancel_me.cancel()
        assert not running.cancel()
        with pytest.raises(Cancelled):
            cancel_me.result(timeout=5)
        with pytest.raises(DeadlineExceeded):
            late_f.result(timeout=5)
        check(running)


def test_failure_isolated_from_batch_mates():
    be = FakeBackend(per_req=0.05)
    with Server(be, slots=1, coalesce=True) as srv:
        blocker = srv.submit(mf_req())
        time.sleep(0.01)
        good = [srv.submit(hv_req("m1", seed=i)) for i in range(3)]
        bad = srv.submit(hv_req("m1", seed=7, tag={"poison": True}))
        good += [srv.submit(hv_req("m1", seed=i + 10)) for i in range(2)]
        for f in [blocker] + good:
            check(f)
        with pytest.raises(RuntimeError, match="poison"):
            bad.result(timeout=5)


def test_plain_path_is_fifo():
    be = FakeBackend()
    with Server(be, slots=1, coalesce=False) as srv:
        futs = [srv.submit(hv_req("m1", seed=i)) for i in range(8)]
        for f in futs:
            f.result(timeout=10)
    ends = [f.request.t_end for f in futs]
    assert ends == sorted(ends)
    assert max(be.batches) == 1


def test_continuous_admission_overlaps_long_job():
    """A short request arriving while a long one runs finishes first."""
    be = FakeBackend(per_req=0.01)
    with Server(be, slots=2) as srv:
        long = srv.submit(mf_req(seed=1, tag={"sleep": 0.5}))
        time.sleep(0.05)
        short = srv.submit(mf_req(seed=2))
        check(short)
        assert not long.done()
        check(long)
    assert be.max_running == 2


def test_shutdown_cancels_pending():
    be = FakeBackend(per_req=0.2)
    srv = Server(be, slots=1)
    srv.submit(mf_req())
    time.sleep(0.02)
    pending = srv.submit(mf_req(seed=5))
    srv.shutdown()
    with pytest.raises(Cancelled):
        pending.result(timeout=5)


class _Dataset:
    def __init__(self, geom, models):
        self.plan = type("P", (), {"geom": geom})()
        self.models = models
        self.dobs = None


def test_serving_trace_draws_and_request_log(tmp_path):
    """The serving trace draws grid, shot count and record length
    independently and misfit / Hessian-vector requests 1:1, and the
    per-request JSONL log has one complete line per request.  Runs the
    closed loop against the simulated backend on CPU tensors."""
    import json

    from paper_2507_10804_amd import synth
    from paper_2507_10804_amd.serve import workload as wl

    be = FakeBackend(per_req=0.0005, per_vec=0.0, budget=10 ** 9)
    be.device = torch.device("cpu")
    be.datasets = {}
    banks = {}
    for grid, (nx, nz) in wl.GRIDS.items():
        nx, nz = nx // 16, nz // 16  # small stand-ins: the draw only needs shapes
        models = {f"m{j}": torch.full((nz, nx), 2000.0 + j) for j in range(len(wl.SMOOTHING))}
        for ns in wl.SHOTS:
            for nt in wl.NTS:
                g = synth.make_geometry(nx, nz, nt=10, ns=2, rec_ix=[1], f0=8.0, v_nominal=5500.0)
                be.datasets[wl.dataset_key(grid, ns, nt)] = _Dataset(g, models)
        banks[grid] = torch.zeros((4, nz, nx))
    with Server(be, slots=4) as srv:
        recs, tw, t1 = wl.run_closed_loop(srv, be, banks, chains=8, rate=4000.0,
                                          requests_per_chain=60, seed=3)
    assert len(recs) == 480 and all(r["ok"] for r in recs)
    kinds = [r["kind"] for r in recs]
    assert abs(kinds.count("misfit") - kinds.count("hvp")) < 0.15 * len(recs)
    for field, values in (("grid", wl.GRIDS), ("shots", wl.SHOTS), ("nt", wl.NTS)):
        counts = [sum(r[field] == v for r in recs) for v in values]
        assert min(counts) > 0.2 * len(recs), (field, counts)
    # independence: every (grid, shots, nt) combination occurs
    assert len({(r["grid"], r["shots"], r["nt"]) for r in recs}) == 27
    path = tmp_path / "requests.jsonl"
    wl.write_log(recs, str(path), tw)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == len(recs)
    for x in lines:
        assert {"grid", "shots", "nt", "kind", "queue_ms", "device_ms", "latency_ms",
                "batch", "ok"} <= set(x)
        assert x["latency_ms"] >= x["device_ms"] >= 0 and x["queue_ms"] >= 0
    s = wl.summarize(recs, tw, t1)
    assert s["requests"] == len(recs) and s["hv_per_s"] > 0 and s["misfit_per_s"] > 0
    assert s["p99_ms"] >= s["p50_ms"]

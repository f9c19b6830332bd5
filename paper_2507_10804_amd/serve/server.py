"""Continuous-batching request server for wave-equation derivative requests.

Clients (MCMC chains evaluating proposals, Section 2.3; probing batches for
the PSF / PDO approximations, Sections 3.2-3.4) submit requests against
datasets kept resident on the GPU.  The server

* admits a request as soon as an execution slot and enough device memory are
  free (every job reserves its workspace bytes, dominated by the forward
  checkpoints, against a fixed budget; a job that can never fit is rejected);
* runs up to ``slots`` jobs at once, each on its own stream, so that work of
  different requests overlaps on the device; a request arriving while others
  run starts when the first slot frees, without waiting for the others;
* merges pending Hessian-vector requests at the same resident model into one
  batched call (one forward solve and recompute shared by the batch);
* isolates failures: a batched job that fails is re-run request by request,
  so only the faulty request reports an error;
* honours cancellation and deadlines of requests that have not started.

The plain path -- one request at a time, first come first served, no
merging -- is the same server with ``slots=1, coalesce=False``.

The execution backend is pluggable (``GpuBackend`` runs the HIP library; the
CPU tests use a simulated backend).  A backend provides
``job_bytes(requests) -> int``, ``max_batch(request) -> int`` and
``run(slot, requests) -> list`` of per-request results (may raise).
"""
from __future__ import annotations

import collections
import itertools
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Optional


class RequestError(RuntimeError):
    pass


class AdmissionError(RequestError):
    """The request can never fit the device-memory budget."""


class DeadlineExceeded(RequestError):
    pass


class Cancelled(RequestError):
    pass


@dataclass
class Request:
    """One unit of client work.

    kind:    "misfit" (Phi at a proposal model), "forward" (data at a
             proposal model) or "hvp" (H v at a resident model, one vector or
             a probe batch)
    dataset: key of a resident dataset (geometry, observed data, models)
    model:   resident model id ("hvp"), or None
    m:       proposal model ("misfit", "forward"), or None
    v:       vector(s) for "hvp": [nz][nx] or [B][nz][nx]
    deadline: absolute time.monotonic() after which the request is dropped
              if it has not started
    """

    kind: str
    dataset: str
    model: Optional[str] = None
    m: Any = None
    v: Any = None
    deadline: Optional[float] = None
    tag: Any = None
    # filled in by the server
    rid: int = -1
    t_submit: float = 0.0
    t_start: float = 0.0
    t_end: float = 0.0
    batch: int = 1
    ready_event: Any = None

    @property
    def nvec(self) -> int:
        if self.kind != "hvp" or self.v is None:
            return 1
        return 1 if self.v.dim() == 2 else int(self.v.shape[0])

    def merge_key(self):
        return (self.kind, self.dataset, self.model) if self.kind == "hvp" else None


class Future:
    def __init__(self, req: Request, lock):
        self.request = req
        self._lock = lock
        self._ev = threading.Event()
        self._result = None
        self._exc = None
        self._cancel = False

    def done(self):
        return self._ev.is_set()

    def cancel(self) -> bool:
        """Cancel if not started yet; returns whether it was cancelled."""
        with self._lock:
            if self.request.t_start:
                return False
            self._cancel = True
            return True

    def cancelled(self):
        return self._cancel

    def result(self, timeout=None):
        if not self._ev.wait(timeout):
            raise TimeoutError("request not finished")
        if self._exc is not None:
            raise self._exc
        return self._result

    def exception(self, timeout=None):
        self._ev.wait(timeout)
        return self._exc

    def _set(self, result=None, exc=None):
        self._result, self._exc = result, exc
        self._ev.set()


@dataclass
class Job:
    futures: list
    nbytes: int
    slot: int = -1


@dataclass
class Stats:
    records: list = field(default_factory=list)  # (kind, nvec, t_submit, t_start, t_end, batch, ok)

    def add(self, r: Request, ok: bool):
        self.records.append((r.kind, r.nvec, r.t_submit, r.t_start, r.t_end, r.batch, ok))


class Server:
    def __init__(self, backend, slots: int = 4, coalesce: bool = True, max_batch: int = 16,
                 mem_budget: Optional[int] = None):
        self.backend = backend
        self.nslots = int(slots)
        self.coalesce = bool(coalesce)
        self.max_batch = int(max_batch)
        self.mem_budget = mem_budget if mem_budget is not None else backend.mem_budget()
        lock = threading.Lock()
        self._cv = threading.Condition(lock)
        self._pending = collections.deque()
        self._free = list(range(self.nslots))
        self._reserved = 0
        self._running = 0
        self._stop = False
        self._ids = itertools.count()
        self.stats = Stats()
        self._slot_jobs = [None] * self.nslots
        self._slot_cv = [threading.Condition(lock) for _ in range(self.nslots)]
        self._workers = [threading.Thread(target=self._worker, args=(i,), daemon=True,
                                          name=f"serve-slot{i}") for i in range(self.nslots)]
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True,
                                            name="serve-dispatch")
        for t in self._workers:
            t.start()
        self._dispatcher.start()

    # ------------------------------------------------------------ client side
    def submit(self, req: Request) -> Future:
        req.rid = next(self._ids)
        req.t_submit = time.monotonic()
        self.backend.prepare(req)
        fut = Future(req, self._cv)
        with self._cv:
            if self._stop:
                raise RuntimeError("server is shut down")
            self._pending.append(fut)
            self._cv.notify_all()
        return fut

    def shutdown(self, wait: bool = True):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
            for c in self._slot_cv:
                c.notify_all()
        if wait:
            self._dispatcher.join()
            for t in self._workers:
                t.join()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.shutdown()

    def busy(self) -> bool:
        with self._cv:
            return bool(self._pending) or self._running > 0

    # ------------------------------------------------------------ dispatcher
    def _drop_dead(self, now):
        """Fail cancelled and expired requests that have not started."""
        keep = collections.deque()
        for f in self._pending:
            if f.cancelled():
                f._set(exc=Cancelled(f"request {f.request.rid} cancelled"))
            elif f.request.deadline is not None and now > f.request.deadline:
                f._set(exc=DeadlineExceeded(f"request {f.request.rid} missed its deadline"))
                self.stats.add(f.request, False)
            else:
                keep.append(f)
        self._pending = keep

    def _take_job(self):
        """Head-of-line request plus mergeable ones; None if nothing fits."""
        head = self._pending[0]
        group = [head]
        key = head.request.merge_key()
        if self.coalesce and key is not None:
            cap = min(self.max_batch, self.backend.max_batch(head.request))
            n = head.request.nvec
            for f in itertools.islice(self._pending, 1, None):
                if f.request.merge_key() == key and n + f.request.nvec <= cap:
                    group.append(f)
                    n += f.request.nvec
        nbytes = self.backend.job_bytes([f.request for f in group])
        return group, nbytes

    def _dispatch(self):
        with self._cv:
            while True:
                while not self._stop and (not self._pending or not self._free):
                    self._cv.wait(0.05)
                    self._drop_dead(time.monotonic())
                if self._stop:
                    for f in self._pending:
                        f._set(exc=Cancelled("server shut down"))
                    self._pending.clear()
                    return
                self._drop_dead(time.monotonic())
                if not self._pending:
                    continue
                group, nbytes = self._take_job()
                if nbytes > self.mem_budget:
                    # can never fit: reject the head alone, merged ones stay
                    head = self._pending.popleft()
                    head._set(exc=AdmissionError(
                        f"request {head.request.rid} needs {nbytes} bytes, budget "
                        f"{self.mem_budget}"))
                    self.stats.add(head.request, False)
                    continue
                if self._reserved + nbytes > self.mem_budget:
                    self._cv.wait(0.05)  # wait for memory to free up (no bypass)
                    continue
                ids = {id(f) for f in group}
                self._pending = collections.deque(f for f in self._pending if id(f) not in ids)
                slot = self._free.pop()
                self._reserved += nbytes
                self._running += 1
                now = time.monotonic()
                for f in group:
                    f.request.t_start = now
                    f.request.batch = sum(x.request.nvec for x in group)
                self._slot_jobs[slot] = Job(group, nbytes, slot)
                self._slot_cv[slot].notify_all()

    # ---------------------------------------------------------------- workers
    def _worker(self, slot):
        while True:
            with self._cv:
                while self._slot_jobs[slot] is None and not self._stop:
                    self._slot_cv[slot].wait(0.1)
                job = self._slot_jobs[slot]
                if job is None and self._stop:
                    return
            self._execute(slot, job)
            with self._cv:
                self._slot_jobs[slot] = None
                self._reserved -= job.nbytes
                self._running -= 1
                self._free.append(slot)
                self._cv.notify_all()

    def _execute(self, slot, job):
        reqs = [f.request for f in job.futures]
        try:
            results = self.backend.run(slot, reqs)
            outcome = [(r, None) for r in results]
        except Exception as exc:  # isolate: re-run one by one
            if len(reqs) == 1:
                outcome = [(None, exc)]
            else:
                outcome = []
                for r in reqs:
                    r.batch = r.nvec
                    try:
                        outcome.append((self.backend.run(slot, [r])[0], None))
                    except Exception as e1:
                        outcome.append((None, e1))
        now = time.monotonic()
        for f, (res, exc) in zip(job.futures, outcome):
            f.request.t_end = now
            self.stats.add(f.request, exc is None)
            f._set(result=res, exc=exc)

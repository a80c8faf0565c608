"""Continuous-batching request loop over the C ABI (sample and log-det requests).

Operators stay resident on the device (their gmrf_op handles, with FFT spectra when
preconditioned).  Requests queue in arrival order.  Whenever a worker is free, the dispatcher
admits the first queued request whose device bytes fit the HBM budget next to everything already
in flight (first fit: a large request at the head does not hold up smaller ones behind it; a
request that has waited longer than `max_wait` seconds is admitted before any later one, so none
starves), and folds into the same job the other queued requests that can share its launches:

  * samples on 2D lattices without preconditioning that agree in order, storage, tolerance and
    m_max, each at most `batch_points` lattice points times right-hand sides, run as one uneven batch
    (gmrf_sample_batch: every Lanczos step is one set of launches over all their columns).  Small
    requests are bound by per-step launch latency, which the batch shares; a larger request already
    fills the device alone, and batching it would only make the small ones wait for its steps;
  * log-det requests on the same operator with the same quadrature length m run as one call
    with all their probes (explicit Rademacher probes, each request's own seed).

A sample whose stored Krylov basis alone would exceed the budget runs the two-pass sampler (O(n)
memory, the recurrence twice) on its own instead of being turned away.  With the library's scratch
in one reserved region (gmrf_pool_reserve, which spares the server the device allocator's irregular
cost) a job can find no free range large enough although its bytes fit the budget; it then goes
back to the head of the queue, and nothing more is admitted until another job has returned its
scratch (when no other job is running, the failure is the request's own and is reported).  Each worker owns a HIP
stream (default priority) and calls the blocking entry points, which release the GIL: admitted
jobs overlap on the GPU.  Every column's arithmetic is independent of the other columns of its
launch (fixed-order reductions, no atomics), so a request's result is bitwise the same alone and
in any mix or batch; a log-det request's mean and standard error are always formed the same way
from its own per-probe values.

This module only schedules; the numerics all run in libgmrf.so.
"""
import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import GmrfError
from ._abi import GMRF_ENOMEM


@dataclass
class ServeRequest:
    rid: int
    kind: str                 # "sample" or "logdet"
    op_index: int
    k: int                    # right-hand sides (sample) or probes (logdet)
    seed: int
    tol: float = 1e-5
    m_max: int = 300          # sample: Krylov cap; logdet: quadrature steps m
    t_arrival: float = 0.0
    # filled in by the server
    t_start: float = 0.0
    t_done: float = 0.0
    bytes: int = 0
    two_pass: bool = False    # sample whose stored Krylov basis does not fit the budget: O(n) two-pass mode
    batched_with: int = 0     # other requests that shared this request's launches
    result: object = None
    error: str = ""
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self):
        return self.t_done - self.t_arrival


class Server:
    def __init__(self, operators, hbm_budget, workers=4, keep_results=True, max_batch_columns=256, max_wait=2.0,
                 batch_points=1 << 22):
        import torch
        self.torch = torch
        self.ops = list(operators)
        self.budget = int(hbm_budget)
        self.workers = int(workers)
        self.keep_results = keep_results
        self.max_batch_columns = int(max_batch_columns)
        self.max_wait = float(max_wait)
        self.batch_points = int(batch_points)
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.in_flight_bytes = 0
        self.peak_bytes = 0
        self.busy = 0
        self.peak_busy = 0
        self.jobs = 0
        self.retries = 0
        self._hold = False         # a job found the region fragmented: admit nothing until another completes
        self.completed = []
        self._stop = False
        self._threads = []
        self._work = collections.deque()
        self._work_cv = threading.Condition()

    # -- sizing -------------------------------------------------------------------------------
    def request_bytes(self, req):
        """Device bytes of the request (library estimate, pool rounding included, plus Z and X in FP64); a
        sample whose stored basis would exceed the budget is switched to the two-pass sampler."""
        op = self.ops[req.op_index]
        vec = op.n * req.k * 8
        if req.kind == "sample":
            stored = op.bytes(req.k, req.m_max, False) + 2 * vec
            req.two_pass = stored > self.budget
            return op.bytes_two_pass(req.k, req.m_max) + 2 * vec if req.two_pass else stored
        # the log-det call keeps three Krylov slots, as the two-pass sampler does, and the probes (int8)
        return op.bytes_two_pass(req.k, req.m_max) + op.n * req.k

    def _batch_key(self, req):
        """Requests with equal keys can share launches (None: never batched)."""
        op = self.ops[req.op_index]
        if req.kind == "logdet":
            return ("logdet", req.op_index, req.m_max)
        shape = getattr(op, "shape", None)
        if req.two_pass or shape is None or len(shape) != 2 or getattr(op, "precond", False) or \
                getattr(op, "has_diag", False) or getattr(op, "order", None) is None or \
                op.n * req.k > self.batch_points:
            return None
        return ("sample2d", op.order, op.storage, req.tol, req.m_max)

    # -- lifecycle ----------------------------------------------------------------------------
    def start(self):
        self._stop = False
        for w in range(self.workers):
            t = threading.Thread(target=self._worker, args=(w,), daemon=True)
            t.start()
            self._threads.append(t)
        d = threading.Thread(target=self._dispatcher, daemon=True)
        d.start()
        self._threads.append(d)
        return self

    def stop(self):
        with self.cv:
            self._stop = True
            self.cv.notify_all()
        with self._work_cv:
            self._work_cv.notify_all()
        for t in self._threads:
            t.join(timeout=60)
        self._threads = []

    def submit(self, req):
        req.bytes = self.request_bytes(req)
        if req.t_arrival == 0.0:
            req.t_arrival = time.perf_counter()
        with self.cv:
            if req.bytes > self.budget:
                req.error = f"request needs {req.bytes} B, above the HBM budget {self.budget} B"
                req.t_done = time.perf_counter()
                req.done.set()
                self.completed.append(req)
                return req
            self.queue.append(req)
            self.cv.notify_all()
        return req

    # -- scheduling ---------------------------------------------------------------------------
    def _admit(self):
        """Under self.cv: the next job (a list of requests) or None.  First fit in arrival order, except that
        a request older than max_wait blocks every later one until it fits; then the compatible requests
        behind it that still fit join its launches."""
        free = self.budget - self.in_flight_bytes
        now = time.perf_counter()
        head = None
        for req in self.queue:
            if req.bytes <= free:
                head = req
                break
            if now - req.t_arrival > self.max_wait:
                return None         # the oldest waiting request keeps its turn
        if head is None:
            return None
        job, used = [head], head.bytes
        key = self._batch_key(head)
        if key is not None:
            cols = head.k
            for req in self.queue:
                if req is head or self._batch_key(req) != key:
                    continue
                if cols + req.k > self.max_batch_columns or used + req.bytes > free:
                    continue
                job.append(req)
                used += req.bytes
                cols += req.k
        for req in job:
            self.queue.remove(req)
            req.batched_with = len(job) - 1
        return job

    def _dispatcher(self):
        while True:
            with self.cv:
                job = None
                while not self._stop:
                    if self.queue and self.busy < self.workers and not self._hold:
                        job = self._admit()
                        if job:
                            break
                    self.cv.wait(timeout=0.02)
                if self._stop:
                    return
                nbytes = sum(r.bytes for r in job)
                self.in_flight_bytes += nbytes
                self.busy += 1
                self.jobs += 1
                self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
                self.peak_busy = max(self.peak_busy, self.busy)
            with self._work_cv:
                self._work.append(job)
                self._work_cv.notify()

    def _worker(self, w):
        stream = None
        while True:
            with self._work_cv:
                while not self._work and not self._stop:
                    self._work_cv.wait(timeout=0.05)
                if self._stop and not self._work:
                    return
                job = self._work.popleft()
            t0 = time.perf_counter()
            for req in job:
                req.t_start = t0
            enomem = False
            try:
                if stream is None:
                    stream = self._new_stream()
                results = self._execute(job, stream)
                for req, res in zip(job, results):
                    req.result = res
            except Exception as e:      # any failure ends this job's requests only, never the worker
                enomem = isinstance(e, GmrfError) and e.status == GMRF_ENOMEM
                msg = f"{type(e).__name__}: {e}" if not isinstance(e, GmrfError) else str(e)
                for req in job:
                    req.error = msg
                    req.result = None
            finally:
                t1 = time.perf_counter()
                with self.cv:
                    self.in_flight_bytes -= sum(r.bytes for r in job)
                    retry = enomem and self.busy > 1
                    self.busy -= 1
                    if retry:
                        self.retries += 1
                        self._hold = True
                        for req in reversed(job):
                            req.error = ""
                            req.batched_with = 0
                            self.queue.appendleft(req)
                    else:
                        self._hold = False
                        for req in job:
                            req.t_done = t1
                            if not self.keep_results:
                                req.result = self._summary(req)
                            self.completed.append(req)
                    self.cv.notify_all()
                if not retry:
                    for req in job:
                        req.done.set()

    def _new_stream(self):
        return self.torch.cuda.Stream()

    def _execute(self, job, stream):
        with self.torch.cuda.stream(stream):
            out = self._run(job, stream)
        stream.synchronize()
        return out

    # -- numerics (all in the library) ----------------------------------------------------------
    def _draw_z(self, req, n):
        g = self.torch.Generator(device="cuda")
        g.manual_seed(req.seed)
        return self.torch.randn((req.k, n), dtype=self.torch.float64, device="cuda", generator=g)

    def _run(self, job, stream):
        from . import rademacher, sample_batch
        torch = self.torch
        head = job[0]
        if head.kind == "sample":
            if len(job) == 1:
                op = self.ops[head.op_index]
                Z = self._draw_z(head, op.n)
                if head.two_pass:
                    X, info = op.sample_two_pass(Z, tol=head.tol, m_max=head.m_max, stream=stream)
                else:
                    X, info = op.sample(Z, tol=head.tol, m_max=head.m_max, reorth=False, stream=stream)
                return [{"X": X, "info": info}]
            ops = [self.ops[r.op_index] for r in job]
            Zs = [self._draw_z(r, op.n) for r, op in zip(job, ops)]
            Xs, info = sample_batch(ops, Zs, tol=head.tol, m_max=head.m_max, stream=stream)
            out, c = [], 0
            for r, X in zip(job, Xs):
                out.append({"X": X, "info": info[c:c + r.k]})
                c += r.k
            return out
        op = self.ops[head.op_index]
        probes = torch.cat([rademacher(r.seed, op.n, r.k, stream=stream) for r in job]) if len(job) > 1 else \
            rademacher(head.seed, op.n, head.k, stream=stream)
        _, _, per = op.logdet(probes.shape[0], head.m_max, probes=probes, stream=stream)
        out, c = [], 0
        for r in job:
            p = np.array(per[c:c + r.k])
            c += r.k
            se = float(np.std(p, ddof=1) / np.sqrt(r.k)) if r.k > 1 else float("nan")
            out.append({"logdet": float(np.mean(p)), "std_err": se, "per_probe": p})
        return out

    @staticmethod
    def _summary(req):
        """What stays of a result when the server does not keep them: per-column statuses of a sample."""
        if req.result is None or req.kind != "sample":
            return None
        return {"info": req.result["info"]}

    # -- traces ---------------------------------------------------------------------------------
    def run_trace(self, requests, time_scale=1.0, window=None):
        """Replay requests at their arrival times (seconds from start, scaled); returns stats over the
        completed requests and the wall time from the first arrival to the last completion."""
        t0 = time.perf_counter()
        for req in sorted(requests, key=lambda r: r.t_arrival):
            target = t0 + req.t_arrival * time_scale
            now = time.perf_counter()
            if target > now:
                time.sleep(target - now)
            req.t_arrival = max(target, t0)
            self.submit(req)
        for req in requests:
            req.done.wait()
        wall = time.perf_counter() - t0
        st = stats(requests, wall)
        st["jobs"] = self.jobs
        st["retries"] = self.retries
        st["peak_in_flight"] = self.peak_busy
        return st


def stats(requests, wall):
    """Throughput and latency of finished requests.  samples_ok counts only the sample columns that
    reached their tolerance (status OK); latency runs from arrival to result."""
    ok = [r for r in requests if not r.error]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[i]

    samples_ok = 0
    for r in ok:
        if r.kind == "sample" and r.result is not None:
            samples_ok += sum(1 for i in r.result["info"] if i["status"] == "OK")
    probes = sum(r.k for r in ok if r.kind == "logdet")
    return {"requests": len(requests), "completed": len(ok), "rejected": len(requests) - len(ok),
            "two_pass": sum(1 for r in ok if r.two_pass),
            "batched": sum(1 for r in ok if r.batched_with > 0),
            "wall_s": wall, "p50_latency_s": pct(50), "p99_latency_s": pct(99),
            "completed_per_s": len(ok) / wall if wall > 0 else 0.0,
            "samples_ok": samples_ok,
            "samples_per_s": samples_ok / wall if wall > 0 else 0.0,
            "probes_per_s": probes / wall if wall > 0 else 0.0}

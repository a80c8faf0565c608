"""Continuous-batching request loop over the C ABI (sample and log-det requests).

Operators stay resident on the device (their gmrf_op handles, with FFT spectra when
preconditioned).  Requests queue in arrival order; the dispatcher admits the head request as
soon as a worker slot is free and its device bytes fit the HBM budget next to everything
already in flight, so requests that arrive while others run start as capacity frees up.  A
sample whose stored Krylov basis alone would exceed the budget runs the two-pass sampler (O(n)
memory, the recurrence twice) instead of being turned away.  Each
worker owns a HIP stream (default priority) and calls the blocking sample / log-det entry
point, which releases the GIL: admitted requests overlap on the GPU.  Every call has its own
scratch and the kernels' reductions are fixed-order, so a request's result does not depend on
what else is in flight.

This module only schedules; the numerics all run in libgmrf.so.
"""
import collections
import threading
import time
from dataclasses import dataclass, field

from . import GmrfError


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
    result: object = None
    error: str = ""
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self):
        return self.t_done - self.t_arrival


class Server:
    def __init__(self, operators, hbm_budget, workers=4, keep_results=True):
        import torch
        self.torch = torch
        self.ops = list(operators)
        self.budget = int(hbm_budget)
        self.workers = int(workers)
        self.keep_results = keep_results
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.in_flight_bytes = 0
        self.peak_bytes = 0
        self.busy = 0
        self.peak_busy = 0
        self.completed = []
        self._stop = False
        self._threads = []
        self._work = collections.deque()
        self._work_cv = threading.Condition()

    # -- sizing -------------------------------------------------------------------------------
    def request_bytes(self, req):
        """Device bytes of the request; a sample whose stored basis would exceed the budget is
        switched to the two-pass sampler (three Krylov slots instead of m_max + 1)."""
        op = self.ops[req.op_index]
        vec = op.n * req.k * 8
        ring3 = op.bytes(req.k, 2, False) + req.k * (req.m_max + 2) * 64   # 3 Krylov slots + scalars
        if req.kind == "sample":
            stored = op.bytes(req.k, req.m_max, False) + 2 * vec          # + Z and X (FP64)
            req.two_pass = stored > self.budget
            return ring3 + 2 * vec if req.two_pass else stored
        return ring3

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
    def _dispatcher(self):
        while True:
            with self.cv:
                while not self._stop and not (self.queue and self.busy < self.workers and
                                              self.in_flight_bytes + self.queue[0].bytes <= self.budget):
                    self.cv.wait(timeout=0.05)
                if self._stop:
                    return
                req = self.queue.popleft()
                self.in_flight_bytes += req.bytes
                self.busy += 1
                self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
                self.peak_busy = max(self.peak_busy, self.busy)
            with self._work_cv:
                self._work.append(req)
                self._work_cv.notify()

    def _worker(self, w):
        stream = None
        while True:
            with self._work_cv:
                while not self._work and not self._stop:
                    self._work_cv.wait(timeout=0.05)
                if self._stop and not self._work:
                    return
                req = self._work.popleft()
            req.t_start = time.perf_counter()
            try:
                if stream is None:
                    stream = self._new_stream()
                req.result = self._execute(req, stream)
            except Exception as e:      # any failure ends this request only, never the worker
                req.error = f"{type(e).__name__}: {e}" if not isinstance(e, GmrfError) else str(e)
                req.result = None
            finally:
                req.t_done = time.perf_counter()
                if not self.keep_results:
                    req.result = None
                with self.cv:
                    self.in_flight_bytes -= req.bytes
                    self.busy -= 1
                    self.completed.append(req)
                    self.cv.notify_all()
                req.done.set()

    def _new_stream(self):
        return self.torch.cuda.Stream()

    def _execute(self, req, stream):
        with self.torch.cuda.stream(stream):
            out = self._run(req, stream)
        stream.synchronize()
        return out

    def _run(self, req, stream):
        torch = self.torch
        op = self.ops[req.op_index]
        if req.kind == "sample":
            g = torch.Generator(device="cuda")
            g.manual_seed(req.seed)
            Z = torch.randn((req.k, op.n), dtype=torch.float64, device="cuda", generator=g)
            if req.two_pass:
                X, info = op.sample_two_pass(Z, tol=req.tol, m_max=req.m_max, stream=stream)
            else:
                X, info = op.sample(Z, tol=req.tol, m_max=req.m_max, reorth=False, stream=stream)
            return {"X": X, "info": info}
        mean, se, per = op.logdet(req.k, req.m_max, seed=req.seed, stream=stream)
        return {"logdet": mean, "std_err": se, "per_probe": per}

    # -- traces ---------------------------------------------------------------------------------
    def run_trace(self, requests, time_scale=1.0):
        """Replay requests at their arrival times (seconds from start, scaled); returns stats."""
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
        return stats(requests, time.perf_counter() - t0)


def stats(requests, wall):
    ok = [r for r in requests if not r.error]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[i]

    samples = sum(r.k for r in ok if r.kind == "sample")
    probes = sum(r.k for r in ok if r.kind == "logdet")
    return {"requests": len(requests), "completed": len(ok), "rejected": len(requests) - len(ok),
            "two_pass": sum(1 for r in ok if r.two_pass),
            "wall_s": wall, "p50_latency_s": pct(50), "p99_latency_s": pct(99),
            "samples_per_s": samples / wall if wall > 0 else 0.0,
            "probes_per_s": probes / wall if wall > 0 else 0.0}

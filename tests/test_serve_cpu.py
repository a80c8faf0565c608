"""Host logic of the serving loop (no GPU): request sizing, the two-pass switch, rejection of requests
too large for either mode, first-fit admission with aging, coalescing of compatible requests into one
job, and worker failure handling, on stand-in operators whose byte counts follow the library's layout
(m_max + 1 Krylov slots of n k values; three slots in two-pass mode)."""
import threading
import time

from paper_1312_1476_amd import serve


class _Op:
    def __init__(self, n, shape=None, order=1, storage=0, precond=False):
        self.n = n
        self.shape = shape
        self.order = order
        self.storage = storage
        self.precond = precond
        self.has_diag = False

    def bytes(self, k, m_max, reorth):
        return (m_max + 1) * self.n * k * 8

    def bytes_two_pass(self, k, m_max):
        return 3 * self.n * k * 8 + k * (m_max + 2) * 64


def _req(kind="sample", k=4, m_max=300, rid=1, op=0):
    return serve.ServeRequest(rid, kind, op, k, 7, m_max=m_max)


def test_stored_mode_when_it_fits():
    srv = serve.Server([_Op(10_000)], hbm_budget=1 << 40)
    r = _req()
    b = srv.request_bytes(r)
    assert not r.two_pass and b == 301 * 10_000 * 4 * 8 + 2 * 10_000 * 4 * 8


def test_two_pass_when_the_basis_does_not_fit():
    op = _Op(10_000)
    stored = serve.Server([op], hbm_budget=1 << 40).request_bytes(_req())
    srv = serve.Server([op], hbm_budget=stored // 10)
    r = _req()
    b = srv.request_bytes(r)
    assert r.two_pass and b < stored // 10
    assert b == 3 * 10_000 * 4 * 8 + 4 * 302 * 64 + 2 * 10_000 * 4 * 8


def test_logdet_is_never_two_pass_and_oversize_is_rejected():
    srv = serve.Server([_Op(10_000)], hbm_budget=1000)
    r = _req("logdet", k=8, m_max=80)
    srv.request_bytes(r)
    assert not r.two_pass
    big = srv.submit(_req(k=32))     # not started: submit rejects before queueing
    assert big.error and "budget" in big.error and big.done.is_set()


class _RecordingServer(serve.Server):
    """Records each job's request ids; requests with an odd id fail with a non-library exception."""

    def __init__(self, *a, fail_odd=False, hold=None, **kw):
        super().__init__(*a, **kw)
        self.job_log = []
        self.fail_odd = fail_odd
        self.hold = hold

    def _new_stream(self):
        return object()

    def _execute(self, job, stream):
        self.job_log.append([r.rid for r in job])
        if self.hold is not None:
            self.hold.wait(timeout=10)
        if self.fail_odd and job[0].rid % 2:
            raise RuntimeError("out of memory while drawing Z")
        return [{"ok": r.rid, "info": [{"status": "OK"}] * r.k} for r in job]


def test_worker_survives_any_exception_and_releases_its_slot():
    srv = _RecordingServer([_Op(1000)], hbm_budget=1 << 40, workers=2, fail_odd=True).start()
    reqs = [serve.ServeRequest(i, "sample", 0, 2, 7, m_max=50) for i in range(8)]
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(timeout=30)
    srv.stop()
    assert [bool(r.error) for r in reqs] == [bool(i % 2) for i in range(8)]
    assert all("RuntimeError" in r.error for r in reqs if r.rid % 2)
    assert all(r.result["ok"] == r.rid for r in reqs if not r.rid % 2)
    assert srv.busy == 0 and srv.in_flight_bytes == 0 and len(srv.completed) == 8


def _queue_then_release(srv, reqs, hold):
    """Submit while the only worker is held on a first job, so that the rest queue up together."""
    srv.start()
    srv.submit(reqs[0])
    deadline = time.time() + 10
    while srv.busy == 0 and time.time() < deadline:
        time.sleep(0.01)
    for r in reqs[1:]:
        srv.submit(r)
    hold.set()
    for r in reqs:
        assert r.done.wait(timeout=30)
    srv.stop()


def test_compatible_samples_share_a_job_and_logdets_merge_by_operator():
    ops = [_Op(64 * 64, (64, 64)), _Op(32 * 32, (32, 32)), _Op(16 ** 3, (16, 16, 16)),
           _Op(48 * 48, (48, 48), order=2), _Op(64 * 64, (64, 64), precond=True), _Op(2048 ** 2, (2048, 2048))]
    hold = threading.Event()
    srv = _RecordingServer(ops, hbm_budget=1 << 40, workers=1, hold=hold)
    R = serve.ServeRequest
    reqs = [R(0, "sample", 0, 2, 1), R(1, "sample", 0, 3, 2), R(2, "sample", 1, 4, 3), R(3, "sample", 2, 2, 4),
            R(4, "sample", 3, 2, 5), R(5, "sample", 4, 2, 6), R(6, "logdet", 0, 8, 7, m_max=80),
            R(7, "logdet", 0, 8, 8, m_max=80), R(8, "logdet", 1, 8, 9, m_max=80), R(9, "sample", 1, 2, 10, tol=1e-8),
            R(10, "sample", 5, 2, 11), R(11, "sample", 5, 2, 12)]
    _queue_then_release(srv, reqs, hold)
    jobs = [sorted(j) for j in srv.job_log]
    assert jobs[0] == [0]
    # small first-order 2D samples with the same tolerance and m_max share one job; 3D, second-order,
    # preconditioned, other-tolerance and large samples run alone; log-dets merge per (operator, m)
    assert [1, 2] in jobs and [3] in jobs and [4] in jobs and [5] in jobs and [9] in jobs
    assert [10] in jobs and [11] in jobs
    assert [6, 7] in jobs and [8] in jobs
    st = serve.stats(reqs, 1.0)
    assert st["samples_ok"] == sum(r.k for r in reqs if r.kind == "sample") and st["batched"] == 4


def test_first_fit_admission_and_aging():
    ops = [_Op(1000, (40, 25))]
    srv = serve.Server(ops, hbm_budget=10_000)
    R = serve.ServeRequest
    big, small = R(1, "sample", 0, 1, 1), R(2, "sample", 0, 1, 2)
    big.bytes, small.bytes = 8_000, 1_000
    big.t_arrival = small.t_arrival = time.perf_counter()
    srv.queue.extend([big, small])
    srv.in_flight_bytes = 4_000                  # the big head does not fit; the small one behind it does
    assert srv._admit() == [small]
    srv.queue.append(small)                      # back behind the big one
    big.t_arrival -= 10 * srv.max_wait           # once the head has waited too long it keeps its turn
    assert srv._admit() is None
    srv.in_flight_bytes = 0
    job = srv._admit()
    assert job[0] is big


def _enomem():
    from paper_1312_1476_amd._abi import GMRF_ENOMEM
    e = serve.GmrfError.__new__(serve.GmrfError)
    e.status = GMRF_ENOMEM
    RuntimeError.__init__(e, "gmrf_sample: ENOMEM: reserved region has no free range")
    return e


class _FragmentedServer(_RecordingServer):
    """Request 1 finds no free range on its first attempt; request 2 never does."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.attempts = {}

    def _execute(self, job, stream):
        rid = job[0].rid
        self.attempts[rid] = self.attempts.get(rid, 0) + 1
        if rid == 2 or (rid == 1 and self.attempts[rid] == 1):
            self.job_log.append([r.rid for r in job])
            raise _enomem()
        return super()._execute(job, stream)


def test_fragmentation_retries_after_a_completion_and_alone_reports():
    hold = threading.Event()
    srv = _FragmentedServer([_Op(1000, (40, 25), order=2)], hbm_budget=1 << 40, workers=2, hold=hold).start()
    r0, r1 = serve.ServeRequest(0, "sample", 0, 1, 1), serve.ServeRequest(1, "sample", 0, 1, 2)
    srv.submit(r0)
    deadline = time.time() + 10
    while srv.busy == 0 and time.time() < deadline:
        time.sleep(0.01)
    srv.submit(r1)
    while srv.retries == 0 and time.time() < deadline:
        time.sleep(0.01)
    assert srv.retries == 1 and not r1.done.is_set() and srv.queue[0] is r1
    time.sleep(0.1)
    assert srv.attempts[1] == 1          # held: nothing is admitted until a job completes
    hold.set()
    assert r0.done.wait(10) and r1.done.wait(10)
    assert not r0.error and not r1.error and r1.result["ok"] == 1 and srv.attempts[1] == 2
    # with nothing else running, the failure is the request's own
    r2 = srv.submit(serve.ServeRequest(2, "sample", 0, 1, 3))
    assert r2.done.wait(10)
    srv.stop()
    assert "ENOMEM" in r2.error and srv.retries == 1 and srv.busy == 0 and srv.in_flight_bytes == 0

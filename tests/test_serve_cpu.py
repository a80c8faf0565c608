"""Host logic of the serving loop (no GPU): request sizing, the two-pass switch and the
rejection of requests too large for either mode, on a stand-in operator whose byte count follows
the library's layout (m_max + 1 Krylov slots of n k values)."""
from paper_1312_1476_amd import serve


class _Op:
    def __init__(self, n):
        self.n = n

    def bytes(self, k, m_max, reorth):
        return (m_max + 1) * self.n * k * 8


def _req(kind="sample", k=4, m_max=300):
    return serve.ServeRequest(1, kind, 0, k, 7, m_max=m_max)


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


class _FailingServer(serve.Server):
    """Requests with an odd id raise a non-library exception inside the worker."""

    def _new_stream(self):
        return object()

    def _execute(self, req, stream):
        if req.rid % 2:
            raise RuntimeError("out of memory while drawing Z")
        return {"ok": req.rid}


def test_worker_survives_any_exception_and_releases_its_slot():
    srv = _FailingServer([_Op(1000)], hbm_budget=1 << 40, workers=2).start()
    reqs = [serve.ServeRequest(i, "sample", 0, 2, 7, m_max=50) for i in range(8)]
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(timeout=30)
    srv.stop()
    assert [bool(r.error) for r in reqs] == [bool(i % 2) for i in range(8)]
    assert all("RuntimeError" in r.error for r in reqs if r.rid % 2)
    assert all(r.result == {"ok": r.rid} for r in reqs if not r.rid % 2)
    assert srv.busy == 0 and srv.in_flight_bytes == 0 and len(srv.completed) == 8

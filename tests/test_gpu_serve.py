"""Serving (continuous batching) over the C ABI: each result is identical alone, in a mix of
overlapping jobs and coalesced into a batched job; admission never exceeds the HBM budget; a sample
whose stored basis does not fit runs the two-pass sampler; requests too large even for that are
rejected; and served samples (FP64 alone, FP32 storage in a batch) and FP32-storage log-dets match the
oracle."""
import numpy as np
import pytest

from oracle import lanczos, lattice, logdet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import os
    import torch
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1312_1476_amd as gm
    from paper_1312_1476_amd import serve
    ops = [gm.Operator.lattice((96, 80), 1, 0.05, 1.0, "free", "f32"),
           gm.Operator.lattice((24, 20, 28), 1, 0.2, 1.0, "free", "f64"),
           gm.Operator.lattice((128, 128), 2, 0.05, 1.0, "free", "f64").set_circulant_precond(),
           gm.Operator.lattice((150, 150), 1, 0.01, 1.0, "free", "f64")]
    return gm, serve, ops


def _same_info(a, b):
    def norm(d):
        return {k: ("nan" if isinstance(v, float) and v != v else v) for k, v in d.items()}
    return [norm(x) for x in a] == [norm(x) for x in b]


def _mix(serve):
    R = serve.ServeRequest
    return [R(1, "sample", 0, 4, 7, tol=1e-6, m_max=300), R(2, "logdet", 1, 8, 11, m_max=40),
            R(3, "sample", 2, 3, 5, tol=1e-8, m_max=400), R(4, "sample", 3, 8, 9, tol=1e-6, m_max=400),
            R(5, "logdet", 2, 6, 13, m_max=60), R(6, "sample", 1, 16, 3, tol=1e-6, m_max=200),
            R(7, "sample", 0, 32, 21, tol=1e-6, m_max=300), R(8, "logdet", 3, 4, 17, m_max=80),
            R(9, "logdet", 1, 8, 19, m_max=40), R(10, "sample", 0, 2, 29, tol=1e-6, m_max=300),
            R(11, "sample", 3, 3, 31, tol=1e-6, m_max=400)]


def _check_same(alone, reqs):
    import torch
    for req in reqs:
        assert not req.error, req.error
        a = alone[req.rid]
        if req.kind == "sample":
            assert torch.equal(a["X"], req.result["X"]), req.rid
            assert _same_info(a["info"], req.result["info"])
        else:
            assert a["logdet"] == req.result["logdet"]
            assert np.array_equal(a["per_probe"], req.result["per_probe"])


def test_alone_equals_mix(env):
    gm, serve, ops = env
    alone = {}
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=1).start()
    for req in _mix(serve):
        srv.submit(req)
        req.done.wait()
        assert not req.error, req.error
        assert req.batched_with == 0
        alone[req.rid] = req.result
    srv.stop()
    # four workers: jobs overlap on the device
    mix = _mix(serve)
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=4).start()
    for req in mix:
        srv.submit(req)
    for req in mix:
        req.done.wait()
    srv.stop()
    assert srv.peak_busy >= 2
    _check_same(alone, mix)
    # one worker busy on the first request: the rest queue up and compatible ones are coalesced
    # (samples on the 96x80 lattice into one uneven batch, log-dets on the 3D lattice into one call)
    mix = _mix(serve)
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=1).start()
    for req in mix:
        srv.submit(req)
    for req in mix:
        req.done.wait()
    srv.stop()
    assert serve.stats(mix, 1.0)["batched"] >= 2 and srv.jobs < len(mix)
    _check_same(alone, mix)


def test_budget_admission_and_rejection(env):
    gm, serve, ops = env
    probe = serve.Server(ops, hbm_budget=1 << 40)
    reqs = _mix(serve)
    sizes = [probe.request_bytes(r) for r in reqs]
    budget = int(max(sizes) * 1.3)
    srv = serve.Server(ops, hbm_budget=budget, workers=4, keep_results=False).start()
    for req in reqs:
        srv.submit(req)
    big = serve.ServeRequest(99, "sample", 3, 2000, 1, m_max=1000)
    srv.submit(big)
    for req in reqs + [big]:
        req.done.wait()
    srv.stop()
    assert all(not r.error for r in reqs)
    assert big.error and "budget" in big.error
    assert srv.peak_bytes <= budget
    st = serve.stats(reqs + [big], 1.0)
    assert st["completed"] == len(reqs) and st["rejected"] == 1


def test_budget_holds_in_the_librarys_own_accounting(env):
    """The admission estimate against what the library really holds: with the library's scratch confined
    to a region of exactly the budget's size (Z and X, which torch allocates, are outside it), every
    admitted mix still runs -- a job that found the region fragmented is retried once others return
    their scratch -- and the library holds nothing afterwards."""
    gm, serve, ops = env
    probe = serve.Server(ops, hbm_budget=1 << 40)
    sizes = [probe.request_bytes(r) for r in _mix(serve)]
    budget = int(max(sizes) * 1.3)
    gm.pool_reserve(budget)
    try:
        a0 = gm.pool_info()["device_allocs"]
        reqs = _mix(serve)
        srv = serve.Server(ops, hbm_budget=budget, workers=4, keep_results=False).start()
        for req in reqs:
            srv.submit(req)
        for req in reqs:
            req.done.wait()
        srv.stop()
        assert all(not r.error for r in reqs), [r.error for r in reqs if r.error]
        info = gm.pool_info()
        assert info["in_use"] == 0 and info["device_allocs"] == a0 and info["largest_free_range"] >= budget
    finally:
        gm.pool_reserve(0)


def test_served_sample_matches_oracle(env):
    import torch
    gm, serve, ops = env
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=2).start()
    req = srv.submit(serve.ServeRequest(1, "sample", 3, 2, 42, tol=1e-8, m_max=500))
    req.done.wait()
    srv.stop()
    assert not req.error
    g = torch.Generator(device="cuda")
    g.manual_seed(42)
    Z = torch.randn((2, ops[3].n), dtype=torch.float64, device="cuda", generator=g).cpu().numpy()
    Q = lattice.lattice_precision((150, 150), 1, 0.01, 1.0, "free")
    X = req.result["X"].cpu().numpy()
    for r in range(2):
        m = req.result["info"][r]["m_used"]
        ref = lanczos.sample_csr(Q, Z[r], m, tol=0.0)
        assert np.linalg.norm(X[r] - ref.x) / np.linalg.norm(ref.x) <= 1e-8


def test_served_fp32_batch_matches_oracle(env):
    """Two requests on the FP32-storage lattice coalesced into one uneven batch at the serving tolerance
    1e-5: every column reaches it, and each sample is within 1e-5 (relative) of the oracle's x_m at the
    same m."""
    import torch
    gm, serve, ops = env
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=1)
    reqs = [serve.ServeRequest(1, "sample", 0, 3, 71, tol=1e-5, m_max=600),
            serve.ServeRequest(2, "sample", 0, 2, 73, tol=1e-5, m_max=600)]
    for r in reqs:
        r.bytes = srv.request_bytes(r)
    assert srv._batch_key(reqs[0]) == srv._batch_key(reqs[1]) is not None
    results = srv._execute(reqs, torch.cuda.Stream())
    Q = lattice.lattice_precision((96, 80), 1, 0.05, 1.0, "free")
    for r, res in zip(reqs, results):
        g = torch.Generator(device="cuda")
        g.manual_seed(r.seed)
        Z = torch.randn((r.k, ops[0].n), dtype=torch.float64, device="cuda", generator=g).cpu().numpy()
        X = res["X"].cpu().numpy()
        assert [i["status"] for i in res["info"]] == ["OK"] * r.k
        for c in range(r.k):
            ref = lanczos.sample_csr(Q, Z[c], res["info"][c]["m_used"], tol=0.0)
            assert np.linalg.norm(X[c] - ref.x) / np.linalg.norm(ref.x) <= 1e-5, (r.rid, c)


def test_served_fp32_logdets_match_oracle(env):
    """Two log-det requests on the FP32-storage lattice merged into one call (each request's own seed's
    Rademacher probes, FP64 scalars), as the serving mix runs them: every per-probe quadrature is within
    1e-5 (relative) of the oracle's on the same probes."""
    import torch
    gm, serve, ops = env
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=1)
    reqs = [serve.ServeRequest(1, "logdet", 0, 5, 81, m_max=40), serve.ServeRequest(2, "logdet", 0, 3, 83, m_max=40)]
    for r in reqs:
        r.bytes = srv.request_bytes(r)
    assert srv._batch_key(reqs[0]) == srv._batch_key(reqs[1]) is not None
    results = srv._execute(reqs, torch.cuda.Stream())
    Q = lattice.lattice_precision((96, 80), 1, 0.05, 1.0, "free")
    for r, res in zip(reqs, results):
        ref = logdet.hutchinson_csr(Q, r.k, r.m_max, seed=r.seed)
        assert np.all(np.abs(res["per_probe"] - ref.per_probe) <= 1e-5 * np.abs(ref.per_probe)), r.rid


def test_two_pass_fallback(env):
    """A budget below the stored basis but above three Krylov slots: the sample is admitted in
    two-pass mode and equals the one-pass sample (same m, 1e-12)."""
    import torch
    gm, serve, ops = env
    probe = serve.Server(ops, hbm_budget=1 << 40)
    req = serve.ServeRequest(1, "sample", 3, 4, 23, tol=1e-8, m_max=500)
    stored = probe.request_bytes(req)
    assert not req.two_pass
    budget = stored // 4
    srv = serve.Server(ops, hbm_budget=budget, workers=2).start()
    req2 = srv.submit(serve.ServeRequest(1, "sample", 3, 4, 23, tol=1e-8, m_max=500))
    req2.done.wait()
    srv.stop()
    assert not req2.error, req2.error
    assert req2.two_pass and req2.bytes <= budget and srv.peak_bytes <= budget
    g = torch.Generator(device="cuda")
    g.manual_seed(23)
    Z = torch.randn((4, ops[3].n), dtype=torch.float64, device="cuda", generator=g)
    X1, i1 = ops[3].sample(Z, tol=1e-8, m_max=500)
    assert [i["m_used"] for i in i1] == [i["m_used"] for i in req2.result["info"]]
    assert float((req2.result["X"] - X1).norm() / X1.norm()) <= 1e-12
    assert serve.stats([req2], 1.0)["two_pass"] == 1


def test_budget_call_returns_cached_scratch(env):
    """Scratch of finished calls stays cached in the library's pool for reuse; setting the HBM budget
    hands it back to the device, so the memory the caller then sees free includes it."""
    import torch
    gm, serve, ops = env
    op = gm.Operator.lattice((256, 256), 1, 0.05, 1.0, "free", "f64")
    Z = torch.randn((8, op.n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    need = op.bytes(8, 600, False)
    assert need > (256 << 20)
    op.sample(Z, tol=0.0, m_max=600)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free_cached, _ = torch.cuda.mem_get_info()
    gm.set_hbm_budget(0)
    free_after, _ = torch.cuda.mem_get_info()
    assert free_after - free_cached >= need // 2, (free_cached, free_after, need)
    op.close()


def test_alone_equals_mix_with_two_pass(env):
    """A budget that sends the larger samples to the two-pass sampler: each result is still the same
    alone and in the mix (the mode depends only on the request and the budget)."""
    import torch
    gm, serve, ops = env
    probe = serve.Server(ops, hbm_budget=1 << 40)
    sizes = [probe.request_bytes(r) for r in _mix(serve)]
    budget = int(sorted(sizes)[len(sizes) // 2])        # about half the samples do not fit stored
    alone = {}
    srv = serve.Server(ops, hbm_budget=budget, workers=1).start()
    reqs = [r for r in _mix(serve)]
    for req in reqs:
        srv.submit(req)
        req.done.wait()
        alone[req.rid] = (req.error, req.two_pass, req.result)
    srv.stop()
    assert any(tp for e, tp, _ in alone.values() if not e)
    mix = _mix(serve)
    srv = serve.Server(ops, hbm_budget=budget, workers=4).start()
    for req in mix:
        srv.submit(req)
    for req in mix:
        req.done.wait()
    srv.stop()
    assert srv.peak_bytes <= budget
    for req in mix:
        err, tp, res = alone[req.rid]
        assert bool(req.error) == bool(err) and req.two_pass == tp, req.rid
        if err:
            continue
        if req.kind == "sample":
            assert torch.equal(res["X"], req.result["X"]), req.rid
            assert _same_info(res["info"], req.result["info"])
        else:
            assert res["logdet"] == req.result["logdet"]

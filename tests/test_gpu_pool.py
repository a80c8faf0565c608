"""The scratch pool's reserved region (gmrf_pool_reserve / gmrf_pool_query), through the C ABI: calls
carve their scratch from the region, make no device allocations, give bitwise the same results as
with the ordinary pool, hand every range back (the free ranges merge into one), and a call larger than
the region is refused without running."""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1312_1476_amd as gm
    yield gm
    gm.pool_reserve(0)


def _z(n, k, seed):
    import torch
    return torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(n, k, seed, 0).T)).to("cuda:0")


def test_region_calls_allocate_nothing_and_match(gm):
    import torch
    ops = [gm.Operator.lattice((128, 96), 1, 0.05, 1.0, "free", "f32"),
           gm.Operator.lattice((24, 20, 28), 1, 0.2, 1.0, "free", "f64"),
           gm.Operator.lattice((128, 128), 2, 0.05, 1.0, "free", "f64").set_circulant_precond()]
    Zs = [_z(op.n, 5, 41 + i) for i, op in enumerate(ops)]
    ref = [op.sample(Z, tol=1e-6, m_max=300) for op, Z in zip(ops, Zs)]
    ref_tp = ops[1].sample_two_pass(Zs[1], tol=1e-6, m_max=300)
    ref_ld = ops[2].logdet(6, 40, seed=3)
    ref_b, _ = gm.sample_batch([ops[0], ops[0]], [Zs[0], Zs[0][:2].contiguous()], tol=1e-6, m_max=300)
    gm.pool_reserve(1 << 30)
    info0 = gm.pool_info()
    assert info0["reserved_bytes"] == 1 << 30 and info0["largest_free_range"] == 1 << 30 and info0["cached"] == 0
    for _ in range(2):
        for op, Z, (X0, i0) in zip(ops, Zs, ref):
            X, i = op.sample(Z, tol=1e-6, m_max=300)
            assert torch.equal(X, X0) and [d["m_used"] for d in i] == [d["m_used"] for d in i0]
        X, _ = ops[1].sample_two_pass(Zs[1], tol=1e-6, m_max=300)
        assert torch.equal(X, ref_tp[0])
        ld = ops[2].logdet(6, 40, seed=3)
        assert ld[0] == ref_ld[0] and np.array_equal(ld[2], ref_ld[2])
        Xb, _ = gm.sample_batch([ops[0], ops[0]], [Zs[0], Zs[0][:2].contiguous()], tol=1e-6, m_max=300)
        assert all(torch.equal(a, b) for a, b in zip(Xb, ref_b))
    info = gm.pool_info()
    assert info["device_allocs"] == info0["device_allocs"] and info["device_frees"] == info0["device_frees"]
    assert info["in_use"] == 0 and info["largest_free_range"] == 1 << 30
    gm.pool_reserve(0)
    assert gm.pool_info()["reserved_bytes"] == 0
    for op in ops:
        op.close()


def test_call_larger_than_region_is_refused(gm):
    import torch
    op = gm.Operator.lattice((256, 256), 1, 0.05, 1.0, "free", "f64")
    Z = _z(op.n, 8, 5)
    assert op.bytes(8, 600) > (64 << 20)
    gm.pool_reserve(64 << 20)
    X = torch.full_like(Z, 7.0)
    with pytest.raises(gm.GmrfError) as e:
        op.sample(Z, tol=1e-6, m_max=600, out=X)
    assert e.value.status == 4 and "free range" in str(e.value)
    assert torch.all(X == 7.0)                       # nothing ran
    info = gm.pool_info()
    assert info["in_use"] == 0 and info["largest_free_range"] == 64 << 20
    # a small call still runs in the same region, and a larger region can replace it
    X1, _ = op.sample(Z[:1].contiguous(), tol=1e-6, m_max=20)
    gm.pool_reserve(1 << 30)
    X2, _ = op.sample(Z[:1].contiguous(), tol=1e-6, m_max=20)
    assert torch.equal(X1, X2)
    gm.pool_reserve(0)
    op.close()


def test_served_mix_with_region_matches_and_allocates_nothing(gm):
    """The serving loop over a reserved region: every result equals the one computed alone with the
    ordinary pool, and the pool makes no device allocation while serving."""
    import torch
    from paper_1312_1476_amd import serve
    ops = [gm.Operator.lattice((96, 80), 1, 0.05, 1.0, "free", "f32"),
           gm.Operator.lattice((150, 150), 1, 0.01, 1.0, "free", "f64")]
    R = serve.ServeRequest
    mk = lambda: [R(1, "sample", 0, 4, 7, tol=1e-5, m_max=600), R(2, "sample", 0, 3, 8, tol=1e-5, m_max=600),
                  R(3, "logdet", 1, 8, 9, m_max=60), R(4, "sample", 1, 6, 10, tol=1e-6, m_max=400),
                  R(5, "logdet", 1, 4, 11, m_max=60), R(6, "sample", 0, 1, 12, tol=1e-5, m_max=600)]
    alone = {}
    srv = serve.Server(ops, hbm_budget=64 << 30, workers=1).start()
    for r in mk():
        srv.submit(r)
        r.done.wait()
        assert not r.error, r.error
        alone[r.rid] = r.result
    srv.stop()
    probe = serve.Server(ops, hbm_budget=1 << 40)
    region = sum(probe.request_bytes(r) for r in mk())
    gm.pool_reserve(region)
    a0 = gm.pool_info()["device_allocs"]
    mix = mk()
    srv = serve.Server(ops, hbm_budget=region, workers=4).start()
    for r in mix:
        srv.submit(r)
    for r in mix:
        r.done.wait()
    srv.stop()
    assert gm.pool_info()["device_allocs"] == a0 and gm.pool_info()["in_use"] == 0
    for r in mix:
        assert not r.error, r.error
        if r.kind == "sample":
            assert torch.equal(alone[r.rid]["X"], r.result["X"]), r.rid
        else:
            assert np.array_equal(alone[r.rid]["per_probe"], r.result["per_probe"]), r.rid
    gm.pool_reserve(0)
    for op in ops:
        op.close()

"""gmrf_sample_noalloc: the sampler with every scratch buffer in the library's static device array (for
callers that cannot allocate), through the C ABI, against gmrf_sample on the same inputs.

Each case makes two calls in a row, the second with a smaller input, so that the second call runs on
the array as the first left it.  The bar is the sampler's parity tolerance (relative 2-norm 1e-8 for
FP64 storage, 1e-5 for FP32) with identical Krylov dimensions and statuses.  A call too large for
the array is refused with ENOMEM before any kernel runs, and the next call still works.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import os
    import torch
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1312_1476_amd as gm
    return gm


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _compare(gm, op, Zh, bar, **kw):
    Z = _t(Zh.T)
    Xn, in_ = op.sample_noalloc(Z, **kw)
    Xs, is_ = op.sample(Z, **kw)
    Xn, Xs = Xn.cpu().numpy(), Xs.cpu().numpy()
    assert [(i["m_used"], i["status"]) for i in in_] == [(i["m_used"], i["status"]) for i in is_]
    for r in range(Zh.shape[1]):
        e = np.linalg.norm(Xn[r] - Xs[r]) / np.linalg.norm(Xs[r])
        assert e <= bar, (r, e)
    return in_


@pytest.mark.parametrize("reorth", [True, False])
def test_noalloc_equals_sample_plain(gm, reorth):
    big = gm.Operator.lattice((64, 64), 1, 0.1, 1.0, "free", "f64")
    small = gm.Operator.lattice((40, 48), 1, 0.3, 1.0, "free", "f64")
    info = _compare(gm, big, workloads.gaussian_block(64 * 64, 4, 90, 0), 1e-8, tol=1e-8, m_max=200, reorth=reorth)
    assert all(i["status"] == "OK" for i in info)
    _compare(gm, small, workloads.gaussian_block(40 * 48, 2, 90, 1), 1e-8, tol=1e-8, m_max=150, reorth=reorth)


def test_noalloc_equals_sample_preconditioned(gm):
    # eight columns: gmrf_sample splits them over two streams, the allocation-free call runs one group
    big = gm.Operator.lattice((64, 64), 2, 0.05, 1.0, "free", "f64").set_circulant_precond()
    small = gm.Operator.lattice((32, 32), 2, 0.1, 1.0, "free", "f64").set_circulant_precond()
    _compare(gm, big, workloads.gaussian_block(64 * 64, 8, 90, 2), 1e-8, tol=1e-10, m_max=300)
    _compare(gm, small, workloads.gaussian_block(32 * 32, 4, 90, 3), 1e-8, tol=1e-10, m_max=300)


def test_noalloc_equals_sample_fp32(gm):
    big = gm.Operator.lattice((48, 48), 1, 0.2, 1.0, "free", "f32")
    small = gm.Operator.lattice((20, 24), 1, 0.2, 1.0, "free", "f32")
    _compare(gm, big, workloads.gaussian_block(48 * 48, 3, 90, 4), 1e-5, tol=1e-5, m_max=300)
    _compare(gm, small, workloads.gaussian_block(20 * 24, 1, 90, 5), 1e-5, tol=1e-5, m_max=300)


def test_noalloc_refuses_oversize_then_runs(gm):
    # 512^2 x 32 columns x 301 Krylov slots in FP64 is ~20 GB, far beyond the 128 MiB array
    big = gm.Operator.lattice((512, 512), 2, 0.01, 1.0, "free", "f64")
    Zb = _t(workloads.gaussian_block(512 * 512, 32, 90, 6).T)
    with pytest.raises(gm.GmrfError) as e:
        big.sample_noalloc(Zb, tol=1e-8, m_max=300)
    assert e.value.status == 4 and "static scratch" in str(e.value)
    small = gm.Operator.lattice((16, 16), 1, 0.5, 1.0, "free", "f64")
    _compare(gm, small, workloads.gaussian_block(256, 2, 90, 7), 1e-8, tol=1e-8, m_max=100)

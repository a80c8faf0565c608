"""GPU parity of the two-pass, O(n)-memory sampler (gmrf_sample_two_pass) through the C ABI.

Pass 2 re-runs the recurrence with the same launches, so the two-pass sample equals the one-pass
sample (stored basis, k_combine) up to the order in which the basis is summed, and both equal the
FP64 oracle's Algorithm 1 at the same m: relative 2-norm 1e-8 (FP64) / 1e-5 (FP32).  Iteration
counts and statuses are identical to the one-pass call.  Under an HBM budget too small for the
stored basis the one-pass call fails with ENOMEM and the two-pass call runs.
"""
import numpy as np
import pytest

import workloads
from oracle import lanczos, lattice, lgcp, precond

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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# conditioned so that every column converges within m_max (an unconverged plain recurrence follows
# rounding, which would test the oracle comparison rather than the two passes)
CASES = [((48, 40), 1, 0.1, "free", "f64"), ((33, 64), 2, 0.5, "free", "f64"), ((64, 64), 2, 0.5, "free", "f32"),
         ((10, 12, 14), 1, 0.2, "periodic", "f64"), ((500,), 2, 0.2, "free", "f64")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-o{c[1]}-{c[4]}")
def test_two_pass_lattice(gm, case):
    shape, order, k2, bc, storage = case
    n = int(np.prod(shape))
    op = gm.Operator.lattice(shape, order, k2, 1.0, bc, storage)
    Zh = workloads.gaussian_block(n, 3, 61, 0)
    X1, info1 = op.sample(_t(Zh.T), tol=1e-7, m_max=300)
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-7, m_max=300)
    X1, X2 = X1.cpu().numpy().T, X2.cpu().numpy().T
    Q = lattice.lattice_precision(shape, order, k2, 1.0, bc)
    tol = 1e-8 if storage == "f64" else 1e-5
    for r in range(3):
        assert info1[r]["status"] == "OK"
        assert info2[r]["m_used"] == info1[r]["m_used"] and info2[r]["status"] == info1[r]["status"]
        assert info2[r]["rel_residual"] == info1[r]["rel_residual"]
        assert _rel(X2[:, r], X1[:, r]) <= (1e-12 if storage == "f64" else 1e-5)
        ref = lanczos.sample_csr(Q, Zh[:, r], info2[r]["m_used"], tol=0.0)
        assert _rel(X2[:, r], ref.x) <= tol, _rel(X2[:, r], ref.x)


def test_two_pass_csr(gm):
    Q = lattice.section52_test_matrix()
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data)
    Zh = workloads.gaussian_block(Q.shape[0], 2, 62, 0)
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=0.0, m_max=60)
    X2 = X2.cpu().numpy().T
    for r in range(2):
        ref = lanczos.sample_csr(Q, Zh[:, r], 60, tol=0.0)
        assert _rel(X2[:, r], ref.x) <= 1e-8


def test_two_pass_preconditioned(gm):
    shape, order, k2 = (64, 64), 2, 0.01
    n = shape[0] * shape[1]
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f64").set_circulant_precond()
    Zh = workloads.gaussian_block(n, 8, 63, 0)     # 8 columns: two column groups
    X1, info1 = op.sample(_t(Zh.T), tol=1e-9, m_max=400)
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-9, m_max=400)
    X1, X2 = X1.cpu().numpy().T, X2.cpu().numpy().T
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    for r in (0, 7):
        assert info2[r]["m_used"] == info1[r]["m_used"]
        assert _rel(X2[:, r], X1[:, r]) <= 1e-12
        ref = precond.sample(Q, shape, order, k2, 1.0, Zh[:, r], info2[r]["m_used"], tol=0.0)
        assert _rel(X2[:, r], ref.x) <= 1e-8


def test_two_pass_lgcp(gm):
    N = 128
    spec = workloads.lgcp_prior(N)
    d = workloads.lgcp_diagonal(N)
    op = gm.Operator.lattice(spec.shape, 2, spec.kappa2, spec.tau, "periodic", "f64")
    op.set_diagonal(d)
    op.set_circulant_precond()
    Zh = workloads.gaussian_block(N * N, 2, 64, 0)
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-8, m_max=40)
    X2 = X2.cpu().numpy().T
    for r in range(2):
        ref = lgcp.sample(spec.shape, 2, spec.kappa2, spec.tau, d, Zh[:, r], 40, tol=1e-8)
        assert info2[r]["m_used"] == ref.m
        assert _rel(X2[:, r], ref.x) <= 1e-8


def test_two_pass_edge_columns(gm):
    # a zero column (x = 0, m = 0) and a non-finite column (EINVAL, NaN) beside a regular one
    shape = (16, 16)
    op = gm.Operator.lattice(shape, 1, 0.2, 1.0, "free", "f64")
    Zh = workloads.gaussian_block(256, 3, 65, 0)
    Zh[:, 1] = 0.0
    Zh[3, 2] = np.nan
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-8, m_max=100)
    X2 = X2.cpu().numpy().T
    assert info2[1]["m_used"] == 0 and np.all(X2[:, 1] == 0.0)
    assert info2[2]["status"] == "EINVAL" and np.all(np.isnan(X2[:, 2]))
    Q = lattice.lattice_precision(shape, 1, 0.2, 1.0, "free")
    ref = lanczos.sample_csr(Q, Zh[:, 0], info2[0]["m_used"], tol=0.0)
    assert _rel(X2[:, 0], ref.x) <= 1e-8


def test_two_pass_fits_where_the_basis_does_not(gm):
    shape, k, m_max = (256, 256), 8, 300
    op = gm.Operator.lattice(shape, 1, 0.01, 1.0, "free", "f64")
    Zh = workloads.gaussian_block(shape[0] * shape[1], k, 66, 0)
    need = op.bytes(k, m_max)
    vec = shape[0] * shape[1] * k * 8
    X1, info1 = op.sample(_t(Zh.T), tol=1e-6, m_max=m_max)     # reference, unconstrained
    try:
        gm.set_hbm_budget(gm.hbm_in_use() + 12 * vec)          # room for ~12 vectors, not the m_max + 1 basis
        assert need > 12 * vec
        with pytest.raises(gm.GmrfError):
            op.sample(_t(Zh.T), tol=1e-6, m_max=m_max)
        X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-6, m_max=m_max)
    finally:
        gm.set_hbm_budget(0)
    assert [i["m_used"] for i in info2] == [i["m_used"] for i in info1]
    assert _rel(X2.cpu().numpy(), X1.cpu().numpy()) <= 1e-12

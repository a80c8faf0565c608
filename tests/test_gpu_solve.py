"""GPU parity of gmrf_solve, the Lanczos form of (preconditioned) conjugate gradients on the sampler's
kernels, against the oracle's x_m = ||b|| V_m T_m^{-1} e_1 (FP64 1e-8 at the oracle's m, FP32 1e-5),
against dense solves at convergence, and with rel_residual equal to the true residual
||b - Q x_m|| / ||b|| (Theorem 1's rho_m).  Covers lattices (one-pass 2D, 3D), CSR, circulant
preconditioning, the LGCP proposal mean (Q + H)^{-1} grad and incomplete Cholesky.
"""
import numpy as np
import pytest

import workloads
from oracle import ichol, lanczos, lattice, lgcp, precond

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


@pytest.mark.parametrize("case", [((40, 36), 1, 0.1, "free", "f64"), ((30, 34), 2, 0.5, "free", "f64"),
                                  ((8, 10, 12), 1, 0.2, "periodic", "f64"), ((48, 48), 2, 0.5, "free", "f32")],
                         ids=lambda c: f"{c[0]}-o{c[1]}-{c[4]}")
def test_solve_lattice(gm, case):
    shape, order, k2, bc, storage = case
    n = int(np.prod(shape))
    op = gm.Operator.lattice(shape, order, k2, 1.0, bc, storage)
    Q = lattice.lattice_precision(shape, order, k2, 1.0, bc)
    Bh = workloads.gaussian_block(n, 3, 81, 0)
    X, info = op.solve(_t(Bh.T), tol=1e-9, m_max=400)
    X = X.cpu().numpy().T
    tol = 1e-8 if storage == "f64" else 1e-5
    for r in range(3):
        assert info[r]["status"] == "OK"
        ref = lanczos.solve(lambda v: Q @ v, Bh[:, r], info[r]["m_used"], tol=0.0)
        assert _rel(X[:, r], ref.x) <= tol, _rel(X[:, r], ref.x)
        res = np.linalg.norm(Bh[:, r] - Q @ X[:, r]) / np.linalg.norm(Bh[:, r])
        if storage == "f64":
            assert res == pytest.approx(info[r]["rel_residual"], rel=1e-3, abs=1e-12)
        exact = np.linalg.solve(Q.toarray(), Bh[:, r])
        assert _rel(X[:, r], exact) <= (1e-7 if storage == "f64" else 1e-4)


def test_solve_csr(gm):
    Q = lattice.lattice_precision((20, 22), 2, 0.3, 1.0, "free")
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data)
    Bh = workloads.gaussian_block(440, 2, 82, 0)
    X, info = op.solve(_t(Bh.T), tol=0.0, m_max=50)
    X = X.cpu().numpy().T
    for r in range(2):
        ref = lanczos.solve(lambda v: Q @ v, Bh[:, r], 50, tol=0.0)
        assert _rel(X[:, r], ref.x) <= 1e-8


def test_solve_circulant_preconditioned(gm):
    shape, order, k2 = (64, 64), 2, 0.01
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f64").set_circulant_precond()
    Bh = workloads.gaussian_block(4096, 8, 83, 0)
    X, info = op.solve(_t(Bh.T), tol=1e-10, m_max=600, reorth=True)
    X = X.cpu().numpy().T
    for r in (0, 7):
        assert info[r]["status"] == "OK"
        ref = precond.solve(Q, shape, order, k2, 1.0, Bh[:, r], info[r]["m_used"], tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= 1e-8
        exact = np.linalg.solve(Q.toarray(), Bh[:, r])
        assert _rel(X[:, r], exact) <= 1e-6


def test_lgcp_proposal_mean(gm):
    N = 128
    spec = workloads.lgcp_prior(N)
    d = workloads.lgcp_diagonal(N)
    op = gm.Operator.lattice(spec.shape, 2, spec.kappa2, spec.tau, "periodic", "f64")
    op.set_diagonal(d)
    op.set_circulant_precond()
    Gh = workloads.gaussian_block(N * N, 2, 84, 0)
    X, info = op.solve(_t(Gh.T), tol=1e-10, m_max=40)
    X = X.cpu().numpy().T
    for r in range(2):
        ref = lgcp.proposal_mean_solve(spec.shape, 2, spec.kappa2, spec.tau, d, Gh[:, r], 40, tol=1e-10)
        assert info[r]["m_used"] == ref.m <= 10
        assert _rel(X[:, r], ref.x) <= 1e-8


def test_solve_ichol(gm):
    Q = lattice.section52_test_matrix()
    op = gm.Operator.csr(900, Q.indptr, Q.indices, Q.data)
    op.set_ichol_precond(1e-3)
    L, _ = ichol.ichol(Q, 1e-3)
    Bh = workloads.gaussian_block(900, 2, 85, 0)
    X, info = op.solve(_t(Bh.T), tol=1e-10, m_max=200, reorth=True)
    X = X.cpu().numpy().T
    for r in range(2):
        ref = ichol.solve(Q, L, Bh[:, r], 200, tol=1e-10, reorth=True)
        assert info[r]["m_used"] == ref.m
        assert _rel(X[:, r], ref.x) <= 1e-8

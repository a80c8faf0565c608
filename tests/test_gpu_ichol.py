"""GPU parity of incomplete-Cholesky preconditioning (Section 5.2, Figure 3) through the C ABI.

The library factorises on the host and solves with L and L^T on the GPU (level-scheduled); the oracle
factorises densely with the same rule.  Checked: the shift the factorisation needed and the number of
nonzeros of L (integers, exact), the iteration count at the tolerance and the sample (FP64 1e-8,
FP32 1e-5) with CGS2, the sample at forced m without it, log det per probe, the complete factor
(one step, exact sample), two-pass sampling, Figure 3's iteration counts.
"""
import numpy as np
import pytest

import workloads
from oracle import ichol, lattice

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


def _op(gm, Q, droptol, storage="f64"):
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data, storage)
    shift = op.set_ichol_precond(droptol)
    return op, shift


SEC52 = lattice.section52_test_matrix()


@pytest.mark.parametrize("droptol", [-1.0, 1e-2, 1e-3, 1e-4])
def test_factor_matches_oracle(gm, droptol):
    op, shift = _op(gm, SEC52, droptol)
    L, oshift = ichol.ichol(SEC52, droptol)
    nnz, levels, sh = op.ichol_info()
    assert shift == oshift == sh
    assert nnz == np.count_nonzero(np.tril(L))
    assert levels >= 1


@pytest.mark.parametrize("droptol", [-1.0, 1e-3, 1e-4])
def test_sample_converged_reorth(gm, droptol):
    op, _ = _op(gm, SEC52, droptol)
    L, _ = ichol.ichol(SEC52, droptol)
    Zh = workloads.gaussian_block(900, 3, 71, 0)
    X, info = op.sample(_t(Zh.T), tol=1e-8, m_max=400, reorth=True)
    X = X.cpu().numpy().T
    for r in range(3):
        ref = ichol.sample(SEC52, L, Zh[:, r], 400, tol=1e-8, reorth=True)
        assert info[r]["status"] == "OK" and info[r]["m_used"] == ref.m
        assert _rel(X[:, r], ref.x) <= 1e-8, _rel(X[:, r], ref.x)


@pytest.mark.parametrize("m", [1, 3, 8, 20])
def test_sample_prefix_plain(gm, m):
    op, _ = _op(gm, SEC52, 1e-3)
    L, _ = ichol.ichol(SEC52, 1e-3)
    Zh = workloads.gaussian_block(900, 2, 72, 0)
    X, info = op.sample(_t(Zh.T), tol=0.0, m_max=m)
    X = X.cpu().numpy().T
    for r in range(2):
        ref = ichol.sample(SEC52, L, Zh[:, r], m, tol=0.0)
        assert info[r]["m_used"] == m
        assert _rel(X[:, r], ref.x) <= 1e-8


def test_sample_fp32(gm):
    # FP32 storage rounds the factor itself: the solves amplify that by cond(L) = cond(Q)^{1/2}, about
    # 390 on Section 5.2's matrix (2.5e-5 measured there), so the FP32 bar is taken on a lattice with
    # cond(Q) ~ 160
    Q = lattice.lattice_precision((24, 20), 1, 0.05, 1.0, "free")
    op, _ = _op(gm, Q, 1e-3, "f32")
    L, _ = ichol.ichol(Q, 1e-3)
    Zh = workloads.gaussian_block(480, 2, 73, 0)
    X, info = op.sample(_t(Zh.T), tol=1e-6, m_max=100, reorth=True)
    X = X.cpu().numpy().T
    for r in range(2):
        ref = ichol.sample(Q, L, Zh[:, r], info[r]["m_used"], tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= 1e-5, _rel(X[:, r], ref.x)


def test_complete_factor_is_one_step(gm):
    Q = lattice.lattice_precision((12, 10), 2, 0.2, 1.0, "free")
    op, shift = _op(gm, Q, 0.0)
    assert shift == 0.0
    Zh = workloads.gaussian_block(120, 2, 74, 0)
    X, info = op.sample(_t(Zh.T), tol=1e-10, m_max=20)
    X = X.cpu().numpy().T
    Lc = np.linalg.cholesky(Q.toarray())
    for r in range(2):
        assert info[r]["m_used"] == 1
        x = np.linalg.solve(Lc.T, Zh[:, r])
        assert _rel(X[:, r], x) <= 1e-12


def test_lattice_as_csr_ic0(gm):
    Q = lattice.lattice_precision((24, 20), 1, 0.05, 1.0, "free")
    op, _ = _op(gm, Q, -1.0)
    L, _ = ichol.ichol(Q, -1.0)
    Zh = workloads.gaussian_block(480, 4, 75, 0)
    X, info = op.sample(_t(Zh.T), tol=1e-9, m_max=300, reorth=True)
    X = X.cpu().numpy().T
    for r in range(4):
        ref = ichol.sample(Q, L, Zh[:, r], 300, tol=1e-9, reorth=True)
        assert info[r]["m_used"] == ref.m
        assert _rel(X[:, r], ref.x) <= 1e-8


@pytest.mark.parametrize("n,w", [(7000, 1), (7000, 20), (7000, 40), (9000, 6)])
def test_banded_exact_factor_large(gm, n, w):
    """Solves too large for the LDS-staged kernels: n = 7000 keeps x in LDS with the factor's tables in
    global memory, n = 9000 keeps x there too.  Half-bandwidths 1 / 6 / 20 / 40 give rows for one
    thread, 4, 8 and 16 lanes.  IC(0) of a banded matrix with a full band is its Cholesky factor, so the
    preconditioned sample is one step and equals L^{-T} z; the reference takes L from LAPACK's banded
    Cholesky and solves with scipy's sparse triangular solve."""
    import scipy.linalg as sl
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    rng = np.random.default_rng(500 + w)
    offs = [rng.uniform(-1.0, 1.0, n - k) for k in range(1, w + 1)]
    diag = np.ones(n)
    for k, o in enumerate(offs, start=1):
        diag[k:] += np.abs(o)
        diag[:-k] += np.abs(o)
    Q = sp.diags([diag] + offs + offs, [0] + list(range(1, w + 1)) + [-k for k in range(1, w + 1)],
                 format="csr")
    Q.sort_indices()
    op, shift = _op(gm, Q, -1.0)
    assert shift == 0.0
    ab = np.zeros((w + 1, n))
    ab[0] = diag
    for k, o in enumerate(offs, start=1):
        ab[k, :n - k] = o
    lb = sl.cholesky_banded(ab, lower=True)
    L = sp.diags([lb[k, :n - k] for k in range(w + 1)], [-k for k in range(w + 1)], format="csr")
    z = rng.standard_normal((2, n))
    X, info = op.sample(_t(z), tol=1e-9, m_max=20, reorth=True)
    X = X.cpu().numpy()
    for r in range(2):
        assert info[r]["status"] == "OK" and info[r]["m_used"] == 1
        x = spl.spsolve_triangular(L.T.tocsr(), z[r], lower=False)
        assert _rel(X[r], x) <= 1e-10
    op.close()


@pytest.mark.parametrize("n,bs", [(2000, 2), (2400, 12)])
def test_block_diagonal_exact_factor_wide_levels(gm, n, bs):
    """Levels wider than one wave's two passes, in a solve that fits LDS: the block form of the LDS
    kernel.  Q is block diagonal with dense SPD blocks of size bs, so IC(0) is its Cholesky factor and
    every level holds one row of each block (n / bs rows).  bs = 2: the entries in LDS, one thread per
    row; bs = 12: the entries in global memory (they do not fit beside the tables), 4 lanes per row.
    One step samples x = L^{-T} z; the reference factors each block with numpy's Cholesky."""
    import scipy.sparse as sp
    import scipy.linalg as sl
    rng = np.random.default_rng(600 + bs)
    blocks = []
    for _ in range(n // bs):
        M = rng.standard_normal((bs, bs))
        blocks.append(M @ M.T + bs * np.eye(bs))
    Q = sp.block_diag(blocks, format="csr")
    Q.sort_indices()
    op, shift = _op(gm, Q, -1.0)
    assert shift == 0.0
    L = sl.block_diag(*[np.linalg.cholesky(B) for B in blocks])
    z = rng.standard_normal((2, n))
    X, info = op.sample(_t(z), tol=1e-9, m_max=20, reorth=True)
    X = X.cpu().numpy()
    for r in range(2):
        assert info[r]["status"] == "OK" and info[r]["m_used"] == 1
        x = sl.solve_triangular(L, z[r], lower=True, trans="T")
        assert _rel(X[r], x) <= 1e-10
    op.close()


def test_logdet(gm):
    op, _ = _op(gm, SEC52, 1e-4)
    L, _ = ichol.ichol(SEC52, 1e-4)
    mean, se, per = op.logdet(6, 30, seed=11)
    ref = ichol.hutchinson(SEC52, L, 6, 30, seed=11)
    assert np.all(np.abs(per - ref.per_probe) <= 1e-10 * np.abs(ref.per_probe))
    from oracle import dense
    exact = dense.cholesky_logdet(SEC52)
    assert abs(mean - exact) < 5 * se + 1e-8 * abs(exact)


def test_two_pass(gm):
    op, _ = _op(gm, SEC52, 1e-3)
    Zh = workloads.gaussian_block(900, 3, 76, 0)
    X1, info1 = op.sample(_t(Zh.T), tol=1e-8, m_max=200)
    X2, info2 = op.sample_two_pass(_t(Zh.T), tol=1e-8, m_max=200)
    assert [i["m_used"] for i in info1] == [i["m_used"] for i in info2]
    assert _rel(X2.cpu().numpy(), X1.cpu().numpy()) <= 1e-12


def test_figure3_counts(gm):
    z = np.random.default_rng(7).standard_normal(900)
    for droptol in (-1.0, 1e-2, 1e-3, 1e-4, 1e-5):
        op, _ = _op(gm, SEC52, droptol)
        X, info = op.sample(_t(z[None, :]), tol=1e-8, m_max=900, reorth=True)
        ref = ichol.sample(SEC52, ichol.ichol(SEC52, droptol)[0], z, 900, tol=1e-8, reorth=True)
        assert info[0]["m_used"] == ref.m
        op.close()


def test_unsupported(gm):
    op = gm.Operator.lattice((8, 8), 1, 0.2, 1.0, "free")
    with pytest.raises(gm.GmrfError):
        op.set_ichol_precond(-1.0)

"""GPU parity of the unpreconditioned path, through the C ABI, against the FP64 oracle.

Tolerances: relative 2-norm error <= 1e-8 for FP64 storage and <= 1e-5 for FP32 storage (the
targets of the sampler's parity definition), forced identical Krylov dimension (the oracle
runs m_fixed = m_gpu); bit-exact for the integer probe generator.  Sizes span several tiles
and ragged tails (sides not multiples of the 64 x 16 / 32 x 8 x 4 tiles).
"""
import numpy as np
import pytest

import workloads
from oracle import closed_form, lanczos, lattice, logdet, philox

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


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# 3D first-order lattices of 2^20 points and more march along z: several row segments with a ragged last
# one and ragged runs of planes (37, 181, 157), rows of the maximum 512 points (5, 410, 512), a single
# segment per plane (4100, 16, 16); rows of 513 points take the box tiles (3, 700, 513)
LATTICES = [((300,), 1), ((300,), 2), ((64, 64), 1), ((45, 70), 2), ((17, 130), 1), ((130, 17), 2),
            ((9, 10, 11), 1), ((16, 16, 16), 1), ((7, 9, 20), 2), ((1, 1), 1), ((2, 2), 2),
            ((37, 181, 157), 1), ((5, 410, 512), 1), ((4100, 16, 16), 1), ((3, 700, 513), 1)]


@pytest.mark.parametrize("shape,order", LATTICES)
@pytest.mark.parametrize("boundary", ["free", "periodic"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_apply_lattice(gm, shape, order, boundary, storage):
    import torch
    k2, tau = 0.07, 1.3
    op = gm.Operator.lattice(shape, order, k2, tau, boundary, storage)
    Q = lattice.lattice_precision(shape, order, k2, tau, boundary)
    n = Q.shape[0]
    X = np.random.default_rng(1).standard_normal((3, n))
    dt = torch.float64 if storage == "f64" else torch.float32
    Xs = X.astype(np.float64 if storage == "f64" else np.float32).astype(np.float64)
    Y = op.apply(_t(X, dt)).double().cpu().numpy()
    ref = (Q @ Xs.T).T
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= (1e-14 if storage == "f64" else 1e-5), err


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_apply_csr(gm, storage):
    import torch
    Q = lattice.section52_test_matrix()
    Q = Q / Q.diagonal().max()
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data, storage)
    X = np.random.default_rng(2).standard_normal((2, Q.shape[0]))
    dt = torch.float64 if storage == "f64" else torch.float32
    Y = op.apply(_t(X, dt)).double().cpu().numpy()
    ref = (Q @ X.T).T
    assert np.abs(Y - ref).max() / np.abs(ref).max() <= (1e-14 if storage == "f64" else 1e-5)


def test_csr_column_blocks_bitwise(gm):
    """The CSR kernel takes 8, 4 or 1 right-hand sides per block by grid size (a 192 x 192 lattice's
    36864 rows: 8 at 32 columns, 4 at 16, 1 at one).  A column's bits do not depend on it, in the
    operator and in the Lanczos step, and the 32-column samples match the oracle."""
    import scipy.sparse as sps
    Q = sps.csr_matrix(lattice.lattice_precision((192, 192), 1, 0.05, 1.0, "free"))
    Q.sort_indices()
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data, "f64")
    Zh = workloads.gaussian_block(Q.shape[0], 32, 95, 0)
    Y32 = op.apply(_t(Zh.T)).cpu().numpy()
    Y16 = op.apply(_t(Zh[:, :16].T)).cpu().numpy()
    Y1 = op.apply(_t(Zh[:, 7:8].T)).cpu().numpy()
    assert np.array_equal(Y16, Y32[:16]) and np.array_equal(Y1[0], Y32[7])
    assert np.abs(Y32 - (Q @ Zh).T).max() <= 1e-13 * np.abs(Y32).max()
    X32, i32, _, _ = _gpu_sample(gm, op, Zh, tol=1e-8, m_max=300)
    X16, _, _, _ = _gpu_sample(gm, op, Zh[:, :16], tol=1e-8, m_max=300)
    assert np.array_equal(X16, X32[:, :16])
    for r in (0, 31):
        X1, i1, _, _ = _gpu_sample(gm, op, Zh[:, r:r + 1], tol=1e-8, m_max=300)
        assert i1[0]["m_used"] == i32[r]["m_used"] and np.array_equal(X1[:, 0], X32[:, r])
        ref = lanczos.sample_csr(Q, Zh[:, r], i32[r]["m_used"], tol=0.0)
        assert i32[r]["status"] == "OK" and _rel(X32[:, r], ref.x) <= 1e-8, (r, _rel(X32[:, r], ref.x))


@pytest.mark.parametrize("n,nprobes,seed", [(1, 1, 0), (255, 2, 7), (1000, 3, 14761315), (70001, 2, 2 ** 63 + 5)])
def test_rademacher_bit_exact(gm, n, nprobes, seed):
    P = gm.rademacher(seed, n, nprobes).cpu().numpy().astype(np.float64)
    ref = philox.rademacher_probes(seed, nprobes, n).T
    assert np.array_equal(P, ref)


def _rand_tridiag(rng, m, cond):
    # SPD tridiagonal with a prescribed spread: T = D^{1/2} B D^{1/2}, B diagonally dominant
    a = rng.uniform(2.0, 3.0, m)
    b = rng.uniform(-0.9, 0.9, m)
    s = np.exp(np.linspace(0.0, np.log(cond) / 2, m))
    rng.shuffle(s)
    alpha = a * s * s
    beta = b * s * np.roll(s, -1)
    beta[-1] = 0.0
    return alpha, beta


@pytest.mark.parametrize("m", [1, 2, 7, 80, 300, 700, 1024, 1025, 3000])
@pytest.mark.parametrize("cond", [1.0, 1e3, 1e6])
def test_tridiag_vs_eigh(gm, m, cond):
    import torch
    rng = np.random.default_rng(m * 7 + int(np.log10(cond)))
    k, ld = 3, max(m, 1)
    A = np.zeros((k, ld))
    B = np.zeros((k, ld))
    for r in range(k):
        A[r, :m], B[r, :m] = _rand_tridiag(rng, m, cond)
    mm = torch.full((k,), m, dtype=torch.int32, device="cuda:0")
    y, st = gm.tridiag_invsqrt_e1(_t(A), _t(B), mm)
    lg, st2 = gm.tridiag_log_e1(_t(A), _t(B), mm)
    y, lg = y.cpu().numpy(), lg.cpu().numpy()
    assert (st.cpu().numpy() == 0).all() and (st2.cpu().numpy() == 0).all()
    for r in range(k):
        T = np.diag(A[r, :m]) + np.diag(B[r, :m - 1], 1) + np.diag(B[r, :m - 1], -1)
        kap = np.linalg.cond(T)
        ref = lanczos.tridiag_inv_sqrt_e1(A[r, :m], B[r, :m])
        assert _rel(y[r, :m], ref) <= max(1e-13, 20 * kap * 2.2e-16), (_rel(y[r, :m], ref), kap)
        lref = lanczos.tridiag_log_e1(A[r, :m], B[r, :m])
        assert abs(lg[r] - lref) <= 1e-13 * max(1.0, abs(lref)) + 20 * kap * 2.2e-16


def test_tridiag_lds_and_global_forms_agree_bitwise(gm):
    """Up to 1024 steps T is staged in LDS; a caller whose rows hold more steps gets the form that reads
    T from global memory.  Same arithmetic in the same order: the same T gives the same bits in both."""
    import torch
    rng = np.random.default_rng(77)
    k = 4
    ms = [1, 64, 700, 1024]
    A = np.zeros((k, 1024))
    B = np.zeros((k, 1024))
    for r, m in enumerate(ms):
        A[r, :m], B[r, :m] = _rand_tridiag(rng, m, 1e4)
    mm = torch.tensor(ms, dtype=torch.int32, device="cuda:0")
    y1, _ = gm.tridiag_invsqrt_e1(_t(A), _t(B), mm)
    l1, _ = gm.tridiag_log_e1(_t(A), _t(B), mm)
    A2, B2 = np.zeros((k, 2000)), np.zeros((k, 2000))
    A2[:, :1024], B2[:, :1024] = A, B
    y2, _ = gm.tridiag_invsqrt_e1(_t(A2), _t(B2), mm)
    l2, _ = gm.tridiag_log_e1(_t(A2), _t(B2), mm)
    y1, y2 = y1.cpu().numpy(), y2.cpu().numpy()
    for r, m in enumerate(ms):
        assert np.array_equal(y1[r, :m], y2[r, :m]), m
    assert torch.equal(l1, l2)


@pytest.mark.parametrize("scale", [1e-8, 1e-4, 1e4, 1e10])
def test_tridiag_log_scaled_spectrum(gm, scale):
    """e_1^T log(T) e_1 for T scaled far from 1 (tau-scaled operators): the quadrature window must cover
    both the spectrum and s = 0, where the log integrand's tails begin."""
    import torch
    rng = np.random.default_rng(int(np.log10(scale)) + 50)
    m, k = 60, 2
    A = np.zeros((k, m))
    B = np.zeros((k, m))
    for r in range(k):
        a, b = _rand_tridiag(rng, m, 1e3)
        A[r], B[r] = scale * a, scale * b
    mm = torch.full((k,), m, dtype=torch.int32, device="cuda:0")
    lg, st = gm.tridiag_log_e1(_t(A), _t(B), mm)
    lg = lg.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    for r in range(k):
        lref = lanczos.tridiag_log_e1(A[r], B[r])
        assert abs(lg[r] - lref) <= 1e-12 * max(1.0, abs(lref)), (scale, lg[r], lref)


def test_tridiag_flags_indefinite(gm):
    import torch
    A = np.array([[1.0, -2.0, 1.0, 0.0]])
    B = np.array([[0.1, 0.1, 0.0, 0.0]])
    mm = torch.tensor([3], dtype=torch.int32, device="cuda:0")
    _, st = gm.tridiag_invsqrt_e1(_t(A), _t(B), mm)
    assert st.cpu().numpy()[0] == 2


def _gpu_sample(gm, op, Zh, **kw):
    Z = _t(Zh.T)
    X, info, al, be = op.sample(Z, coeffs=True, **kw)
    return X.cpu().numpy().T, info, al, be


def test_sample_plain_fp64_workload(gm):
    """The plain FP64 workload: 64 x 64, first order, kappa2 = 0.1, full reorth, tol 1e-8."""
    c = workloads.C0
    sp = c.lattice
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f64")
    Zh = workloads.gaussian_block(sp.n, c.k, 0, 0)
    X, info, al, be = _gpu_sample(gm, op, Zh, tol=c.tol, m_max=c.m_max, reorth=c.reorth)
    m = info[0]["m_used"]
    assert info[0]["status"] == "OK" and info[0]["rel_residual"] <= c.tol and 20 < m < c.m_max
    Q = lattice.lattice_precision(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    ref = lanczos.sample_csr(Q, Zh[:, 0], m, tol=0.0, reorth=True)
    assert _rel(X[:, 0], ref.x) <= 1e-8
    assert np.allclose(al[0, :m], ref.alpha[:m], rtol=1e-10, atol=0)
    assert np.allclose(be[0, 1:m + 1], ref.beta[:m], rtol=1e-9, atol=0)
    # the oracle stops at the same m when given the same tolerance
    ref_tol = lanczos.sample_csr(Q, Zh[:, 0], c.m_max, tol=c.tol, reorth=True)
    assert ref_tol.m == m
    exact = closed_form.exact_sample_free(sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, 0])
    lmin, lmax = closed_form.exact_lambda_min_max(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    assert _rel(X[:, 0], exact) <= np.sqrt(lmax / lmin) * info[0]["rel_residual"]


CASES = [
    ("lat", (45, 70), 2, 0.3, "free", 3, 40),
    ("lat", (10, 12, 9), 1, 0.2, "free", 2, 50),
    ("lat", (33, 40), 1, 0.05, "periodic", 2, 60),
    ("lat", (500,), 2, 0.5, "free", 2, 30),
    ("lat", (7, 9, 20), 2, 0.4, "periodic", 1, 30),
    ("lat", (37, 181, 157), 1, 0.2, "free", 2, 40),
    ("lat", (4100, 16, 16), 1, 0.3, "periodic", 2, 30),
    ("csr", None, None, None, None, 2, 60),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}-{c[4]}")
@pytest.mark.parametrize("reorth", [False, True])
def test_sample_fixed_m_fp64(gm, case, reorth):
    kind, shape, order, k2, bc, k, m = case
    if kind == "lat":
        op = gm.Operator.lattice(shape, order, k2, 1.0, bc, "f64")
        Q = lattice.lattice_precision(shape, order, k2, 1.0, bc)
    else:
        Q = lattice.section52_test_matrix()
        Q = Q / Q.diagonal().max()
        op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data, "f64")
    Zh = workloads.gaussian_block(Q.shape[0], k, 90, 1)
    X, info, al, be = _gpu_sample(gm, op, Zh, tol=0.0, m_max=m, reorth=reorth)
    for r in range(k):
        mr = info[r]["m_used"]
        ref = lanczos.sample_csr(Q, Zh[:, r], mr, tol=0.0, reorth=reorth)
        assert ref.m == mr
        assert _rel(X[:, r], ref.x) <= 1e-8, (r, _rel(X[:, r], ref.x))


@pytest.mark.parametrize("reorth", [False, True])
def test_sample_fp32_storage(gm, reorth):
    shape, k2 = (60, 75), 0.5
    op = gm.Operator.lattice(shape, 1, k2, 1.0, "free", "f32")
    Q = lattice.lattice_precision(shape, 1, k2, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], 4, 91, 0)
    X, info, _, _ = _gpu_sample(gm, op, Zh, tol=1e-6, m_max=100, reorth=reorth)
    for r in range(4):
        ref = lanczos.sample_csr(Q, Zh[:, r], info[r]["m_used"], tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= 1e-5


@pytest.mark.parametrize("shape,k,m,storage", [((300, 300), 2, 30, "f64"), ((300, 300), 2, 20, "f32"),
                                               ((128, 128), 2, 25, "f64"), ((16385,), 1, 20, "f64"),
                                               ((64, 64), 24, 40, "f64"), ((33, 31), 3, 45, "f32")],
                         ids=["long-f64", "long-f32", "at-limit", "limit+1", "many-columns", "odd-f32"])
def test_reorth_tilings(gm, shape, k, m, storage):
    """Both reorthogonalisation tilings (vectors of up to 16384 elements in 64- or 128-element chunks per
    block, and longer), the slices of basis vectors the general dot kernel takes on small grids, and the
    FP32 combine with and without float4 loads, at a forced m against the oracle with CGS2."""
    op = gm.Operator.lattice(shape, 1, 0.05, 1.0, "free", storage)
    Q = lattice.lattice_precision(shape, 1, 0.05, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], k, 97, 0)
    X, info, _, _ = _gpu_sample(gm, op, Zh, tol=0.0, m_max=m, reorth=True)
    tol = 1e-8 if storage == "f64" else 1e-5
    for r in range(k):
        assert info[r]["m_used"] == m
        ref = lanczos.sample_csr(Q, Zh[:, r], m, tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= tol, (r, _rel(X[:, r], ref.x))


def test_reorth_many_sweeps(gm):
    """CGS2 past 128 basis vectors, which the short-vector kernels take in sweeps of 128: a 1D lattice of
    800 points with kappa^2 = 0.002 needs about 510 steps to rho <= 1e-10 (four sweeps, the last one
    partial); parity with the oracle at the GPU's m."""
    op = gm.Operator.lattice((800,), 1, 0.002, 1.0, "free", "f64")
    Q = lattice.lattice_precision((800,), 1, 0.002, 1.0, "free")
    Zh = workloads.gaussian_block(800, 2, 96, 0)
    X, info, _, _ = _gpu_sample(gm, op, Zh, tol=1e-10, m_max=700, reorth=True)
    for r in range(2):
        assert info[r]["status"] == "OK" and info[r]["m_used"] > 3 * 128, info[r]
        ref = lanczos.sample_csr(Q, Zh[:, r], info[r]["m_used"], tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= 1e-8, (r, _rel(X[:, r], ref.x))


def test_edge_cases(gm):
    shape = (20, 20)
    op = gm.Operator.lattice(shape, 1, 0.3, 1.0, "free", "f64")
    Zh = workloads.gaussian_block(400, 3, 92, 0)
    Zh[:, 1] = 0.0
    Zh[5, 2] = np.nan
    X, info, _, _ = _gpu_sample(gm, op, Zh, tol=1e-8, m_max=50, reorth=False)
    assert info[0]["status"] == "OK"
    assert info[1]["status"] == "OK" and info[1]["m_used"] == 0 and np.all(X[:, 1] == 0.0)
    assert info[2]["status"] == "EINVAL" and np.all(np.isnan(X[:, 2]))
    # scalar lattice: Q = tau kappa2, breakdown after one step, x = z / sqrt(tau kappa2)
    op1 = gm.Operator.lattice((1,), 1, 0.3, 2.0, "free", "f64")
    X1, info1, _, _ = _gpu_sample(gm, op1, np.array([[1.7, -0.4]]), tol=1e-8, m_max=5)
    assert [i["m_used"] for i in info1] == [1, 1]
    assert np.allclose(X1[0], np.array([1.7, -0.4]) / np.sqrt(0.6), rtol=1e-15)
    # not positive definite
    opn = gm.Operator.lattice((12, 12), 1, -0.5, 1.0, "free", "f64")
    Xn, infon, _, _ = _gpu_sample(gm, opn, workloads.gaussian_block(144, 1, 92, 1), tol=1e-12, m_max=144,
                                  reorth=True)
    assert infon[0]["status"] == "ENOTSPD" and np.all(np.isnan(Xn))
    # no convergence by m_max: x_{m_max} is still returned
    opc = gm.Operator.lattice((40, 40), 1, 0.001, 1.0, "free", "f64")
    Zc = workloads.gaussian_block(1600, 1, 92, 2)
    Xc, infoc, _, _ = _gpu_sample(gm, opc, Zc, tol=1e-10, m_max=7)
    assert infoc[0]["status"] == "ENOCONV" and infoc[0]["m_used"] == 7
    Q = lattice.lattice_precision((40, 40), 1, 0.001, 1.0, "free")
    assert _rel(Xc[:, 0], lanczos.sample_csr(Q, Zc[:, 0], 7).x) <= 1e-8


def test_deterministic(gm):
    op = gm.Operator.lattice((70, 90), 2, 0.02, 1.0, "free", "f64")
    Zh = workloads.gaussian_block(6300, 3, 93, 0)
    X1, i1, _, _ = _gpu_sample(gm, op, Zh, tol=1e-8, m_max=120, reorth=False)
    X2, i2, _, _ = _gpu_sample(gm, op, Zh, tol=1e-8, m_max=120, reorth=False)
    assert np.array_equal(X1, X2) and i1 == i2


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_logdet_per_probe(gm, storage, tol):
    shape, k2, npb, m, seed = (32, 32), 0.05, 8, 40, 12345
    op = gm.Operator.lattice(shape, 2, k2, 1.0, "free", storage)
    Q = lattice.lattice_precision(shape, 2, k2, 1.0, "free")
    mean, se, per = op.logdet(npb, m, seed=seed)
    ref = logdet.hutchinson_csr(Q, npb, m, seed=seed)
    assert np.all(np.abs(per - ref.per_probe) <= tol * np.abs(ref.per_probe))
    assert abs(mean - ref.logdet) <= tol * abs(ref.logdet)
    assert se == pytest.approx(ref.std_err, rel=1e-6 if storage == "f64" else 1e-2)
    # explicit probes give the same numbers as the seed rule
    P = gm.rademacher(seed, Q.shape[0], npb)
    mean2, _, per2 = op.logdet(npb, m, probes=P)
    assert np.array_equal(per, per2) and mean == mean2

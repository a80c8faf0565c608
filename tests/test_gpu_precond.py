"""GPU parity of the block-circulant preconditioned path (Proposition 1, Section 5.1) and of
the preconditioned log-det split (Section 6.2), through the C ABI, against the FP64 oracle.

The GPU runs Algorithm 1 on F A F^H in the packed spectral basis (two FFTs per step); the
oracle runs it on A = M^{-1/2} Q M^{-1/2} in real space (four FFTs per step).  Both give the
same Lanczos coefficients and the same x in exact arithmetic.

Conditioning.  A = I + (boundary terms) has a large eigenvalue cluster at 1, and its Krylov
space is ill-conditioned with respect to rounding until the iteration has converged: a
relative perturbation of 1e-16 of the oracle's own operator moves x_40 by 4e-6 on a 32 x 32
lattice (rho_40 = 1e-2) and x_150 by 8e-5 on 128 x 128, while converged results
(rho <= 1e-6) move by 1e-14.  Tight parity (1e-8 FP64, 1e-5 FP32, forced identical m) is
therefore asserted at convergence and on the first steps, where the process is well
conditioned; an unconverged full-size run is compared at the truncation level 10 rho_m.
"""
import numpy as np
import pytest

import workloads
from oracle import closed_form, lanczos, lattice, logdet, precond

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


@pytest.mark.parametrize("shape", [(8, 8), (16, 32), (64, 8), (8, 128), (256, 64), (512, 512), (32, 4096)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_precond_apply(gm, shape, order, storage):
    import torch
    k2, tau = 0.03, 1.7
    op = gm.Operator.lattice(shape, order, k2, tau, "free", storage).set_circulant_precond()
    n = shape[0] * shape[1]
    X = np.random.default_rng(3).standard_normal((2, n))
    dt = torch.float64 if storage == "f64" else torch.float32
    Y = op.precond_apply(_t(X, dt)).double().cpu().numpy()
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, tau)
    for r in range(2):
        ref = precond.apply_inv_sqrt_M(shape, mult, X[r])
        assert _rel(Y[r], ref) <= (1e-13 if storage == "f64" else 1e-5), _rel(Y[r], ref)


def test_precond_unsupported(gm):
    with pytest.raises(gm.GmrfError):
        gm.Operator.lattice((12, 16), 1, 0.1).set_circulant_precond()
    with pytest.raises(gm.GmrfError):
        gm.Operator.lattice((8, 8, 8), 1, 0.1).set_circulant_precond()


def _sample(gm, op, Zh, **kw):
    X, info, al, be = op.sample(_t(Zh.T), coeffs=True, **kw)
    return X.cpu().numpy().T, info, al, be


CASES = [((32, 32), 2, 0.01, 3), ((64, 128), 2, 0.05, 2), ((16, 64), 1, 0.02, 2), ((128, 16), 1, 0.2, 1)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-o{c[1]}")
@pytest.mark.parametrize("reorth", [False, True])
def test_precond_sample_converged_fp64(gm, case, reorth):
    shape, order, k2, k = case
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f64").set_circulant_precond()
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], k, 95, 0)
    X, info, al, be = _sample(gm, op, Zh, tol=1e-10, m_max=400, reorth=reorth)
    for r in range(k):
        mr = info[r]["m_used"]
        assert info[r]["status"] == "OK" and info[r]["rel_residual"] <= 1e-10
        ref = precond.sample(Q, shape, order, k2, 1.0, Zh[:, r], mr, tol=0.0, reorth=reorth)
        assert ref.m == mr
        # the first steps are well conditioned: coefficients agree closely there
        assert np.allclose(al[r, :8], ref.alpha[:8], rtol=1e-11, atol=0)
        assert _rel(X[:, r], ref.x) <= 1e-8, _rel(X[:, r], ref.x)


@pytest.mark.parametrize("m", [1, 2, 5, 10])
def test_precond_sample_prefix_fp64(gm, m):
    shape, order, k2 = (64, 64), 2, 0.01
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f64").set_circulant_precond()
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], 2, 95, 1)
    X, info, al, be = _sample(gm, op, Zh, tol=0.0, m_max=m)
    for r in range(2):
        ref = precond.sample(Q, shape, order, k2, 1.0, Zh[:, r], m, tol=0.0)
        assert info[r]["m_used"] == m
        assert _rel(X[:, r], ref.x) <= 1e-8


@pytest.mark.parametrize("shape,storage,tol", [((16, 2048), "f64", 1e-8), ((2048, 16), "f64", 1e-8),
                                               ((8, 4096), "f32", 1e-5)])
def test_precond_wide_lattice_prefix(gm, shape, storage, tol):
    """Sides beyond the on-chip band kernel (4 N > LDS FFT capacity: 1024 in FP64, 2048 in
    FP32) take the band kernel that stages the boundary rows in global scratch."""
    order, k2, m = 2, 0.05, 6
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", storage).set_circulant_precond()
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], 2, 98, 0)
    X, info, al, _ = _sample(gm, op, Zh, tol=0.0, m_max=m)
    for r in range(2):
        ref = precond.sample(Q, shape, order, k2, 1.0, Zh[:, r], m, tol=0.0)
        assert info[r]["m_used"] == m
        assert _rel(X[:, r], ref.x) <= tol, _rel(X[:, r], ref.x)


def test_precond_sample_fp32(gm):
    shape, order, k2, k = (64, 64), 2, 0.05, 3
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f32").set_circulant_precond()
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    Zh = workloads.gaussian_block(Q.shape[0], k, 96, 0)
    X, info, _, _ = _sample(gm, op, Zh, tol=1e-6, m_max=200, reorth=True)
    for r in range(k):
        ref = precond.sample(Q, shape, order, k2, 1.0, Zh[:, r], info[r]["m_used"], tol=0.0, reorth=True)
        assert _rel(X[:, r], ref.x) <= 1e-5


def test_perfect_preconditioner_one_step(gm):
    # periodic Q preconditioned by itself: A = I, one step, x = Q^{-1/2} z (closed form)
    shape, k2 = (32, 64), 0.2
    op = gm.Operator.lattice(shape, 2, k2, 1.0, "periodic", "f64").set_circulant_precond()
    Zh = workloads.gaussian_block(shape[0] * shape[1], 2, 97, 0)
    X, info, _, _ = _sample(gm, op, Zh, tol=1e-10, m_max=10)
    assert [i["m_used"] for i in info] == [1, 1]
    for r in range(2):
        ex = closed_form.exact_sample_periodic(shape, 2, k2, 1.0, Zh[:, r])
        assert _rel(X[:, r], ex) <= 1e-13


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_precond_logdet(gm, storage, tol):
    # m = 80 (the log-det workload's m): the quadrature has converged (rho ~ 1e-13)
    shape, k2, npb, m, seed = (32, 32), 0.05, 6, 80, 777
    op = gm.Operator.lattice(shape, 2, k2, 1.0, "free", storage).set_circulant_precond()
    Q = lattice.lattice_precision(shape, 2, k2, 1.0, "free")
    mean, se, per = op.logdet(npb, m, seed=seed)
    ref = logdet.hutchinson_preconditioned(Q, shape, 2, k2, 1.0, npb, m, seed=seed)
    assert np.all(np.abs(per - ref.per_probe) <= tol * np.abs(ref.per_probe))
    assert abs(mean - ref.logdet) <= tol * abs(ref.logdet)
    exact = closed_form.exact_logdet(shape, 2, k2, 1.0, "free")
    assert abs(mean - exact) < 5 * se + 1e-6 * abs(exact)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_preconditioned_batch_full_size(gm, storage):
    """The 512 x 512 preconditioned batch at its real shape and launch configuration (32
    right-hand sides, m_max = 300, no reorthogonalisation); columns 0 and 31 are compared
    with the oracle.  Prefix (m = 10, well conditioned): 1e-8 / 1e-5.  Full run (m = 300,
    unconverged, rho ~ 1e-4): truncation level 10 rho_m."""
    c = workloads.C1
    sp = c.lattice
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, storage).set_circulant_precond()
    Zh = workloads.gaussian_block(sp.n, c.k, 1, 0)
    Q = lattice.lattice_precision(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    Xp, infop, _, _ = _sample(gm, op, Zh, tol=0.0, m_max=10)
    tight = 1e-8 if storage == "f64" else 1e-5
    for r in (0, 31):
        ref = precond.sample(Q, sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, r], 10, tol=0.0)
        assert _rel(Xp[:, r], ref.x) <= tight, _rel(Xp[:, r], ref.x)
    X, info, _, _ = _sample(gm, op, Zh, tol=c.tol, m_max=c.m_max, reorth=False)
    assert all(i["m_used"] == c.m_max and i["status"] == "ENOCONV" for i in info)
    ref = precond.sample(Q, sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, 0], c.m_max, tol=0.0)
    assert _rel(X[:, 0], ref.x) <= 10 * ref.rho[-1], (_rel(X[:, 0], ref.x), ref.rho[-1])


@pytest.mark.timeout(900)
def test_preconditioned_batch_full_size_converged(gm):
    """The benchmark's configuration run to convergence: 512 x 512, 13-point, 32 right-hand sides in
    the launch configuration of the benchmark (two column groups of 16 on two streams), FP64 storage,
    no reorthogonalisation, stop at rho <= 1e-10 (m ~ 970-990, under m_max = 1024).  Every column
    converges; columns 0 (first group) and 31 (second group) equal the oracle at the same m to 1e-8."""
    c = workloads.C1
    sp = c.lattice
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f64").set_circulant_precond()
    Zh = workloads.gaussian_block(sp.n, c.k, 1, 0)
    X, info, _, _ = _sample(gm, op, Zh, tol=1e-10, m_max=1024, reorth=False)
    assert all(i["status"] == "OK" and i["rel_residual"] <= 1e-10 for i in info), info
    Q = lattice.lattice_precision(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    for r in (0, 31):
        ref = precond.sample(Q, sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, r], info[r]["m_used"], tol=0.0)
        assert _rel(X[:, r], ref.x) <= 1e-8, (r, info[r]["m_used"], _rel(X[:, r], ref.x))

"""Pins for oracle.lanczos (Algorithm 1 and the Theorem 1 stopping quantity).

  * m = n with full reorthogonalisation reproduces the dense principal-root sample
    (Krylov space = R^n), including the Section 5.2 test matrix (31^2 P_30)^2.
  * Theorem 1: the a posteriori bound ||x - x_m|| <= lambda_min^{-1/2} ||r_m|| and the a
    priori bound hold for every m, with x exact (closed form) and lambda_min exact.
  * The rho recursion equals the explicitly computed conjugate-gradient residual.
  * Special cases: Q = cI breaks down at m = 1 with x = z / sqrt(c); a diagonal Q with d
    distinct values breaks down at m = d with the exact sample.
  * At the plain FP64 workload (64 x 64, kappa2 = 0.1) the tol-stopped sample meets the
    relative-error bound sqrt(cond) * rho_m against the DCT-exact sample.
"""
import numpy as np
import pytest

from oracle import closed_form, dense, lanczos, lattice


def _z(n, seed=0):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("shape,order", [((8, 8), 1), ((6, 7), 2), ((4, 4, 4), 1), ((20,), 2)])
def test_full_dimension_equals_dense(shape, order):
    Q = lattice.lattice_precision(shape, order, 0.3, 1.0, "free")
    n = Q.shape[0]
    z = _z(n)
    res = lanczos.sample_csr(Q, z, n, tol=0.0, reorth=True)
    x = dense.inv_sqrt_apply(Q, z)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-11


def test_section52_matrix_full_dimension():
    Q = lattice.section52_test_matrix()
    z = _z(900, 3)
    x = dense.inv_sqrt_apply(Q, z)
    # P_30 has 451 distinct eigenvalues (lambda_kl = lambda_lk, and lambda_{k,31-k} = 4),
    # so the Krylov space of a generic z is exhausted at m = 451: exact from there on.
    lam = np.linalg.eigvalsh(lattice.poisson_dirichlet_2d(30).toarray())
    n_distinct = 1 + int(np.sum(np.diff(np.sort(lam)) > 1e-9))
    assert n_distinct == 451
    # cond(Q) ~ 1.5e5, so rounding alone allows ~ cond * eps ~ 3e-11; bound at 30x that
    for m in (n_distinct, 900):
        res = lanczos.sample_csr(Q, z, m, tol=0.0, reorth=True)
        assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-9


def test_theorem1_bounds_every_m():
    shape, k2 = (24, 24), 0.05
    Q = lattice.lattice_precision(shape, 1, k2, 1.0, "free")
    z = _z(Q.shape[0], 5)
    x = closed_form.exact_sample_free(shape, 1, k2, 1.0, z)
    lmin, lmax = closed_form.exact_lambda_min_max(shape, 1, k2, 1.0, "free")
    kappa = lmax / lmin
    alpha, beta, beta0, rho, m, status, V = lanczos.lanczos_tridiag(lambda v: Q @ v, z, 120, 0.0, True)
    for j in range(1, m + 1):
        y = lanczos.tridiag_inv_sqrt_e1(alpha[:j], beta[:j])
        xm = beta0 * (V[:, :j] @ y)
        err = np.linalg.norm(x - xm)
        rj = lanczos.cg_relative_residual(Q, z, V, alpha, beta, beta0, j) * beta0
        assert err <= lmin ** -0.5 * rj * (1 + 1e-9) + 1e-12
        apriori = 2 * lmin ** -0.5 * np.sqrt(kappa) * ((np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)) ** j * beta0
        assert err <= apriori * (1 + 1e-9)


def test_rho_recursion_equals_cg_residual():
    Q = lattice.lattice_precision((16, 16), 2, 0.1, 1.0, "free")
    z = _z(256, 7)
    alpha, beta, beta0, rho, m, status, V = lanczos.lanczos_tridiag(lambda v: Q @ v, z, 60, 0.0, True)
    for j in range(1, m + 1):
        r = lanczos.cg_relative_residual(Q, z, V, alpha, beta, beta0, j)
        if r < 1e-10:
            break
        assert rho[j - 1] == pytest.approx(r, rel=1e-8)


def test_scalar_identity_breaks_down_at_one():
    c = 3.7
    z = _z(50, 1)
    res = lanczos.sample(lambda v: c * v, z, 20, tol=1e-8)
    assert res.m == 1 and res.status == lanczos.OK
    assert np.allclose(res.x, z / np.sqrt(c), rtol=1e-14, atol=0)


def test_diagonal_with_d_distinct_values():
    vals = np.repeat([0.5, 1.0, 2.0, 7.0, 30.0], 8)
    z = _z(vals.size, 2)
    res = lanczos.sample(lambda v: vals * v, z, 40, tol=1e-10, reorth=True)
    assert res.m == 5 and res.beta[4] < 1e-9 * res.beta[0]
    assert np.linalg.norm(res.x - z / np.sqrt(vals)) / np.linalg.norm(z / np.sqrt(vals)) < 1e-12


def test_plain_workload_meets_relative_bound():
    shape, k2 = (64, 64), 0.1
    Q = lattice.lattice_precision(shape, 1, k2, 1.0, "free")
    z = _z(4096, 11)
    res = lanczos.sample_csr(Q, z, 200, tol=1e-8, reorth=True)
    assert res.status == lanczos.OK and res.rho[-1] <= 1e-8
    x = closed_form.exact_sample_free(shape, 1, k2, 1.0, z)
    lmin, lmax = closed_form.exact_lambda_min_max(shape, 1, k2, 1.0, "free")
    rel = np.linalg.norm(res.x - x) / np.linalg.norm(x)
    assert rel <= np.sqrt(lmax / lmin) * res.rho[-1]


def test_not_positive_definite_is_flagged():
    res = lanczos.sample(lambda v: -v, _z(10), 5, tol=1e-8)
    assert res.status == lanczos.ENOTSPD and res.x is None
    # indefinite lattice operator: kappa2 < 0 moves the constant mode below zero
    Q = lattice.lattice_precision((10, 10), 1, -0.5, 1.0, "free")
    res = lanczos.sample_csr(Q, _z(100, 4), 100, tol=1e-12, reorth=True)
    assert res.status == lanczos.ENOTSPD


def test_noconv_when_m_max_too_small():
    Q = lattice.lattice_precision((32, 32), 1, 0.01, 1.0, "free")
    res = lanczos.sample_csr(Q, _z(1024), 5, tol=1e-8)
    assert res.status == lanczos.ENOCONV and res.m == 5 and res.x is not None


def test_tridiag_inv_sqrt_against_dense():
    rng = np.random.default_rng(9)
    m = 40
    a = rng.uniform(2.0, 3.0, m)
    b = rng.uniform(0.1, 0.9, m)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    y = lanczos.tridiag_inv_sqrt_e1(a, b)
    e1 = np.zeros(m); e1[0] = 1
    assert np.allclose(y, dense.inv_sqrt_matrix(T) @ e1, atol=1e-14)
    assert lanczos.tridiag_log_e1(a, b) == pytest.approx(dense.log_matrix(T)[0, 0], abs=1e-14)

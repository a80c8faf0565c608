"""Pins for the closed-form samples and log-determinants (oracle.closed_form, oracle.dense).

Exact samples by the DCT (free) and DFT (periodic) are compared with a dense symmetric
eigendecomposition of the explicitly assembled matrix; exact log-determinants with a dense
Cholesky factorisation and, at the 128 x 128 size of the log-det workload's subgrid, with a
sparse LU factorisation (SuperLU) of the assembled matrix.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import closed_form, dense, lattice


CASES = [((12,), 1), ((6, 9), 1), ((8, 8), 2), ((4, 3, 5), 1), ((5, 4, 3), 2)]


@pytest.mark.parametrize("shape,order", CASES)
def test_exact_sample_free_vs_dense(shape, order):
    Q = lattice.lattice_precision(shape, order, 0.2, 1.5, "free")
    z = np.random.default_rng(0).standard_normal((Q.shape[0], 3))
    x_cf = closed_form.exact_sample_free(shape, order, 0.2, 1.5, z)
    x_d = dense.inv_sqrt_apply(Q, z)
    assert np.linalg.norm(x_cf - x_d) / np.linalg.norm(x_d) < 1e-12


@pytest.mark.parametrize("shape,order", CASES)
def test_exact_sample_periodic_vs_dense(shape, order):
    Q = lattice.lattice_precision(shape, order, 0.2, 1.5, "periodic")
    z = np.random.default_rng(1).standard_normal((Q.shape[0], 2))
    x_cf = closed_form.exact_sample_periodic(shape, order, 0.2, 1.5, z)
    x_d = dense.inv_sqrt_apply(Q, z)
    assert np.linalg.norm(x_cf - x_d) / np.linalg.norm(x_d) < 1e-12


@pytest.mark.parametrize("shape,order", CASES)
@pytest.mark.parametrize("boundary", ["free", "periodic"])
def test_exact_logdet_vs_cholesky(shape, order, boundary):
    Q = lattice.lattice_precision(shape, order, 0.05, 0.7, boundary)
    ld = closed_form.exact_logdet(shape, order, 0.05, 0.7, boundary)
    assert ld == pytest.approx(dense.cholesky_logdet(Q), rel=1e-12, abs=1e-10)


def test_exact_logdet_subgrid_128_vs_sparse_lu():
    # The 128 x 128 subgrid of the log-det workload (second order, kappa2 = 0.05).
    shape = (128, 128)
    Q = lattice.lattice_precision(shape, 2, 0.05, 1.0, "free").tocsc()
    lu = spla.splu(Q, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options={"SymmetricMode": True})
    diag = lu.U.diagonal()
    assert np.all(diag > 0)
    ld_lu = float(np.sum(np.log(diag)))
    ld_cf = closed_form.exact_logdet(shape, 2, 0.05, 1.0, "free")
    assert ld_cf == pytest.approx(ld_lu, rel=1e-11)


def test_principal_root_is_symmetric_and_squares_to_inverse():
    Q = lattice.lattice_precision((5, 6), 2, 0.3, 1.0, "free")
    S = dense.inv_sqrt_matrix(Q)
    assert np.allclose(S, S.T, atol=1e-13)
    assert np.allclose(S @ S @ Q.toarray(), np.eye(30), atol=1e-10)
    assert np.all(np.linalg.eigvalsh(S) > 0)


@pytest.mark.parametrize("shape,order", CASES)
@pytest.mark.parametrize("boundary", ["free", "periodic"])
def test_exact_log_quadratic_form_vs_dense_logm(shape, order, boundary):
    Q = lattice.lattice_precision(shape, order, 0.05, 0.7, boundary)
    v = np.where(np.random.default_rng(3).uniform(size=Q.shape[0]) < 0.5, -1.0, 1.0)
    q = closed_form.exact_log_quadratic_form(shape, order, 0.05, 0.7, boundary, v)
    ref = float(v @ dense.log_matrix(Q) @ v)
    assert abs(q - ref) <= 1e-11 * abs(ref)


def test_gauss_quadrature_of_log_decreases_to_the_quadratic_form():
    """Section 6's quadrature is the m-node Gauss rule for the spectral measure of v; log has negative
    even derivatives, so the rule over-estimates v^T log(Q) v and the error shrinks as m grows."""
    from oracle import logdet
    shape, order, k2 = (16, 16), 2, 0.05
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    v = np.where(np.random.default_rng(4).uniform(size=Q.shape[0]) < 0.5, -1.0, 1.0)
    q = closed_form.exact_log_quadratic_form(shape, order, k2, 1.0, "free", v)
    g = [logdet.quadrature(lambda x: Q @ x, v, m)[0] for m in (5, 10, 20, 40, 256)]   # m = n: exact
    assert all(a > b for a, b in zip(g, g[1:])), g
    assert all(x > q for x in g[:-1]), (g, q)
    assert abs(g[-1] - q) <= 1e-10 * abs(q), (g[-1], q)

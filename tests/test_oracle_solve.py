"""Pins for the Lanczos linear solve x_m = ||b|| V_m T_m^{-1} e_1 (oracle.lanczos.solve and its
preconditioned forms), used for the sMMALA proposal mean (Q + H)^{-1} grad (Section 3).

  * At m = n (CGS2) it is the exact solve (dense numpy.linalg.solve).
  * Its residual ||b - Q x_m|| / ||b|| equals the sampler's stopping quantity rho_m at every m: the
    conjugate-gradient link of Theorem 1.
  * Circulant-, LGCP- and incomplete-Cholesky-preconditioned solves converge to the same exact
    Q^{-1} b.
"""
import numpy as np
import pytest

import workloads
from oracle import ichol, lanczos, lattice, lgcp, precond


def test_full_dimension_is_exact():
    Q = lattice.lattice_precision((6, 5), 2, 0.2, 1.0, "free")
    b = np.random.default_rng(0).standard_normal(30)
    res = lanczos.solve(lambda v: Q @ v, b, 30, tol=0.0, reorth=True)
    x = np.linalg.solve(Q.toarray(), b)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-10


def test_residual_is_rho():
    Q = lattice.lattice_precision((10, 9), 1, 0.05, 1.0, "free")
    b = np.random.default_rng(1).standard_normal(90)
    for m in (1, 5, 20, 40):
        res = lanczos.solve(lambda v: Q @ v, b, m, tol=0.0, reorth=True)
        r = np.linalg.norm(b - Q @ res.x) / np.linalg.norm(b)
        assert r == pytest.approx(res.rho[m - 1], rel=1e-7)


def test_preconditioned_solves_converge_to_the_solution():
    shape, order, k2 = (16, 16), 2, 0.05
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    b = np.random.default_rng(2).standard_normal(256)
    x = np.linalg.solve(Q.toarray(), b)
    res = precond.solve(Q, shape, order, k2, 1.0, b, 400, tol=1e-12, reorth=True)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-8
    L, _ = ichol.ichol(Q, 1e-3)
    res = ichol.solve(Q, L, b, 400, tol=1e-12, reorth=True)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-8


def test_lgcp_proposal_mean():
    N = 32
    spec = workloads.lgcp_prior(N)
    d = workloads.lgcp_diagonal(N)
    g = np.random.default_rng(3).standard_normal(N * N)
    P = lgcp.posterior_precision(spec.shape, 2, spec.kappa2, spec.tau, d).toarray()
    res = lgcp.proposal_mean_solve(spec.shape, 2, spec.kappa2, spec.tau, d, g, 60, tol=1e-12)
    x = np.linalg.solve(P, g)
    assert res.m <= 10
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-9

"""Pins for oracle.lgcp: the log-Gaussian Cox process proposal (Section 3) sampled with the
prior as preconditioner (Section 5.1, Theorem 2 with alpha_n = 0).

  * Proposition 1 with Q + H: S = M^{-1/2} A^{-1/2} satisfies S S^T = (Q + H)^{-1}, and the
    sampler at m = n equals S z.
  * The spectrum of A = I + M^{-1/2} H M^{-1/2} lies in [1 + min H / lambda_max(M),
    1 + max H / lambda_min(M)] (a wrong sign or a dropped term leaves it).
  * The trace identity of the appendix proof: tr(A) - n = tr(M^{-1} H) = [M^{-1}]_{11} sum H,
    the circulant inverse having a constant diagonal (the mean of 1 / lambda_M).
  * H = 0 makes A the identity: one step, and the direct periodic sample of the closed form.
  * Section 6.2 split with H: log det A + log det M = log det (Q + H).
  * Table 1, qualitatively (its inputs are not given): the preconditioned count to 1e-8 does not
    grow with N, the unpreconditioned one does (tests/golden/table1_iterations.txt).
"""
import os

import numpy as np
import pytest

import workloads
from oracle import closed_form, dense, lgcp, precond

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_A(P, shape, mult):
    n = P.shape[0]
    op = precond.preconditioned_operator(P, shape, mult)
    return np.column_stack([op(e) for e in np.eye(n)])


def _case(shape=(6, 8), order=2, kappa2=0.3, tau=2.0, seed=0):
    n = int(np.prod(shape))
    d = np.random.default_rng(seed).uniform(0.05, 1.5, n)
    return shape, order, kappa2, tau, d


@pytest.mark.parametrize("order", [1, 2])
def test_proposition1_factor_with_diagonal(order):
    shape, _, k2, tau, d = _case(order=order)
    n = int(np.prod(shape))
    P = lgcp.posterior_precision(shape, order, k2, tau, d)
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, tau)
    A = _dense_A(P, shape, mult)
    M = lgcp.posterior_precision(shape, order, k2, tau, np.zeros(n))
    S = dense.inv_sqrt_matrix(M) @ dense.inv_sqrt_matrix(A)
    Pinv = np.linalg.inv(P.toarray())
    assert np.linalg.norm(S @ S.T - Pinv) / np.linalg.norm(Pinv) < 1e-11
    z = np.random.default_rng(3).standard_normal(n)
    res = lgcp.sample(shape, order, k2, tau, d, z, n, tol=0.0, reorth=True)
    assert np.linalg.norm(res.x - S @ z) / np.linalg.norm(S @ z) < 1e-10


def test_spectrum_is_identity_plus_bounded_perturbation():
    shape, order, k2, tau, d = _case()
    P = lgcp.posterior_precision(shape, order, k2, tau, d)
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, tau)
    ev = np.linalg.eigvalsh(_dense_A(P, shape, mult))
    lam = closed_form.lattice_spectrum(shape, order, k2, tau, "periodic")
    assert ev.min() >= 1.0 + d.min() / lam.max() - 1e-12
    assert ev.max() <= 1.0 + d.max() / lam.min() + 1e-12


def test_appendix_trace_identity():
    shape, order, k2, tau, d = _case(shape=(8, 8), seed=5)
    n = 64
    P = lgcp.posterior_precision(shape, order, k2, tau, d)
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, tau)
    A = _dense_A(P, shape, mult)
    lam = closed_form.lattice_spectrum(shape, order, k2, tau, "periodic")
    minv11 = float(np.mean(1.0 / lam))
    Minv = np.linalg.inv(lgcp.posterior_precision(shape, order, k2, tau, np.zeros(n)).toarray())
    assert np.allclose(np.diag(Minv), minv11, rtol=1e-12)
    assert np.trace(A) - n == pytest.approx(minv11 * d.sum(), rel=1e-11)


def test_zero_diagonal_is_one_step_and_the_direct_sample():
    shape, order, k2, tau = (8, 16), 2, 0.2, 3.0
    z = np.random.default_rng(7).standard_normal(128)
    res = lgcp.sample(shape, order, k2, tau, np.zeros(128), z, 20, tol=1e-10)
    assert res.m == 1
    x = closed_form.exact_sample_periodic(shape, order, k2, tau, z)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-13


@pytest.mark.parametrize("order", [1, 2])
def test_logdet_split_with_diagonal(order):
    shape, _, k2, tau, d = _case(order=order, seed=2)
    P = lgcp.posterior_precision(shape, order, k2, tau, d)
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, tau)
    ldA = np.linalg.slogdet(_dense_A(P, shape, mult))[1]
    assert ldA + lgcp.logdet_split(shape, order, k2, tau) == pytest.approx(dense.cholesky_logdet(P), rel=1e-12)


def _golden_table1():
    out = {}
    with open(os.path.join(GOLDEN, "table1_iterations.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = line.split("=")
                out[key.strip()] = [None if v == "-" else int(v) for v in val.split()]
    return out


def test_table1_iteration_counts_qualitatively():
    g = _golden_table1()
    paper_pre = dict(zip(g["N"], g["preconditioned"]))
    paper_un = dict(zip(g["N"], g["unpreconditioned"]))
    pre, un = {}, {}
    for N in (16, 32, 64):
        spec = workloads.lgcp_prior(N)
        d = workloads.lgcp_diagonal(N)
        z = workloads.gaussian_block(N * N, 1, 5, 1)[:, 0]
        pre[N] = lgcp.sample(spec.shape, 2, spec.kappa2, spec.tau, d, z, 100, tol=1e-8).m
        un[N] = lgcp.sample_unpreconditioned(spec.shape, 2, spec.kappa2, spec.tau, d, z, 4000, tol=1e-8).m
    # preconditioned: flat in N and of the paper's size; unpreconditioned: grows at least as fast
    assert max(pre.values()) - min(pre.values()) <= 1
    assert max(pre.values()) <= 2 * paper_pre[16]
    assert un[32] / un[16] >= 0.9 * paper_un[32] / paper_un[16]
    assert un[64] / un[16] >= 0.9 * paper_un[64] / paper_un[16]

"""Pins for oracle.ichol: incomplete-Cholesky preconditioning (Section 5.2, Figure 3).

  * droptol = 0 keeps every entry: L is numpy's complete Cholesky factor, A = I, one step, and the
    sample is the exact L^{-T} z.
  * IC(0) on a tridiagonal matrix (no fill in the exact factor) is the exact factor.
  * IC(0) reproduces Q on Q's pattern: (L L^T)_ij = Q_ij wherever Q_ij != 0 (the defining property
    of the zero-fill factorisation), and L stays inside tril(Q)'s pattern.
  * The threshold rule: every kept off-diagonal |l_ij l_jj| >= droptol ||Q[:, j]||, and the error of
    L L^T falls with droptol; IC(0) needs a diagonal shift on Section 5.2's matrix (breakdown).
  * Proposition 1 with F = L on Section 5.2's matrix: S = L^{-T} A^{-1/2} gives S S^T = Q^{-1}; the
    log-det split log det A + 2 sum log L_ii = log det Q.
  * Figure 3, qualitatively: iterations to rho <= 1e-8 fall as the threshold falls, all below the
    unpreconditioned count.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dense, ichol, lanczos, lattice


def test_zero_droptol_is_complete_cholesky():
    Q = lattice.lattice_precision((6, 7), 2, 0.2, 1.0, "free")
    L, shift = ichol.ichol(Q, 0.0)
    assert shift == 0.0
    assert np.allclose(L, np.linalg.cholesky(Q.toarray()), rtol=1e-12, atol=1e-12)
    z = np.random.default_rng(1).standard_normal(42)
    res = ichol.sample(Q, L, z, 10, tol=1e-12)
    assert res.m == 1
    x = np.linalg.solve(L.T, z)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-12


def test_ic0_tridiagonal_is_exact():
    Q = lattice.lattice_precision((30,), 1, 0.3, 1.0, "free")
    assert np.allclose(ichol.ichol(Q, -1.0)[0], np.linalg.cholesky(Q.toarray()), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("Q", [lattice.section52_test_matrix(), lattice.lattice_precision((9, 8), 1, 0.1, 1.0, "free")],
                         ids=["sec52", "5pt"])
def test_ic0_matches_q_on_its_pattern(Q):
    L, shift = ichol.ichol(Q, -1.0)
    Qd = Q.toarray() + shift * np.diag(Q.diagonal())
    pat = Qd != 0
    assert np.all(L[~np.tril(pat)] == 0.0)
    R = L @ L.T - Qd
    assert np.max(np.abs(R[pat])) < 1e-9 * np.max(np.abs(Qd))
    assert np.max(np.abs(R[~pat])) > 0.0            # fill was dropped, so L L^T != Q


def test_threshold_rule_and_accuracy():
    Q = lattice.section52_test_matrix()
    Qd = Q.toarray()
    cn = np.linalg.norm(Qd, axis=0)
    errs = []
    for tol in (1e-2, 1e-3, 1e-4, 1e-5):
        L, shift = ichol.ichol(Q, tol)
        off = np.tril(L, -1)
        i, j = np.nonzero(off)
        assert np.all(np.abs(off[i, j] * L[j, j]) >= tol * cn[j] * (1 - 1e-12))
        errs.append(np.linalg.norm(L @ L.T - Qd) / np.linalg.norm(Qd))
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_proposition1_and_logdet_with_ic0():
    Q = lattice.section52_test_matrix()
    L, shift = ichol.ichol(Q, -1.0)
    assert shift > 0.0                              # IC(0) breaks down unshifted on this matrix
    n = Q.shape[0]
    Linv = np.linalg.inv(L)
    A = Linv @ Q.toarray() @ Linv.T
    S = Linv.T @ dense.inv_sqrt_matrix(A)
    Qinv = np.linalg.inv(Q.toarray())
    assert np.linalg.norm(S @ S.T - Qinv) / np.linalg.norm(Qinv) < 1e-9
    ldA = np.linalg.slogdet(A)[1]
    assert ldA + 2 * np.sum(np.log(np.diag(L))) == pytest.approx(dense.cholesky_logdet(Q), rel=1e-11)
    z = np.random.default_rng(5).standard_normal(n)
    res = ichol.sample(Q, L, z, 200, tol=0.0, reorth=True)
    assert np.linalg.norm(res.x - S @ z) / np.linalg.norm(S @ z) < 1e-8


def test_figure3_iterations_fall_with_threshold():
    Q = lattice.section52_test_matrix()
    z = np.random.default_rng(7).standard_normal(Q.shape[0])
    m_plain = lanczos.sample_csr(Q, z, 900, tol=1e-8, reorth=True).m
    ms = [ichol.sample(Q, ichol.ichol(Q, t)[0], z, 900, tol=1e-8, reorth=True).m for t in (-1.0, 1e-3, 1e-4, 1e-5)]
    assert m_plain > ms[0]
    assert all(a >= b for a, b in zip(ms, ms[1:])) and ms[0] > ms[-1]

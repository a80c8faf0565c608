"""Incomplete-Cholesky preconditioning (Section 5.2) for a general sparse SPD Q.

Proposition 1 with M = L L^T from an incomplete Cholesky factorisation and F = L: Algorithm 1 runs
on A = L^{-1} Q L^{-T} and the sample is x = L^{-T} u_m; log det Q = log det A + 2 sum log L_ii
(Section 6.2 with F = L).  The paper compares factorisations with several drop thresholds (Figure 3)
without fixing the dropping rule; the one used here, column by column (left looking, FP64):

    l_jj = sqrt(c_jj - sum_{k<j} l_jk^2),   l_ij = (c_ij - sum_{k<j} l_ik l_jk) / l_jj   (i > j),

with C = Q + shift * diag(Q).  A non-positive pivot is a breakdown; the factorisation then restarts
with the next shift of the sequence 0, 1e-3, 2e-3, 4e-3, ... (at most 30 doublings), the diagonal
compensation that keeps it defined on matrices that are not M-matrices (Section 5.2's is not).
Threshold rule (droptol >= 0): an off-diagonal l_ij is dropped (set to zero before the next column
uses it) when its numerator |c_ij - sum_{k<j} l_ik l_jk| < droptol * ||Q[:, j]||_2, the scale of the
column it updates (dropping before the division by the pivot, as in Saad's ILUT); droptol = 0 keeps
everything (the complete Cholesky factor).  Level-0 rule (droptol < 0): l_ij is kept only where
Q_ij != 0 (IC(0)).

Dense arithmetic: the oracle is meant for the paper's 900-point test matrix and smaller.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import lanczos, logdet


SHIFTS = [0.0] + [1e-3 * 2.0 ** i for i in range(31)]


def ichol(Q, droptol):
    """(L, shift): the lower-triangular factor (dense FP64) for the first shift of SHIFTS without a
    breakdown."""
    for shift in SHIFTS:
        try:
            return ichol_shifted(Q, droptol, shift), shift
        except ValueError:
            pass
    raise ValueError("incomplete Cholesky broke down for every shift")


def ichol_shifted(Q, droptol, shift):
    """The factor of C = Q + shift diag(Q) (ValueError on a non-positive pivot)."""
    Qd = np.asarray(sp.csr_matrix(Q).toarray(), dtype=np.float64)
    n = Qd.shape[0]
    C = Qd + shift * np.diag(np.diag(Qd))
    colnorm = np.linalg.norm(Qd, axis=0)
    keep0 = Qd != 0.0
    L = np.zeros((n, n))
    for j in range(n):
        col = C[j:, j] - L[j:, :j] @ L[j, :j]
        if not col[0] > 0.0:
            raise ValueError(f"incomplete Cholesky breakdown at column {j}")
        d = np.sqrt(col[0])
        num = col[1:]
        if droptol < 0:
            num = np.where(keep0[j + 1:, j], num, 0.0)
        else:
            num = np.where(np.abs(num) >= droptol * colnorm[j], num, 0.0)
        off = num / d
        L[j, j] = d
        L[j + 1:, j] = off
    return L


def operator(Q, L):
    """v -> A v = L^{-1} Q L^{-T} v."""
    Q = sp.csr_matrix(Q)

    def matvec(v):
        t = sla.solve_triangular(L, v, lower=True, trans="T")
        return sla.solve_triangular(L, Q @ t, lower=True)
    return matvec


def sample(Q, L, z, m_max, tol=0.0, reorth=False):
    """x = L^{-T} u_m with u_m Algorithm 1's sample for A (Proposition 1, F = L)."""
    res = lanczos.sample(operator(Q, L), z, m_max, tol, reorth)
    if res.x is not None:
        res.x = sla.solve_triangular(L, res.x, lower=True, trans="T")
    return res


def hutchinson(Q, L, n_probes, m, seed=0):
    """Section 6.2 with F = L: Hutchinson on A plus 2 sum log L_ii."""
    shift = 2.0 * float(np.sum(np.log(np.diag(L))))
    return logdet.hutchinson(operator(Q, L), Q.shape[0], n_probes, m, seed, shift=shift)


def solve(Q, L, b, m_max, tol=0.0, reorth=False):
    """Q^{-1} b = L^{-T} A^{-1} L^{-1} b (incomplete-Cholesky preconditioned conjugate gradients)."""
    res = lanczos.solve(operator(Q, L), sla.solve_triangular(L, b, lower=True), m_max, tol, reorth)
    if res.x is not None:
        res.x = sla.solve_triangular(L, res.x, lower=True, trans="T")
    return res

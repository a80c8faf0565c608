"""Section 6: the Hutchinson estimator of log det Q with Lanczos (Gauss) quadrature.

    log det Q = E[ V^T log(Q) V ] ~= N^{-1} sum_p v_p^T log(Q) v_p,  v_p Rademacher.

The quadratic form v^T log(Q) v is evaluated by running m steps of Algorithm 1's
recurrence from v (the paper cites Bai, Fahey & Golub 1996 and does not print the rule):
with T_m = U diag(theta) U^T,

    v^T log(Q) v ~= ||v||^2 e_1^T log(T_m) e_1 = ||v||^2 sum_k U_{1k}^2 log theta_k,

exact once m reaches the dimension of the Krylov space.  ||v||^2 = n for Rademacher
probes.  The estimate is the probe mean; its standard error is sd(Gamma)/sqrt(N).

Variance reading: for Rademacher probes Var(v^T B v) = 2 sum_{i != j} B_ij^2 (the printed
expression lacks the factor 2 and uses the Gaussian-probe form); the tests check the
factor-2 form by simulation.

Preconditioned split (Section 6.2, sign corrected): log det Q = log det A + log det M with
A = M^{-1/2} Q M^{-1/2}.

Coloured Hutchinson (Section 6.1, after Aune et al. with the colouring suggested by Tang & Saad):
partition the nodes into colour classes c such that two nodes of one class are more than p steps
apart in the graph of Q, i.e. colour the graph of Q^p.  With V^c the probe restricted to class c
(zero elsewhere) the estimate of one probe is sum_c (V^c)^T log(Q) V^c, unbiased for log det Q,
with variance 2 sum_c sum_{i != j in c} B_ij^2 for Rademacher entries (the factor 2 as above).
Here V^c is the Rademacher probe v_p masked to class c, so a coloured probe is the plain probe
split by colour; each class takes its own quadrature.  The colouring is first fit in node order
on the pattern of (I + |Q|)^p.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import lanczos, philox, precond


@dataclass
class LogdetResult:
    logdet: float
    std_err: float
    per_probe: np.ndarray
    m_used: np.ndarray


def quadrature(matvec, v, m):
    """Gamma = ||v||^2 e_1^T log(T_m) e_1 from m steps of the recurrence (no reorth)."""
    alpha, beta, beta0, rho, mu, status, _ = lanczos.lanczos_tridiag(matvec, v, m, 0.0, False)
    if status == lanczos.ENOTSPD:
        raise ValueError("operator is not positive definite")
    return beta0 ** 2 * lanczos.tridiag_log_e1(alpha[:mu], beta[:mu]), mu


def hutchinson(matvec, n, n_probes, m, seed=0, probes=None, shift=0.0):
    """Mean and standard error of Gamma_p over the probes; `shift` adds a known constant
    (log det M in the preconditioned split)."""
    if probes is None:
        probes = philox.rademacher_probes(seed, n_probes, n)
    gam = np.empty(n_probes)
    mus = np.empty(n_probes, dtype=np.int64)
    for p in range(n_probes):
        gam[p], mus[p] = quadrature(matvec, probes[:, p], m)
    gam = gam + shift
    se = float(np.std(gam, ddof=1) / np.sqrt(n_probes)) if n_probes > 1 else float("nan")
    return LogdetResult(float(np.mean(gam)), se, gam, mus)


def hutchinson_csr(Q, n_probes, m, seed=0, probes=None):
    return hutchinson(lambda v: Q @ v, Q.shape[0], n_probes, m, seed, probes)


def hutchinson_preconditioned(Q, shape, order, kappa2, tau, n_probes, m, seed=0, probes=None):
    """Section 6.2: estimate log det A by Hutchinson and add the closed-form log det M."""
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, kappa2, tau)
    A = precond.preconditioned_operator(Q, shape, mult)
    shift = precond.logdet_M(shape, order, kappa2, tau)
    return hutchinson(A, Q.shape[0], n_probes, m, seed, probes, shift=shift)


def distance_colouring(Q, p):
    """Colour of every node such that nodes within p steps of each other in the graph of Q differ:
    first fit in node order on the pattern of (I + |Q|)^p (p = 0: one colour)."""
    n = Q.shape[0]
    if p <= 0:
        return np.zeros(n, dtype=np.int64)
    A = (abs(sp.csr_matrix(Q)) + sp.identity(n)).tocsr()
    A.data[:] = 1.0
    R = sp.identity(n, format="csr")
    for _ in range(p):
        R = (R @ A).tocsr()
        R.data[:] = 1.0
    colour = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = {int(colour[j]) for j in R.indices[R.indptr[i]:R.indptr[i + 1]] if colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def hutchinson_coloured(matvec, n, colour, n_probes, m, seed=0, shift=0.0):
    """Section 6.1: Gamma_p = sum_c Gamma(v_p masked to class c) + shift; mean and standard error
    over the probes (v_p: the Philox Rademacher probes)."""
    colour = np.asarray(colour)
    K = int(colour.max()) + 1
    probes = philox.rademacher_probes(seed, n_probes, n)
    gam = np.zeros(n_probes)
    for q in range(n_probes):
        for c in range(K):
            v = np.where(colour == c, probes[:, q], 0.0)
            gam[q] += quadrature(matvec, v, m)[0]
    gam = gam + shift
    se = float(np.std(gam, ddof=1) / np.sqrt(n_probes)) if n_probes > 1 else float("nan")
    return LogdetResult(float(np.mean(gam)), se, gam, np.full(n_probes, m))


def coloured_variance(B, colour):
    """2 sum_c sum_{i != j in c} B_ij^2: the variance of one coloured Rademacher probe (dense B)."""
    colour = np.asarray(colour)
    same = colour[:, None] == colour[None, :]
    off = np.where(same & ~np.eye(B.shape[0], dtype=bool), B, 0.0)
    return float(2.0 * np.sum(off ** 2))

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
"""
from dataclasses import dataclass

import numpy as np

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

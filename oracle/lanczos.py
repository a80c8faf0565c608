"""Algorithm 1 (Section 4): the Lanczos Krylov sampler x_m ~= Q^{-1/2} z, in FP64.

The steps follow Algorithm 1 in the paper's order:
    beta0 = ||z||, v_1 = z / beta0
    for j = 1..m:   q = Q v_j;  if j > 1: q -= beta_{j-1} v_{j-1}
                    alpha_j = v_j^T q;  q -= alpha_j v_j
                    beta_j = ||q||;     v_{j+1} = q / beta_j
    T_m = tridiag(beta, alpha, beta),  x_m = ||z|| V_m T_m^{-1/2} e_1

Readings where the paper is silent (each also listed in the design notes):
  * Stopping.  Algorithm 1 takes a fixed m; Section 1 says m can be chosen adaptively and
    Theorem 1 bounds the error by lambda_min^{-1/2} ||r_m|| with r_m the conjugate-gradient
    residual for Q y = z.  The relative residual rho_j = ||r_j|| / ||z|| is obtained from the
    Lanczos coefficients through the LDL^T pivots of T_j:  d_1 = alpha_1,
    d_j = alpha_j - beta_{j-1}^2 / d_{j-1},  rho_j = rho_{j-1} * beta_j / d_j  (rho_0 = 1).
    Iteration stops at the first j with rho_j <= tol, or at breakdown
    (beta_j <= 64 eps (|alpha_j| + beta_{j-1})), or at m_max.  tol <= 0 runs exactly m_max
    steps (breakdown still stops).
  * Reorthogonalisation is not mentioned.  ``reorth=True`` applies classical Gram-Schmidt
    twice (CGS2) against all stored v_1..v_j after the three-term update.
  * Definiteness.  alpha_j <= 0 or d_j <= 0 means T_j (hence Q) is not positive definite:
    status ENOTSPD and no sample.
  * T_m^{-1/2} e_1 is taken from the exact eigendecomposition of T_m (LAPACK stemr via
    scipy.linalg.eigh_tridiagonal): T_m = U diag(theta) U^T,
    y = U (theta^{-1/2} * U^T e_1).  stemr (relatively robust representations) can fail to
    converge on the tight Ritz-value clusters of long runs without reorthogonalisation; the
    implicit QL/QR driver stev, which always converges, then computes the same decomposition.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

OK, ENOTSPD, ENOCONV = 0, 2, 3
EPS = np.finfo(np.float64).eps


@dataclass
class LanczosResult:
    x: np.ndarray               # the sample x_m (None if not SPD)
    m: int                      # Krylov dimension used
    alpha: np.ndarray           # alpha_1..alpha_m
    beta: np.ndarray            # beta_1..beta_m (beta_m is the last, unused in T_m)
    beta0: float                # ||z||
    rho: np.ndarray             # rho_1..rho_m
    status: int
    V: np.ndarray = field(default=None, repr=False)   # n x m basis (kept for tests)


def lanczos_tridiag(matvec, z, m_max, tol=0.0, reorth=False, keep_basis=False):
    """Run Algorithm 1's recurrence; return coefficients, rho and (optionally) V_m."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    beta0 = float(np.linalg.norm(z))
    V = np.zeros((n, m_max + 1))
    V[:, 0] = z / beta0
    alpha, beta, rho = [], [], []
    d_prev, rho_prev = None, 1.0
    status, m, converged = OK, 0, False
    for j in range(1, m_max + 1):
        vj = V[:, j - 1]
        q = matvec(vj)
        if j > 1:
            q = q - beta[-1] * V[:, j - 2]
        a = float(vj @ q)
        q = q - a * vj
        if reorth:
            for _ in range(2):
                Vj = V[:, :j]
                q = q - Vj @ (Vj.T @ q)
        b = float(np.linalg.norm(q))
        d = a if j == 1 else a - beta[-1] ** 2 / d_prev
        r = rho_prev * b / d if d != 0 else np.inf
        prev_beta = beta[-1] if j > 1 else 0.0
        alpha.append(a)
        beta.append(b)
        rho.append(r)
        m = j
        if a <= 0 or d <= 0:
            status = ENOTSPD
            break
        if b <= 64.0 * EPS * (abs(a) + prev_beta) or (tol > 0 and r <= tol):
            converged = True
            break
        V[:, j] = q / b
        d_prev, rho_prev = d, r
    if status == OK and tol > 0 and not converged:
        status = ENOCONV
    return np.array(alpha), np.array(beta), beta0, np.array(rho), m, status, V[:, :m]


def _eigh_tridiag(alpha, beta_off):
    """Eigendecomposition of the symmetric tridiagonal T (LAPACK stemr; stev if stemr fails)."""
    try:
        return sla.eigh_tridiagonal(alpha, beta_off)
    except np.linalg.LinAlgError:
        return sla.eigh_tridiagonal(alpha, beta_off, lapack_driver="stev")


def tridiag_inv_sqrt_e1(alpha, beta):
    """y = T^{-1/2} e_1 with T = tridiag(beta[:m-1], alpha, beta[:m-1]) via eigh."""
    m = len(alpha)
    if m == 1:
        return np.array([alpha[0] ** -0.5])
    theta, U = _eigh_tridiag(alpha, beta[: m - 1])
    if theta.min() <= 0:
        raise ValueError("T_m is not positive definite")
    return U @ (theta ** -0.5 * U[0, :])


def tridiag_log_e1(alpha, beta):
    """e_1^T log(T) e_1 = sum_k tau_k^2 log theta_k (Gauss quadrature nodes/weights)."""
    m = len(alpha)
    if m == 1:
        return float(np.log(alpha[0]))
    theta, U = _eigh_tridiag(alpha, beta[: m - 1])
    if theta.min() <= 0:
        raise ValueError("T_m is not positive definite")
    return float(np.sum(U[0, :] ** 2 * np.log(theta)))


def sample(matvec, z, m_max, tol=0.0, reorth=False, keep_basis=False):
    """x_m = ||z|| V_m T_m^{-1/2} e_1 (Algorithm 1, final step)."""
    alpha, beta, beta0, rho, m, status, V = lanczos_tridiag(matvec, z, m_max, tol, reorth)
    if status == ENOTSPD:
        return LanczosResult(None, m, alpha, beta, beta0, rho, status,
                             V if keep_basis else None)
    y = tridiag_inv_sqrt_e1(alpha[:m], beta[:m])
    x = beta0 * (V[:, :m] @ y)
    return LanczosResult(x, m, alpha, beta, beta0, rho, status, V if keep_basis else None)


def sample_csr(Q, z, m_max, tol=0.0, reorth=False, keep_basis=False):
    return sample(lambda v: Q @ v, z, m_max, tol, reorth, keep_basis)


def sample_many(matvec, Z, m_max, tol=0.0, reorth=False, m_fixed=None):
    """Column-by-column samples of an n x k block; m_fixed[r] forces the Krylov dimension."""
    Z = np.asarray(Z, dtype=np.float64)
    k = Z.shape[1]
    X = np.full_like(Z, np.nan)
    infos = []
    for r in range(k):
        if m_fixed is not None:
            res = sample(matvec, Z[:, r], int(m_fixed[r]), 0.0, reorth)
        else:
            res = sample(matvec, Z[:, r], m_max, tol, reorth)
        if res.x is not None:
            X[:, r] = res.x
        infos.append(res)
    return X, infos


def cg_relative_residual(Q, z, V, alpha, beta, beta0, j):
    """||z - Q V_j y_j|| / ||z|| with y_j = beta0 T_j^{-1} e_1: the conjugate-gradient
    residual written out explicitly (used to check the rho recursion)."""
    T = np.diag(alpha[:j]) + np.diag(beta[: j - 1], 1) + np.diag(beta[: j - 1], -1)
    e1 = np.zeros(j)
    e1[0] = 1.0
    y = beta0 * np.linalg.solve(T, e1)
    r = z - Q @ (V[:, :j] @ y)
    return float(np.linalg.norm(r) / beta0)


def tridiag_solve_e1(alpha, beta):
    """y = T^{-1} e_1 (T = tridiag(beta[:m-1], alpha, beta[:m-1])) by a dense solve."""
    m = len(alpha)
    T = np.diag(alpha[:m]) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    e1 = np.zeros(m)
    e1[0] = 1.0
    return np.linalg.solve(T, e1)


def solve(matvec, b, m_max, tol=0.0, reorth=False):
    """x_m = ||b|| V_m T_m^{-1} e_1: the Lanczos form of the conjugate-gradient iterate for Q x = b
    (Theorem 1 ties the sampler's stopping quantity rho_m to this iterate's residual ||b - Q x_m||)."""
    alpha, beta, beta0, rho, m, status, V = lanczos_tridiag(matvec, b, m_max, tol, reorth)
    if status == ENOTSPD:
        return LanczosResult(None, m, alpha, beta, beta0, rho, status)
    y = tridiag_solve_e1(alpha[:m], beta[:m])
    return LanczosResult(beta0 * (V[:, :m] @ y), m, alpha, beta, beta0, rho, status)

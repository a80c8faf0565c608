"""Dense references: the plain definitions the Krylov method approximates.

Section 4: the target sample is x = Q^{-1/2} z with Q^{-1/2} the inverse of the principal
square root.  Section 6: the determinant term is log det Q = tr log Q.  These are written
out with a dense symmetric eigendecomposition (LAPACK syevd via numpy) and a dense
Cholesky factorisation; they are only used on small n.
"""
import numpy as np
import scipy.sparse as sp


def _dense(Q):
    return Q.toarray() if sp.issparse(Q) else np.asarray(Q, dtype=np.float64)


def inv_sqrt_apply(Q, z):
    """Q^{-1/2} z through Q = U diag(lam) U^T (principal root)."""
    lam, U = np.linalg.eigh(_dense(Q))
    if lam.min() <= 0:
        raise ValueError("Q is not positive definite")
    return U @ ((U.T @ z) / (np.sqrt(lam)[:, None] if np.ndim(z) == 2 else np.sqrt(lam)))


def inv_sqrt_matrix(Q):
    lam, U = np.linalg.eigh(_dense(Q))
    return (U / np.sqrt(lam)) @ U.T


def sqrt_matrix(Q):
    lam, U = np.linalg.eigh(_dense(Q))
    return (U * np.sqrt(lam)) @ U.T


def log_matrix(Q):
    """log Q through the eigendecomposition."""
    lam, U = np.linalg.eigh(_dense(Q))
    return (U * np.log(lam)) @ U.T


def cholesky_logdet(Q):
    """log det Q = 2 sum log L_ii with Q = L L^T."""
    L = np.linalg.cholesky(_dense(Q))
    return float(2.0 * np.sum(np.log(np.diag(L))))


def eig_extremes(Q):
    lam = np.linalg.eigvalsh(_dense(Q))
    return float(lam[0]), float(lam[-1])

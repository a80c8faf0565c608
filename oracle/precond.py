"""Proposition 1 (Section 5) with the block-circulant preconditioner of Section 5.1.

With M = F F^T, draw u ~ N(0, (F^{-1} Q F^{-T})^{-1}) by Algorithm 1 on
A = F^{-1} Q F^{-T}, then x solves F^T x = u and has precision Q.  Here M is the periodic
(block-circulant) version of the lattice precision and F = M^{1/2} is its symmetric root,
so F^{-1} = F^{-T} = M^{-1/2} is applied with the FFT:

    M^{-1/2} v = IFFT( lambda_M^{-1/2} * FFT(v) ),

lambda_M being the DFT eigenvalues of M.  Per Lanczos step this costs two FFT pairs (four
FFTs) and one stencil, which is the count Section 5.1 gives; the back-transform
x = M^{-1/2} u_m is one more pair.

Preconditioned determinant (Section 6.2): log det Q = log det(F^{-1} Q F^{-T}) + 2 log det F
= log det A + log det M.  The printed formula has "- 2 log det F"; since
det(F^{-1} Q F^{-T}) = det Q / det(F)^2 the sign must be "+", which a dense check confirms.
"""
import numpy as np

from . import closed_form, lanczos


def circulant_inv_sqrt_multiplier(shape, order, kappa2, tau):
    """lambda_M^{-1/2} on the DFT grid for M = periodic version of the lattice precision."""
    lam = closed_form.lattice_spectrum(shape, order, kappa2, tau, "periodic")
    return 1.0 / np.sqrt(lam)


def apply_inv_sqrt_M(shape, mult, v):
    """M^{-1/2} v by the n-dimensional FFT (real input, real output)."""
    V = np.asarray(v, dtype=np.float64).reshape(shape)
    return np.real(np.fft.ifftn(np.fft.fftn(V) * mult)).ravel()


def preconditioned_operator(Q, shape, mult):
    """v -> A v = M^{-1/2} Q M^{-1/2} v."""
    def matvec(v):
        return apply_inv_sqrt_M(shape, mult, Q @ apply_inv_sqrt_M(shape, mult, v))
    return matvec


def sample(Q, shape, order, kappa2, tau, z, m_max, tol=0.0, reorth=False):
    """x = M^{-1/2} u_m with u_m the Algorithm 1 sample for A (Proposition 1)."""
    mult = circulant_inv_sqrt_multiplier(shape, order, kappa2, tau)
    res = lanczos.sample(preconditioned_operator(Q, shape, mult), z, m_max, tol, reorth)
    if res.x is not None:
        res.x = apply_inv_sqrt_M(shape, mult, res.x)
    return res


def sample_many(Q, shape, order, kappa2, tau, Z, m_max, tol=0.0, reorth=False, m_fixed=None):
    Z = np.asarray(Z, dtype=np.float64)
    X = np.full_like(Z, np.nan)
    infos = []
    for r in range(Z.shape[1]):
        mm = int(m_fixed[r]) if m_fixed is not None else m_max
        tt = 0.0 if m_fixed is not None else tol
        res = sample(Q, shape, order, kappa2, tau, Z[:, r], mm, tt, reorth)
        if res.x is not None:
            X[:, r] = res.x
        infos.append(res)
    return X, infos


def logdet_M(shape, order, kappa2, tau):
    """log det M = sum log lambda_M (closed form)."""
    return closed_form.exact_logdet(shape, order, kappa2, tau, "periodic")


def solve(Q, shape, order, kappa2, tau, b, m_max, tol=0.0, reorth=False):
    """Q^{-1} b = M^{-1/2} A^{-1} M^{-1/2} b with A^{-1} by the Lanczos iterate (Proposition 1's
    factorisation used for a linear solve, i.e. preconditioned conjugate gradients)."""
    mult = circulant_inv_sqrt_multiplier(shape, order, kappa2, tau)
    res = lanczos.solve(preconditioned_operator(Q, shape, mult), apply_inv_sqrt_M(shape, mult, b), m_max, tol, reorth)
    if res.x is not None:
        res.x = apply_inv_sqrt_M(shape, mult, res.x)
    return res

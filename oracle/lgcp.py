"""The log-Gaussian Cox process example (Section 3) and its preconditioned sampler (Section 5.1).

The sMMALA proposal of Section 3 needs samples of N(0, (Q + H)^{-1}), Q the block-circulant
prior precision on the torus and H the diagonal Fisher information of the Poisson counts.
Section 5.1 (Theorem 2, with alpha_n = 0) preconditions with M = Q itself: Proposition 1 with
F = M^{1/2} runs Algorithm 1 on

    A = M^{-1/2} (Q + H) M^{-1/2} = I + M^{-1/2} H M^{-1/2},

whose spectrum lies in [1, 1 + max(H) / lambda_min(M)] whatever the lattice size, so the
iteration count to a fixed tolerance does not grow with n (Table 1).  The sample is
x = M^{-1/2} u_m.  Here everything is delegated to ``precond`` with the explicit sparse
Q + diag(H): the same four-FFT real-space form that Section 5.1 counts.
"""
import numpy as np
import scipy.sparse as sp

from . import lanczos, lattice, precond


def posterior_precision(shape, order, kappa2, tau, d):
    """Q + diag(d), Q the periodic lattice precision (the LGCP prior on the torus)."""
    Q = lattice.lattice_precision(shape, order, kappa2, tau, "periodic")
    return (Q + sp.diags(np.asarray(d, dtype=np.float64))).tocsr()


def sample(shape, order, kappa2, tau, d, z, m_max, tol=0.0, reorth=False):
    """Proposition 1 with M = Q: x = M^{-1/2} u_m, u_m Algorithm 1's sample for A."""
    P = posterior_precision(shape, order, kappa2, tau, d)
    return precond.sample(P, shape, order, kappa2, tau, z, m_max, tol, reorth)


def sample_many(shape, order, kappa2, tau, d, Z, m_max, tol=0.0, reorth=False, m_fixed=None):
    P = posterior_precision(shape, order, kappa2, tau, d)
    return precond.sample_many(P, shape, order, kappa2, tau, Z, m_max, tol, reorth, m_fixed)


def sample_unpreconditioned(shape, order, kappa2, tau, d, z, m_max, tol=0.0, reorth=False):
    """Algorithm 1 on Q + H directly (the second row of Table 1)."""
    return lanczos.sample_csr(posterior_precision(shape, order, kappa2, tau, d), z, m_max, tol, reorth)


def logdet_split(shape, order, kappa2, tau):
    """log det M, added to the Hutchinson estimate of log det A (Section 6.2, sign corrected)."""
    return precond.logdet_M(shape, order, kappa2, tau)


def proposal_mean_solve(shape, order, kappa2, tau, d, g, m_max, tol=0.0, reorth=False):
    """(Q + H)^{-1} g with M = Q (the drift of the sMMALA proposal of Section 3)."""
    P = posterior_precision(shape, order, kappa2, tau, d)
    return precond.solve(P, shape, order, kappa2, tau, g, m_max, tol, reorth)

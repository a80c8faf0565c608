"""Closed-form spectra, exact samples and exact log-determinants of lattice precisions.

Section 1 / Section 2: a (block) circulant precision is diagonalised by the discrete
Fourier transform, so its samples and determinant cost O(n log n).  The free-boundary
lattice is diagonalised the same way by the type-II discrete cosine transform (the path
Laplacian's eigenvectors), which makes exact samples available at every lattice size.

1D spectra (N nodes, k = 0..N-1):
    free (path)      mu_k = 4 sin^2(pi k / (2N)),   u_k(i) = c_k cos(pi k (i + 1/2) / N)
    periodic (cycle) mu_k = 4 sin^2(pi k / N),      Fourier modes
with c_0 = sqrt(1/N), c_k = sqrt(2/N).  The lattice Laplacian is a Kronecker sum, so
its eigenvalues add over axes; Q's eigenvalues are tau*(kappa2 + sum mu) (first order)
or tau*(kappa2 + sum mu)^2 (second order).
"""
import numpy as np


def path_spectrum(N, periodic):
    k = np.arange(N, dtype=np.float64)
    if periodic:
        return 4.0 * np.sin(np.pi * k / N) ** 2
    return 4.0 * np.sin(np.pi * k / (2.0 * N)) ** 2


def dct2_matrix(N):
    """Orthonormal DCT-II eigenvector matrix U (columns u_k) of the free path Laplacian."""
    i = np.arange(N, dtype=np.float64)[:, None]
    k = np.arange(N, dtype=np.float64)[None, :]
    U = np.cos(np.pi * k * (i + 0.5) / N) * np.sqrt(2.0 / N)
    U[:, 0] = np.sqrt(1.0 / N)
    return U


def lattice_spectrum(shape, order=1, kappa2=1.0, tau=1.0, boundary="free"):
    """Eigenvalues of Q laid out on the lattice's frequency grid (array of `shape`)."""
    periodic = boundary == "periodic"
    shape = tuple(int(s) for s in shape)
    mu = np.zeros(shape)
    for d, Nd in enumerate(shape):
        sl = [None] * len(shape)
        sl[d] = slice(None)
        mu = mu + path_spectrum(Nd, periodic)[tuple(sl)]
    base = kappa2 + mu
    if order == 1:
        return tau * base
    if order == 2:
        return tau * base ** 2
    raise ValueError("order must be 1 or 2")


def _apply_axes(X, mats):
    """Apply matrix mats[d] along axis d of X (X reshaped to the lattice)."""
    for d, A in enumerate(mats):
        X = np.moveaxis(np.tensordot(A, X, axes=([1], [d])), 0, d)
    return X


def exact_sample_free(shape, order, kappa2, tau, z):
    """x = Q^{-1/2} z for the free-boundary lattice (principal root), z of length n or n x k."""
    shape = tuple(int(s) for s in shape)
    lam = lattice_spectrum(shape, order, kappa2, tau, "free")
    Us = [dct2_matrix(N) for N in shape]
    z = np.asarray(z, dtype=np.float64)
    cols = z.reshape(z.shape[0], -1)
    out = np.empty_like(cols)
    for r in range(cols.shape[1]):
        Zr = cols[:, r].reshape(shape)
        C = _apply_axes(Zr, [U.T for U in Us])
        C = C / np.sqrt(lam)
        out[:, r] = _apply_axes(C, Us).ravel()
    return out.reshape(z.shape)


def exact_sample_periodic(shape, order, kappa2, tau, z):
    """x = Q^{-1/2} z for the periodic (block-circulant) lattice via the DFT."""
    shape = tuple(int(s) for s in shape)
    lam = lattice_spectrum(shape, order, kappa2, tau, "periodic")
    z = np.asarray(z, dtype=np.float64)
    cols = z.reshape(z.shape[0], -1)
    out = np.empty_like(cols)
    for r in range(cols.shape[1]):
        Zr = cols[:, r].reshape(shape)
        out[:, r] = np.real(np.fft.ifftn(np.fft.fftn(Zr) / np.sqrt(lam))).ravel()
    return out.reshape(z.shape)


def exact_logdet(shape, order, kappa2, tau, boundary):
    """log det Q = sum of log eigenvalues."""
    lam = lattice_spectrum(shape, order, kappa2, tau, boundary)
    return float(np.sum(np.log(lam)))


def exact_lambda_min_max(shape, order, kappa2, tau, boundary):
    lam = lattice_spectrum(shape, order, kappa2, tau, boundary)
    return float(lam.min()), float(lam.max())


def exact_log_quadratic_form(shape, order, kappa2, tau, boundary, v):
    """v^T log(Q) v for a lattice precision: the quantity that Section 6's Lanczos quadrature
    approximates for one probe v.  log Q = U diag(log lambda) U^T with U the DCT-II (free) or the
    unitary DFT (periodic) eigenvectors, so v^T log(Q) v = sum_k log(lambda_k) |(U^T v)_k|^2."""
    shape = tuple(int(s) for s in shape)
    lam = lattice_spectrum(shape, order, kappa2, tau, boundary)
    V = np.asarray(v, dtype=np.float64).reshape(shape)
    if boundary == "periodic":
        c2 = np.abs(np.fft.fftn(V)) ** 2 / V.size
    else:
        c2 = _apply_axes(V, [dct2_matrix(N).T for N in shape]) ** 2
    return float(np.sum(np.log(lam) * c2))

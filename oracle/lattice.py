"""Explicit sparse lattice precision matrices (oracle side).

Section 2: a GMRF precision Q is sparse and only products Qv are needed.  Section 3
places the field on a regular lattice (a torus in the running example).  The operators
used throughout are

    first order   Q = tau * (kappa2 * I + L)
    second order  Q = tau * (kappa2 * I + L)^2

with L the graph Laplacian (degree minus adjacency) of the lattice graph: the grid graph
for a free boundary, the torus graph for a periodic one.  Lattice points are ordered
row-major, i = (i1 * N2 + i2) * N3 + i3.  The second-order operator is built as an explicit
sparse product, so on a free 2D N x N lattice it has the 13-point pattern.
"""
import numpy as np
import scipy.sparse as sp


def path_laplacian(N, periodic):
    """1D graph Laplacian of a path (free) or a cycle (periodic) with N nodes.

    The cycle is built edge by edge, so N = 2 gives a doubled edge and N = 1 a self loop
    (whose Laplacian is zero): the degree counts every edge end.
    """
    rows, cols = [], []
    n_edges = N if periodic else N - 1
    for e in range(n_edges):
        a, b = e, (e + 1) % N
        rows += [a, b]
        cols += [b, a]
    W = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N)).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    return (sp.diags(deg) - W).tocsr()


def lattice_laplacian(shape, boundary="free"):
    """Graph Laplacian of a 1D/2D/3D lattice as the Kronecker sum of path Laplacians."""
    periodic = boundary == "periodic"
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    L = sp.csr_matrix((n, n))
    for d, Nd in enumerate(shape):
        left = int(np.prod(shape[:d])) if d > 0 else 1
        right = int(np.prod(shape[d + 1:])) if d + 1 < len(shape) else 1
        term = sp.kron(sp.kron(sp.identity(left), path_laplacian(Nd, periodic)),
                       sp.identity(right))
        L = L + term
    return L.tocsr()


def lattice_precision(shape, order=1, kappa2=1.0, tau=1.0, boundary="free"):
    """Q = tau*(kappa2 I + L) for order 1, tau*(kappa2 I + L)^2 for order 2 (CSR, FP64)."""
    L = lattice_laplacian(shape, boundary)
    n = L.shape[0]
    K = (kappa2 * sp.identity(n) + L).tocsr()
    if order == 1:
        Q = tau * K
    elif order == 2:
        Q = tau * (K @ K)
    else:
        raise ValueError("order must be 1 or 2")
    Q = sp.csr_matrix(Q)
    Q.eliminate_zeros()
    Q.sort_indices()
    return Q


def poisson_dirichlet_2d(N):
    """The 5-point Dirichlet Laplacian on an N x N interior grid (4 on the diagonal, -1 to
    each neighbour).  Section 5.2 builds its test matrix as (31^2 * P_30)^2 from this
    operator with N = 30."""
    T = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    return (sp.kron(T, I) + sp.kron(I, T)).tocsr()


def section52_test_matrix():
    """Q = (31^2 P_30)^2 of Section 5.2 (n = 900): a second-order random walk on a 30 x 30
    lattice with a Dirichlet-type boundary that makes it proper."""
    P = 31.0 ** 2 * poisson_dirichlet_2d(30)
    return sp.csr_matrix(P @ P)

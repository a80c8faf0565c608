"""Pins for oracle.lattice and oracle.closed_form.

The builder (Kronecker sum of path Laplacians) is checked against a brute-force edge
enumeration of the lattice graph, against the entry pattern stated for the first-order
operator (Q_ii = kappa2 + degree, Q_ij = -1), against the 13-point count of the squared
free operator, and against its closed-form spectrum (path and cycle eigenvalues, Section 1's
diagonalisation of circulant matrices).  A mistake in any one of the three constructions
fails at least one of these.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import closed_form, dense, lattice


def brute_force_laplacian(shape, periodic):
    """Graph Laplacian by enumerating every lattice point and its +1 neighbour per axis."""
    shape = tuple(shape)
    n = int(np.prod(shape))
    L = np.zeros((n, n))
    idx = lambda c: int(np.ravel_multi_index(c, shape))
    for c in itertools.product(*[range(s) for s in shape]):
        for d in range(len(shape)):
            if c[d] + 1 < shape[d]:
                nb = list(c); nb[d] += 1
            elif periodic:
                nb = list(c); nb[d] = 0
            else:
                continue
            a, b = idx(c), idx(tuple(nb))
            L[a, a] += 1; L[b, b] += 1
            L[a, b] -= 1; L[b, a] -= 1
    return L


SHAPES = [(1,), (2,), (7,), (3, 4), (5, 5), (2, 6), (1, 5), (3, 2, 4), (4, 4, 4)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("boundary", ["free", "periodic"])
def test_laplacian_matches_edge_enumeration(shape, boundary):
    L = lattice.lattice_laplacian(shape, boundary).toarray()
    B = brute_force_laplacian(shape, boundary == "periodic")
    assert np.array_equal(L, B)


def test_first_order_entries_c0_statement():
    # Q_ii = kappa2 + degree, Q_ij = -1 on the free 4-neighbour lattice, tau = 1
    N, k2 = 6, 0.1
    Q = lattice.lattice_precision((N, N), 1, k2, 1.0, "free").toarray()
    for i1 in range(N):
        for i2 in range(N):
            i = i1 * N + i2
            deg = (i1 > 0) + (i1 < N - 1) + (i2 > 0) + (i2 < N - 1)
            assert Q[i, i] == pytest.approx(k2 + deg, abs=1e-15)
            nbs = [(i1 + a, i2 + b) for a, b in ((1, 0), (-1, 0), (0, 1), (0, -1))
                   if 0 <= i1 + a < N and 0 <= i2 + b < N]
            for (a, b) in nbs:
                assert Q[i, a * N + b] == -1.0
            assert np.count_nonzero(Q[i]) == 1 + len(nbs)


@pytest.mark.parametrize("N", [3, 4, 8, 17, 32])
def test_second_order_is_13_point(N):
    Q = lattice.lattice_precision((N, N), 2, 0.01, 1.0, "free")
    # pattern = ordered pairs of lattice points at L1 distance <= 2
    pairs = sum(1 for a in range(N) for b in range(N) for c in range(N) for d in range(N)
                if abs(a - c) + abs(b - d) <= 2)
    assert Q.nnz == pairs
    if N >= 4:
        assert Q.nnz == 13 * N * N - 20 * N + 4
    if N >= 5:
        assert np.diff(Q.indptr).max() == 13
    # symmetric
    assert abs(Q - Q.T).max() == 0


@pytest.mark.parametrize("order,boundary", [(1, "free"), (2, "free"), (1, "periodic"), (2, "periodic")])
def test_constant_vector_eigenpair(order, boundary):
    # L 1 = 0 so Q 1 = tau kappa2 1 (order 1) or tau kappa2^2 1 (order 2)
    Q = lattice.lattice_precision((5, 7), order, 0.3, 2.0, boundary)
    one = np.ones(35)
    expect = 2.0 * (0.3 if order == 1 else 0.09)
    assert np.allclose(Q @ one, expect * one, rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(9,), (6, 5), (8, 8), (3, 4, 5)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("boundary", ["free", "periodic"])
def test_closed_form_spectrum(shape, order, boundary):
    Q = lattice.lattice_precision(shape, order, 0.07, 1.3, boundary)
    lam = np.sort(np.linalg.eigvalsh(Q.toarray()))
    cf = np.sort(closed_form.lattice_spectrum(shape, order, 0.07, 1.3, boundary).ravel())
    assert np.allclose(lam, cf, rtol=1e-12, atol=1e-12 * lam.max())


@pytest.mark.parametrize("N", [1, 2, 5, 16])
def test_dct2_is_orthonormal_eigenbasis(N):
    U = closed_form.dct2_matrix(N)
    assert np.allclose(U.T @ U, np.eye(N), atol=1e-14)
    L = lattice.path_laplacian(N, False).toarray()
    mu = closed_form.path_spectrum(N, False)
    assert np.allclose(L @ U, U * mu, atol=1e-13)


def test_section52_matrix_dirichlet_spectrum():
    # P_30: 5-point Dirichlet Laplacian, eigenvalues 4 - 2cos(pi k/31) - 2cos(pi l/31)
    P = lattice.poisson_dirichlet_2d(30).toarray()
    assert P[0, 0] == 4 and P[0, 1] == -1 and P[0, 30] == -1
    k = np.arange(1, 31)
    ev = (2 - 2 * np.cos(np.pi * k / 31))[:, None] + (2 - 2 * np.cos(np.pi * k / 31))[None, :]
    assert np.allclose(np.sort(np.linalg.eigvalsh(P)), np.sort(ev.ravel()), atol=1e-12)
    Q = lattice.section52_test_matrix()
    assert Q.shape == (900, 900)
    lam = np.sort(np.linalg.eigvalsh(Q.toarray()))
    assert np.allclose(lam, np.sort((961.0 * ev.ravel()) ** 2), rtol=1e-10)

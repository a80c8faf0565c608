"""Pins for the coloured Hutchinson estimator of Section 6.1 (oracle.logdet).

  * The colouring separates every pair of nodes within p steps of each other in the graph of Q
    (brute-force breadth-first distances), and first fit on the 5-point lattice with p = 1 is the
    checkerboard.
  * One colour is the plain estimator; one colour per node is exact (each class a single +-e_i,
    so the estimate is sum_i B_ii = log det Q with no variance).
  * At m = n the quadrature of each class is exact: the estimate equals sum_c v_c^T B v_c.
  * Unbiased within four standard errors, and the empirical variance of one coloured probe matches
    2 sum_c sum_{i != j in c} B_ij^2; on Section 5.2's matrix (Figure 4) that variance falls as p
    grows from 0 to 3.
"""
from collections import deque

import numpy as np
import pytest

from oracle import dense, lattice, logdet, philox


def _bfs_dist(Q, s):
    Q = Q.tocsr()
    dist = {s: 0}
    dq = deque([s])
    while dq:
        i = dq.popleft()
        for j in Q.indices[Q.indptr[i]:Q.indptr[i + 1]]:
            if j not in dist:
                dist[j] = dist[i] + 1
                dq.append(j)
    return dist


@pytest.mark.parametrize("shape,order,bc,p", [((7, 9), 1, "free", 1), ((7, 9), 2, "free", 1), ((6, 8), 1, "periodic", 2),
                                             ((5, 6), 2, "free", 2), ((4, 4, 4), 1, "free", 2), ((12,), 2, "periodic", 3)])
def test_colouring_separates_within_p(shape, order, bc, p):
    Q = lattice.lattice_precision(shape, order, 0.3, 1.0, bc)
    col = logdet.distance_colouring(Q, p)
    n = Q.shape[0]
    for s in range(n):
        for t, d in _bfs_dist(Q, s).items():
            if t != s and d <= p:
                assert col[s] != col[t], (s, t, d)


def test_checkerboard():
    shape = (6, 7)
    Q = lattice.lattice_precision(shape, 1, 0.3, 1.0, "free")
    col = logdet.distance_colouring(Q, 1).reshape(shape)
    i1, i2 = np.meshgrid(np.arange(6), np.arange(7), indexing="ij")
    assert np.array_equal(col, (i1 + i2) % 2)


def test_single_colour_is_plain_hutchinson():
    Q = lattice.lattice_precision((6, 6), 2, 0.2, 1.0, "free")
    mv = lambda v: Q @ v
    plain = logdet.hutchinson(mv, 36, 5, 20, seed=9)
    col = logdet.hutchinson_coloured(mv, 36, np.zeros(36, dtype=int), 5, 20, seed=9)
    assert np.allclose(col.per_probe, plain.per_probe, rtol=1e-14, atol=0)


def test_one_colour_per_node_is_exact():
    Q = lattice.lattice_precision((4, 5), 1, 0.4, 1.0, "free")
    res = logdet.hutchinson_coloured(lambda v: Q @ v, 20, np.arange(20), 3, 20, seed=1)
    exact = dense.cholesky_logdet(Q)
    assert np.allclose(res.per_probe, exact, rtol=1e-12)
    assert res.std_err < 1e-12 * abs(exact)


def test_full_dimension_quadrature_is_the_coloured_form():
    Q = lattice.lattice_precision((5, 5), 2, 0.2, 1.0, "free")
    B = dense.log_matrix(Q)
    col = logdet.distance_colouring(Q, 1)
    v = philox.rademacher_probes(4, 1, 25)[:, 0]
    res = logdet.hutchinson_coloured(lambda x: Q @ x, 25, col, 1, 25, seed=4)
    want = sum(np.where(col == c, v, 0.0) @ B @ np.where(col == c, v, 0.0) for c in range(col.max() + 1))
    assert res.per_probe[0] == pytest.approx(want, rel=1e-10)


def test_variance_falls_with_p_on_section52_matrix():
    # Figure 4's matrix: the exact variance of one coloured probe for the uncoloured, 1-, 2- and
    # 3-coloured estimators
    Q = lattice.section52_test_matrix()
    B = dense.log_matrix(Q)
    var = [logdet.coloured_variance(B, logdet.distance_colouring(Q, p)) for p in (0, 1, 2, 3)]
    assert var[0] > var[1] > var[2] > var[3] > 0


def test_coloured_unbiased_and_variance():
    Q = lattice.lattice_precision((10, 10), 2, 0.5, 1.0, "free")
    n = Q.shape[0]
    B = dense.log_matrix(Q)
    exact = dense.cholesky_logdet(Q)
    col = logdet.distance_colouring(Q, 1)
    res = logdet.hutchinson_coloured(lambda v: Q @ v, n, col, 300, 40, seed=21)
    assert abs(res.logdet - exact) < 4 * res.std_err
    assert np.var(res.per_probe, ddof=1) == pytest.approx(logdet.coloured_variance(B, col), rel=0.25)

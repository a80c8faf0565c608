"""GPU parity of the coloured Hutchinson estimator (Section 6.1) through the C ABI.

  * gmrf_distance_colouring equals the oracle's first-fit colouring of the graph of Q^p exactly
    (integer output, bit-exact) on lattices (free and periodic, orders 1 and 2, 1D/2D/3D) and on
    Section 5.2's CSR matrix.
  * gmrf_logdet_coloured with the oracle's colouring matches the oracle's coloured estimator probe
    by probe (FP64 1e-10, FP32 1e-5 relative), plain and preconditioned (Section 6.2).
  * One colour reproduces gmrf_logdet bit for bit; a colour out of range is rejected.
"""
import numpy as np
import pytest

from oracle import lattice, logdet, precond

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import os
    import torch
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1312_1476_amd as gm
    return gm


LATTICES = [((9, 11), 1, "free"), ((9, 11), 2, "free"), ((8, 12), 1, "periodic"), ((10, 10), 2, "periodic"),
            ((5, 6, 7), 1, "free"), ((30,), 2, "periodic")]


@pytest.mark.parametrize("lat", LATTICES, ids=lambda l: f"{l[0]}-o{l[1]}-{l[2]}")
@pytest.mark.parametrize("p", [1, 2, 3])
def test_distance_colouring_matches_oracle(gm, lat, p):
    shape, order, bc = lat
    op = gm.Operator.lattice(shape, order, 0.3, 1.0, bc)
    Q = lattice.lattice_precision(shape, order, 0.3, 1.0, bc)
    assert np.array_equal(op.distance_colouring(p), logdet.distance_colouring(Q, p))


@pytest.mark.parametrize("p", [0, 1, 2])
def test_distance_colouring_csr(gm, p):
    Q = lattice.section52_test_matrix()
    op = gm.Operator.csr(Q.shape[0], Q.indptr, Q.indices, Q.data)
    assert np.array_equal(op.distance_colouring(p), logdet.distance_colouring(Q, p))


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("p", [1, 2])
def test_coloured_logdet_matches_oracle(gm, storage, tol, p):
    shape, order, k2, npb, m, seed = (12, 12), 2, 0.3, 4, 30, 99
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    col = logdet.distance_colouring(Q, p)
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", storage)
    mean, se, per = op.logdet_coloured(npb, m, col, seed=seed)
    ref = logdet.hutchinson_coloured(lambda v: Q @ v, Q.shape[0], col, npb, m, seed=seed)
    assert np.all(np.abs(per - ref.per_probe) <= tol * np.abs(ref.per_probe))
    assert abs(mean - ref.logdet) <= tol * abs(ref.logdet)
    assert abs(se - ref.std_err) <= 1e-6 * abs(ref.logdet) + tol * ref.std_err


def test_coloured_logdet_preconditioned(gm):
    shape, order, k2, npb, m, seed = (16, 16), 2, 0.05, 3, 40, 5
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    col = logdet.distance_colouring(Q, 1)
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", "f64").set_circulant_precond()
    mean, se, per = op.logdet_coloured(npb, m, col, seed=seed)
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, 1.0)
    A = precond.preconditioned_operator(Q, shape, mult)
    ref = logdet.hutchinson_coloured(A, Q.shape[0], col, npb, m, seed=seed,
                                     shift=precond.logdet_M(shape, order, k2, 1.0))
    assert np.all(np.abs(per - ref.per_probe) <= 1e-10 * np.abs(ref.per_probe))


def test_single_colour_is_plain(gm):
    shape, npb, m = (20, 24), 6, 25
    op = gm.Operator.lattice(shape, 2, 0.2, 1.0, "free", "f64")
    mean0, se0, per0 = op.logdet(npb, m, seed=3)
    mean1, se1, per1 = op.logdet_coloured(npb, m, np.zeros(shape[0] * shape[1], dtype=np.int32), seed=3)
    assert np.array_equal(per0, per1) and mean0 == mean1


def test_colour_out_of_range(gm):
    op = gm.Operator.lattice((8, 8), 1, 0.2, 1.0, "free")
    col = np.zeros(64, dtype=np.int32)
    col[5] = -1
    with pytest.raises(gm.GmrfError):
        op.logdet_coloured(2, 10, col)

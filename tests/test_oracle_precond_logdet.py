"""Pins for oracle.precond (Proposition 1, Section 5.1) and oracle.logdet (Section 6).

  * The FFT multiplier M^{-1/2} equals the dense principal inverse root of the assembled
    periodic operator.
  * Proposition 1: S = M^{-1/2} A^{-1/2} with A = M^{-1/2} Q M^{-1/2} satisfies
    S S^T = Q^{-1}; the preconditioned sampler at m = n equals S z.
  * A perfect preconditioner (M = Q) collapses to one step and the direct sample.
  * Section 5.1's count: Algorithm 1 on A costs four FFTs per step (24 for 6 steps), with
    one more pair for the back-transform (fixture tests/golden/fft_count.txt).
  * Section 6.2 split, sign corrected: log det A + log det M = log det Q, and the printed
    sign is off by 2 log det M.
  * Quadrature at m = n equals v^T log(Q) v; the Hutchinson mean lies within 4 standard
    errors of the exact log det; the Rademacher variance is 2 sum_{i != j} B_ij^2.
  * Philox4x64-10 equals numpy's independent implementation (numpy.random.Philox), and the
    probe rule picks bits as documented.
"""
import os

import numpy as np
import pytest

from oracle import closed_form, dense, lanczos, lattice, logdet, philox, precond

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("shape,order", [((8, 8), 1), ((8, 8), 2), ((4, 6), 2), ((4, 4, 4), 1)])
def test_fft_multiplier_is_dense_inverse_root(shape, order):
    M = lattice.lattice_precision(shape, order, 0.2, 1.7, "periodic")
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, 0.2, 1.7)
    v = np.random.default_rng(0).standard_normal(M.shape[0])
    assert np.allclose(precond.apply_inv_sqrt_M(shape, mult, v), dense.inv_sqrt_apply(M, v), atol=1e-12)


def _dense_A(Q, shape, mult):
    n = Q.shape[0]
    op = precond.preconditioned_operator(Q, shape, mult)
    return np.column_stack([op(e) for e in np.eye(n)])


@pytest.mark.parametrize("order", [1, 2])
def test_proposition1_factor(order):
    shape, k2 = (6, 8), 0.1
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, 1.0)
    A = _dense_A(Q, shape, mult)
    Minv = dense.inv_sqrt_matrix(lattice.lattice_precision(shape, order, k2, 1.0, "periodic"))
    S = Minv @ dense.inv_sqrt_matrix(A)
    Qinv = np.linalg.inv(Q.toarray())
    assert np.linalg.norm(S @ S.T - Qinv) / np.linalg.norm(Qinv) < 1e-11
    z = np.random.default_rng(2).standard_normal(48)
    res = precond.sample(Q, shape, order, k2, 1.0, z, 48, tol=0.0, reorth=True)
    assert np.linalg.norm(res.x - S @ z) / np.linalg.norm(S @ z) < 1e-10


def test_perfect_preconditioner_collapses():
    shape, k2 = (8, 8), 0.3
    Q = lattice.lattice_precision(shape, 2, k2, 1.0, "periodic")
    z = np.random.default_rng(4).standard_normal(64)
    res = precond.sample(Q, shape, 2, k2, 1.0, z, 10, tol=1e-10)
    assert res.m == 1
    x = dense.inv_sqrt_apply(Q, z)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-13


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = line.split("=")
                out[key.strip()] = val.strip()
    return out


def test_fft_count_per_iteration(monkeypatch):
    g = _read_golden("fft_count.txt")
    iters, ffts = int(g["iterations"]), int(g["ffts"])
    calls = {"fft": 0}
    real_fftn, real_ifftn = np.fft.fftn, np.fft.ifftn

    def cfft(*a, **k):
        calls["fft"] += 1
        return real_fftn(*a, **k)

    def cifft(*a, **k):
        calls["fft"] += 1
        return real_ifftn(*a, **k)

    monkeypatch.setattr(np.fft, "fftn", cfft)
    monkeypatch.setattr(np.fft, "ifftn", cifft)
    shape = (16, 16)
    Q = lattice.lattice_precision(shape, 2, 0.1, 1.0, "free")
    z = np.random.default_rng(0).standard_normal(256)
    res = precond.sample(Q, shape, 2, 0.1, 1.0, z, iters, tol=0.0)
    assert res.m == iters
    assert calls["fft"] == ffts + 2      # plus one FFT pair for x = M^{-1/2} u_m


@pytest.mark.parametrize("order", [1, 2])
def test_preconditioned_logdet_split_sign(order):
    shape, k2 = (6, 6), 0.08
    Q = lattice.lattice_precision(shape, order, k2, 1.0, "free")
    mult = precond.circulant_inv_sqrt_multiplier(shape, order, k2, 1.0)
    A = _dense_A(Q, shape, mult)
    ldA = np.linalg.slogdet(A)[1]
    ldM = precond.logdet_M(shape, order, k2, 1.0)
    ldQ = dense.cholesky_logdet(Q)
    assert ldA + ldM == pytest.approx(ldQ, rel=1e-12)
    # the printed "- 2 log det F" is off by exactly 2 log det M
    assert abs((ldA - ldM) - ldQ) == pytest.approx(2 * abs(ldM), rel=1e-9)


def test_quadrature_full_dimension_is_quadratic_form():
    Q = lattice.lattice_precision((5, 5), 2, 0.2, 1.0, "free")
    B = dense.log_matrix(Q)
    v = philox.rademacher_probe(123, 0, 25)
    g, m = logdet.quadrature(lambda x: Q @ x, v, 25)
    assert g == pytest.approx(v @ B @ v, rel=1e-10, abs=1e-10)


def test_hutchinson_unbiased_within_se():
    shape, k2 = (8, 8), 0.2
    Q = lattice.lattice_precision(shape, 1, k2, 1.0, "free")
    res = logdet.hutchinson_csr(Q, 400, 30, seed=77)
    exact = closed_form.exact_logdet(shape, 1, k2, 1.0, "free")
    assert abs(res.logdet - exact) < 4 * res.std_err


def test_hutchinson_variance_factor_two():
    Q = lattice.lattice_precision((4, 4), 1, 0.3, 1.0, "free")
    B = dense.log_matrix(Q)
    res = logdet.hutchinson_csr(Q, 4000, 16, seed=5)
    off = B - np.diag(np.diag(B))
    var_theory = 2.0 * np.sum(off ** 2)
    var_emp = np.var(res.per_probe, ddof=1)
    # chi-square-like spread of the sample variance at N = 4000: a few percent
    assert var_emp == pytest.approx(var_theory, rel=0.1)
    # the printed Gaussian-probe form ||B||_F^2 - tr(B)^2 is not the Rademacher variance
    assert abs(var_emp - (np.sum(B ** 2) - np.trace(B) ** 2)) > 0.5 * var_theory


def test_preconditioned_hutchinson_within_se():
    shape, k2 = (8, 8), 0.1
    Q = lattice.lattice_precision(shape, 2, k2, 1.0, "free")
    res = logdet.hutchinson_preconditioned(Q, shape, 2, k2, 1.0, 200, 40, seed=3)
    exact = closed_form.exact_logdet(shape, 2, k2, 1.0, "free")
    assert abs(res.logdet - exact) < 4 * res.std_err + 1e-9


@pytest.mark.parametrize("ctr,key", [
    ((5, 7, 11, 13), (17, 19)),
    ((2 ** 63 + 3, 2 ** 64 - 1, 123456789, 42), (2 ** 64 - 5, 99)),
    ((1, 0, 0, 0), (0, 0)),
    ((2 ** 40 + 1, 2 ** 33, 2 ** 64 - 2, 2 ** 62), (0xDEADBEEFCAFEBABE, 2 ** 64 - 1)),
])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox increments its counter before each block: start one below
    bg = np.random.Philox(counter=np.array([ctr[0] - 1, ctr[1], ctr[2], ctr[3]], dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    ref = [int(x) for x in bg.random_raw(4)]
    mine = philox.philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
    assert ref == [int(x) for x in mine]


def test_probe_rule_bits():
    # Each probe bit is read straight from numpy's Philox stream: numpy adds one to the
    # counter (with carry) before each block, so block b of probe p starts from
    # (b - 1, p) or, for b = 0, from (2^64 - 1, p - 1).
    seed, p, n = 987654321, 5, 700
    v = philox.rademacher_probe(seed, p, n)
    for i in [0, 1, 63, 64, 200, 255, 256, 511, 699]:
        b, t = i // 256, i % 256
        start = [b - 1, p, 0, 0] if b > 0 else [2 ** 64 - 1, p - 1, 0, 0]
        bg = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                              key=np.array([seed, 0], dtype=np.uint64))
        words = [int(x) for x in bg.random_raw(4)]
        bit = (words[t // 64] >> (t % 64)) & 1
        assert v[i] == (1.0 if bit == 0 else -1.0)
    assert set(np.unique(v)) <= {-1.0, 1.0}
    big = philox.rademacher_probe(seed, 0, 200000)
    assert abs(big.mean()) < 4.0 / np.sqrt(200000)

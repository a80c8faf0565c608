"""Autotuner (gmrf_autotune and the tuning table), through the C ABI.

The tuner chooses launch options that change no result bit: the tile order (linear or XCD-contiguous),
the store policy (ordinary or non-temporal) and, for the SpMM alone, its tile shape (rows per wave,
columns per lane).  So every option set must give bitwise-identical
outputs -- the SpMM, the one-pass Lanczos sampler (coefficients and samples), and a field sampled
alone versus inside an uneven batch -- and the table must round-trip through its JSON form.
"""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ALL_OPTIONS = (0, 1, 2, 3)
SPMM_OPTIONS = tuple(range(64))       # with every tile shape code (rows per wave, columns per lane)


@pytest.fixture(scope="module")
def gm():
    import torch
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1312_1476_amd as gm
    yield gm
    gm.clear_tune()


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).to("cuda:0")


def _set(gm, kernel, op, k, bits):
    """Table entry for (kernel, op's key, k) = bits."""
    from paper_1312_1476_amd import _abi
    import ctypes as C
    cl = lambda v: int(np.ceil(np.log2(v))) if v > 1 else 0
    n1, n2 = op.shape
    e = (C.c_int32 * 7)(gm.TUNE_KERNELS.index(kernel), op.order_, op.storage, cl(n1), cl(n2), cl(k), bits)
    _abi.check(_abi.lib().gmrf_tune_import(e, 1), "gmrf_tune_import")


def _op(gm, shape, order, storage, k2=0.05):
    op = gm.Operator.lattice(shape, order, k2, 1.0, "free", storage)
    op.order_ = order
    return op


@pytest.mark.parametrize("shape,order,storage", [((512, 512), 2, "f64"), ((512, 512), 2, "f32"),
                                                 ((1024, 1024), 1, "f32"), ((100, 76), 2, "f64"),
                                                 ((37, 64), 1, "f32")])
def test_spmm_bitwise_under_every_option(gm, shape, order, storage):
    import torch
    gm.clear_tune()
    k = 5
    op = _op(gm, shape, order, storage)
    dt = torch.float64 if storage == "f64" else torch.float32
    X = _t(np.random.default_rng(11).standard_normal((k, shape[0] * shape[1])), dt)
    ref = op.apply(X).clone()
    for bits in SPMM_OPTIONS:
        _set(gm, "spmv", op, k, bits)
        assert torch.equal(op.apply(X), ref), bits
    gm.clear_tune()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_one_pass_sampler_bitwise_under_every_option(gm, storage):
    import torch
    gm.clear_tune()
    shape, k = (200, 136), 3
    op = _op(gm, shape, 2, storage, 0.1)
    Z = _t(workloads.gaussian_block(shape[0] * shape[1], k, 93, 0).T)
    X0, i0, a0, b0 = op.sample(Z, tol=1e-6, m_max=300, coeffs=True)
    for bits in ALL_OPTIONS:
        _set(gm, "lz2d", op, k, bits)
        X, info, a, b = op.sample(Z, tol=1e-6, m_max=300, coeffs=True)
        assert torch.equal(X, X0) and np.array_equal(a, a0) and np.array_equal(b, b0), bits
        assert [d["m_used"] for d in info] == [d["m_used"] for d in i0]
    gm.clear_tune()


def test_autotune_records_choices_and_batch_stays_bitwise(gm, tmp_path):
    import torch
    gm.clear_tune()
    specs = [((64, 64), 0.2), ((96, 80), 0.05), ((128, 128), 0.01)]
    ops = [_op(gm, sh, 1, "f32", k2) for sh, k2 in specs]
    Zs = [_t(workloads.gaussian_block(sh[0] * sh[1], 4, 93, 1 + f).T) for f, (sh, _) in enumerate(specs)]
    alone0 = [op.sample(Z, tol=1e-5, m_max=400)[0] for op, Z in zip(ops, Zs)]
    Xb0, _ = gm.sample_batch(ops, Zs, tol=1e-5, m_max=400)
    for op in ops:
        ch = gm.autotune(op, 4, reps=3)
        assert set(ch) == {"spmv", "lz2d"} and all(isinstance(v, list) for v in ch.values())
    table = gm.tune_table()
    assert len(table) >= 2 and all(r["options"] is not None for r in table)
    for op, Z, X0 in zip(ops, Zs, alone0):
        assert torch.equal(op.sample(Z, tol=1e-5, m_max=400)[0], X0)
    Xb, _ = gm.sample_batch(ops, Zs, tol=1e-5, m_max=400)
    for f in range(len(ops)):
        assert torch.equal(Xb[f], Xb0[f]) and torch.equal(Xb[f], alone0[f])
    # JSON round trip
    path = str(tmp_path / "tune.json")
    gm.save_tune(path)
    gm.clear_tune()
    assert gm.tune_table() == []
    gm.load_tune(path)
    assert gm.tune_table() == table
    assert json.load(open(path)) == table
    gm.clear_tune()


def test_tune_import_rejects_invalid_entries(gm):
    import ctypes as C
    from paper_1312_1476_amd import _abi
    gm.clear_tune()
    bad = (C.c_int32 * 7)(0, 2, 0, 9, 9, 5, 64)       # option bit 64 does not exist
    assert _abi.lib().gmrf_tune_import(bad, 1) == _abi.GMRF_EINVAL
    bad1 = (C.c_int32 * 7)(1, 2, 0, 9, 9, 5, 4)       # tile shapes are for the SpMM alone
    assert _abi.lib().gmrf_tune_import(bad1, 1) == _abi.GMRF_EINVAL
    bad2 = (C.c_int32 * 7)(5, 2, 0, 9, 9, 5, 1)       # no kernel 5
    assert _abi.lib().gmrf_tune_import(bad2, 1) == _abi.GMRF_EINVAL
    assert gm.tune_table() == []
    # a CSR operator is left untuned
    op = gm.Operator.csr(3, [0, 1, 2, 3], [0, 1, 2], [2.0, 2.0, 2.0])
    assert gm.autotune(op, 1) == {"spmv": None, "lz2d": None}

"""Uneven batches (gmrf_sample_batch): many independent lattice fields of different sizes and
kappa2 in one set of launches per Lanczos step.

  * every field's result is bitwise identical to the same field sampled on its own, and
    matches the oracle at the same Krylov dimension (FP64 1e-8, FP32 1e-5);
  * incompatible fields are rejected;
  * the uneven-batch workload at its real shape (256 fields, side uniform in 32..256,
    kappa2 log-uniform in [1e-3, 1], 8 right-hand sides each), sampled fields vs the oracle.
"""
import numpy as np
import pytest

import workloads
from oracle import lanczos, lattice

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


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("storage,tol_par", [("f64", 1e-8), ("f32", 1e-5)])
def test_batch_matches_single_and_oracle(gm, storage, tol_par):
    rng = np.random.default_rng(2024)
    specs = []
    for f in range(12):
        s1, s2 = int(rng.integers(17, 97)), int(rng.integers(17, 97))
        k2 = float(10 ** rng.uniform(-1.0, 0.0)) if storage == "f32" else float(10 ** rng.uniform(-3.0, 0.0))
        specs.append(((s1, s2), k2, 1 + f % 3))
    ops = [gm.Operator.lattice(sh, 1, k2, 1.0, "free", storage) for sh, k2, _ in specs]
    Zs = [workloads.gaussian_block(sh[0] * sh[1], k, 94, f) for f, (sh, k2, k) in enumerate(specs)]
    Xs, info = gm.sample_batch(ops, [_t(Z.T) for Z in Zs], tol=1e-7, m_max=600)
    col = 0
    for f, ((sh, k2, k), op, Z) in enumerate(zip(specs, ops, Zs)):
        Xb = Xs[f].cpu().numpy()
        Xa, ia = op.sample(_t(Z.T), tol=1e-7, m_max=600)
        assert np.array_equal(Xb, Xa.cpu().numpy()), f
        nan = lambda d: {kk: ("nan" if isinstance(v, float) and v != v else v) for kk, v in d.items()}
        assert [nan(info[col + r]) for r in range(k)] == [nan(d) for d in ia]
        Q = lattice.lattice_precision(sh, 1, k2, 1.0, "free")
        for r in range(k):
            m = info[col + r]["m_used"]
            ref = lanczos.sample_csr(Q, Z[:, r], m, tol=0.0)
            assert _rel(Xb[r], ref.x) <= tol_par, (f, r, _rel(Xb[r], ref.x))
        col += k


@pytest.mark.parametrize("storage,tol_par", [("f64", 1e-8), ("f32", 1e-5)])
def test_batch_of_3d_fields(gm, storage, tol_par):
    """3D first-order fields in one batch: small ones (box tiles) and, separately, fields of 2^20 points
    and more (z-marching kernel, each block taking its lane width from its own field: odd and even row
    lengths mixed).  Each field bitwise equal to the field alone and within tol of the oracle at its m."""
    groups = [[((9, 10, 11), 0.2, 2), ((12, 8, 16), 0.05, 1), ((7, 7, 7), 0.5, 3)],
              [((34, 181, 175), 0.3, 2), ((17, 256, 256), 0.1, 1), ((64, 128, 130), 0.5, 1)]]
    for gi, specs in enumerate(groups):
        ops = [gm.Operator.lattice(sh, 1, k2, 1.0, "free", storage) for sh, k2, _ in specs]
        Zs = [workloads.gaussian_block(int(np.prod(sh)), k, 95, 10 * gi + f) for f, (sh, k2, k) in enumerate(specs)]
        Xs, info = gm.sample_batch(ops, [_t(Z.T) for Z in Zs], tol=1e-7, m_max=300)
        col = 0
        for f, ((sh, k2, k), op, Z) in enumerate(zip(specs, ops, Zs)):
            Xb = Xs[f].cpu().numpy()
            Xa, ia = op.sample(_t(Z.T), tol=1e-7, m_max=300)
            assert np.array_equal(Xb, Xa.cpu().numpy()), (gi, f)
            Q = lattice.lattice_precision(sh, 1, k2, 1.0, "free")
            for r in range(k):
                m = info[col + r]["m_used"]
                assert info[col + r]["status"] == "OK" and m == ia[r]["m_used"]
                ref = lanczos.sample_csr(Q, Z[:, r], m, tol=0.0)
                assert _rel(Xb[r], ref.x) <= tol_par, (gi, f, r, _rel(Xb[r], ref.x))
            col += k
        for op in ops:
            op.close()
    # a batch mixing the two kernels is refused
    a = gm.Operator.lattice((9, 10, 11), 1, 0.2, 1.0, "free", storage)
    b = gm.Operator.lattice((17, 256, 256), 1, 0.1, 1.0, "free", storage)
    with pytest.raises(gm.GmrfError):
        gm.sample_batch([a, b], [_t(np.ones((1, a.n))), _t(np.ones((1, b.n)))])


def test_batch_rejects_incompatible(gm):
    a = gm.Operator.lattice((16, 16), 1, 0.1)
    b = gm.Operator.lattice((16, 16), 2, 0.1)
    Z = [_t(np.ones((1, 256))), _t(np.ones((1, 256)))]
    with pytest.raises(gm.GmrfError):
        gm.sample_batch([a, b], Z)
    c = gm.Operator.lattice((16, 16), 1, 0.1).set_circulant_precond()
    with pytest.raises(gm.GmrfError):
        gm.sample_batch([a, c], Z)


def test_uneven_batch_workload_full_size(gm):
    """FP64 storage so that the stored Krylov basis of all 2048 columns (about 0.4 GB per
    slot) fits for m_max = 400.  Converged columns: 1e-8 against the oracle at the same m;
    columns that stop at m_max (the smallest kappa2, cond(Q) ~ 8e3): truncation level 10 rho."""
    fields = workloads.uneven_fields()
    ops = [gm.Operator.lattice((s, s), 1, k2, 1.0, "free", "f64") for s, k2 in fields]
    Zs = [workloads.uneven_field_rhs(f, s) for f, (s, _) in enumerate(fields)]
    Xs, info = gm.sample_batch(ops, [_t(Z.T) for Z in Zs], tol=1e-6, m_max=400)
    assert len(info) == 8 * len(fields)
    assert all(i["status"] in ("OK", "ENOCONV") for i in info)
    order = np.argsort([k2 for _, k2 in fields])
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    for f in picks:
        s, k2 = fields[f]
        Q = lattice.lattice_precision((s, s), 1, k2, 1.0, "free")
        X = Xs[f].cpu().numpy()
        for r in (0, 7):
            i = info[8 * f + r]
            ref = lanczos.sample_csr(Q, Zs[f][:, r], i["m_used"], tol=0.0)
            tol = 1e-8 if i["status"] == "OK" else 10 * ref.rho[-1]
            assert _rel(X[r], ref.x) <= tol, (f, r, _rel(X[r], ref.x), i)


def test_batch_edge_columns(gm):
    """Columns that stop at the first step inside a batch: a zero right-hand side (m = 0, x = 0) and a
    non-finite one (EINVAL, NaN). The other columns keep running on the shrinking (column, tile) list and
    equal the same fields sampled on their own, bit for bit."""
    import torch
    specs = [((20, 20), 0.3), ((33, 17), 0.05), ((64, 64), 0.01)]
    ops = [gm.Operator.lattice(sh, 1, k2, 1.0, "free", "f64") for sh, k2 in specs]
    Zs = [workloads.gaussian_block(sh[0] * sh[1], 2, 95, f) for f, (sh, _) in enumerate(specs)]
    Zs[1][:, 0] = 0.0
    Zs[2][7, 1] = np.nan
    Xs, info = gm.sample_batch(ops, [_t(Z.T) for Z in Zs], tol=1e-8, m_max=400)
    assert info[2]["status"] == "OK" and info[2]["m_used"] == 0
    assert torch.all(Xs[1][0] == 0)
    assert info[5]["status"] == "EINVAL" and torch.all(torch.isnan(Xs[2][1]))
    for f, (op, Z) in enumerate(zip(ops, Zs)):
        Xa, ia = op.sample(_t(Z.T), tol=1e-8, m_max=400)
        for r in range(2):
            c = 2 * f + r
            if c in (2, 5):
                continue
            assert info[c]["status"] == "OK" and info[c]["m_used"] == ia[r]["m_used"]
            assert torch.equal(Xs[f][r], Xa[r]), (f, r)


@pytest.mark.timeout(600)
def test_uneven_batch_workload_fp32_as_benchmarked(gm):
    """The uneven batch exactly as the benchmark runs it: 256 fields, 8 right-hand sides each, FP32
    storage with FP64 scalars, stop at rho <= 1e-5, m_max = 600.  Every column converges.  Eight fields
    across the kappa2 range (the smallest kappa2 = 1e-3 end included, cond(Q) ~ 8e3) x columns 0 and 7
    equal the FP64 oracle at the same m within the FP32 tolerance 1e-5."""
    fields = workloads.uneven_fields()
    ops = [gm.Operator.lattice((s, s), 1, k2, 1.0, "free", "f32") for s, k2 in fields]
    Zs = [workloads.uneven_field_rhs(f, s) for f, (s, _) in enumerate(fields)]
    Xs, info = gm.sample_batch(ops, [_t(Z.T) for Z in Zs], tol=1e-5, m_max=600)
    assert all(i["status"] == "OK" for i in info), [i for i in info if i["status"] != "OK"][:4]
    order = np.argsort([k2 for _, k2 in fields])
    picks = [int(order[(len(order) - 1) * q // 7]) for q in range(8)]
    worst = 0.0
    for f in picks:
        s, k2 = fields[f]
        Q = lattice.lattice_precision((s, s), 1, k2, 1.0, "free")
        X = Xs[f].cpu().numpy()
        for r in (0, 7):
            ref = lanczos.sample_csr(Q, Zs[f][:, r], info[8 * f + r]["m_used"], tol=0.0)
            e = _rel(X[r].astype(np.float64), ref.x)
            worst = max(worst, e)
            assert e <= 1e-5, (f, s, k2, r, info[8 * f + r], e)
    print(f"uneven batch FP32 vs oracle: worst rel err {worst:.2e} over {2 * len(picks)} columns")
    for op in ops:
        op.close()

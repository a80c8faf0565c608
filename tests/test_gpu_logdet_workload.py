"""The Hutchinson log-det workload (Section 6) at its real shape: 1024 x 1024 lattice,
second-order Q with kappa2 = 0.05, 64 Rademacher probes, m = 80 Lanczos steps, FP32 storage
with FP64 scalars.  Checked against
  * the oracle per probe (two probes at full size, same probe rule), FP32 tolerance 1e-5;
  * the closed-form log det of the periodic (block-circulant) version (DFT eigenvalues),
    statistically: |mean - exact| < 5 standard errors;
  * the free-boundary closed form (DCT eigenvalues), statistically;
  * the oracle on the 128 x 128 subgrid, every probe, FP32 1e-5 and FP64 1e-10.
"""
import numpy as np
import pytest

import workloads
from oracle import closed_form, lattice, logdet

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


def test_logdet_full_size_free(gm):
    sp, npb, m, seed = workloads.C3_LATTICE, workloads.C3_PROBES, workloads.C3_M, workloads.c3_probe_seed()
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f32")
    mean, se, per = op.logdet(npb, m, seed=seed)
    exact = closed_form.exact_logdet(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    assert abs(mean - exact) < 5 * se, (mean, exact, se)
    Q = lattice.lattice_precision(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    from oracle import philox
    for p in (0, npb - 1):
        v = philox.rademacher_probe(seed, p, sp.n)
        g, _ = logdet.quadrature(lambda x: Q @ x, v, m)
        assert abs(per[p] - g) <= 1e-5 * abs(g), (p, per[p], g)


def test_logdet_full_size_periodic_closed_form(gm):
    sp, npb, m, seed = workloads.C3_LATTICE, workloads.C3_PROBES, workloads.C3_M, workloads.c3_probe_seed()
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, "periodic", "f32")
    mean, se, per = op.logdet(npb, m, seed=seed)
    exact = closed_form.exact_logdet(sp.shape, sp.order, sp.kappa2, sp.tau, "periodic")
    assert abs(mean - exact) < 5 * se, (mean, exact, se)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f64", 1e-10)])
def test_logdet_subgrid_128(gm, storage, tol):
    sp, npb, m, seed = workloads.C3_LATTICE, workloads.C3_PROBES, workloads.C3_M, workloads.c3_probe_seed()
    shape = (128, 128)
    op = gm.Operator.lattice(shape, sp.order, sp.kappa2, sp.tau, sp.boundary, storage)
    mean, se, per = op.logdet(npb, m, seed=seed)
    Q = lattice.lattice_precision(shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    ref = logdet.hutchinson_csr(Q, npb, m, seed=seed)
    assert np.all(np.abs(per - ref.per_probe) <= tol * np.abs(ref.per_probe))
    assert abs(mean - ref.logdet) <= tol * abs(ref.logdet)
    exact = closed_form.exact_logdet(shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    assert abs(mean - exact) < 5 * se


def test_logdet_full_size_preconditioned(gm):
    """Section 6.2 split at full size: Hutchinson on A plus the closed-form log det M."""
    sp, npb, m, seed = workloads.C3_LATTICE, 16, workloads.C3_M, workloads.c3_probe_seed()
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f32").set_circulant_precond()
    mean, se, per = op.logdet(npb, m, seed=seed)
    exact = closed_form.exact_logdet(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
    assert abs(mean - exact) < 5 * se + 1e-6 * abs(exact), (mean, exact, se)

"""Plain FP64 CPU oracle for the Krylov GMRF sampler and the Lanczos log-det estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.  The
library ``paper_1312_1476_amd`` never imports it, and this package imports nothing from
the library: the two share no kernels, helpers, tables or constants.  The only module
both sides use is ``workloads`` (seeded inputs, no arithmetic of the method).

Everything here is deliberately slow and literal: NumPy / SciPy in IEEE FP64, no blocking,
fusion or reordering beyond the definitions it follows.  Each function cites the part of
Simpson, Turner, Strickland & Pettitt, "Scalable iterative methods for sampling from
massive Gaussian random vectors" (arXiv 1312.1476) it restates.

Modules
  lattice      -- explicit sparse lattice precisions (Sections 2-3)
  closed_form  -- DCT / DFT spectra, exact samples and log-determinants
  dense        -- dense eigendecomposition and Cholesky references
  lanczos      -- Algorithm 1 (Section 4) with the Theorem 1 stopping quantity
  precond      -- Proposition 1 with the block-circulant preconditioner (Section 5)
  lgcp         -- the log-Gaussian Cox process proposal Q + H with M = Q (Sections 3, 5.1)
  ichol        -- incomplete-Cholesky preconditioning of a general sparse Q (Section 5.2)
  logdet       -- Hutchinson estimator with Lanczos (Gauss) quadrature (Section 6)
  philox       -- Philox4x64-10 counter-based generator for Rademacher probes

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against dense
linear algebra, closed forms, published invariants or an independent library routine,
except the items listed in ``PARITY_UNPINNED`` below.
"""

# Functions for which no independent pin exists (their parity is partial).
PARITY_UNPINNED = (
    # Table 1 iteration counts: the paper's LGCP inputs (covariance, point pattern,
    # intensity) are never given, so its printed counts cannot be reproduced.
    "table1_iteration_counts",
)

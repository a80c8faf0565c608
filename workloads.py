"""Seeded synthetic inputs shared by the library's tests and benchmarks and by the oracle.

This module holds NO arithmetic of the method: it only draws random inputs and lists the
workload shapes.  Both the HIP path and the CPU oracle receive exactly the arrays built
here.  Base seed 14761312; every stream is numpy.random.default_rng([SEED, config, stream]).

Workloads (synthetic lattices standing in for the paper's unspecified LGCP lattices):
  C0  plain FP64 sample: 64 x 64 lattice, first order, kappa2 = 0.1, tau = 1, free boundary,
      one N(0, I) right-hand side, full reorthogonalisation, m_max = 200, tol 1e-8
  C1  preconditioned batch: 512 x 512, second order, kappa2 = 0.01, free boundary,
      periodic (block-circulant) preconditioner, 32 right-hand sides, m_max = 300
  C2  uneven batch: 256 fields, side uniform in {32..256}, first order,
      kappa2 log-uniform in [1e-3, 1], 8 right-hand sides each
  C3  Hutchinson log det: 1024 x 1024, second order, kappa2 = 0.05, 64 Rademacher probes,
      m = 80 (probe seed SEED + 3)
  C4  serving mix: Poisson arrivals (mean 200 req/s), sample and log-det requests on 2D
      lattices of side 64..2048 and 3D 7-point lattices up to 128^3
  C5  log-Gaussian Cox process proposal (Sections 3 and 5.1, Table 1): N x N lattice on the
      unit torus (h = 1/N), prior Q = tau (kappa2 I + L)^2 with tau = N^2, kappa2 = kc^2 / N^2
      (kc = 10: the same continuum field at every N), and the diagonal Fisher information
      H = h^2 exp(x) of Poisson cell counts at a smooth log-intensity x (mean log 500, unit
      variance, a fixed sum of low-frequency cosines, so every N sees the same surface).  The
      paper does not give its covariance, point pattern or intensity; this stands in for them.
"""
from dataclasses import dataclass, field

import numpy as np

SEED = 14761312


def rng(config, stream=0):
    return np.random.default_rng([SEED, int(config), int(stream)])


def gaussian_block(n, k, config, stream=0):
    """n x k block of i.i.d. N(0, 1) draws, column-major (each column one right-hand side)."""
    Z = rng(config, stream).standard_normal((k, n))
    return np.asfortranarray(Z.T)


@dataclass
class LatticeSpec:
    shape: tuple
    order: int = 1
    kappa2: float = 1.0
    tau: float = 1.0
    boundary: str = "free"

    @property
    def n(self):
        return int(np.prod(self.shape))


@dataclass
class SampleConfig:
    name: str
    lattice: LatticeSpec
    k: int
    m_max: int
    tol: float
    reorth: bool
    precond: bool
    storage: str = "f64"
    extra: dict = field(default_factory=dict)


C0 = SampleConfig("C0 plain FP64 64x64 first order", LatticeSpec((64, 64), 1, 0.1, 1.0),
                  k=1, m_max=200, tol=1e-8, reorth=True, precond=False)
C1 = SampleConfig("C1 preconditioned batch 512x512 second order",
                  LatticeSpec((512, 512), 2, 0.01, 1.0), k=32, m_max=300, tol=1e-8,
                  reorth=False, precond=True)
C3_LATTICE = LatticeSpec((1024, 1024), 2, 0.05, 1.0)
C3_PROBES, C3_M = 64, 80


def c3_probe_seed():
    return SEED + 3


def uneven_fields(n_fields=256, side_lo=32, side_hi=256, k=8):
    """C2 field list: (side, kappa2) per field, then each field's Z block (stream 1 + f)."""
    g = rng(2, 0)
    sides = g.integers(side_lo, side_hi + 1, size=n_fields)
    kappa2 = 10.0 ** g.uniform(-3.0, 0.0, size=n_fields)
    return [(int(s), float(kk)) for s, kk in zip(sides, kappa2)]


def uneven_field_rhs(f, side, k=8):
    return gaussian_block(side * side, k, 2, 1 + f)


@dataclass
class Request:
    t_arrival: float
    kind: str          # "sample" or "logdet"
    op_index: int      # index into the operator pool
    k: int             # right-hand sides (samples) or probes
    seed: int


def serving_pool(n_ops=64, side_lo=64, side_hi=2048, side3_lo=16, side3_hi=128, frac_3d=0.2):
    """C4 operator pool: 2D first-order lattices with log-uniform side, 3D 7-point lattices
    with log-uniform side, kappa2 log-uniform in [1e-3, 1]."""
    g = rng(4, 1)
    pool = []
    for _ in range(n_ops):
        kappa2 = float(10.0 ** g.uniform(-3.0, 0.0))
        if g.uniform() < frac_3d:
            s = int(round(np.exp(g.uniform(np.log(side3_lo), np.log(side3_hi)))))
            pool.append(LatticeSpec((s, s, s), 1, kappa2, 1.0))
        else:
            s = int(round(np.exp(g.uniform(np.log(side_lo), np.log(side_hi)))))
            pool.append(LatticeSpec((s, s), 1, kappa2, 1.0))
    return pool


def serving_trace(rate=200.0, duration=30.0, n_ops=64, frac_logdet=0.25, k_max=32):
    """Poisson arrival times with request kinds, operator indices and sizes."""
    g = rng(4, 0)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration:
            break
        kind = "logdet" if g.uniform() < frac_logdet else "sample"
        out.append(Request(t, kind, int(g.integers(0, n_ops)), int(g.integers(1, k_max + 1)),
                           int(g.integers(0, 2 ** 62))))
    return out


# ---- C5: log-Gaussian Cox process proposal ---------------------------------------------------------
LGCP_KC = 10.0                 # prior inverse range on the unit torus
LGCP_MEAN = float(np.log(500.0))
LGCP_MODES = 24                # cosine modes of the log-intensity surface
LGCP_KMAX = 4                  # largest wave number per axis


def lgcp_prior(N, kc=LGCP_KC):
    """Second-order periodic lattice on the unit torus at spacing h = 1/N."""
    return LatticeSpec((N, N), 2, kc * kc / float(N * N), float(N * N), "periodic")


def lgcp_log_intensity(N, stream=0):
    """x at the cell centres s = ((i + 1/2) / N, (j + 1/2) / N), row-major: LGCP_MEAN plus
    sum_k a_k g_k cos(2 pi (k . s) + phi_k) with integer wave vectors |k_i| <= LGCP_KMAX,
    a_k proportional to (1 + |k|^2)^{-1/2} and g_k ~ N(0, 1), scaled to unit variance."""
    g = rng(5, stream)
    kv = g.integers(-LGCP_KMAX, LGCP_KMAX + 1, size=(LGCP_MODES, 2))
    phase = g.uniform(0.0, 2.0 * np.pi, size=LGCP_MODES)
    gain = g.standard_normal(LGCP_MODES)
    amp = 1.0 / np.sqrt(1.0 + (kv.astype(np.float64) ** 2).sum(axis=1))
    amp *= np.sqrt(2.0 / (amp ** 2).sum())
    s = (np.arange(N, dtype=np.float64) + 0.5) / N
    x = np.full((N, N), LGCP_MEAN)
    for (k1, k2), ph, gk, ak in zip(kv, phase, gain, amp):
        x += ak * gk * np.cos(2.0 * np.pi * (k1 * s[:, None] + k2 * s[None, :]) + ph)
    return x.ravel()


def lgcp_diagonal(N, stream=0):
    """H = h^2 exp(x): the Fisher information of the cell counts y_ij ~ Po(h^2 exp(x_ij))
    at the log-intensity above (the input of the sMMALA proposal; diagonal, length N^2)."""
    return np.exp(lgcp_log_intensity(N, stream)) / float(N * N)

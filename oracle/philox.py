"""Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11) and the Rademacher probe rule built on it (oracle side, NumPy uint64).

Section 6 draws Hutchinson probes with i.i.d. Rademacher (+-1, equal probability)
entries; the paper fixes no generator.  The probe rule used on both sides of the parity
check is:

    seed s (64 bit), probe p, lattice index i:
        block b = i // 256, bit t = i % 256
        (w0, w1, w2, w3) = Philox4x64-10(counter = (b, p, 0, 0), key = (s, 0))
        v_p[i] = +1 if bit (t % 64) of w_{t // 64} is 0, else -1

Philox4x64 round (multipliers M0, M1, Weyl increments W0, W1 from the SC'11 paper):
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2   (full 128-bit products)
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);  then k <- (k0 + W0, k1 + W1)
Ten rounds, the key bumped between rounds.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit product as (hi, lo), vectorised over uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, c0)
            hi1, lo1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        return c0, c1, c2, c3


def rademacher_probe(seed, p, n):
    """v_p in {-1, +1}^n for the probe rule above (float64)."""
    nblocks = (n + 255) // 256
    b = np.arange(nblocks, dtype=np.uint64)
    words = philox4x64_10(b, np.uint64(p), np.uint64(0), np.uint64(0),
                          np.uint64(seed), np.uint64(0))
    W = np.stack(words, axis=1)                      # nblocks x 4
    i = np.arange(n, dtype=np.int64)
    blk, t = i // 256, i % 256
    w = W[blk, t // 64]
    bits = (w >> (t % 64).astype(np.uint64)) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def rademacher_probes(seed, n_probes, n):
    """n x n_probes block of probes (column p is probe p)."""
    return np.stack([rademacher_probe(seed, p, n) for p in range(n_probes)], axis=1)

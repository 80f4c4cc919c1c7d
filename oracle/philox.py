"""Philox4x32-10 counter-based generator and the normal draws built on it.

TEST INFRASTRUCTURE: this package is the CPU oracle.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The solver draws random numbers in two places: the start vector v1 of the
Lanczos bidiagonalization (Alg. 1, first step: v1 = randn(n,1), normalized) when
the caller passes none, and the replacement vector after a breakdown (a reading
of the paper: it is silent on breakdowns).  Both sides implement the same
published generator independently:

  Philox4x32-10 -- J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC'11.  Round function on the
  4x32-bit counter (c0,c1,c2,c3) with 2x32-bit key (k0,k1):
      (hi0, lo0) = mulhilo(0xD2511F53, c0); (hi1, lo1) = mulhilo(0xCD9E8D57, c2)
      c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
  ten rounds, the key advanced by the Weyl constants (0x9E3779B9, 0xBB67AE85)
  between rounds.

Normal vector of length L for seed s and stream q (this library's encoding):
  key = (s mod 2^32, s >> 32); for block b = 0 .. ceil(L/2)-1:
  (x0,x1,x2,x3) = Philox4x32-10(counter = (b mod 2^32, b >> 32, q, 0), key)
  u1 = (((x1<<32 | x0) >> 11) + 1) * 2^-53   in (0, 1]
  u2 = ((x3<<32 | x2) >> 11) * 2^-53         in [0, 1)
  z[2b] = sqrt(-2 ln u1) cos(2 pi u2), z[2b+1] = sqrt(-2 ln u1) sin(2 pi u2)
  (Box-Muller, 1958).  Stream 0 is the default start vector; stream 1+b is the
  replacement vector of the b-th breakdown of a solve.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Arguments are uint32-valued arrays (any int
    dtype); returns four uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK32 for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0          # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def normal_vector(length: int, seed: int, stream: int) -> np.ndarray:
    """N(0,1) vector of ``length`` entries for (seed, stream), as defined above."""
    nb = (length + 1) // 2
    b = np.arange(nb, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    x0, x1, x2, x3 = philox4x32_10(b & MASK32, b >> np.uint64(32),
                                   np.full(nb, stream, dtype=np.uint64),
                                   np.zeros(nb, dtype=np.uint64),
                                   s & MASK32, s >> np.uint64(32))
    a = ((x1 << np.uint64(32)) | x0) >> np.uint64(11)
    c = ((x3 << np.uint64(32)) | x2) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = c.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    z = np.empty(2 * nb)
    z[0::2] = rad * np.cos(th)
    z[1::2] = rad * np.sin(th)
    return z[:length]

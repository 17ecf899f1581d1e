"""Oracle: counter-based Gaussian noise for RapidPT recovery.  TEST INFRASTRUCTURE.

Alg. 2 draws the residual s ~ i.i.d. N(0, sigma^2) for each of the v entries of
every recovered column.  The paper does not name a generator; we read it as a
counter-based one so that the v x L draws need never be stored and the HIP
library and this oracle produce the same draw for the same (column, voxel):

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key, ten rounds;
  each round multiplies counter words 0 and 2 by the constants 0xD2511F53 and
  0xCD9E8D57, forms the new words from the high/low product halves xor'd with
  the other counter words and the key, and the key is bumped by the Weyl
  constants (0x9E3779B9, 0xBB67AE85) between rounds.
* Each 32-bit output word x maps to u = ((x >> 8) + 0.5) * 2^-24 in (0, 1).
* Box-Muller (Box & Muller, 1958): from (u_a, u_b), z = sqrt(-2 ln u_a) times
  cos(2 pi u_b), and the sine for the second normal.

Noise layout: key = (seed mod 2^32, seed >> 32); counter = (k, i >> 2, stream,
study) for voxel k of column i, so one call serves four consecutive columns at
one voxel.  Words (x0, x1) give the normals of columns i = 4q and 4q+1 (cos,
then sin), words (x2, x3) those of 4q+2 and 4q+3.  Since u >= 2^-25,
|z| <= sqrt(50 ln 2) < 5.8872 for every draw.

Pins (tests/test_oracle_philox.py): the published Random123 known-answer
vectors for Philox4x32-10, the uniform map's range, moments and a
Kolmogorov-Smirnov test of the normals.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_RECOVERY = 2
STREAM_TRAINING = 4

Z_BOUND = float(np.sqrt(-2.0 * np.log(2.0 ** -25)))  # largest |z| the map can give


def philox4x32_10(ctr, key):
    """Philox4x32-10 on broadcastable arrays.

    ctr: sequence of 4 integer arrays (uint32 values), key: 2 integers or
    arrays.  Returns a (4, ...) uint32 array of output words.
    """
    c = [np.asarray(x, dtype=np.uint64) & MASK32 for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * c[0]               # < 2^64, exact in uint64
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in np.broadcast_arrays(*c)])


def uniform_from_word(x) -> np.ndarray:
    """Top 24 bits of a 32-bit word, centred in its cell: ((x>>8)+0.5)/2^24."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(8)).astype(np.float64) + 0.5) * (2.0 ** -24)


def normals(seed: int, stream: int, i: int, k, study: int = 0) -> np.ndarray:
    """z(seed, stream, i, k) for an array of voxel indices k (int)."""
    k = np.asarray(k, dtype=np.int64).astype(np.uint64)
    i = int(i)
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    w = philox4x32_10((k, np.uint64(i >> 2), np.uint64(stream), np.uint64(study)), key)
    u = uniform_from_word(w)                      # (4, ...)
    sel = i & 3
    ua, ub = (u[0], u[1]) if sel < 2 else (u[2], u[3])
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return rad * np.cos(ang) if (sel & 1) == 0 else rad * np.sin(ang)

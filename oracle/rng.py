"""Counter-based random numbers of the method's draws (TEST INFRASTRUCTURE ONLY).

Philox4x32-10 as published by Salmon, Moraes, Dror & Shaw (2011), "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): ten rounds on a 4 x 32-bit counter under a 2 x 32-bit key; each
round multiplies counter words 0 and 2 by fixed 32-bit multipliers, swaps and xors the halves
of the products with words 1 and 3 and the key, and the key is bumped by two Weyl constants
between rounds. Uniforms take 52 bits from two words; normals use the Box-Muller transform
(cosine branch). Written here from that definition so that the oracle can draw the same
numbers as the kernels from the same (seed, counter) without taking any value from them.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """counter: uint32 array [..., 4]; key: two uint32 (scalars or arrays broadcast against
    the counter's leading shape). Returns uint32 [..., 4]."""
    c = np.asarray(counter, np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., i] for i in range(4))
    k0 = np.asarray(key[0], np.uint64) & _MASK
    k1 = np.asarray(key[1], np.uint64) & _MASK
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(_W0)) & _MASK
        k1 = (k1 + np.uint64(_W1)) & _MASK
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def u01(a, b):
    """Uniform in (0, 1) from two words: k = 26 high bits of a above 26 high bits of b,
    u = (k + 1/2) / 2^52 (exact, so never 0 or 1)."""
    a = np.asarray(a, np.uint64) >> np.uint64(6)
    b = np.asarray(b, np.uint64) >> np.uint64(6)
    return (a.astype(np.float64) * 67108864.0 + b.astype(np.float64) + 0.5) / 4503599627370496.0


def split_seed(seed: int):
    return np.uint32(seed & 0xFFFFFFFF), np.uint32((seed >> 32) & 0xFFFFFFFF)


def normals(seed: int, w0, w1, w2, tag: int):
    """Standard normals for counters (w0, w1, w2, tag) (arrays broadcast together): the
    first two words give u1, the last two u2, n = sqrt(-2 ln u1) cos(2 pi u2)."""
    w0, w1, w2 = np.broadcast_arrays(np.asarray(w0, np.uint64), np.asarray(w1, np.uint64),
                                     np.asarray(w2, np.uint64))
    ctr = np.stack([w0, w1, w2, np.full(w0.shape, tag, np.uint64)], axis=-1)
    r = philox4x32_10(ctr, split_seed(seed))
    u1, u2 = u01(r[..., 0], r[..., 1]), u01(r[..., 2], r[..., 3])
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)

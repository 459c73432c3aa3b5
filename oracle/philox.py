"""Philox4x32-10 (oracle copy), written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11), section on the Philox family: a 4 x 32-bit counter block and a
2 x 32-bit key; each of the 10 rounds multiplies counter words 0 and 2 by the
constants M0, M1 (full 64-bit products split into high and low halves),
mixes the high halves with the other two counter words and the round key, and
the key is advanced by the Weyl constants W0, W1 between rounds.

Vectorised over any number of counters with numpy uint64 arithmetic (every
product of two 32-bit values fits in 64 bits, so nothing overflows).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SHIFT32 = np.uint64(32)


def philox4x32_10(counter, key):
    """Encrypt counter blocks.

    counter: array of shape (..., 4) of integers in [0, 2^32).
    key:     array of shape (..., 2) (broadcast against counter[..., 0]).
    Returns an array of shape (..., 4) of uint32 words.
    """
    ctr = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i] & MASK32 for i in range(4))
    k0 = np.broadcast_to(k[..., 0] & MASK32, x0.shape)
    k1 = np.broadcast_to(k[..., 1] & MASK32, x0.shape)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> SHIFT32, p0 & MASK32
        hi1, lo1 = p1 >> SHIFT32, p1 & MASK32
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)

"""Philox4x32-10 counter-based generator, from its published definition.

Test infrastructure (the oracle).  Written from J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11:
a 4x32-bit counter and a 2x32-bit key; each of the 10 rounds multiplies words
0 and 2 by two fixed odd constants, takes the high and low halves of the two
64-bit products and mixes them with words 1 and 3 and the key; between rounds
the key is bumped by two Weyl constants.  Pinned against the published
known-answer vectors in ``tests/test_oracle_philox.py``.

Vectorised over arbitrary numpy arrays of counters (uint32).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words for counters (c0..c3) and key (k0, k1).

    Counters may be numpy arrays (broadcast together); the key is scalar.
    """
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    key0 = int(k0) & 0xFFFFFFFF
    key1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            key0 = (key0 + _W0) & 0xFFFFFFFF
            key1 = (key1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(key0), lo1, hi0 ^ c[3] ^ np.uint64(key1), lo0]
    return tuple(x.astype(np.uint32) for x in c)


def uniform_open01(x):
    """Map 32-bit words to (0, 1) as (x + 1/2) * 2^-32 (exact in FP64)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32

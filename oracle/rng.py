"""Counter-based random numbers for the learned proposal's draws (test infrastructure).

Philox-4x64 with 10 rounds, from its published definition (Salmon, Moraes, Dror
and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a block of four
64-bit words is a keyed bijection of a four-word counter; each round multiplies
words 0 and 2 by fixed constants, mixes the high halves of the products with
the other two words and the key, and the key is bumped by two Weyl constants
between rounds.

The streams the library and this oracle both use:
* element i of stream (seed, offset) is word 0 of the block with counter
  (offset + i, 0, 0, 0) and key (seed, 0);
* uniform = (w0 >> 11) * 2^-53 in [0, 1); randint(hi) = floor(uniform * hi).

Pins: numpy's own Philox bit generator (an independent implementation of the
same definition) and the block function written with Python integers.
"""

import numpy as np

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_int(counter, key, rounds=10):
    """One block with Python integers (exact 128-bit products); counter 4 words, key 2 words."""
    x = [int(v) & _MASK for v in counter]
    k = [int(v) & _MASK for v in key]
    for _ in range(rounds):
        p0 = _M0 * x[0]
        p1 = _M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ x[3] ^ k[1], p0 & _MASK]
        k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
    return x


def _mulhilo(a, b):
    """(hi, lo) of the 128-bit products of uint64 arrays a and a constant b."""
    a = np.asarray(a, dtype=np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    al, ah = a & m32, a >> s32
    bl, bh = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    ll = al * bl
    lh = al * bh
    hl = ah * bl
    hh = ah * bh
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64(c0, key0, rounds=10):
    """Word 0..3 of the blocks with counters (c0, 0, 0, 0) (uint64 array) and key (key0, 0)."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64).copy()
        x1 = np.zeros_like(x0)
        x2 = np.zeros_like(x0)
        x3 = np.zeros_like(x0)
        k0 = np.uint64(int(key0) & _MASK)
        k1 = np.uint64(0)
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(x0, _M0)
            hi1, lo1 = _mulhilo(x2, _M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + np.uint64(_W0)
            k1 = k1 + np.uint64(_W1)
    return x0, x1, x2, x3


def uniform(seed, offset, n):
    """Elements offset .. offset + n - 1 of the uniform stream of seed, as float64 in [0, 1)."""
    c = np.uint64(offset) + np.arange(n, dtype=np.uint64)
    w0 = philox4x64(c, seed)[0]
    return (w0 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def randint(seed, offset, n, hi):
    """floor(uniform * hi) of the same stream (int64 in [0, hi))."""
    return np.floor(uniform(seed, offset, n) * hi).astype(np.int64)

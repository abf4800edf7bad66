"""Philox4x64-10 counter-based generator, vectorised over counters.

Test infrastructure (see ``oracle/__init__.py``).  Written from the published
definition (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a 2-word
key; each of 10 rounds multiplies counter words 0 and 2 by the constants
M0 = 0xD2E7470EE14C6C93 and M1 = 0xCA5A826395121157 (full 128-bit
products), then permutes and XORs with the key; the key is bumped by the
Weyl constants W0 = 0x9E3779B97F4A7C15, W1 = 0xBB67AE8584CAA73B between
rounds.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays: (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | ((mid & _M32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(counter, key) -> np.ndarray:
    """counter [..., 4] uint64, key [..., 2] uint64 (broadcast) -> [..., 4]."""
    counter = np.asarray(counter, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (counter[..., i] for i in range(4))
    k0, k1 = key[..., 0], key[..., 1]
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = k0 + W0
                k1 = k1 + W1
            h0, l0 = mulhilo64(M0, c0)
            h1, l1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0
    return np.stack(np.broadcast_arrays(c0, c1, c2, c3), axis=-1)


def block(seed: int, stream: int, generation, unit, blk) -> np.ndarray:
    """The GA's draw convention: key = (seed, stream),
    counter = (generation, unit, block, 0).  Broadcasts its index arguments."""
    g, u, b = np.broadcast_arrays(np.asarray(generation, dtype=np.uint64),
                                  np.asarray(unit, dtype=np.uint64),
                                  np.asarray(blk, dtype=np.uint64))
    ctr = np.stack([g, u, b, np.zeros_like(g)], axis=-1)
    key = np.array([np.uint64(seed), np.uint64(stream)], dtype=np.uint64)
    return philox4x64_10(ctr, key)

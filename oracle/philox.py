"""Philox4x32-10, written from its published description (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4.2).

State: a 128-bit counter (four 32-bit words) and a 64-bit key (two words).
One round multiplies counter words 0 and 2 by two fixed odd constants, keeps
the high and low halves of the 64-bit products, and mixes them with the other
two counter words and the key; the key is bumped by two Weyl constants between
rounds.  Ten rounds are applied.

The Metropolis sampler draws one Philox block per (chain, sweep, link):
key = (seed & 0xffffffff, seed >> 32), counter = (chain, sweep, link, 0).
The uniform is u = (((x1 << 32) | x0) >> 11) * 2^-53 in [0, 1), and the Z_N
proposal step is 1 + (x2 mod (N - 1)) (1 for Z2, 1 + (x2 & 1) for Z3).  This is
the sampler reading for Sec. 5.1 (the paper does not name a sampler).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Scalar reference: ctr = 4 ints, key = 2 ints -> 4 ints."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def philox_vec(c0, c1, c2, c3, k0, k1):
    """Vectorised over uint64 arrays holding 32-bit values (same rounds as above)."""
    c0 = np.asarray(c0, np.uint64) & MASK
    c1 = np.asarray(c1, np.uint64) & MASK
    c2 = np.asarray(c2, np.uint64) & MASK
    c3 = np.asarray(c3, np.uint64) & MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    m = np.uint64(MASK)
    for _ in range(10):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & m
        k1 = (k1 + np.uint64(W1)) & m
    return c0, c1, c2, c3


def uniform_from_words(x0, x1):
    """53-bit uniform double in [0, 1) from two 32-bit words."""
    x0 = np.asarray(x0, np.uint64)
    x1 = np.asarray(x1, np.uint64)
    bits = ((x1 << np.uint64(32)) | x0) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -53)


def draw(seed: int, chain, sweep, link, group: int = 3):
    """(u, step) for the Z_N proposal at (chain, sweep, link); arrays broadcast.  The step
    1 + (x2 mod (N - 1)) is uniform over the N - 1 other elements (symmetric proposal)."""
    x0, x1, x2, _ = philox_vec(chain, sweep, link, 0, seed & MASK, (seed >> 32) & MASK)
    u = uniform_from_words(x0, x1)
    step = 1 + (x2 % np.uint64(group - 1)).astype(np.int64)
    return u, step

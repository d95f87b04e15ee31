"""Philox counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written generically for 4 words
of W = 32 or 64 bits.

The paper reconstructs the winning candidate on the host by running the same
random process as the GPU workers, sending only the seed (sec. 2.5, the
implementation detail after Algorithm 2).  A counter-based generator keyed by
(candidate index, iteration) gives that property without any stream state.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

# Multipliers and Weyl key increments from the SC'11 paper.
_CONST = {
    32: ((0xD2511F53, 0xCD9E8D57), (0x9E3779B9, 0xBB67AE85)),
    64: ((0xD2E7470EE14C6C93, 0xCA5A826395121157),
         (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def philox4(counter, key, bits: int = 32, rounds: int = 10):
    """One Philox-4xW block: 4 output words for a 4-word counter and 2-word key.

    Each round multiplies words 0 and 2 by the two constants, keeps the high
    and low halves of each product, and mixes the high halves with the odd
    words and the round key; the key is bumped by the Weyl constants between
    rounds.
    """
    (m0, m1), (w0, w1) = _CONST[bits]
    mask = (1 << bits) - 1
    x0, x1, x2, x3 = (int(c) & mask for c in counter)
    k0, k1 = (int(k) & mask for k in key)
    for _ in range(rounds):
        p0 = m0 * x0
        p1 = m1 * x2
        hi0, lo0 = p0 >> bits, p0 & mask
        hi1, lo1 = p1 >> bits, p1 & mask
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + w0) & mask
        k1 = (k1 + w1) & mask
    return [x0, x1, x2, x3]


def seed_key(seed: int):
    """Run seed (64 bit) -> Philox-4x32 key (low word, high word)."""
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def draw_words(seed: int, a: int, b: int, c: int, d: int):
    """Philox-4x32-10 block for counter (a, b, c, d) under the run seed."""
    return philox4((a, b, c, d), seed_key(seed), bits=32, rounds=10)


def scale(word: int, m: int) -> int:
    """Map a uniform 32-bit word to {0..m-1}: floor(word * m / 2^32)."""
    return (word * m) >> 32

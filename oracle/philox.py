"""Philox4x64-10, written from its published definition (test infrastructure).

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11.  Philox4x64 maps a 256-bit counter
(four 64-bit words) and a 128-bit key (two words) through R = 10 rounds.  Each
round multiplies counter words 0 and 2 by two fixed odd constants, producing
64x64->128-bit products (hi, lo), and permutes/xors:

    out = (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))

Between rounds the key is bumped by two Weyl constants (golden ratio and
sqrt(3) - 1 in 64-bit fixed point).  Arithmetic is done with Python integers
and masked to 64 bits, so it is exact and independent of any GPU code.

The randomized decomposition draws all its randomness from this function: the
Gaussian test matrix G_n of Alg. 1/2/4/5 and the column draws of RANDSAMPLE
(Section 3.2).  The counter layout used for each is documented in
``oracle.tucker``.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1

# Round multipliers and key-schedule (Weyl) increments of Philox4x64.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

ROUNDS = 10


def philox4x64(counter, key, rounds: int = ROUNDS):
    """Return the four 64-bit output words for a 4-word counter, 2-word key."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        x0, x1, x2, x3 = (((p1 >> 64) ^ x1 ^ k0) & MASK64, p1 & MASK64,
                          ((p0 >> 64) ^ x3 ^ k1) & MASK64, p0 & MASK64)
    return (x0, x1, x2, x3)

"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition with Python integers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper only says the classical variable is "randomly modified" (Sec. II(c),
Fig. 2 step (c)) and decided "via the Metropolis algorithm" (Sec. I); it fixes
no generator.  Reading used here: one Philox4x64-10 block per
(key=(seed, 0), counter=(c0, c1, c2, c3)) where the counter words are
(sweep, site, stream, attempt).  Draws therefore do not depend on how updates
are batched or scheduled.

Pinned by: ``numpy.random.Philox`` (an independent implementation) — our
block at counter c equals numpy's first block when numpy is seeded with
counter c-1 (numpy advances the counter before producing output).
"""

MASK64 = (1 << 64) - 1

# Round multipliers and Weyl key increments of Philox4x64 (SC'11, Sec. 5).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
ROUNDS = 10


def _mulhilo(a: int, b: int):
    p = a * b
    return p >> 64, p & MASK64


def philox4x64(key, counter):
    """Return the four 64-bit words of the Philox4x64-10 block.

    key: (k0, k1) 64-bit ints; counter: (c0, c1, c2, c3) 64-bit ints.
    Each round: two 64x64->128 multiplies of words 0 and 2, a permutation and
    an xor with the round key; the key is bumped by the Weyl constants between
    rounds.
    """
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for _ in range(ROUNDS):
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return (c0, c1, c2, c3)

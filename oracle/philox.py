"""Philox4x32-10 counter-based generator: TEST INFRASTRUCTURE ONLY.

Written from its published definition (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011, the Philox-4x32
family with ten rounds): the state is four 32-bit counter words and two key
words.  A round multiplies counter words 0 and 2 by the two round
multipliers into 64-bit products; the new word 0 is the high half of the
second product xored with counter word 1 and key word 0, word 1 is the low
half of the second product, word 2 the high half of the first product xored
with counter word 3 and key word 1, word 3 the low half of the first
product.  Between rounds the key words grow by the two Weyl increments
(the golden ratio and sqrt(3) - 1 scaled to 32 bits).  Plain Python
integers, one block at a time.

The device sampler draws its proposals and acceptance uniforms from the same
generator; tests compare the library's host and device implementations with
this one.  Parity unpinned against the generator's published known-answer
values (none is reproduced here); pinned by statistical properties instead
(tests/test_philox.py).
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
MULT = (0xD2511F53, 0xCD9E8D57)   # round multipliers of Philox-4x32
WEYL = (0x9E3779B9, 0xBB67AE85)   # key increments: 2^32 (phi - 1), 2^32 (sqrt 3 - 1)


def philox4x32(ctr, key, rounds: int = 10):
    """Four output words for counter ctr (4 words) and key (2 words)."""
    c = [int(x) & MASK32 for x in ctr]
    k = [int(x) & MASK32 for x in key]
    for _ in range(rounds):
        p0 = MULT[0] * c[0]
        p1 = MULT[1] * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & MASK32, p1 & MASK32,
             ((p0 >> 32) ^ c[3] ^ k[1]) & MASK32, p0 & MASK32]
        k = [(k[0] + WEYL[0]) & MASK32, (k[1] + WEYL[1]) & MASK32]
    return c


def uniform53(a: int, b: int) -> float:
    """A uniform in (0, 1] from two words: the top 27 bits of a and 26 of b."""
    return 1.0 - ((a >> 5) * 67108864.0 + (b >> 6)) / 9007199254740992.0

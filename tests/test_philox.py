"""The counter-based generator of the device sampler: the oracle's
Philox4x32-10 (written from its published definition) against properties
that fix it independently of the code, and the library's host
implementation against the oracle's, bit for bit."""
import math

import numpy as np

from oracle import philox
from paper_2312_05647_amd import mjp


def test_key_increments_are_the_weyl_constants():
    # 2^32 (golden ratio - 1) and 2^32 (sqrt 3 - 1), rounded down
    assert philox.WEYL[0] == math.floor(2 ** 32 * (math.sqrt(5) - 1) / 2)
    assert philox.WEYL[1] == math.floor(2 ** 32 * (math.sqrt(3) - 1))


def test_zero_rounds_is_the_identity_and_rounds_mix():
    assert philox.philox4x32([1, 2, 3, 4], [5, 6], rounds=0) == [1, 2, 3, 4]
    # one round by hand: words 0 and 2 multiplied, halves exchanged
    c, k = [3, 7, 11, 13], [17, 19]
    p0, p1 = philox.MULT[0] * 3, philox.MULT[1] * 11
    want = [((p1 >> 32) ^ 7 ^ 17), p1 & 0xFFFFFFFF, ((p0 >> 32) ^ 13 ^ 19), p0 & 0xFFFFFFFF]
    assert philox.philox4x32(c, k, rounds=1) == want


def test_outputs_are_uniform_and_independent():
    g = np.random.default_rng(11)
    key = [int(x) for x in g.integers(0, 2 ** 32, 2)]
    words = np.array([philox.philox4x32([i, 0, 0, 0], key) for i in range(20000)], np.uint64)
    bits = ((words[:, :, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(np.float64)
    freq = bits.mean(axis=0)                       # every bit of every word
    assert np.abs(freq - 0.5).max() < 5 * 0.5 / math.sqrt(len(words))
    # top-4-bit histogram of each word: chi-square with 15 degrees of freedom
    for w in range(4):
        h = np.bincount((words[:, w] >> np.uint64(28)).astype(np.int64), minlength=16)
        e = len(words) / 16
        assert ((h - e) ** 2 / e).sum() < 45.0
    # consecutive counters: words uncorrelated
    u = words[:, 0].astype(np.float64) / 2 ** 32
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.03


def test_avalanche():
    g = np.random.default_rng(12)
    flips = []
    for _ in range(400):
        ctr = [int(x) for x in g.integers(0, 2 ** 32, 4)]
        key = [int(x) for x in g.integers(0, 2 ** 32, 2)]
        w, b = int(g.integers(0, 4)), int(g.integers(0, 32))
        c2 = list(ctr)
        c2[w] ^= 1 << b
        x, y = philox.philox4x32(ctr, key), philox.philox4x32(c2, key)
        flips.append(sum(bin(p ^ q).count("1") for p, q in zip(x, y)))
    assert abs(np.mean(flips) - 64.0) < 2.0


def test_box_muller_normals():
    z = []
    for i in range(10000):
        r = philox.philox4x32([i, 5, 0, 0], [123, 456])
        u1, u2 = philox.uniform53(r[0], r[1]), philox.uniform53(r[2], r[3])
        rad = math.sqrt(-2.0 * math.log(u1))
        z += [rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2)]
    z = np.array(z)
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.04
    assert abs((z ** 4).mean() - 3.0) < 0.25


def test_library_host_generator_matches_oracle():
    g = np.random.default_rng(13)
    for _ in range(2000):
        ctr = g.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = g.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        got = mjp.mjp_philox4x32_10(ctr, key)
        assert list(map(int, got)) == philox.philox4x32(ctr, key)

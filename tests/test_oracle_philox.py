"""Pins of the oracle's counter-based generator (Philox, Salmon et al. SC'11).

The oracle instantiates ONE generic Philox-4xW-10 round function for W = 32
and W = 64 bits.  numpy ships Philox4x64-10, so the 64-bit instantiation is
checked bit-for-bit against numpy; that pins the round structure, the word
permutation and the Weyl key schedule shared by both widths.  The 32-bit
instantiation is pinned by the published known-answer vectors of
Philox4x32-10 (tests/golden/philox4x32_10_kat.txt), which fix its multipliers
and Weyl constants, and is additionally checked statistically.
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def test_philox4x32_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = np.array([int(x, 16) for x in r], dtype=np.uint32)
        got = oracle.philox4x32(w[:4].copy(), w[4:6].copy())
        assert np.array_equal(got, w[6:]), (r, [f"{x:08x}" for x in got])


def _numpy_block(ctr, key):
    # numpy increments the 256-bit counter before each block
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("seed", range(6))
def test_philox4x64_matches_numpy(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ctr = rng.integers(0, 2**63, 4, dtype=np.uint64)
    ctr[0] = ctr[0] & np.uint64(2**62 - 1)      # no carry out of word 0 on the increment
    key = rng.integers(0, 2**63, 2, dtype=np.uint64)
    got = oracle.philox4x64(ctr + np.array([1, 0, 0, 0], dtype=np.uint64), key)
    assert np.array_equal(got, _numpy_block(ctr, key))


def test_philox4x64_zero_key_counter():
    got = oracle.philox4x64(np.array([1, 0, 0, 0], dtype=np.uint64), np.zeros(2, dtype=np.uint64))
    assert np.array_equal(got, _numpy_block([0, 0, 0, 0], [0, 0]))


def _stream_words(n, step=0):
    out = np.empty((n, 4), dtype=np.uint32)
    key = np.array([0x12345678, 0x9ABCDEF0], dtype=np.uint32)
    for i in range(n):
        out[i] = oracle.philox4x32(np.array([i, step, 0, 0], dtype=np.uint32), key)
    return out


def test_philox4x32_uniformity_and_bits():
    w = _stream_words(20000).ravel()
    # top-byte histogram chi-square (255 dof): mean 255, sd ~22.6
    h = np.bincount(w >> 24, minlength=256)
    e = len(w) / 256
    chi2 = ((h - e) ** 2 / e).sum()
    assert 160 < chi2 < 360
    # each bit set half the time
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(w)))
    # lag-1 serial correlation of uniforms
    u = (w >> 8).astype(np.float64) / 2**24
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 5 / np.sqrt(len(u))


def test_philox4x32_avalanche():
    key = np.array([1, 2], dtype=np.uint32)
    base = oracle.philox4x32(np.array([7, 11, 0, 0], dtype=np.uint32), key)
    flips = []
    for b in range(32):
        c = np.array([7 ^ (1 << b), 11, 0, 0], dtype=np.uint32)
        o = oracle.philox4x32(c, key)
        flips.append(sum(bin(int(x)).count("1") for x in (o ^ base)))
    m = np.mean(flips)
    assert 56 < m < 72           # half of 128 output bits on average


def test_philox4x32_distinct_over_counters_and_keys():
    a = _stream_words(2000, step=0)
    b = _stream_words(2000, step=1)
    allw = np.concatenate([a.ravel(), b.ravel()])
    assert len(np.unique(allw)) > 0.999 * len(allw)

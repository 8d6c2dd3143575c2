"""Pins of the oracle's random-number layer: Philox-4x32-10, the step stream, Lemire draws,
inverse-transform group selection.  CPU only."""
import os
import random

import numpy as np
import pytest

import oracle as O
from oracle import pyref
from conftest import GOLDEN


def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    # Published known-answer vectors: pins the round function, constants and round count.
    assert O.philox(ctr, key) == out
    assert pyref.philox4x32_10(ctr, key) == out


def test_philox_two_implementations_agree():
    rng = random.Random(7)
    for _ in range(300):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        assert O.philox(ctr, key) == pyref.philox4x32_10(ctr, key)


def test_stream_layout_matches_independent_stream():
    rng = random.Random(11)
    for _ in range(50):
        seed, walk, step = rng.getrandbits(64), rng.getrandbits(64), rng.getrandbits(32)
        words = O.stream_words(seed, walk, step, 11)
        s = pyref.Stream(seed, walk, step)
        assert [int(x) for x in words] == [s.next32() for _ in range(11)]
        # block 1 continues the counter's last word: it is not a re-draw of block 0
        assert list(words[4:8]) != list(words[0:4])


def test_lemire_width16_exhaustive():
    # Every output value of an exact draw on [0, n) must have exactly floor(2^16 / n) accepted
    # preimages among the 2^16 words, and exactly 2^16 mod n words must be rejected.
    W = 16
    for n in [1, 2, 3, 5, 7, 10, 255, 1000, 4097, 40000, 65535, 65536]:
        counts, rejected = O.below_all_words(n, W)
        assert rejected == (1 << W) % n, n
        assert (counts == (1 << W) // n).all(), n
    # the same on 20-bit words for a few awkward n
    for n in [3, 999_983, 1 << 19, (1 << 20) - 1]:
        counts, rejected = O.below_all_words(n, 20)
        assert rejected == (1 << 20) % n and (counts == (1 << 20) // n).all(), n


def test_lemire_matches_pure_python_on_random_words():
    rng = random.Random(3)
    for W in (32, 64):
        for _ in range(400):
            n = rng.randrange(1, 1 << (W - rng.randrange(0, W - 1)))
            words = [rng.getrandbits(W) for _ in range(8)]
            it = iter(words)
            expect = pyref.below(n, W, lambda: next(it))
            got, used = O.below_words(n, W, words)
            assert got == expect
            assert used is not None


def test_lemire_rejection_consumes_next_word():
    # n = 3 on 16-bit words: x = 0 gives low part 0 < (2^16 - 3) mod 3 = 1, so it is rejected
    # and the next word decides.
    v, used = O.below_words(3, 16, [0, 0x8000])
    assert used == 2 and v == (0x8000 * 3) >> 16


def test_below32_below64_follow_stream_words():
    rng = random.Random(5)
    for _ in range(200):
        seed, walk, step = rng.getrandbits(64), rng.getrandbits(40), rng.getrandbits(8)
        n32 = rng.randrange(1, 1 << 32)
        n64 = rng.randrange(1, 1 << 60)
        s = pyref.Stream(seed, walk, step)
        assert O.below32(seed, walk, step, n32) == pyref.below(n32, 32, s.next32)
        s = pyref.Stream(seed, walk, step)
        assert O.below64(seed, walk, step, n64) == pyref.below(n64, 64, s.next64)


def test_below64_uniform_chi2():
    from scipy.stats import chisquare
    n = 10
    vals = [O.below64(99, i, 0, n) for i in range(20000)]
    counts = np.bincount(vals, minlength=n)
    assert chisquare(counts).pvalue > 1e-4


def test_group_selection_exhaustive():
    # Inverse transform over groups: each group k must receive exactly c_k * 2^k of the W values
    # of r, in one contiguous run, groups in ascending bit order (Eq. eq:group_prob).
    rng = random.Random(1)
    for _ in range(40):
        K = rng.randrange(1, 9)
        counts = [rng.choice([0, 0, 1, 2, 3, 5]) for _ in range(K)]
        if sum(counts) == 0:
            counts[0] = 1
        W = sum(c << k for k, c in enumerate(counts))
        ks = [O.pick_group(counts, r) for r in range(W)]
        for k, c in enumerate(counts):
            assert ks.count(k) == c << k
        assert ks == sorted(ks)
        assert ks == [pyref.pick_group(counts, r) for r in range(W)]

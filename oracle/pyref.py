"""Second, pure-Python implementation of the oracle's random-number pieces.

TEST INFRASTRUCTURE.  Written separately from ``bingo_oracle.c`` and used only
to cross-check it on small cases: Philox-4x32-10 from its published description
(Salmon et al., SC'11), the per-step stream layout, and Lemire's exact bounded
draw (ACM TOMACS 2019).  Slow on purpose: every operation is a Python int.
"""
from __future__ import annotations

M32 = 0xFFFFFFFF
_MUL = (0xD2511F53, 0xCD9E8D57)
_WEYL = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(ctr, key):
    x = [int(v) & M32 for v in ctr]
    k = [int(v) & M32 for v in key]
    for _ in range(10):
        a = _MUL[0] * x[0]
        b = _MUL[1] * x[2]
        x = [((b >> 32) ^ x[1] ^ k[0]) & M32, b & M32, ((a >> 32) ^ x[3] ^ k[1]) & M32, a & M32]
        k = [(k[0] + _WEYL[0]) & M32, (k[1] + _WEYL[1]) & M32]
    return x


class Stream:
    """Words of the step stream (seed, walk, step): block 0, 1, ... in order."""

    def __init__(self, seed, walk, step):
        self.key = (seed & M32, (seed >> 32) & M32)
        self.ctr = (walk & M32, (walk >> 32) & M32, step & M32)
        self.blk = 0
        self.buf = []

    def next32(self):
        if not self.buf:
            self.buf = philox4x32_10(self.ctr + (self.blk,), self.key)
            self.blk += 1
        return self.buf.pop(0)

    def next64(self):
        hi = self.next32()
        return (hi << 32) | self.next32()


def below(n, width, next_word):
    """Uniform integer on [0, n) from ``width``-bit words (multiply, then reject the biased low part)."""
    two = 1 << width
    x = next_word()
    m = x * n
    low = m % two
    if low < n:
        thresh = (two - n) % n
        while low < thresh:
            x = next_word()
            m = x * n
            low = m % two
    return m >> width


def pick_group(counts, r):
    acc = 0
    for k, c in enumerate(counts):
        acc += c << k
        if r < acc:
            return k
    return -1

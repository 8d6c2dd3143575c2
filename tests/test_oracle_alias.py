"""Pins of the oracle's inter-group alias table (Sec. 4.1, the paper's inter-group sampler).

Pinned against: brute force over every (slot, value) pair for small totals (group k must be chosen by
exactly 32 T_k of the 32 W pairs), the paper's running example of Sec. 4.1 (group totals 2, 2, 8), and the
closed-form transition distribution P(v_i) = w_i / sum w (Theorem 1) for one-step samples."""
import json
import os
import random

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def brute(totals):
    W = int(sum(totals))
    cut, al = O.alias_table(totals)
    hits = [0] * 32
    for j in range(32):
        c = int(cut[j])
        assert 0 <= c <= W
        hits[j] += c
        hits[int(al[j])] += W - c
    return hits


@pytest.mark.parametrize("seed", range(12))
def test_alias_table_brute_force(seed):
    rng = random.Random(seed)
    totals = [0] * 32
    for k in rng.sample(range(12), rng.randrange(1, 12)):
        totals[k] = rng.randrange(1, 40) << k
    hits = brute(totals)
    assert list(hits) == [32 * t for t in totals]
    W = sum(totals)
    if W <= 1 << 13:  # every (slot, x) pair through the selection rule itself
        counts = np.zeros(32, np.int64)
        for j in range(32):
            for x in range(W):
                counts[O.alias_pick(totals, j, x)] += 1
        assert list(counts) == [32 * t for t in totals]


def test_alias_table_running_example():
    ex = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))["running"]
    # group totals of vertex 2 in the running example: 2^0 {1,5} -> 2, 2^1 {5} -> 2, 2^2 {1,4} -> 8
    totals = [0] * 32
    for _, _, w in ex["edges"]:
        for k in range(32):
            if (w >> k) & 1:
                totals[k] += 1 << k
    assert totals[:3] == [2, 2, 8]
    assert list(brute(totals))[:3] == [64, 64, 256]


def test_alias_table_edge_cases():
    assert brute([0, 0, 0, 5 << 3]) == [0, 0, 0, 32 * (5 << 3)] + [0] * 28  # one group: always chosen
    big = [(1 << 32) - 1 << k for k in range(32)]  # totals near 2^63 each: 128-bit intermediate values
    big[31] = ((1 << 32) - 1) << 31
    W = sum(big)
    assert W < 1 << 64
    hits = brute(big)
    assert list(hits) == [32 * t for t in big]


@pytest.mark.parametrize("adaptive", [True, False])
def test_alias_walk_distribution(adaptive):
    rng = random.Random(4)
    d = 14
    w = [rng.choice([1, 3, 8, 100, rng.randrange(1, 1 << 20)]) for _ in range(d)]
    g = O.Graph(d + 1, [0] * d, list(range(1, d + 1)), w, adaptive=adaptive, alias=True)
    n_samples = 200_000
    paths, _ = g.deepwalk(np.zeros(n_samples, np.uint32), 1, 33, threads=8)
    obs = np.bincount(paths[:, 1].astype(np.int64), minlength=d + 1)[1:]
    p = np.asarray(w, np.float64) / sum(w)
    chi2 = float((((obs - n_samples * p) ** 2) / (n_samples * p)).sum())
    assert stats.chi2.sf(chi2, d - 1) > 1e-6
    # the same graph with inverse transform: another stream use, the same distribution
    gi = O.Graph(d + 1, [0] * d, list(range(1, d + 1)), w, adaptive=adaptive)
    pi, _ = gi.deepwalk(np.zeros(2000, np.uint32), 1, 33)
    assert not np.array_equal(pi, paths[:2000])


def test_alias_rejects_fixed_point():
    with pytest.raises(O.OracleError):
        O.Graph(3, [0], [1], [256], frac_bits=8, alias=True)

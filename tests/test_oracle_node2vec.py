"""Pins of the oracle's node2vec walks (Sec. 2.2, Eq. node2vec), CPU only.

The oracle samples the second-order transition by rejection on the first-order sampler.  These
tests check it against what the definition fixes: the closed-form transition law
P(v | w, u) proportional to w_uv * f(w, v) (chi-square), its change when an update adds or
removes the edge w -> v, the exact reduction to DeepWalk at p = q = 1, the acceptance thresholds,
and the degenerate cases."""
from collections import Counter

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle as O

A, B, C, D, E, X = 0, 1, 2, 3, 4, 5


def f_factor(prev, v, nbrs_prev, p, q):
    if v == prev:
        return 1.0 / p
    if v in nbrs_prev:
        return 1.0
    return 1.0 / q


def second_step_law(edges, prev, u, p, q):
    """Closed form of Eq. node2vec: P(v) proportional to sum over parallel edges u->v of w * f."""
    nbrs_prev = {d for s, d, _ in edges if s == prev}
    mass = Counter()
    for s, d, w in edges:
        if s == u:
            mass[d] += w * f_factor(prev, d, nbrs_prev, p, q)
    tot = sum(mass.values())
    return {v: m / tot for v, m in mass.items()}


def empirical_second_step(g, prev, u, p, q, nsamp, seed):
    paths, _ = g.node2vec([prev] * nsamp, 2, seed, p, q)
    keep = paths[paths[:, 1] == u]
    return Counter(keep[:, 2].tolist()), len(keep)


# B's neighbours: A (back, distance 0), C (A -> C exists: distance 1), D twice (parallel edges),
# E (distance 2).  A reaches B or C.
EDGES = [(A, B, 10), (A, C, 1), (B, A, 3), (B, C, 5), (B, D, 1), (B, D, 6), (B, E, 2), (C, A, 1),
         (D, B, 1), (E, B, 4)]


def graph(edges, n=6, adaptive=True):
    return O.Graph(n, [e[0] for e in edges], [e[1] for e in edges], [e[2] for e in edges], adaptive=adaptive)


def test_thresholds():
    assert O.node2vec_thresholds(0.5, 2.0).tolist() == [1 << 32, 1 << 31, 1 << 30]
    assert O.node2vec_thresholds(1.0, 1.0).tolist() == [1 << 32] * 3
    assert O.node2vec_thresholds(2.0, 0.5).tolist() == [1 << 30, 1 << 31, 1 << 32]
    assert O.node2vec_thresholds(1.0, 3.0).tolist() == [1 << 32, 1 << 32, (1 << 32) // 3]
    with pytest.raises(ValueError):
        O.node2vec_thresholds(0.0, 1.0)
    with pytest.raises(ValueError):
        O.node2vec_thresholds(1.0, -2.0)


@pytest.mark.parametrize("p,q", [(0.5, 2.0), (2.0, 0.5), (1.0, 3.0)])
@pytest.mark.parametrize("adaptive", [True, False])
def test_second_order_law_chi2(p, q, adaptive):
    g = graph(EDGES, adaptive=adaptive)
    law = second_step_law(EDGES, A, B, p, q)
    obs, n = empirical_second_step(g, A, B, p, q, 120_000, seed=77)
    assert n > 100_000
    keys = sorted(law)
    assert set(obs) <= set(keys)
    o = np.array([obs[k] for k in keys], float)
    e = np.array([law[k] * n for k in keys])
    assert chisquare(o, e).pvalue > 1e-4


def test_law_follows_updates():
    # deleting A -> C turns C from distance 1 into distance 2; inserting A -> E does the opposite
    g = graph(EDGES)
    g.update([A], [E], [1], [A], [C])
    edges = [e for e in EDGES if e[:2] != (A, C)] + [(A, E, 1)]
    for p, q in [(0.5, 2.0), (2.0, 0.25)]:
        law = second_step_law(edges, A, B, p, q)
        obs, n = empirical_second_step(g, A, B, p, q, 100_000, seed=5)
        keys = sorted(law)
        o = np.array([obs[k] for k in keys], float)
        e = np.array([law[k] * n for k in keys])
        assert chisquare(o, e).pvalue > 1e-4


@pytest.mark.parametrize("adaptive", [True, False])
def test_p_q_one_is_deepwalk(adaptive):
    rng = np.random.default_rng(3)
    n = 200
    src = rng.integers(0, n, 3000)
    dst = rng.integers(0, n, 3000)
    w = rng.integers(1, 1 << 20, 3000)
    g = O.Graph(n, src, dst, w, adaptive=adaptive)
    starts = rng.integers(0, n, 500)
    a, sa = g.node2vec(starts, 30, seed=11, p=1.0, q=1.0, base=7)
    b, sb = g.deepwalk(starts, 30, seed=11, base=7)
    assert np.array_equal(a, b) and sa == sb


def test_degenerate_cases():
    # a sink start stops at once; a walk reaching a sink stops there
    g2 = O.Graph(4, [0, 1], [1, 2], [1, 1])  # 0 -> 1 -> 2, vertex 2 is a sink
    paths, steps = g2.node2vec([0, 2], 4, seed=3, p=0.5, q=2.0)
    assert paths[0].tolist() == [0, 1, 2, O.STOP, O.STOP] and steps == 2
    assert paths[1].tolist() == [2] + [O.STOP] * 4
    # a walk that can never accept gives up after 2^15 proposals and stops: from 0 -> 1 the only
    # move is 1 -> 2 (distance 2), whose threshold is 0 when 1/q is negligible next to 1/p
    assert O.node2vec_thresholds(1e-12, 1.0)[2] == 0
    paths, steps, props = g2.node2vec([0], 3, seed=3, p=1e-12, q=1.0, with_proposals=True)
    assert paths[0].tolist() == [0, 1, O.STOP, O.STOP] and steps == 1
    assert props == 1 + (1 << 15)


def test_first_step_is_first_order():
    # the first transition has no previous vertex: the first-order law w / sum w
    g = graph(EDGES)
    paths, _ = g.node2vec([B] * 60_000, 1, seed=21, p=0.25, q=4.0)
    obs = Counter(paths[:, 1].tolist())
    mass = Counter()
    for s, d, w in EDGES:
        if s == B:
            mass[d] += w
    keys = sorted(mass)
    tot = sum(mass.values())
    o = np.array([obs[k] for k in keys], float)
    e = np.array([mass[k] / tot * 60_000 for k in keys])
    assert chisquare(o, e).pvalue > 1e-4


def test_thread_count_invariance():
    rng = np.random.default_rng(8)
    n = 300
    g = O.Graph(n, rng.integers(0, n, 4000), rng.integers(0, n, 4000), rng.integers(1, 1 << 16, 4000))
    starts = rng.integers(0, n, 2000)
    a, _ = g.node2vec(starts, 20, seed=4, p=0.5, q=2.0, threads=1)
    b, _ = g.node2vec(starts, 20, seed=4, p=0.5, q=2.0, threads=8)
    assert np.array_equal(a, b)

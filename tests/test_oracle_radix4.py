"""Radix base 4 (Supplement S.2, Fig. 17) in the oracle: groups by base-4 digit, split into subgroups
of equal digit so that every subgroup is uniform.  Pinned by brute force over the subgroup draw, by
exact transition probabilities (Theorem 1 carried over: P(v_i) = w_i / sum w), by chi-square tests of
one-step samples and by special cases that reduce to uniform or deterministic moves."""
import random
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def digits4(w):
    return [(w >> (2 * k)) & 3 for k in range(16)]


def test_subgroup_counts_follow_the_base4_digits():
    """The supplement's example has two members with digit 2 and three with digit 3 in group 4^0;
    any vertex with those digits gets c(0,2) = 2 and c(0,3) = 3, its other subgroups from the
    remaining digits, each subgroup listed or dense by the type rule on (c, d)."""
    w = [2, 2 + 4, 3, 3 + 16, 3, 4 * 3]
    g = O.Graph4(7, [0] * 6, [1, 2, 3, 4, 5, 6], w)
    v = O.parse_dump4(g.dump(), 7)[0]
    c = {s: cc for s, (t, cc, m) in v["subgroups"].items()}
    assert c[0 * 3 + 1] == 2 and c[0 * 3 + 2] == 3           # digit 0: two 2s, three 3s
    assert c[1 * 3 + 0] == 1 and c[1 * 3 + 2] == 1           # digit 1: one 1 (w = 6), one 3 (w = 12)
    assert c[2 * 3 + 0] == 1                                  # digit 2: one 1 (w = 19)
    assert sum(c.values()) == sum(sum(1 for x in digits4(ww) if x) for ww in w)
    for s, (t, cc, m) in v["subgroups"].items():
        assert t == O.type_of(cc, 6)
        k, dv = s // 3, s % 3 + 1
        members = [i for i in range(6) if digits4(w[i])[k] == dv]
        if t in (O.T_SPARSE, O.T_REGULAR):
            assert m == members                               # ascending
        elif t == O.T_ONE:
            assert m == members


def test_subgroup_draw_exhaustive():
    """For a small W every r in [0, W) goes through the selection: subgroup s gets exactly
    c_s * v * 4^k values, in ascending runs."""
    rng = random.Random(5)
    for _ in range(30):
        c = [0] * 48
        for s in rng.sample(range(0, 21), 6):
            c[s] = rng.randrange(1, 4)
        W = sum(c[s] * (s % 3 + 1) * 4 ** (s // 3) for s in range(48))
        got = [O.pick_subgroup(c, r) for r in range(W)]
        exp = [s for s in range(48) for _ in range(c[s] * (s % 3 + 1) * 4 ** (s // 3))]
        assert got == exp


def exact_probabilities4(v):
    """P(edge i) from the structure: subgroup s with probability T_s / W, then its member rule
    (one element; uniform over the list; dense rejection = uniform over the members)."""
    d = v["d"]
    W = int(v["w"].astype(np.int64).sum())
    P = [Fraction(0)] * d
    for s, (t, c, members) in v["subgroups"].items():
        k, dv = s // 3, s % 3 + 1
        ps = Fraction(c * dv * 4 ** k, W)
        if t == O.T_ONE:
            P[members[0]] += ps
        elif t in (O.T_SPARSE, O.T_REGULAR):
            for i in members:
                P[i] += ps / c
        else:
            acc = [i for i in range(d) if (int(v["w"][i]) >> (2 * k)) & 3 == dv]
            assert len(acc) == c
            for i in acc:
                P[i] += ps * (Fraction(1, d) / Fraction(len(acc), d))
    return P, W


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_theorem1_exact_base4(adaptive, seed):
    rng = random.Random(seed)
    n, m = 12, 90
    src = [rng.randrange(n) for _ in range(m)]
    w = [rng.choice([1, 2, 3, 5, 15, 16, 63, rng.randrange(1, 1 << 20), rng.randrange(1, 1 << 32)]) for _ in range(m)]
    g = O.Graph4(n, src, [rng.randrange(n) for _ in range(m)], w, adaptive=adaptive)
    for v in O.parse_dump4(g.dump(), n):
        if v["d"] == 0:
            continue
        P, W = exact_probabilities4(v)
        assert all(P[i] == Fraction(int(v["w"][i]), W) for i in range(v["d"]))


def test_one_step_chi2_base4():
    from scipy.stats import chisquare
    rng = random.Random(9)
    d = 60
    w = [rng.choice([1, 2, 3, 7, 11, 48, 255, 1000, 70000]) for _ in range(d)]
    g = O.Graph4(d + 1, [0] * d, list(range(1, d + 1)), w)
    nsamp = 200_000
    paths, steps = g.deepwalk([0] * nsamp, 1, seed=77)
    assert steps == nsamp
    obs = Counter(paths[:, 1].tolist())
    W = sum(w)
    o = np.array([obs[i + 1] for i in range(d)], float)
    e = np.array([w[i] * nsamp / W for i in range(d)])
    assert chisquare(o, e).pvalue > 1e-4


def test_special_cases_base4():
    # every weight 3: one subgroup (digit 0 = 3) holding all edges, dense: uniform moves
    g = O.Graph4(5, [0] * 4, [1, 2, 3, 4], [3] * 4)
    v = O.parse_dump4(g.dump(), 5)[0]
    assert list(v["subgroups"]) == [2] and v["subgroups"][2][0] == O.T_DENSE
    paths, _ = g.deepwalk([0] * 40_000, 1, seed=3)
    cnt = Counter(paths[:, 1].tolist())
    assert all(abs(cnt[x] - 10_000) < 600 for x in (1, 2, 3, 4))
    # degree one: deterministic; sink: stop
    g = O.Graph4(3, [0], [2], [123456])
    paths, steps = g.deepwalk([0, 1], 3, seed=1)
    assert paths[0].tolist() == [0, 2, 0xFFFFFFFF, 0xFFFFFFFF] and steps == 1
    assert paths[1].tolist() == [1] + [0xFFFFFFFF] * 3
    # powers of four: each edge in exactly one subgroup (digit 1 of its power)
    w = [4 ** k for k in range(16)]
    g = O.Graph4(17, [0] * 16, list(range(1, 17)), w)
    v = O.parse_dump4(g.dump(), 17)[0]
    assert sorted(v["subgroups"]) == [3 * k for k in range(16)]


def test_bad_input_base4():
    with pytest.raises(O.OracleError):
        O.Graph4(3, [0], [5], [1])
    with pytest.raises(O.OracleError):
        O.Graph4(3, [0], [1], [0])

"""Pins of the oracle's floating-point-bias mode (Sec. 4.3, Fig. SAMPLING2; Sec. 4.4 complexity).

Pinned against: the paper's worked example (tests/golden/paper_examples.json, "floating"),
hand-computed quantizations, the closed-form transition distribution P(v_i) = w_i / sum w
(Theorem 1) under the quantized weights, and the invariant that an updated structure equals a
fresh build of the same adjacency up to the order inside kept lists.
"""
import json
import os
import random

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
EX = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))["floating"]


def test_quantize_hand_values():
    F = 8
    cases = [(0.5, 1.0, 128), (1.0, 1.0, 256), (3.75, 2.0, 1920), (1.0 / 256, 1.0, 1), (255.99609375, 1.0, 65535),
             (16777215.0, 1.0, 4294967040)]
    got = O.quantize([c[0] for c in cases], 1.0, F)
    # lambda differs per case: quantize them one by one
    for b, lam, want in cases:
        assert int(O.quantize([b], lam, F)[0]) == want, (b, lam)
    assert len(got) == len(cases)
    # 4 fraction bits: 3.75 * 2 = 7.5 -> 120
    assert int(O.quantize([3.75], 2.0, 4)[0]) == 120
    # float32 inputs: 0.1f = 0.100000001490116..., times 10 rounds to 1.0000000149..., floor(x * 256) = 256
    assert int(O.quantize([0.1], 10.0, 8)[0]) == 256


@pytest.mark.parametrize("b,lam,F", [(-1.0, 1.0, 8), (float("nan"), 1.0, 8), (float("inf"), 1.0, 8),
                                     (1e-6, 1.0, 8), (16777216.0, 1.0, 8), (0.0, 5.0, 4), (1.0, -1.0, 8)])
def test_quantize_rejects(b, lam, F):
    assert int(O.quantize([b], lam, F)[0]) == 0


def test_paper_example_groups():
    """Fig. SAMPLING2: integer-part groups and the decimal group of vertex 2, and the 1/16 share."""
    F = 8
    src = [e[0] for e in EX["edges"]]
    dst = [e[1] for e in EX["edges"]]
    w = O.quantize([e[2] for e in EX["edges"]], EX["lambda"], F)
    g = O.Graph(6, src, dst, w, adaptive=False, frac_bits=F)  # every group listed: members are dumped
    v = O.parse_dump(g.dump(), 6)[EX["vertex"]]
    dsts = [int(x) for x in v["dst"]]
    for j, members in EX["integer_groups_logical"].items():
        t, c, lst = v["groups"][F + int(j)]
        assert sorted(dsts[i] for i in lst) == members, j
    t, c, lst = v["groups"][0]
    assert sorted(dsts[i] for i in lst) == EX["decimal_group_logical"]
    assert set(v["groups"]) == {0} | {F + int(j) for j in EX["integer_groups_logical"]}
    frac = sum(int(x) & ((1 << F) - 1) for x in v["w"])
    share = frac / sum(int(x) for x in v["w"])
    assert abs(share - EX["decimal_share"]) < 3 * 2.0 ** -F / 15  # three truncated fractions


def _freq_check(biases, lam, F, adaptive=True, n_samples=200_000, seed=77):
    d = len(biases)
    w = O.quantize(biases, lam, F)
    assert (w > 0).all()
    g = O.Graph(d + 1, [0] * d, list(range(1, d + 1)), w, adaptive=adaptive, frac_bits=F)
    paths, _ = g.deepwalk(np.zeros(n_samples, np.uint32), 1, seed, threads=8)
    obs = np.bincount(paths[:, 1].astype(np.int64), minlength=d + 1)[1:]
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    chi2 = float((((obs - n_samples * p) ** 2) / (n_samples * p)).sum())
    assert stats.chi2.sf(chi2, d - 1) > 1e-6, (chi2, obs, n_samples * p)
    return g


def _types(g, u):
    v = O.parse_dump(g.dump(), g.n)[u]
    return {k: t for k, (t, c, m) in v["groups"].items()}


def test_distribution_dense_decimal_group():
    g = _freq_check([0.554, 0.726, 0.320], 10.0, 8)
    assert _types(g, 0)[0] == O.T_DENSE


def test_distribution_heavy_decimal_group():
    # lambda = 1: fractions carry about half of the total, so the decimal group is drawn often
    rng = random.Random(5)
    g = _freq_check([rng.uniform(0.05, 2.0) for _ in range(12)], 1.0, 6)
    assert _types(g, 0)[0] == O.T_DENSE


def test_distribution_listed_decimal_group():
    rng = random.Random(6)
    b = [float(rng.randrange(1, 9)) for _ in range(20)]
    b[3] += 0.75; b[11] += 0.5; b[17] += 0.25  # 3 of 20 edges with fractions: regular (15 %)
    g = _freq_check(b, 1.0, 8)
    assert _types(g, 0)[0] == O.T_REGULAR
    b = [float(rng.randrange(1, 9)) for _ in range(50)]
    b[7] += 0.5; b[40] += 0.875  # 2 of 50: sparse
    g = _freq_check(b, 1.0, 8)
    assert _types(g, 0)[0] == O.T_SPARSE


def test_distribution_one_element_decimal_group():
    b = [float(x) for x in (3, 1, 4, 1, 5, 9, 2, 6)]
    b[5] += 0.375
    g = _freq_check(b, 1.0, 8)
    assert _types(g, 0)[0] == O.T_ONE


def test_distribution_without_adaption():
    rng = random.Random(8)
    _freq_check([rng.uniform(0.5, 30.0) for _ in range(9)], 3.0, 10, adaptive=False)


def test_update_matches_fresh_build():
    """After float-bias batches, counts, types, one-element members and list contents equal a fresh
    build of the resulting adjacency (list order may differ: kept lists are edited in place)."""
    rng = random.Random(9)
    F, n = 8, 30
    src = [rng.randrange(n) for _ in range(300)] + [0] * 200
    dst = [rng.randrange(n) for _ in range(500)]
    bias = [rng.choice([rng.uniform(0.01, 1.0), float(rng.randrange(1, 50)), rng.uniform(1.0, 4000.0)])
            for _ in range(500)]
    g = O.Graph(n, src, dst, O.quantize(bias, 4.0, F), frac_bits=F)
    for b in range(6):
        cur = O.parse_dump(g.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ins = [(rng.randrange(n) if rng.random() < 0.5 else 0, rng.randrange(n)) for _ in range(rng.randrange(40))]
        iw = O.quantize([rng.uniform(0.01, 300.0) for _ in ins], 4.0, F)
        dels = [rng.choice(live) for _ in range(rng.randrange(60))]
        g.update([a for a, _ in ins], [c for _, c in ins], iw, [a for a, _ in dels], [c for _, c in dels])
        after = O.parse_dump(g.dump(), n)
        fsrc = [u for u, v in enumerate(after) for _ in v["dst"]]
        fresh = O.parse_dump(O.Graph(n, fsrc, np.concatenate([v["dst"] for v in after]),
                                     np.concatenate([v["w"] for v in after]), frac_bits=F).dump(), n)
        for u in range(n):
            a, f = after[u], fresh[u]
            assert np.array_equal(a["dst"], f["dst"]) and np.array_equal(a["w"], f["w"])
            assert set(a["groups"]) == set(f["groups"]), (b, u)
            for k, (t, c, m) in a["groups"].items():
                tf, cf, mf = f["groups"][k]
                assert (t, c) == (tf, cf), (b, u, k)
                if m is not None:
                    assert sorted(m) == sorted(mf), (b, u, k)
                if 1 <= k < F:
                    raise AssertionError("slots 1..F-1 must stay empty")

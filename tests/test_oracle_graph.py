"""Pins of the oracle's structures, sampling step, walks and batched updates.  CPU only.

Each check compares the oracle with something other than itself: the paper's worked examples
(tests/golden/paper_examples.json), closed forms (Theorem 1: P(v_i) = w_i / sum w; group
totals c_k 2^k), invariants, rebuild-from-scratch equality, multiset bookkeeping of the batch,
brute force on tiny inputs and statistical tests."""
import json
import os
import random
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import GOLDEN

EX = json.load(open(os.path.join(GOLDEN, "paper_examples.json")))


def one_vertex_graph(edges, n=8, adaptive=False):
    src = [e[0] for e in edges]; dst = [e[1] for e in edges]; w = [e[2] for e in edges]
    return O.Graph(n, src, dst, w, adaptive=adaptive)


def vertex(g, u):
    return O.parse_dump(g.dump(), g.n)[u]


def logical(v, k):
    t, c, members = v["groups"][k]
    return [int(v["dst"][i]) for i in members]


# --------------------------------------------------------------------------- paper examples
def test_running_example_groups():
    ex = EX["running"]
    g = one_vertex_graph(ex["edges"])
    v = vertex(g, ex["vertex"])
    for k, members in ex["group_members_logical"].items():
        k = int(k)
        t, c, _ = v["groups"][k]
        assert t == O.T_REGULAR
        assert sorted(logical(v, k)) == sorted(members)
        assert c << k == ex["group_bias"][str(k)]
    # with adaption: c/d = 2/3 > 40% -> dense for 2^0 and 2^2, 2^1 holds one element
    ga = one_vertex_graph(ex["edges"], adaptive=True)
    vg = vertex(ga, ex["vertex"])
    assert vg["groups"][0][0] == O.T_DENSE and vg["groups"][2][0] == O.T_DENSE
    assert vg["groups"][1][0] == O.T_ONE and logical(vg, 1) == [5]


def test_insertion_example():
    ex = EX["insert"]
    g = one_vertex_graph(EX["running"]["edges"])
    s, d, w = ex["edge"]
    g.update([s], [d], [w], [], [])
    v = vertex(g, s)
    idx = v["d"] - 1
    assert int(v["dst"][idx]) == d
    for k in range(3):
        members = v["groups"][k][2]
        assert (idx in members) == (k in ex["groups_joined"])
        if k in ex["groups_joined"]:
            assert members[-1] == idx  # appended at the end of the group list
    for k, b in ex["group_bias_after"].items():
        assert v["groups"][int(k)][1] << int(k) == b
    assert sum(ex["group_bias_after"].values()) == int(v["w"].sum())


def test_deletion_example():
    ex = EX["delete"]
    g = one_vertex_graph(EX["running"]["edges"])
    ins = EX["insert"]["edge"]
    g.update([ins[0]], [ins[1]], [ins[2]], [], [])
    before = vertex(g, 2)
    assert before["groups"][0][2] == ex["group0_list_before"]
    s, d, w = ex["edge"]
    assert int(before["dst"][ex["neighbor_index"]]) == d
    st = g.update([], [], [], [s], [d])
    assert st["deleted"] == 1 and st["not_found"] == 0
    v = vertex(g, 2)
    # group 2^0: the deleted index 0 was replaced by the tail index 3 (renamed to its new slot 0)
    assert logical(v, 0)[0] == before["dst"][ex["group0_tail_swapped_in"]]
    for k, members in ex["group_members_logical_after"].items():
        assert logical(v, int(k)) == members
    for k, b in ex["group_bias_after"].items():
        assert v["groups"][int(k)][1] << int(k) == b


def test_dense_example_and_type_rule():
    ex = EX["dense"]
    assert O.type_of(ex["c"], ex["d"]) == O.T_DENSE
    # precedence and strict comparisons (alpha = 40, beta = 10)
    assert O.type_of(0, 10) == O.T_EMPTY
    assert O.type_of(1, 2) == O.T_ONE          # 50% but one element
    assert O.type_of(1, 100) == O.T_ONE        # 1% but one element
    assert O.type_of(2, 5) == O.T_REGULAR      # exactly 40% is not dense
    assert O.type_of(3, 5) == O.T_DENSE
    assert O.type_of(2, 20) == O.T_REGULAR     # exactly 10% is not sparse
    assert O.type_of(2, 21) == O.T_SPARSE
    assert O.type_of(7, 8, adaptive=False) == O.T_REGULAR
    assert O.type_of(10**9, 2 * 10**9 + 1) == O.T_DENSE  # no 32-bit overflow in 100c
    for c in range(0, 60):
        for d in range(max(c, 1), 60):
            t = O.type_of(c, d)
            if c == 0:
                assert t == O.T_EMPTY
            elif c == 1:
                assert t == O.T_ONE
            elif Fraction(c, d) > Fraction(40, 100):
                assert t == O.T_DENSE
            elif Fraction(c, d) < Fraction(10, 100):
                assert t == O.T_SPARSE
            else:
                assert t == O.T_REGULAR


def test_two_phase_example():
    ex = EX["two_phase"]
    flags = [1 if i in ex["delete_positions"] else 0 for i in range(len(ex["array"]))]
    out = O.two_phase(ex["array"], flags)
    assert len(out) == len(ex["array"]) - len(ex["delete_positions"])
    assert ex["filled_with_not"] not in out.tolist()
    assert out[0] == 8
    # a small case: deleting positions {0,1} of [a,b,c,d] pairs the holes with the tail by rank
    assert O.two_phase([10, 11, 12, 13], [1, 1, 0, 0]).tolist() == [12, 13]


def test_two_phase_brute_force():
    rng = random.Random(0)
    for _ in range(500):
        n = rng.randrange(0, 20)
        arr = list(range(100, 100 + n))
        dele = [rng.random() < 0.4 for _ in range(n)]
        out = O.two_phase(arr, dele).tolist()
        N = sum(dele)
        nl = n - N
        assert sorted(out) == sorted(a for a, d in zip(arr, dele) if not d)
        holes = [i for i in range(nl) if dele[i]]
        tail = [arr[i] for i in range(nl, n) if not dele[i]]
        assert len(holes) == len(tail)
        for i in range(nl):
            if not dele[i]:
                assert out[i] == arr[i]        # untouched entries stay in place
        assert [out[h] for h in holes] == tail  # holes filled by tail survivors in rank order


# --------------------------------------------------------------------------- sampling exactness
def exact_probabilities(v):
    """P(neighbor index i) of one step, enumerated exactly from the dumped structure:
    inter-group ITS over every r in [0, W) through the oracle's selection function, then the
    group's own member rule (list entry j uniform, the single member, or rejection on the
    adjacency whose acceptance set is enumerated)."""
    d = v["d"]
    counts = [0] * 32
    for k, (t, c, _) in v["groups"].items():
        counts[k] = c
    W = sum(c << k for k, c in enumerate(counts))
    hits = Counter(O.pick_group(counts, r) for r in range(W))
    P = [Fraction(0)] * d
    for k, nr in hits.items():
        pk = Fraction(nr, W)
        t, c, members = v["groups"][k]
        if t == O.T_ONE:
            P[members[0]] += pk
        elif t in (O.T_SPARSE, O.T_REGULAR):
            for j in range(c):
                P[members[j]] += pk / c
        else:
            acc = [i for i in range(d) if (int(v["w"][i]) >> k) & 1]
            # each attempt is uniform over the d slots; the geometric series gives 1/|acc| each
            for i in acc:
                P[i] += pk * (Fraction(1, d) / Fraction(len(acc), d))
    return P, W


def small_graph(seed, n=12, m=70, wmax=40, adaptive=True):
    rng = random.Random(seed)
    src = [rng.randrange(n) for _ in range(m)]
    dst = [rng.randrange(n) for _ in range(m)]
    w = [rng.randrange(1, wmax) for _ in range(m)]
    return O.Graph(n, src, dst, w, adaptive=adaptive)


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_theorem1_exact(adaptive, seed):
    g = small_graph(seed, adaptive=adaptive)
    for v in O.parse_dump(g.dump(), g.n):
        if v["d"] == 0:
            continue
        P, W = exact_probabilities(v)
        assert W == int(v["w"].astype(np.int64).sum())
        for i in range(v["d"]):
            assert P[i] == Fraction(int(v["w"][i]), W)


def skew_graph(adaptive=True):
    """A hand-made vertex 0 that holds every group type: d = 40."""
    w = [1] * 40                                   # bit 0 in all: dense
    for i in range(0, 12):
        w[i] |= 2                                  # bit 1 in 12 of 40 = 30%: regular
    for i in (5, 9, 17):
        w[i] |= 4                                  # bit 2 in 3 of 40 = 7.5%: sparse
    w[33] |= 1 << 9                                # bit 9 once: one-element
    for i in range(0, 40, 2):
        w[i] |= 8                                  # bit 3 in 20 of 40 = 50%: dense
    src = [0] * 40 + [1, 1, 2]
    dst = list(range(1, 41)) + [0, 2, 1]
    w = w + [3, 6, 1]
    return O.Graph(45, src, dst, w, adaptive=adaptive)


def test_skew_vertex_types_and_exactness():
    g = skew_graph()
    v = vertex(g, 0)
    types = {k: t for k, (t, c, m) in v["groups"].items()}
    assert types == {0: O.T_DENSE, 1: O.T_REGULAR, 2: O.T_SPARSE, 3: O.T_DENSE, 9: O.T_ONE}
    P, W = exact_probabilities(v)
    assert all(P[i] == Fraction(int(v["w"][i]), W) for i in range(40))


def test_one_step_chi2():
    from scipy.stats import chisquare
    g = skew_graph()
    v = vertex(g, 0)
    nsamp = 200_000
    paths, steps = g.deepwalk([0] * nsamp, 1, seed=1234)
    assert steps == nsamp
    obs = Counter(paths[:, 1].tolist())
    W = int(v["w"].astype(np.int64).sum())
    exp = Counter()
    for i in range(v["d"]):
        exp[int(v["dst"][i])] += int(v["w"][i])
    keys = sorted(exp)
    o = np.array([obs[k] for k in keys], float)
    e = np.array([exp[k] * nsamp / W for k in keys])
    assert chisquare(o, e).pvalue > 1e-4


def test_special_cases():
    # all weights 1: a single dense group, the walk is uniform over slots
    g = O.Graph(5, [0] * 4, [1, 2, 3, 4], [1] * 4)
    v = vertex(g, 0)
    assert list(v["groups"]) == [0] and v["groups"][0][0] == O.T_DENSE
    paths, _ = g.deepwalk([0] * 40000, 1, seed=9)
    cnt = np.bincount(paths[:, 1], minlength=5)[1:]
    assert cnt.min() > 9400 and cnt.max() < 10600
    # powers of two: each edge in exactly one group
    g = O.Graph(5, [0] * 4, [1, 2, 3, 4], [1, 2, 4, 8], adaptive=False)
    v = vertex(g, 0)
    assert all(v["groups"][k][1] == 1 for k in range(4))
    # degree one: a deterministic move; sinks stop the walk
    g = O.Graph(3, [0], [2], [77])
    paths, steps = g.deepwalk([0, 1], 3, seed=5)
    assert paths[0].tolist() == [0, 2, O.STOP, O.STOP] and paths[1].tolist() == [1, O.STOP, O.STOP, O.STOP]
    assert steps == 1


# --------------------------------------------------------------------------- updates
def check_invariants(g):
    for u, v in enumerate(O.parse_dump(g.dump(), g.n)):
        d = v["d"]
        w = v["w"].astype(np.int64)
        assert len(set(v["seq"].tolist())) == d and (d == 0 or v["seq"].max() < v["next_seq"])
        total = 0
        for k in range(32):
            members = {i for i in range(d) if (w[i] >> k) & 1}
            if not members:
                assert k not in v["groups"]
                continue
            t, c, lst = v["groups"][k]
            assert c == len(members)
            assert t == O.type_of(c, d, g.adaptive)
            if t == O.T_ONE:
                assert set(lst) == members
            elif t in (O.T_SPARSE, O.T_REGULAR):
                assert len(lst) == c and set(lst) == members
            total += c << k
        assert total == int(w.sum())


def rebuilt_equal(g):
    """Rebuild from scratch from the current adjacency; structures must agree up to list order."""
    vs = O.parse_dump(g.dump(), g.n)
    src = np.concatenate([np.full(v["d"], u, np.uint32) for u, v in enumerate(vs)])
    dst = np.concatenate([v["dst"] for v in vs]); w = np.concatenate([v["w"] for v in vs])
    h = O.Graph(g.n, src, dst, w, adaptive=g.adaptive)
    for a, b in zip(vs, O.parse_dump(h.dump(), g.n)):
        assert a["d"] == b["d"]
        assert (a["dst"] == b["dst"]).all() and (a["w"] == b["w"]).all()
        assert set(a["groups"]) == set(b["groups"])
        for k in a["groups"]:
            ta, ca, ma = a["groups"][k]
            tb, cb, mb = b["groups"][k]
            assert (ta, ca) == (tb, cb)
            if ma is not None:
                assert sorted(ma) == sorted(mb)


def batch_multiset_expectation(before, ins, dels):
    """Per vertex multiset of (dst, w, seq) after the batch, from bookkeeping alone: inserts get
    seq = next_seq, next_seq + 1, ... in batch order; a delete of (u, t) removes the live
    occurrence of (u, t) with the smallest seq; surplus deletes are not found."""
    state = {u: {"edges": [(int(a), int(b), int(c)) for a, b, c in zip(v["dst"], v["w"], v["seq"])],
                 "next": v["next_seq"]} for u, v in enumerate(before)}
    for (s, d, w) in ins:
        st = state[s]
        st["edges"].append((d, w, st["next"]))
        st["next"] += 1
    nf = 0
    for (s, d) in dels:
        cands = [e for e in state[s]["edges"] if e[0] == d]
        if not cands:
            nf += 1
            continue
        state[s]["edges"].remove(min(cands, key=lambda e: e[2]))
    return state, nf


@pytest.mark.parametrize("adaptive", [True, False])
def test_update_batches_invariants_and_rebuild(adaptive):
    rng = random.Random(42)
    n = 30
    src = [rng.randrange(n) for _ in range(300)] + [0] * 60
    dst = [rng.randrange(n) for _ in range(300)] + [rng.randrange(4) for _ in range(60)]  # duplicates
    w = [rng.choice([1, 2, 3, 7, 64, 1000, rng.randrange(1, 1 << 20)]) for _ in range(360)]
    g = O.Graph(n, src, dst, w, adaptive=adaptive)
    check_invariants(g)
    for b in range(12):
        before = O.parse_dump(g.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(before) for t in v["dst"]]
        ni = rng.randrange(0, 40)
        nd = rng.randrange(0, 40)
        hub = rng.random() < 0.5
        ins = [(0 if hub and rng.random() < 0.7 else rng.randrange(n), rng.randrange(n),
                rng.choice([1, 3, 5, 1 << rng.randrange(31), rng.randrange(1, 1 << 31)])) for _ in range(ni)]
        dels = [rng.choice(live) if live and rng.random() < 0.85 else (rng.randrange(n), rng.randrange(n))
                for _ in range(nd)]
        # occasionally delete an edge inserted in this same batch
        if ins and rng.random() < 0.5:
            dels.append(ins[0][:2])
        st = g.update([a for a, _, _ in ins], [b for _, b, _ in ins], [c for _, _, c in ins],
                      [a for a, _ in dels], [b for _, b in dels])
        exp, nf = batch_multiset_expectation(before, ins, dels)
        assert st["inserted"] == len(ins) and st["not_found"] == nf and st["deleted"] == len(dels) - nf
        after = O.parse_dump(g.dump(), n)
        for u, v in enumerate(after):
            got = sorted(zip(v["dst"].tolist(), v["w"].tolist(), v["seq"].tolist()))
            assert got == sorted(exp[u]["edges"]), (b, u)
            assert v["next_seq"] == exp[u]["next"]
        check_invariants(g)
        rebuilt_equal(g)


def test_update_rejects_bad_input_without_change():
    g = small_graph(5)
    before = g.dump().copy()
    with pytest.raises(O.OracleError):
        g.update([0], [1], [0], [], [])          # zero weight
    with pytest.raises(O.OracleError):
        g.update([0], [99], [3], [], [])         # vertex out of range
    with pytest.raises(O.OracleError):
        g.update([], [], [], [100], [1])
    assert (g.dump() == before).all()


def test_paper_tail_delete_example_on_adjacency():
    # deleting two edges where one is the tail: the tail one disappears, the other hole is
    # filled by the last survivor of the tail window
    g = O.Graph(12, [0] * 10, list(range(1, 11)), [1] * 10, adaptive=False)
    g.update([], [], [], [0, 0], [1, 10])
    v = vertex(g, 0)
    assert v["dst"].tolist() == [9, 2, 3, 4, 5, 6, 7, 8]
    assert v["groups"][0][2] == list(range(8)) or sorted(v["groups"][0][2]) == list(range(8))


# --------------------------------------------------------------------------- PPR
def test_ppr_matches_linear_solve():
    """Expected visits per walk solve x = e_s + (1 - p) P^T x over non-sink rows (the cap of 200
    changes the expectation by less than 0.85^200)."""
    rng = random.Random(8)
    n = 9
    src, dst, w = [], [], []
    for u in range(n - 1):              # vertex n-1 is a sink
        for _ in range(rng.randrange(1, 5)):
            src.append(u); dst.append(rng.randrange(n)); w.append(rng.randrange(1, 50))
    g = O.Graph(n, src, dst, w)
    p = 0.15
    thr = int(p * 2**32)
    Pm = np.zeros((n, n))
    for s, d, ww in zip(src, dst, w):
        Pm[s, d] += ww
    Pm = Pm / np.maximum(Pm.sum(1, keepdims=True), 1)
    M = (1 - p) * Pm
    sources = [0, 3]
    R = 40000
    off, vtx, cnt, steps = g.ppr(sources, R, thr, 200, seed=77, base=0)
    assert int(cnt.sum()) == len(sources) * R + steps
    for q, s in enumerate(sources):
        x = np.linalg.solve(np.eye(n) - M.T, np.eye(n)[s])
        got = np.zeros(n)
        got[vtx[off[q]:off[q + 1]]] = cnt[off[q]:off[q + 1]]
        assert (np.diff(vtx[off[q]:off[q + 1]].astype(np.int64)) > 0).all()
        mean = got / R
        # per-walk visit counts have variance below E[L^2]; a 6-sigma band on the mean
        sd = np.sqrt(np.maximum(x * (1 + 2 / p), 1e-9) / R)
        assert (np.abs(mean - x) < 6 * sd + 1e-12).all(), (mean, x)


def test_walks_thread_count_invariant():
    g = small_graph(4, n=40, m=300)
    starts = list(range(40)) * 5
    a, sa = g.deepwalk(starts, 20, seed=3, threads=1)
    b, sb = g.deepwalk(starts, 20, seed=3, threads=4)
    assert (a == b).all() and sa == sb
    r1 = g.ppr([0, 1, 2], 300, int(0.15 * 2**32), 200, seed=5, threads=1)
    r2 = g.ppr([0, 1, 2], 300, int(0.15 * 2**32), 200, seed=5, threads=3)
    for x, y in zip(r1, r2):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_memory_model_orders():
    g = small_graph(6, n=50, m=2000, wmax=1 << 20)
    mem = g.memory()
    assert mem["adjacency"] == 12 * 2000
    ga = mem["one"] + mem["sparse"] + mem["regular"] + mem["sparse_reduced_lists"]
    assert ga < mem["all_regular_groups"] < mem["naive_bound"]


# ---- memory model (Sec. 4.4 space formula; Sec. 5.1 per-type structures; Sec. 6.3 all-regular baseline)
# Expected byte counts are worked out by hand from the per-type rules: one-element 4 B (the member),
# dense nothing, regular 4(c + d) (its list and a full inverted index over the d neighbour indices),
# sparse 4c + 4|S| (its list and an inverted index over the reduced list S(u) of edges in at least one
# sparse group) plus 4|S| once per vertex for S(u) itself; the all-regular baseline charges 4(c + d)
# for every non-empty group; the naive bound is 4(dK + sum_i popc w_i) with K = 32.

def test_memory_model_running_example():
    """Sec. 4.1 running example, vertex 2 with weights 5, 4, 3: groups 2^0 = {5, 3} (c = 2 of d = 3,
    dense), 2^1 = {3} (one-element), 2^2 = {5, 4} (dense)."""
    g = O.Graph(6, [2, 2, 2], [1, 4, 5], [5, 4, 3])
    mem = g.memory()
    assert mem == {"adjacency": 36, "one": 4, "dense": 0, "sparse": 0, "regular": 0, "reserved": 0,
                   "sparse_reduced_lists": 0,
                   "all_regular_groups": 4 * ((2 + 3) + (1 + 3) + (2 + 3)),   # 56
                   "naive_bound": 4 * (3 * 32 + 2 + 1 + 2)}                   # 404
    bs = O.Graph(6, [2, 2, 2], [1, 4, 5], [5, 4, 3], adaptive=False).memory()
    assert bs["regular"] == 56 and bs["one"] == 0 and bs["all_regular_groups"] == 56


def test_memory_model_skew_graph():
    """The skew graph: vertex 0 (d = 40) with dense groups 0 and 3, regular group 1 (c = 12), sparse
    group 2 (edges 5, 9, 17) and one-element group 9; vertex 1 (weights 3, 6: one-element groups 0
    and 2, dense group 1); vertex 2 (weight 1: one-element group 0)."""
    mem = skew_graph().memory()
    assert mem["adjacency"] == 12 * 43
    assert mem["one"] == 4 + 2 * 4 + 4
    assert mem["dense"] == 0
    assert mem["sparse"] == 4 * 3 + 4 * 3            # list of 3, inverted index over |S| = 3
    assert mem["sparse_reduced_lists"] == 4 * 3
    assert mem["regular"] == 4 * (12 + 40)
    assert mem["all_regular_groups"] == 4 * ((40 + 40) + (12 + 40) + (3 + 40) + (20 + 40) + (1 + 40)
                                             + (1 + 2) + (2 + 2) + (1 + 2) + (1 + 1))
    popc0 = 40 + 12 + 3 + 20 + 1
    assert mem["naive_bound"] == 4 * (40 * 32 + popc0) + 4 * (2 * 32 + 4) + 4 * (32 + 1)
    bs = skew_graph(adaptive=False).memory()
    assert bs["regular"] == mem["all_regular_groups"] and bs["sparse"] == 0 and bs["one"] == 0


def test_memory_model_two_sparse_groups_share_reduced_list():
    """A vertex of d = 30 with one group of each type and two sparse groups sharing an edge:
    e0..e4 weight 3 (bits 0, 1), e5..e14 weight 1, e20 weight 4, e21 weight 12 (bits 2, 3), e22 weight
    8, e25 weight 16, the other eleven weight 32.  Group 0: c = 15 (dense, 5c > 2d); group 1: c = 5
    (regular); groups 2 = {e20, e21} and 3 = {e21, e22}: c = 2 each (sparse, 10c < d); group 4 = {e25}
    (one-element); group 5: c = 11 (regular).  S(u) = {e20, e21, e22}, |S| = 3."""
    w = [3] * 5 + [1] * 10 + [32] * 5 + [4, 12, 8, 32, 32, 16, 32, 32, 32, 32]
    assert len(w) == 30
    g = O.Graph(31, [0] * 30, list(range(1, 31)), w)
    types = {k: t for k, (t, c, m) in vertex(g, 0)["groups"].items()}
    assert types == {0: O.T_DENSE, 1: O.T_REGULAR, 2: O.T_SPARSE, 3: O.T_SPARSE, 4: O.T_ONE, 5: O.T_REGULAR}
    mem = g.memory()
    assert mem["adjacency"] == 360
    assert mem["one"] == 4
    assert mem["sparse"] == 2 * (4 * 2 + 4 * 3)      # 40
    assert mem["sparse_reduced_lists"] == 4 * 3
    assert mem["regular"] == 4 * (5 + 30) + 4 * (11 + 30)   # 304
    assert mem["all_regular_groups"] == 4 * ((15 + 30) + (5 + 30) + (2 + 30) + (2 + 30) + (1 + 30) + (11 + 30))
    popc = 5 * 2 + 10 * 1 + 11 * 1 + 1 + 2 + 1 + 1
    assert mem["naive_bound"] == 4 * (30 * 32 + popc)

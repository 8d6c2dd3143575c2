"""Group indexes in the oracle (Sec. 4.2 inverted index; Sec. 5.1 sparse groups and the reduced
neighbour list S(u)), pinned by hand-computed dumps: a vertex with one regular, two sparse (sharing a
member), one one-element and one dense group, before and after a batch that deletes the shared sparse
member; the paper's running example in the all-regular mode; and invariants on random graphs."""
import random

import numpy as np

import oracle as O

NF = 0xFFFFFFFF


def hand_vertex():
    """25 edges of vertex 0.  Bit 0 on every edge (dense, 25/25); bit 2 on edges 0..7 (8/25 = 32 %,
    regular); bit 3 on edges 4 and 17 (2/25 = 8 %, sparse); bit 5 on edge 9 (one element); bit 6 on
    edges 2 and 4 (sparse).  S(0) = edges in a sparse group = [2, 4, 17]."""
    w = []
    for i in range(25):
        x = 1
        if i < 8:
            x |= 4
        if i in (4, 17):
            x |= 8
        if i == 9:
            x |= 32
        if i in (2, 4):
            x |= 64
        w.append(x)
    dst = [(i * 7) % 30 + 1 for i in range(25)]
    return 31, [0] * 25, dst, w


def test_index_dump_by_hand():
    n, src, dst, w = hand_vertex()
    g = O.Graph(n, np.array(src), np.array(dst), np.array(w))
    types = {k: t for k, (t, c, m) in O.parse_dump(g.dump(0, 1), 1)[0]["groups"].items()}
    assert types == {0: O.T_DENSE, 2: O.T_REGULAR, 3: O.T_SPARSE, 5: O.T_ONE, 6: O.T_SPARSE}
    expect = [3, 2, 4, 17,                  # |S| = 3, S = [2, 4, 17]
              2, 0, 1, 2, 3, 4, 5, 6, 7,    # regular group 2^2: list [0..7], inverted index at its members
              3, NF, 0, 1,                  # sparse 2^3 = [4, 17] over S: 2 absent, 4 at 0, 17 at 1
              6, 0, 1, NF]                  # sparse 2^6 = [2, 4] over S
    assert g.index_dump(0, 1).tolist() == expect
    # vertices without edges: |S| = 0 and no listed groups
    assert g.index_dump(1, 3).tolist() == [0, 0]
    # delete edge 4 (the shared sparse member): the last edge (24, weight 1) fills index 4; groups 2^3
    # and 2^6 drop to one element, so S is empty; group 2^2 (7/24 regular) loses position 4 to its
    # tail entry 7, giving [0, 1, 2, 3, 7, 5, 6]
    g.update(np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64), np.array([0]), np.array([dst[4]]))
    v = O.parse_dump(g.dump(0, 1), 1)[0]
    assert v["groups"][2] == (O.T_REGULAR, 7, [0, 1, 2, 3, 7, 5, 6])
    assert g.index_dump(0, 1).tolist() == [0, 2, 0, 1, 2, 3, 4, 5, 6]


def test_index_dump_running_example_all_regular():
    """Running example vertex 2 (weights 5, 4, 3) without adaption: groups 2^0 = [0, 2], 2^1 = [2],
    2^2 = [0, 1], each with its inverted index at its members; no sparse group, so S is empty.
    After inserting (2, 3, 3) at index 3, 2^0 = [0, 2, 3] and 2^1 = [2, 3]."""
    g = O.Graph(6, np.array([2, 2, 2]), np.array([1, 4, 5]), np.array([5, 4, 3]), adaptive=False)
    assert g.index_dump(2, 3).tolist() == [0, 0, 0, 1, 1, 0, 2, 0, 1]
    g.update(np.array([2]), np.array([3]), np.array([3]), np.zeros(0, np.int64), np.zeros(0, np.int64))
    assert g.index_dump(2, 3).tolist() == [0, 0, 0, 1, 2, 1, 0, 1, 2, 0, 1]


def test_index_invariants_random():
    """On random graphs, after random batches: S is ascending and holds exactly the edges with a bit
    in a sparse group; a regular group's entries are 0..c-1; a sparse group's index over S names each
    member's list position once and is 0xFFFFFFFF elsewhere."""
    rng = random.Random(9)
    n = 30
    src = [rng.randrange(n) for _ in range(900)]
    dst = [rng.randrange(n) for _ in range(900)]
    w = [rng.choice([1, 3, 1 << rng.randrange(20), rng.randrange(1, 1 << 20), 0x30000 | rng.randrange(8)])
         for _ in range(900)]
    g = O.Graph(n, np.array(src), np.array(dst), np.array(w))
    for b in range(4):
        verts = O.parse_dump(g.dump(), n)
        idx = g.index_dump()
        o = 0
        seen_sparse = False
        for u, v in enumerate(verts):
            ns = int(idx[o]); S = idx[o + 1:o + 1 + ns].tolist(); o += 1 + ns
            smask = sum(1 << k for k, (t, c, m) in v["groups"].items() if t == O.T_SPARSE)
            assert S == [i for i in range(v["d"]) if int(v["w"][i]) & smask]
            for k, (t, c, m) in sorted(v["groups"].items()):
                if t not in (O.T_SPARSE, O.T_REGULAR):
                    continue
                assert int(idx[o]) == k; o += 1
                if t == O.T_REGULAR:
                    assert idx[o:o + c].tolist() == list(range(c)); o += c
                else:
                    seen_sparse = True
                    J = idx[o:o + ns].tolist(); o += ns
                    assert [J[S.index(x)] for x in m] == list(range(c))
                    assert sum(1 for j in J if j != NF) == c
        assert o == len(idx)
        assert seen_sparse
        cur = O.parse_dump(g.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ins = [(rng.randrange(n), rng.randrange(n), rng.choice([1, 0x30000, rng.randrange(1, 1 << 20)]))
               for _ in range(60)]
        dels = [rng.choice(live) for _ in range(60)]
        g.update(*(np.array(c) for c in zip(*ins)), *(np.array(c) for c in zip(*dels)))

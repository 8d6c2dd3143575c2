"""Group indexes on the GPU (Sec. 4.2 inverted index of regular groups; Sec. 5.1 the reduced neighbour
list S(u) and the sparse groups' indexes over it), compared word for word with the oracle's index dump:
the hand-made vertex with every group type before and after deleting its shared sparse member, the
running example without adaption, random batches that convert groups between sparse and regular,
streaming records, compaction, and the memory identity that ties the stored structures to the paper's
memory model.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_parity import B, assert_same_structure, both
from test_oracle_index import hand_vertex

pytestmark = pytest.mark.gpu
NF = 0xFFFFFFFF
E = np.zeros(0, dtype=np.int64)


def t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int64))


def test_hand_vertex_index():
    n, src, dst, w = hand_vertex()
    og, gg = both(n, src, dst, w)
    assert gg.export_index(0, 1).tolist() == [3, 2, 4, 17, 2, 0, 1, 2, 3, 4, 5, 6, 7, 3, NF, 0, 1, 6, 0, 1, NF]
    assert_same_structure(og, gg, "build")
    og.update(E, E, E, np.array([0]), np.array([dst[4]]))
    gg.update(t(E), t(E), t(E), t([0]), t([dst[4]]))
    assert gg.export_index(0, 1).tolist() == [0, 2, 0, 1, 2, 3, 4, 5, 6]
    assert_same_structure(og, gg, "after deleting the shared sparse member")


def test_running_example_all_regular():
    og, gg = both(6, [2, 2, 2], [1, 4, 5], [5, 4, 3], adaptive=False)
    assert gg.export_index(2, 3).tolist() == [0, 0, 0, 1, 1, 0, 2, 0, 1]
    og.update(np.array([2]), np.array([3]), np.array([3]), E, E)
    gg.update(t([2]), t([3]), t([3]), t(E), t(E))
    assert gg.export_index(2, 3).tolist() == [0, 0, 0, 1, 2, 1, 0, 1, 2, 0, 1]
    assert_same_structure(og, gg, "insert")


def _weights(rng, k):
    return [rng.choice([1, 3, 1 << rng.randrange(20), rng.randrange(1, 1 << 20), 0x30000 | rng.randrange(8)])
            for _ in range(k)]


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("split", [0, 64])
def test_random_batches_convert_groups(adaptive, split):
    """Small graph with hubs: every batch grows and shrinks vertices across the sparse / regular /
    dense boundaries and the adjacency capacities, so lists and indexes move and are rebuilt; with
    split = 64 the hubs go through the split work."""
    rng = random.Random(11 + split)
    n = 40
    src = [rng.choice([0, 1, 2, rng.randrange(n)]) for _ in range(3000)]
    dst = [rng.randrange(n) for _ in range(3000)]
    w = _weights(rng, 3000)
    og, gg = both(n, src, dst, w, adaptive=adaptive)
    gg.set_tuning(update_split=split)
    assert_same_structure(og, gg, "build")
    for b in range(6):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(x)) for u, v in enumerate(cur) for x in v["dst"]]
        k = rng.choice([5, 100, 900])
        ins = [(rng.choice([0, 1, 2, rng.randrange(n)]), rng.randrange(n), x) for x in _weights(rng, k)]
        dels = [rng.choice(live) for _ in range(rng.choice([5, 100, 1200]))]
        a = [np.array(c, dtype=np.int64) for c in zip(*ins)]
        d = [np.array(c, dtype=np.int64) for c in zip(*dels)]
        og.update(*a, *d)
        gg.update(*[t(x) for x in a], *[t(x) for x in d])
        assert_same_structure(og, gg, "batch %d" % b)


@pytest.mark.parametrize("adaptive", [True, False])
def test_streaming_records_keep_the_index(adaptive):
    rng = random.Random(5)
    n = 30
    src = [rng.choice([0, 1, rng.randrange(n)]) for _ in range(1500)]
    dst = [rng.randrange(n) for _ in range(1500)]
    w = _weights(rng, 1500)
    og, gg = both(n, src, dst, w, adaptive=adaptive)
    for r in range(4):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(x)) for u, v in enumerate(cur) for x in v["dst"]]
        recs = []
        for _ in range(400):
            if rng.random() < 0.5:
                recs.append((0, rng.choice([0, 1, rng.randrange(n)]), rng.randrange(n), _weights(rng, 1)[0]))
            else:
                u, x = rng.choice(live)
                recs.append((1, u, x, 0))
        ops, s, d, ww = (np.array(c, dtype=np.int64) for c in zip(*recs))
        og.update_stream(ops, s, d, ww)
        gg.update_stream(*[t(x) for x in (ops, s, d, ww)])
        assert_same_structure(og, gg, "stream %d" % r)


def test_compaction_keeps_the_index():
    rng = random.Random(8)
    n = 30
    src = [rng.choice([0, 1, rng.randrange(n)]) for _ in range(2000)]
    dst = [rng.randrange(n) for _ in range(2000)]
    og, gg = both(n, src, dst, _weights(rng, 2000))
    ins = [(rng.choice([0, 1]), rng.randrange(n), x) for x in _weights(rng, 800)]
    a = [np.array(c, dtype=np.int64) for c in zip(*ins)]
    og.update(*a, E, E)
    gg.update(*[t(x) for x in a], t(E), t(E))
    assert gg.memory()["pool_garbage_bytes"] > 0
    gg.compact()
    assert gg.memory()["pool_garbage_bytes"] == 0
    assert_same_structure(og, gg, "after compaction")


@pytest.mark.parametrize("kind", ["uniform", "zipf", "lognormal"])
def test_memory_identity_rmat(kind):
    """The stored structures are exactly the paper's memory model with adaption: 12 bytes per edge, a
    one-element group's 4 bytes, every list's live entries and the indexes' live entries (4 d per
    regular group, 4 |S(u)| per sparse group and for S(u)) add up to model_ga_bytes; the index dump
    equals the oracle's on R-MAT 12."""
    n = 1 << 12
    src, dst = synth.rmat_graph(12, 16 * n, 51)
    m = src.numel()
    w = {"uniform": lambda: synth.weights_uniform(m, 1, 1 << 24, 52),
         "zipf": lambda: synth.weights_zipf(m, 1.5, (1 << 20) - 1, 52),
         "lognormal": lambda: synth.weights_lognormal(m, 8.0, 3.0, 52)}[kind]()
    og = O.Graph(n, src.numpy(), dst.numpy(), w.numpy())
    gg = B().Graph(n, src, dst, w)
    assert_same_structure(og, gg, kind)
    mem = gg.memory()
    ones = mem["groups_by_type"][1]
    assert mem["index_bytes"] + mem["list_bytes"] + 4 * ones + mem["adjacency_bytes"] == mem["model_ga_bytes"]
    assert mem["index_reserved_bytes"] >= mem["index_bytes"]
    gg.close()


@pytest.mark.parametrize("split", [0, 4096])
def test_sparse_rebuild_at_every_vertex_size(split):
    """S(u) and the sparse indexes rebuilt for vertices of every size class the rebuild has: 70,000
    edges (several adjacency chunks, one block each), 3,000 and 1,030 edges (one block per vertex),
    1,000 edges and fewer (one wave per vertex); weights mostly 1, so every group above bit 0 is
    sparse and each batch changes S(u) of the vertices it touches; then a stream of records."""
    rng = np.random.default_rng(21)
    n = 200
    sizes = {0: 70000, 1: 3000, 2: 1030, 3: 1000}
    src = np.concatenate([np.full(d, v) for v, d in sizes.items()] + [rng.integers(4, n, 3000)])
    m = src.size
    dst = rng.integers(0, n, m)
    w = np.where(rng.random(m) < 0.9, 1, rng.integers(1, 1 << 20, m))
    og, gg = both(n, src, dst, w)
    gg.set_tuning(update_split=split)
    assert_same_structure(og, gg, "build")
    for b in range(3):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(x)) for u, v in enumerate(cur) for x in v["dst"]]
        k = 600
        isrc = rng.choice([0, 1, 2, 3, int(rng.integers(4, n))], size=k)
        idst = rng.integers(0, n, k)
        iw = np.where(rng.random(k) < 0.5, 1, rng.integers(1, 1 << 20, k))
        pick = rng.choice(len(live), size=700, replace=False)
        dsrc = np.array([live[i][0] for i in pick])
        ddst = np.array([live[i][1] for i in pick])
        og.update(isrc, idst, iw, dsrc, ddst)
        gg.update(t(isrc), t(idst), t(iw), t(dsrc), t(ddst))
        assert_same_structure(og, gg, "batch %d" % b)
    cur = O.parse_dump(og.dump(), n)
    live = [(u, int(x)) for u, v in enumerate(cur) for x in v["dst"]]
    recs = []
    for _ in range(300):
        if rng.random() < 0.5:
            recs.append((0, int(rng.integers(0, 4)), int(rng.integers(0, n)), int(rng.integers(1, 1 << 20))))
        else:
            u, x = live[int(rng.integers(0, len(live)))]
            recs.append((1, u, x, 0))
    ops, s, d, ww = (np.array(c, dtype=np.int64) for c in zip(*recs))
    og.update_stream(ops, s, d, ww)
    gg.update_stream(*[t(x) for x in (ops, s, d, ww)])
    assert_same_structure(og, gg, "stream")

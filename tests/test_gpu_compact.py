"""Pool compaction on the HIP path: the canonical dump, every walk and PPR histogram stay equal to the
oracle's after the pool is compacted (by hand and by a batch that did not fit), the bookkeeping of
used and replaced blocks is exact, and batches after a compaction (with freshly captured graphs)
still match.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, apply_both, assert_same_structure, skew_edges, u32

pytestmark = pytest.mark.gpu


def build(n, src, dst, w, pool_bytes=0, **kw):
    src, dst, w = (np.asarray(x, dtype=np.int64) for x in (src, dst, w))
    og = O.Graph(n, src, dst, w, frac_bits=kw.get("frac_bits", 0), alias=kw.get("alias_table", False),
                 adaptive=kw.get("adaptive", True))
    gg = B().Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), pool_bytes=pool_bytes, **kw)
    return og, gg


def random_batch(og, rng, n, hub=6, size=300):
    cur = O.parse_dump(og.dump(), n)
    live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
    ins = [(hub if rng.random() < 0.5 else rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 32))
           for _ in range(rng.randrange(1, size))]
    dels = [rng.choice(live) for _ in range(rng.randrange(1, size))]
    return ins, dels


def check_walks(og, gg, seed):
    starts = np.array([0, 5, 6, 3, 1, 2, 7] * 30)
    for mode in (0, 1):
        paths, steps = gg.walk(starts, 20, seed, mode=mode)
        opaths, osteps = og.deepwalk(starts, 20, seed)
        assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps
    thr = int(0.15 * 2**32)
    ooff, ovtx, ocnt, _ = og.ppr(np.array([0, 5, 6]), 100, thr, 200, seed=seed)
    off, vtx, cnt, _ = gg.ppr(np.array([0, 5, 6]), 100, thr, 200, seed=seed)
    assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
    assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt)


@pytest.mark.parametrize("kind", ["ga", "bs", "fixed", "alias"])
def test_compact_keeps_structure_and_walks(kind):
    n, src, dst, w = skew_edges()
    kw = {"bs": {"adaptive": False}, "fixed": {"frac_bits": 8}, "alias": {"alias_table": True}}.get(kind, {})
    og, gg = build(n, src, dst, w, **kw)
    rng = random.Random(21)
    for b in range(6):
        ins, dels = random_batch(og, rng, n)
        apply_both(og, gg, ins, dels, "%s batch %d" % (kind, b))
    before = gg.memory()
    assert before["pool_garbage_bytes"] > 0
    gg.compact()
    after = gg.memory()
    assert after["pool_garbage_bytes"] == 0
    assert after["pool_used_bytes"] == before["pool_used_bytes"] - before["pool_garbage_bytes"]
    assert after["pool_bytes"] == before["pool_bytes"]
    assert_same_structure(og, gg, "%s after compaction" % kind)
    check_walks(og, gg, 40)
    # batches after the move (the captured graphs are made again) and a second compaction
    for b in range(4):
        ins, dels = random_batch(og, rng, n)
        apply_both(og, gg, ins, dels, "%s batch %d after compaction" % (kind, b))
    gg.compact(pool_bytes=after["pool_bytes"] * 2)
    assert gg.memory()["pool_bytes"] == after["pool_bytes"] * 2
    assert_same_structure(og, gg, "%s after the second compaction" % kind)
    check_walks(og, gg, 41)


def test_batches_compact_when_the_pool_is_full():
    # 1500 vertices of two weight-1 edges (capacity 2); each batch takes 300 of them to degree 4
    # (three inserts, one delete), so their adjacency moves to a block of capacity 4 and 300 blocks
    # are replaced: live blocks grow by as many words as the garbage does, and the pool holds all
    # five batches only if the replaced blocks are reclaimed
    n = 2000
    src = [v for v in range(1500) for _ in range(2)]
    dst = [(v * 7 + j) % n for v in range(1500) for j in range(2)]
    w = [1] * len(src)
    _, probe = build(n, src, dst, w)
    used = probe.memory()["pool_used_bytes"]
    probe.close()
    og, gg = build(n, src, dst, w, pool_bytes=used + 18000 * 4)
    pool = gg.memory()["pool_bytes"]
    saw_compaction = False
    for b in range(5):
        vs = range(300 * b, 300 * (b + 1))
        ins = [(v, (v * 11 + j) % n, 1) for v in vs for j in range(3)]
        dels = [(v, (v * 7) % n) for v in vs]
        g0 = gg.memory()["pool_garbage_bytes"]
        apply_both(og, gg, ins, dels, "tight pool, batch %d" % b)
        m = gg.memory()
        assert m["pool_bytes"] == pool and m["pool_used_bytes"] <= pool
        saw_compaction |= m["pool_garbage_bytes"] < g0
    assert saw_compaction
    check_walks(og, gg, 42)


def test_compact_rejections_leave_the_graph_unchanged():
    n, src, dst, w = skew_edges()
    og, gg = build(n, src, dst, w)
    b = B()
    used = gg.memory()["pool_used_bytes"]
    with pytest.raises(b.BingoError):
        gg.compact(pool_bytes=used // 2)  # the live blocks do not fit
    with pytest.raises(b.BingoError):
        gg.compact(pool_bytes=(1 << 37) + 4)  # beyond 32-bit list offsets
    assert gg.memory()["pool_used_bytes"] == used
    assert_same_structure(og, gg, "after refused compactions")
    check_walks(og, gg, 43)


def test_compact_after_streaming_updates():
    # streaming records grow the hub and other vertices past their capacities and convert groups;
    # the replaced blocks they leave are counted exactly and reclaimed
    n, src, dst, w = skew_edges()
    og, gg = build(n, src, dst, w)
    rng = random.Random(22)
    for b in range(3):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        recs = []
        for _ in range(400):
            if rng.random() < 0.7:
                recs.append((0, 6 if rng.random() < 0.5 else rng.randrange(n), rng.randrange(n),
                             rng.randrange(1, 1 << 32)))
            else:
                s_, d_ = rng.choice(live)
                recs.append((1, s_, d_, 0))
        ops, ss, dd, ww = (list(x) for x in zip(*recs))
        og.update_stream(ops, ss, dd, ww)
        gg.update_stream(*[torch.tensor(x) for x in (ops, ss, dd, ww)])
        assert_same_structure(og, gg, "stream %d" % b)
    before = gg.memory()
    assert before["pool_garbage_bytes"] > 0
    gg.compact()
    after = gg.memory()
    assert after["pool_garbage_bytes"] == 0
    assert after["pool_used_bytes"] == before["pool_used_bytes"] - before["pool_garbage_bytes"]
    assert_same_structure(og, gg, "after compaction")
    check_walks(og, gg, 44)


def test_library_sized_pool_grows():
    # a graph whose library-sized pool (twice the input plus 16 MB) cannot hold the edges inserted
    # later: a batch that does not fit even after compaction moves the pool to an arena twice the size
    n, m = 5000, 20000
    rng = np.random.default_rng(23)
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    w = rng.integers(1, 1 << 20, m)
    og, gg = build(n, src, dst, w)
    pool0 = gg.memory()["pool_bytes"]
    empty = np.zeros(0, np.int64)
    for b in range(4):
        k = 500_000
        isrc, idst, iw = rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(1, 1 << 20, k)
        so = og.update(isrc, idst, iw, empty, empty)
        sg = gg.update(*[torch.from_numpy(x) for x in (isrc, idst, iw, empty, empty)])
        assert sg["inserted"] == so["inserted"] == k
        assert np.array_equal(sg["transitions"], so["transitions"])
    mem = gg.memory()
    assert mem["pool_bytes"] > pool0 and mem["pool_used_bytes"] <= mem["pool_bytes"]
    assert np.array_equal(gg.export(), og.dump())
    assert np.array_equal(gg.export_index(), og.index_dump())
    starts = rng.integers(0, n, 500)
    paths, steps = gg.walk(starts, 30, 45)
    opaths, osteps = og.deepwalk(starts, 30, 45)
    assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps

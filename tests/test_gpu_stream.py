"""Streaming updates (Sec. 4.2) through bingo_update_stream: every record applied on its own, in order.
Bit-exact against the oracle applying one batch per record (structure dump, statistics, walks), and
against the GPU's own batch path fed one record at a time.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, assert_same_structure, both, skew_edges, u32

pytestmark = pytest.mark.gpu


def random_stream(rng, cur, n, count, hub=0, hub_share=0.5, wgen=None):
    """Interleaved inserts and deletes; deletes mostly of live edges (including ones this stream
    inserted), some absent; a share of the records on one hub."""
    live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
    ops, src, dst, w = [], [], [], []
    for _ in range(count):
        u = hub if rng.random() < hub_share else rng.randrange(n)
        if rng.random() < 0.5:
            v = rng.randrange(n)
            ops.append(0); src.append(u); dst.append(v)
            w.append(wgen() if wgen else rng.choice([1, 3, 255, 1 << rng.randrange(32), rng.randrange(1, 1 << 32)]))
            live.append((u, v))
        else:
            if live and rng.random() < 0.85:
                u, v = live[rng.randrange(len(live))]
            else:
                v = rng.randrange(n)
            ops.append(1); src.append(u); dst.append(v); w.append(0)
    return ops, src, dst, w


def run_both(og, gg, ops, src, dst, w, where):
    s2 = og.update_stream(ops, src, dst, w)
    t = [torch.tensor(np.asarray(x, np.int64)) for x in (ops, src, dst, w)]
    s1 = gg.update_stream(*t)
    for key in ("inserted", "deleted", "not_found"):
        assert s1[key] == s2[key], (where, key, s1[key], s2[key])
    assert np.array_equal(s1["transitions"], s2["transitions"]), where
    assert s1["touched_vertices"] == len(set(src))
    assert_same_structure(og, gg, where)


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_streams(adaptive, seed):
    rng = random.Random(seed)
    n = 40
    src = [rng.randrange(n) for _ in range(400)] + [0] * 300
    dst = [rng.randrange(n) for _ in range(700)]
    w = [rng.choice([1, 2, 3, 7, 64, 1000, rng.randrange(1, 1 << 20), 1 << rng.randrange(32)]) for _ in range(700)]
    og, gg = both(n, src, dst, w, adaptive)
    for b in range(6):
        cur = O.parse_dump(og.dump(), n)
        ops, s, d, ww = random_stream(rng, cur, n, rng.randrange(1, 600))
        run_both(og, gg, ops, s, d, ww, "stream %d" % b)
        starts = np.arange(n).repeat(3)
        paths, _ = gg.walk(starts, 12, 500 + b)
        opaths, _ = og.deepwalk(starts, 12, 500 + b)
        assert np.array_equal(u32(paths), opaths), b


def test_hub_and_edge_cases():
    og, gg = both(*skew_edges())
    n = og.n
    run_both(og, gg, [1], [9], [9], [0], "delete from an isolated vertex")
    run_both(og, gg, [0, 1, 1], [7, 7, 7], [1, 1, 1], [5, 0, 0], "insert, delete it, delete again")
    run_both(og, gg, [0] * 300 + [1] * 300, [6] * 600, [2] * 600, [1 << 31] * 300 + [0] * 300,
             "hub grows past its capacity, then loses the same edges")
    cur = O.parse_dump(og.dump(), n)
    hub_dels = [int(t) for t in cur[6]["dst"][::3]]
    run_both(og, gg, [1] * len(hub_dels), [6] * len(hub_dels), hub_dels, [0] * len(hub_dels),
             "a third of the hub deleted one record at a time")
    cur = O.parse_dump(og.dump(), n)
    all5 = [int(t) for t in cur[5]["dst"]]
    run_both(og, gg, [1] * len(all5) + [0], [5] * (len(all5) + 1), all5 + [3], [0] * len(all5) + [7],
             "every edge of a vertex deleted, then one inserted")
    rng = random.Random(4)
    for b in range(3):
        cur = O.parse_dump(og.dump(), n)
        ops, s, d, ww = random_stream(rng, cur, n, 2000, hub=6, hub_share=0.7)
        run_both(og, gg, ops, s, d, ww, "hub stream %d" % b)


def test_float_biases_stream():
    F = 8
    rng = random.Random(7)
    n = 30
    src = [rng.randrange(n) for _ in range(400)] + [0] * 200
    dst = [rng.randrange(n) for _ in range(600)]
    bias = [rng.choice([rng.uniform(0.01, 2.0), float(rng.randrange(1, 100)), rng.randrange(1, 50) + rng.random()])
            for _ in range(600)]
    w = O.quantize(bias, 4.0, F)
    og = O.Graph(n, src, dst, w, frac_bits=F)
    gg = B().Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w.astype(np.int64)), frac_bits=F)
    for b in range(4):
        cur = O.parse_dump(og.dump(), n)
        wgen = lambda: int(O.quantize([rng.choice([rng.uniform(0.01, 2.0), float(rng.randrange(1, 100))])], 4.0, F)[0])
        ops, s, d, ww = random_stream(rng, cur, n, 500, wgen=wgen)
        run_both(og, gg, ops, s, d, ww, "float stream %d" % b)
        paths, _ = gg.walk(np.arange(n).repeat(4), 10, 9 + b)
        opaths, _ = og.deepwalk(np.arange(n).repeat(4), 10, 9 + b)
        assert np.array_equal(u32(paths), opaths)


def test_stream_equals_batches_of_one_on_gpu():
    rng = random.Random(11)
    n = 50
    src = [rng.randrange(n) for _ in range(800)]
    dst = [rng.randrange(n) for _ in range(800)]
    w = [rng.randrange(1, 1 << 24) for _ in range(800)]
    og, ga = both(n, src, dst, w)
    gb = B().Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w))
    cur = O.parse_dump(og.dump(), n)
    ops, s, d, ww = random_stream(rng, cur, n, 120, hub=3)
    ga.update_stream(*[torch.tensor(x) for x in (ops, s, d, ww)])
    for o, a, c, x in zip(ops, s, d, ww):
        if o == 0:
            gb.update(torch.tensor([a]), torch.tensor([c]), torch.tensor([x]), torch.tensor([], dtype=torch.int64),
                      torch.tensor([], dtype=torch.int64))
        else:
            e = torch.tensor([], dtype=torch.int64)
            gb.update(e, e, e, torch.tensor([a]), torch.tensor([c]))
    assert np.array_equal(ga.export(), gb.export())
    assert np.array_equal(ga.export_index(), gb.export_index())


def test_stream_rejects_bad_records():
    b = B()
    og, gg = both(*skew_edges())
    before = gg.export()
    for ops, s, d, w, code in [([0], [0], [1], [0], -3), ([2], [0], [1], [1], -2), ([0, 1], [0, 99], [1, 1], [1, 0], -2)]:
        with pytest.raises(b.BingoError) as e:
            gg.update_stream(*[torch.tensor(x) for x in (ops, s, d, w)])
        assert e.value.code == code
        assert np.array_equal(gg.export(), before)


def test_stream_out_of_pool_keeps_a_consistent_prefix():
    """A stream that outgrows the device pool returns BINGO_E_OOM; the vertex that ran out keeps exactly
    the records before the failing one (here the inserts fit until its adjacency or a list must grow),
    which the oracle reproduces by applying that prefix."""
    b = B()
    n, src, dst, w = skew_edges()
    probe = b.Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w))
    used = probe.memory()["pool_used_bytes"]
    probe.close()
    gg = b.Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w), pool_bytes=used + (64 << 10))
    og = O.Graph(n, src, dst, w)
    d0 = O.parse_dump(gg.export(), n)[6]["d"]
    rng = random.Random(12)
    k = 30000
    ops, s, d, ww = [0] * k, [6] * k, [rng.randrange(n) for _ in range(k)], [rng.randrange(1, 1 << 32) for _ in range(k)]
    with pytest.raises(b.BingoError) as e:
        gg.update_stream(*[torch.tensor(x) for x in (ops, s, d, ww)])
    assert e.value.code == -4
    applied = O.parse_dump(gg.export(), n)[6]["d"] - d0
    assert 0 < applied < k
    og.update_stream(ops[:applied], s[:applied], d[:applied], ww[:applied])
    assert_same_structure(og, gg, "prefix of %d inserts" % applied)


def test_stream_grows_a_library_sized_pool():
    """A stream that outgrows a pool the library sized: the sources that ran out stop, the pool moves
    to an arena twice the size, and their remaining records are applied in order; the result equals the
    same stream on a graph whose pool never ran out (and the records counted once each)."""
    b = B()
    n, m = 5000, 20000
    rng = np.random.default_rng(31)
    src, dst, w = rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(1, 1 << 20, m)
    g1 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w))
    g2 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), pool_bytes=1 << 31)
    pool0 = g1.memory()["pool_bytes"]
    k = 1_200_000
    rec = [np.zeros(k, np.int64), rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(1, 1 << 20, k)]
    rec[0][rng.random(k) < 0.1] = 1  # some deletes (most not found, some of earlier inserts)
    s1 = g1.update_stream(*[torch.from_numpy(x) for x in rec])
    s2 = g2.update_stream(*[torch.from_numpy(x) for x in rec])
    assert g1.memory()["pool_bytes"] > pool0
    for key in ("inserted", "deleted", "not_found"):
        assert s1[key] == s2[key], key
    assert s1["inserted"] + s1["deleted"] + s1["not_found"] == k
    assert np.array_equal(g1.export(), g2.export())
    assert np.array_equal(g1.export_index(), g2.export_index())


def test_stream_grows_with_many_more_sources_than_resident_waves():
    """The same growth with 2 x 10^5 distinct sources, many more segments than the waves the apply
    kernel keeps resident: blocks that start after another source has run out of pool still apply
    their own segments, so every record is counted once and the result equals the stream on a pool
    that never ran out."""
    b = B()
    n, m = 200_000, 800_000
    rng = np.random.default_rng(47)
    src, dst, w = rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(1, 1 << 20, m)
    g1 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w))
    g2 = b.Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), pool_bytes=1 << 31)
    pool0 = g1.memory()["pool_bytes"]
    k = 1_200_000
    rec = [np.zeros(k, np.int64), rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(1, 1 << 20, k)]
    dels = rng.random(k) < 0.1
    rec[0][dels] = 1
    # half of the deletes name an input edge, so they are found
    pick = rng.integers(0, m, int(dels.sum()))
    half = rng.random(pick.size) < 0.5
    rec[1][np.flatnonzero(dels)[half]] = src[pick[half]]
    rec[2][np.flatnonzero(dels)[half]] = dst[pick[half]]
    assert np.unique(rec[1]).size > 100_000
    s1 = g1.update_stream(*[torch.from_numpy(x) for x in rec])
    s2 = g2.update_stream(*[torch.from_numpy(x) for x in rec])
    assert g1.memory()["pool_bytes"] > pool0
    for key in ("inserted", "deleted", "not_found"):
        assert s1[key] == s2[key], key
    assert s1["inserted"] + s1["deleted"] + s1["not_found"] == k
    assert s1["deleted"] > 0
    assert np.array_equal(g1.export(), g2.export())
    assert np.array_equal(g1.export_index(), g2.export_index())
    g1.close()
    g2.close()


def test_stream_hub_above_block_threshold():
    """Sources of at least 16,384 edges take a block each (every wave scans a share of the adjacency
    for a delete, wave 0 applies the records): a 40,000-edge hub's interleaved streams equal the
    oracle's, and a fixed pool that runs out in the middle of the hub's inserts keeps exactly the
    records before the failing one."""
    b = B()
    rng = random.Random(77)
    n = 300
    m = 46000
    src = [0] * 40000 + [rng.randrange(1, n) for _ in range(m - 40000)]
    dst = [rng.randrange(n) for _ in range(m)]
    w = [rng.choice([1, 3, 255, 1 << rng.randrange(32), rng.randrange(1, 1 << 32)]) for _ in range(m)]
    og, gg = both(n, src, dst, w)
    for r in range(2):
        cur = O.parse_dump(og.dump(), n)
        ops, s, d, ww = random_stream(rng, cur, n, 3000, hub=0, hub_share=0.6)
        run_both(og, gg, ops, s, d, ww, "hub stream %d" % r)
    gg.close()
    probe = b.Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w))
    used = probe.memory()["pool_used_bytes"]
    probe.close()
    gg = b.Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w), pool_bytes=used + (256 << 10))
    og = O.Graph(n, src, dst, w)
    d0 = O.parse_dump(gg.export(), n)[0]["d"]
    k = 60000
    ops, s, d, ww = [0] * k, [0] * k, [rng.randrange(n) for _ in range(k)], [rng.randrange(1, 1 << 32) for _ in range(k)]
    with pytest.raises(b.BingoError) as e:
        gg.update_stream(*[torch.tensor(x) for x in (ops, s, d, ww)])
    assert e.value.code == -4
    applied = O.parse_dump(gg.export(), n)[0]["d"] - d0
    assert 0 < applied < k
    og.update_stream(ops[:applied], s[:applied], d[:applied], ww[:applied])
    assert_same_structure(og, gg, "prefix of %d hub inserts" % applied)
    gg.close()

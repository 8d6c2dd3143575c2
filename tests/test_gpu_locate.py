"""The edge locator of the batch pipeline (update_locate): batches that locate their deletes through it
leave exactly the structure, statistics and walks of batches that scan for them (and of the oracle),
and after every batch the locator holds one slot per live edge at the edge's neighbour index -- across
duplicate edges, hubs on the split path, growth of the table, captured-graph replays, streaming
updates (which make it stale) and toggling the tuning.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, apply_both, both, skew_edges, u32

pytestmark = pytest.mark.gpu


def live_edges(gg):
    return int(gg.memory()["edges"])


def assert_in_step(gg, where=""):
    r = gg.check_locator()
    assert r is not None, (where, "no locator in step")
    bad, live = r
    assert bad == 0 and live == live_edges(gg), (where, bad, live, live_edges(gg))


def tensors(ins, dels):
    cols = [np.array([x[i] for x in ins], np.int64) for i in range(3)] + \
           [np.array([x[i] for x in dels], np.int64) for i in range(2)]
    return [torch.from_numpy(c) for c in cols]


@pytest.mark.parametrize("split", [0, 64, 4096])
@pytest.mark.parametrize("graphs", [0, 1])
def test_locate_equals_scan_and_oracle(split, graphs):
    rng = random.Random(17 + split + graphs)
    n = 50
    src = [rng.randrange(n) for _ in range(500)] + [0] * 300 + [2] * 200
    # vertex 2 holds many copies of few edges: long runs of one key in the table
    dst = [rng.randrange(n) for _ in range(500)] + [rng.randrange(8) for _ in range(300)] + \
          [rng.randrange(3) for _ in range(200)]
    w = [rng.choice([1, 3, 255, 1 << rng.randrange(32), rng.randrange(1, 1 << 32)]) for _ in range(1000)]
    og, gg = both(n, src, dst, w)
    gs = B().Graph(n, *(torch.tensor(x, dtype=torch.int64) for x in (src, dst, w)))
    for g in (gg, gs):
        g.set_tuning(update_split=split, update_graphs=graphs)
    gs.set_tuning(update_locate=0)
    assert gg.get_tuning()["update_locate"] == 1 and gs.get_tuning()["update_locate"] == 0
    assert gg.check_locator() is None  # built by the first batch
    for b in range(12):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ni, nd = rng.randrange(0, 150), rng.randrange(0, 150)
        ins = [(rng.choice([0, 2, rng.randrange(n)]), rng.randrange(n) if rng.random() < 0.7 else rng.randrange(3),
                rng.randrange(1, 1 << 32)) for _ in range(ni)]
        dels = [rng.choice(live) if live and rng.random() < 0.85 else (rng.randrange(n), rng.randrange(n))
                for _ in range(nd)]
        dels += [(2, rng.randrange(3))] * rng.randrange(0, 40)  # runs longer or shorter than the copies
        if ins:
            dels += [ins[0][:2], ins[-1][:2]]  # deletes of this batch's inserts
        if b == 6:
            dels += [(0, int(t)) for t in cur[0]["dst"]]  # every edge of vertex 0
        if b == 9:
            ins += [(0, rng.randrange(n), 7) for _ in range(6000)]  # vertex 0 onto the split path
        apply_both(og, gg, ins, dels, "batch %d" % b)
        ss = gs.update(*tensors(ins, dels))
        assert np.array_equal(gs.export(), gg.export()), b
        assert np.array_equal(gs.export_index(), gg.export_index()), b
        assert ss["deleted"] + ss["not_found"] == len(dels)
        assert_in_step(gg, "batch %d" % b)
        assert gs.check_locator() is None
        starts = np.arange(n).repeat(2)
        p1, _ = gg.walk(starts, 9, 70 + b)
        p2, _ = gs.walk(starts, 9, 70 + b)
        assert np.array_equal(u32(p1), u32(p2)), b


def test_locate_reads_few_entries():
    """With the locator, the entries read to locate a batch's deletes on a hub are a few slots per
    delete, not the hub's adjacency."""
    rng = random.Random(4)
    n = 30000
    src = [6] * 20000 + [rng.randrange(n) for _ in range(5000)]
    dst = [rng.randrange(n) for _ in range(25000)]
    w = [rng.randrange(1, 1 << 32) for _ in range(25000)]
    og, gg = both(n, src, dst, w)
    apply_both(og, gg, [(6, 1, 1)], [], "first batch builds the locator")
    dels = [(6, t) for t in dst[:50]]
    s2 = og.update(*(np.array(c, np.int64) for c in ([], [], [], [a for a, _ in dels], [b for _, b in dels])))
    s1 = gg.update(*tensors([], dels))
    assert s1["deleted"] == s2["deleted"] == 50
    assert np.array_equal(gg.export(), og.dump())
    assert s1["match_candidates"] >= 50 and s1["match_scanned"] < 400, s1  # the scan would read 20001
    assert_in_step(gg)


def test_locator_stale_after_streaming_and_rebuilt():
    og, gg = both(*skew_edges())
    apply_both(og, gg, [(6, 3, 9)] * 5, [(0, 1)], "first batch builds the locator")
    assert_in_step(gg, "after the first batch")
    gg.update_stream(torch.tensor([0, 1, 0]), torch.tensor([6, 6, 2]), torch.tensor([4, 3, 5]),
                     torch.tensor([11, 0, 12]))
    og.update_stream(np.array([0, 1, 0]), np.array([6, 6, 2]), np.array([4, 3, 5]), np.array([11, 0, 12]))
    assert gg.check_locator() is None  # streaming moved edges without it
    apply_both(og, gg, [(2, 6, 3)], [(6, 3), (6, 4)], "batch after streaming rebuilds it")
    assert_in_step(gg, "after the rebuild")


def test_locator_grows_and_toggles():
    """Inserts past the table's load limit move it to a larger table (the captured graphs with the old
    one are dropped); a batch run with update_locate = 0 makes it stale, and turning it back on
    rebuilds it."""
    rng = random.Random(8)
    n = 3000
    src = [rng.randrange(n) for _ in range(30000)]
    dst = [rng.randrange(n) for _ in range(30000)]
    w = [rng.randrange(1, 1 << 24) for _ in range(30000)]
    og, gg = both(n, src, dst, w)
    sizes = []
    for b in range(4):
        ins = [(rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 24)) for _ in range(20000)]
        dels = [(src[i], dst[i]) for i in rng.sample(range(30000), 3000)]  # input edges, live or not
        apply_both(og, gg, ins, dels, "growth batch %d" % b)
        assert_in_step(gg, "growth batch %d" % b)
        sizes.append(gg.memory()["locator_bytes"])
    assert sizes[-1] > sizes[0] > 0, sizes
    gg.set_tuning(update_locate=0)
    apply_both(og, gg, [(1, 2, 3)], [(src[0], dst[0])], "batch without the locator")
    assert gg.check_locator() is None
    gg.set_tuning(update_locate=1)
    apply_both(og, gg, [(1, 2, 5)], [(1, 2)], "batch with the locator again")
    assert_in_step(gg, "after toggling back")


def test_locator_in_step_after_compaction():
    """Compaction moves blocks but keeps every neighbour index, so the locator stays in step through
    it and the batches after it still equal the oracle's."""
    rng = random.Random(12)
    n = 300
    src = [rng.randrange(n) for _ in range(4000)] + [1] * 2000
    dst = [rng.randrange(n) for _ in range(6000)]
    w = [rng.randrange(1, 1 << 24) for _ in range(6000)]
    og, gg = both(n, src, dst, w)
    for b in range(3):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ins = [(rng.choice([1, rng.randrange(n)]), rng.randrange(n), rng.randrange(1, 1 << 24)) for _ in range(3000)]
        dels = [rng.choice(live) for _ in range(1500)]
        apply_both(og, gg, ins, dels, "before compaction %d" % b)
    assert_in_step(gg, "before compaction")
    gg.compact()
    assert_in_step(gg, "after compaction")
    cur = O.parse_dump(og.dump(), n)
    live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
    apply_both(og, gg, [(1, 2, 3)] * 10, [rng.choice(live) for _ in range(800)], "after compaction")
    assert_in_step(gg, "batch after compaction")

"""Batched DeepWalk queries (bingo_walk_batch, the serving loop's continuous batching): every query of a
batch gets exactly the paths and step count of its own bingo_walk call and of the oracle, for queries
of every size (empty ones included), length (0 included), seed and id base, with integer biases,
fixed-point biases and alias rows, and every dense speculation.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, skew_edges, u32

pytestmark = pytest.mark.gpu


def graphs(kind):
    n, src, dst, w = skew_edges()
    kw = {"fixed": {"frac_bits": 8}, "alias": {"alias_table": True}}.get(kind, {})
    og = O.Graph(n, np.array(src), np.array(dst), np.array(w), frac_bits=kw.get("frac_bits", 0),
                 alias=kw.get("alias_table", False))
    gg = B().Graph(n, torch.tensor(src), torch.tensor(dst), torch.tensor(w), **kw)
    return n, og, gg


@pytest.mark.parametrize("kind", ["integer", "fixed", "alias"])
@pytest.mark.parametrize("spec", [1, 2, 4])
def test_batch_equals_single_queries(kind, spec):
    n, og, gg = graphs(kind)
    gg.set_tuning(dense_spec=spec)
    rng = random.Random(31 + spec)
    sizes = [0, 1, 5, 1000, 0, 300, 64, 2, 0]
    queries = []
    for k in sizes:
        starts = np.array([rng.choice([0, 5, 6, 3, rng.randrange(n)]) for _ in range(k)], dtype=np.int64)
        queries.append((starts, rng.choice([0, 1, 7, 80]), rng.getrandbits(63), rng.getrandbits(40)))
    out = gg.walk_batch(queries)
    torch.cuda.synchronize()
    for (starts, L, seed, base), (paths, steps) in zip(queries, out):
        p1, s1 = gg.walk(starts, L, seed, base=base)
        op, os_ = og.deepwalk(starts, L, seed, base=base)
        assert np.array_equal(u32(paths), op) and np.array_equal(u32(p1), op)
        assert int(steps.item()) == int(s1.item()) == os_


def test_batch_of_the_maximum_size_and_one():
    n, og, gg = graphs("integer")
    b = B()
    rng = random.Random(7)
    queries = [(np.array([rng.randrange(n) for _ in range(rng.randrange(0, 40))], dtype=np.int64), 12, 1000 + i,
                i << 20) for i in range(b.WALK_BATCH_MAX)]
    for qs in (queries, queries[:1]):
        out = gg.walk_batch(qs)
        torch.cuda.synchronize()
        for (starts, L, seed, base), (paths, steps) in zip(qs, out):
            op, os_ = og.deepwalk(starts, L, seed, base=base)
            assert np.array_equal(u32(paths), op) and int(steps.item()) == os_


def test_batch_rejects_bad_arguments():
    n, og, gg = graphs("integer")
    b = B()
    q = (np.array([0, 1], dtype=np.int64), 5, 1, 0)
    with pytest.raises(b.BingoError):
        gg.walk_batch([q] * (b.WALK_BATCH_MAX + 1))
    # a descriptor with walks but no buffers, through the C ABI
    from paper_2504_10233_amd import binding
    qs = (binding._WalkQuery * 1)()
    qs[0] = binding._WalkQuery(1, None, 0, 5, 0, 1, None, None)
    assert b.load().bingo_walk_batch(gg.h, 1, qs, None) != 0


def test_more_overlapping_calls_than_counter_slots():
    """200 bingo_walk / bingo_walk_batch calls issued on 8 streams without a synchronization between
    them: more calls in flight than the handle's 64 counter slots, so slots are reused while their
    previous holders may still run on another stream.  Every call's paths and transition count equal
    the same call issued alone, and the oracle's."""
    n, og, gg = graphs("integer")
    rng = random.Random(97)
    streams = [torch.cuda.Stream() for _ in range(8)]
    calls, results = [], []
    for i in range(200):
        starts = np.array([rng.randrange(n) for _ in range(rng.choice([1, 50, 2000]))], dtype=np.int64)
        L, seed, base = rng.choice([5, 40, 80]), rng.getrandbits(63), rng.getrandbits(40)
        s = streams[i % len(streams)]
        with torch.cuda.stream(s):
            if i % 5 == 4:
                (paths, steps), = gg.walk_batch([(starts, L, seed, base)], stream=s)
            else:
                paths, steps = gg.walk(starts, L, seed, base=base, stream=s)
        calls.append((starts, L, seed, base))
        results.append((paths, steps))
    torch.cuda.synchronize()
    for i, ((starts, L, seed, base), (paths, steps)) in enumerate(zip(calls, results)):
        p1, s1 = gg.walk(starts, L, seed, base=base)
        torch.cuda.synchronize()
        assert torch.equal(paths, p1), i
        assert int(steps.item()) == int(s1.item()), i
        if i % 20 == 0:
            op, ost = og.deepwalk(starts, L, seed=seed, base=base)
            assert np.array_equal(u32(paths), op), i
            assert int(steps.item()) == ost, i

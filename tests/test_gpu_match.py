"""Delete matching at its boundaries, against the oracle: ranges of the flat matching space that span
more touched vertices than are staged in LDS (the vertex search then runs in global memory), and
ranges whose delete targets are too many to stage (every 2^s-th one is staged and each search ends
in global memory), with duplicate (src, dst) pairs deleted oldest first.  Needs an MI355X."""
import random

import numpy as np
import pytest

from test_gpu_parity import apply_both, both

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("split", [0, 64])
def test_ranges_spanning_many_small_vertices(split):
    # 6000 vertices of one or two edges; one batch deletes most of them and inserts into some, so a
    # range of 1024 matching entries spans several hundred touched vertices
    rng = random.Random(11)
    n = 7000
    src, dst, w = [], [], []
    for v in range(6000):
        for _ in range(1 + (v % 3 == 0)):
            src.append(v); dst.append(rng.randrange(n)); w.append(rng.randrange(1, 1 << 32))
    og, gg = both(n, src, dst, w)
    gg.set_tuning(update_split=split)
    edges = list(zip(src, dst))
    dels = [e for e in edges if rng.random() < 0.8] + [(rng.randrange(6000), rng.randrange(n)) for _ in range(200)]
    ins = [(rng.randrange(6000), rng.randrange(n), rng.randrange(1, 1 << 32)) for _ in range(1500)]
    apply_both(og, gg, ins, dels, "many small vertices")
    # a second batch on the result, deleting some of the new edges too
    cur = [(int(a), int(b)) for a, b, _ in ins]
    apply_both(og, gg, [], [e for e in cur if rng.random() < 0.5] + dels[:300], "many small vertices, second")


@pytest.mark.parametrize("split", [0, 64])
def test_hub_with_more_delete_targets_than_staged(split):
    # a hub with 24000 edges over 6000 distinct destinations (each about four times), and a batch of
    # 7000 deletes on it (several per destination: the oldest occurrences go first), plus inserts
    rng = random.Random(12)
    n = 8000
    src = [0] * 24000 + [rng.randrange(1, n) for _ in range(3000)]
    dst = [rng.randrange(6000) for _ in range(24000)] + [rng.randrange(n) for _ in range(3000)]
    w = [rng.choice([1, 6, 1 << rng.randrange(32), rng.randrange(1, 1 << 32)]) for _ in range(27000)]
    og, gg = both(n, src, dst, w)
    gg.set_tuning(update_split=split)
    dels = [(0, rng.randrange(6500)) for _ in range(7000)] + [(rng.randrange(1, n), rng.randrange(n))
                                                               for _ in range(500)]
    ins = [(0, rng.randrange(6000), rng.randrange(1, 1 << 32)) for _ in range(2000)]
    apply_both(og, gg, ins, dels, "hub, sampled targets")
    apply_both(og, gg, [], [(0, d) for d in range(0, 6000, 2)] * 2, "hub, every other destination twice")

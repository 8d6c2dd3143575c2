"""bingo_ppr_async: a PPR query whose visit histogram is left running on another stream while the
next update batch (and the next query's walk, which waits for it on the device) is issued.  Every
result equals the synchronous bingo_ppr on a twin graph given the same calls, and the oracle's.
Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, both, skew_edges, u32

pytestmark = pytest.mark.gpu


def twin(n, src, dst, w):
    return B().Graph(n, *(torch.tensor(x, dtype=torch.int64) for x in (src, dst, w)))


def batch(rng, n, live):
    ins = [(rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 24)) for _ in range(rng.randrange(50, 400))]
    dels = [rng.choice(live) for _ in range(rng.randrange(50, 400))]
    cols = [[x[i] for x in ins] for i in range(3)] + [[x[i] for x in dels] for i in range(2)]
    return [np.array(c, np.int64) for c in cols]


def same(a, b):
    return all(np.array_equal(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(a, b))


@pytest.mark.parametrize("fetch_between", [True, False])
def test_async_queries_overlapping_updates(fetch_between):
    """Query, then update, on the default stream with each query's histogram on another stream.
    fetch_between: the result is fetched after the update; else the next query follows at once (its
    walk waits for the previous histogram on the device) and only the last result is fetched."""
    rng = random.Random(5 if fetch_between else 6)
    n = 400
    src = [rng.randrange(n) for _ in range(6000)] + [0] * 1500
    dst = [rng.randrange(n) for _ in range(7500)]
    w = [rng.randrange(1, 1 << 24) for _ in range(7500)]
    og, ga = both(n, src, dst, w)
    gs = twin(n, src, dst, w)
    sh = torch.cuda.Stream()
    thr = B().ppr_threshold(0.15)
    sources = np.array([0, 3, 17, 399, 0, 250], dtype=np.int64)
    live = list(zip(src, dst))
    for b in range(5):
        steps_a = ga.ppr_async(sources, 300, thr, 60, seed=11 + b, base=b << 20, hist_stream=sh)
        cols = batch(rng, n, live)
        ga.update(*[torch.from_numpy(c) for c in cols])  # runs beside the histogram
        off_s, vtx_s, cnt_s, steps_s = gs.ppr(sources, 300, thr, 60, seed=11 + b, base=b << 20)
        gs.update(*[torch.from_numpy(c) for c in cols])
        assert steps_a == steps_s
        if fetch_between or b == 4:
            res = ga.ppr_result()
            assert same(res, (off_s, vtx_s, cnt_s)), b
            assert ga.ppr_wait() == (int(vtx_s.numel()), 0.0)  # nothing pending after the fetch
            if b == 0:
                ooff, ovtx, ocnt, osteps = og.ppr(sources, 300, thr, 60, seed=11, base=0)
                assert np.array_equal(res[0].cpu().numpy().astype(np.uint64), ooff)
                assert np.array_equal(u32(res[1]), ovtx) and np.array_equal(u32(res[2]), ocnt)
                assert osteps == steps_a
        cur = O.parse_dump(gs.export(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
    assert np.array_equal(ga.export(), gs.export())
    torch.cuda.synchronize()


def test_async_then_other_calls_wait():
    """Calls other than updates and queries wait for a pending histogram: a fetch, an export and a
    synchronous query right after an asynchronous one see its complete result."""
    og, ga = both(*skew_edges())
    gs = twin(*skew_edges())
    sh = torch.cuda.Stream()
    thr = B().ppr_threshold(0.2)
    sources = np.array([0, 6, 6, 5, 3], dtype=np.int64)
    ga.ppr_async(sources, 500, thr, 40, seed=3, hist_stream=sh)
    assert np.array_equal(ga.export(), gs.export())
    res = ga.ppr_result()
    ref = gs.ppr(sources, 500, thr, 40, seed=3)
    assert same(res, ref[:3])
    ne, ms = ga.ppr_wait()  # nothing pending: the count of the last result
    assert ne == int(ref[1].numel()) and ms == 0.0
    # an asynchronous query followed at once by a synchronous one: the second waits on the device
    ga.ppr_async(sources, 500, thr, 40, seed=4, hist_stream=sh)
    r2 = ga.ppr(sources, 500, thr, 40, seed=5)
    assert same(r2[:3], gs.ppr(sources, 500, thr, 40, seed=5)[:3])

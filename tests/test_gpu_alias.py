"""Alias-table inter-group selection (Sec. 4.1 as printed) on the HIP path, bit-exact against the oracle's
alias mode: walks in every form, PPR, node2vec, and the tables after batched and streaming updates.
Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, assert_same_structure, skew_edges, u32

pytestmark = pytest.mark.gpu


def aboth(n, src, dst, w, adaptive=True):
    src, dst, w = (np.asarray(x, dtype=np.int64) for x in (src, dst, w))
    og = O.Graph(n, src, dst, w, adaptive=adaptive, alias=True)
    gg = B().Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), adaptive=adaptive,
                   alias_table=True)
    return og, gg


def random_graph(seed, n=64):
    rng = random.Random(seed)
    src = [rng.randrange(n) for _ in range(3000)] + [6] * 4000
    dst = [rng.randrange(n) for _ in range(7000)]
    w = [rng.choice([1, 3, 255, 1 << rng.randrange(32), rng.randrange(1, 1 << 32), rng.randrange(1, 1 << 20)])
         for _ in range(7000)]
    return n, src, dst, w


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("variant,spec", [(0, 1), (1, 2), (1, 4)])
def test_walks_and_ppr(adaptive, variant, spec):
    n, src, dst, w = random_graph(1)
    og, gg = aboth(n, src, dst, w, adaptive)
    assert_same_structure(og, gg, "alias build")
    assert gg.memory()["alias_bytes"] == n * 32 * 16
    gg.set_tuning(walk_variant=variant, dense_spec=spec)
    starts = np.array([0, 5, 6, 3, 1, 2, 7, 40, 6, 6] * 40)
    for mode in (0, 1):
        paths, steps = gg.walk(starts, 25, 7, base=11, mode=mode)
        opaths, osteps = og.deepwalk(starts, 25, 7, base=11)
        assert np.array_equal(u32(paths), opaths), mode
        assert int(steps.item()) == osteps
    thr = int(0.15 * 2**32)
    sources = np.array([0, 5, 6, 3, 63])
    ooff, ovtx, ocnt, osteps = og.ppr(sources, 150, thr, 200, seed=3)
    for mode in (0, 1):
        off, vtx, cnt, st = gg.ppr(sources, 150, thr, 200, seed=3, mode=mode)
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == osteps


def test_node2vec():
    n, src, dst, w = random_graph(2)
    og, gg = aboth(n, src, dst, w)
    starts = np.arange(n).repeat(6)
    paths, _ = gg.node2vec(starts, 15, 4, 0.5, 2.0)
    opaths, _ = og.node2vec(starts, 15, 4, 0.5, 2.0)
    assert np.array_equal(u32(paths), opaths)


@pytest.mark.parametrize("split", [0, 64])
def test_tables_follow_batched_and_streaming_updates(split):
    og, gg = aboth(*skew_edges())
    gg.set_tuning(update_split=split)
    n = og.n
    rng = random.Random(3 + split)
    for b in range(6):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ins = [(6 if rng.random() < 0.5 else rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 32))
               for _ in range(rng.randrange(1, 300))]
        dels = [rng.choice(live) for _ in range(rng.randrange(1, 300))]
        a = [np.array(x, np.int64) for x in zip(*ins)] + [np.array(x, np.int64) for x in zip(*dels)]
        if b % 2 == 0:
            og.update(*a)
            gg.update(*[torch.from_numpy(x) for x in a])
        else:
            ops = [0] * len(ins) + [1] * len(dels)
            s = [x[0] for x in ins] + [x[0] for x in dels]
            d = [x[1] for x in ins] + [x[1] for x in dels]
            w = [x[2] for x in ins] + [0] * len(dels)
            order = list(range(len(ops)))
            rng.shuffle(order)
            ops, s, d, w = ([v[i] for i in order] for v in (ops, s, d, w))
            og.update_stream(ops, s, d, w)
            gg.update_stream(*[torch.tensor(x) for x in (ops, s, d, w)])
        assert_same_structure(og, gg, "batch %d" % b)
        starts = np.array([0, 5, 6, 3, 1, 2, 7] * 30)
        paths, _ = gg.walk(starts, 20, 100 + b)
        opaths, _ = og.deepwalk(starts, 20, 100 + b)
        assert np.array_equal(u32(paths), opaths), b


def test_alias_with_fixed_point_is_rejected():
    b = B()
    with pytest.raises(b.BingoError):
        b.Graph(4, torch.tensor([0]), torch.tensor([1]), torch.tensor([256]), frac_bits=8, alias_table=True)

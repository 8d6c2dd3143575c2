"""node2vec walks through the C ABI against the CPU oracle, bit for bit.  Needs an MI355X.

Covers several (p, q) settings, the p = q = 1 reduction to DeepWalk, vertices without out-edges,
hubs with parallel edges, the neighbour index rebuilt after update batches, every dense
speculation width, and bad arguments."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

from test_gpu_parity import B, both, c1, skew_edges, u32


@pytest.mark.parametrize("p,q", [(0.5, 2.0), (2.0, 0.5), (1.0, 3.0), (0.25, 0.25)])
def test_node2vec_c1(p, q):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    paths, counts = gg.node2vec(c["starts"], 40, c["seed"], p, q, base=9)
    opaths, osteps, oprops = og.node2vec(c["starts"], 40, c["seed"], p, q, base=9, with_proposals=True)
    assert np.array_equal(u32(paths), opaths)
    assert counts.tolist() == [osteps, oprops]


def test_node2vec_p_q_one_is_deepwalk():
    c = c1()
    _, gg = both(c["n"], c["src"], c["dst"], c["w"])
    a, ca = gg.node2vec(c["starts"], 30, 5, 1.0, 1.0, base=3)
    b, sb = gg.walk(c["starts"], 30, 5, base=3)
    assert np.array_equal(u32(a), u32(b)) and int(ca[0]) == int(sb.item()) == int(ca[1])


def test_node2vec_skew_graph_and_sinks():
    n, src, dst, w = skew_edges()
    og, gg = both(n, src, dst, w)
    starts = np.array(list(range(n)) * 20)  # includes sinks and isolated vertices
    for p, q in [(0.5, 2.0), (4.0, 0.25)]:
        paths, counts = gg.node2vec(starts, 25, 17, p, q)
        opaths, osteps, oprops = og.node2vec(starts, 25, 17, p, q, with_proposals=True)
        assert np.array_equal(u32(paths), opaths), (p, q)
        assert counts.tolist() == [osteps, oprops]


@pytest.mark.parametrize("spec", [1, 2, 4])
def test_node2vec_after_updates(spec):
    rng = random.Random(spec)
    n = 60
    src = [rng.randrange(n) for _ in range(700)] + [0] * 300
    dst = [rng.randrange(n) for _ in range(1000)]
    w = [rng.choice([1, 3, 1 << rng.randrange(32), rng.randrange(1, 1 << 24)]) for _ in range(1000)]
    og, gg = both(n, src, dst, w)
    gg.set_tuning(dense_spec=spec)
    starts = np.arange(n).repeat(10)
    for b in range(4):
        paths, counts = gg.node2vec(starts, 20, 100 + b, 0.5, 2.0)
        opaths, osteps, oprops = og.node2vec(starts, 20, 100 + b, 0.5, 2.0, with_proposals=True)
        assert np.array_equal(u32(paths), opaths), b
        assert counts.tolist() == [osteps, oprops], b
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ins = [(rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 24)) for _ in range(150)]
        dels = [rng.choice(live) for _ in range(150)]
        isrc, idst, iw = (np.array(x, np.int64) for x in zip(*ins))
        dsrc, ddst = (np.array(x, np.int64) for x in zip(*dels))
        og.update(isrc, idst, iw, dsrc, ddst)
        gg.update(*(torch.from_numpy(x) for x in (isrc, idst, iw, dsrc, ddst)))


def test_node2vec_rmat14():
    scale, ef = 14, 16
    m = ef << scale
    s, d = synth.rmat_graph(scale, m, 1014)
    w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, 2014)
    og, gg = both(1 << scale, s.numpy(), d.numpy(), w.numpy())
    starts = np.arange(0, 1 << scale, 7)
    paths, counts = gg.node2vec(starts, 30, 31, 0.5, 2.0)
    opaths, osteps, oprops = og.node2vec(starts, 30, 31, 0.5, 2.0, threads=8, with_proposals=True)
    assert np.array_equal(u32(paths), opaths)
    assert counts.tolist() == [osteps, oprops]


def test_node2vec_rejects_bad_arguments():
    b = B()
    c = c1()
    _, gg = both(c["n"], c["src"], c["dst"], c["w"])
    for p, q in [(0.0, 1.0), (1.0, -1.0), (float("nan"), 1.0), (1.0, float("inf"))]:
        with pytest.raises(b.BingoError):
            gg.node2vec(c["starts"][:4], 5, 1, p, q)

"""Floating-point biases (Sec. 4.3) on the HIP path, bit-exact against the oracle: the quantization
kernel, the structure after build and after update batches, DeepWalk / PPR / node2vec paths in every
walk form.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_parity import B, assert_same_structure, skew_edges, u32

pytestmark = pytest.mark.gpu


def qboth(n, src, dst, bias, lam, F, adaptive=True):
    w = O.quantize(bias, lam, F)
    assert (w > 0).all()
    og = O.Graph(n, src, dst, w, adaptive=adaptive, frac_bits=F)
    gg = B().Graph(n, torch.tensor(np.asarray(src, np.int64)), torch.tensor(np.asarray(dst, np.int64)),
                   torch.tensor(w.astype(np.int64)), adaptive=adaptive, frac_bits=F)
    return og, gg


def float_graph(seed, n=64, m=3000, hub=True, int_share=0.3):
    """Random graph with a hub (vertex 6); int_share of the biases are whole numbers, so with a high
    share the decimal groups are sparse, regular or one-element instead of dense."""
    rng = random.Random(seed)
    src = [rng.randrange(n) for _ in range(m)]
    if hub:
        src += [6] * 5000
    dst = [rng.randrange(n) for _ in range(len(src))]
    bias = []
    for _ in src:
        r = rng.random()
        if r < int_share:
            bias.append(float(rng.randrange(1, 1000)))            # integer: no decimal part
        elif r < int_share + (1 - int_share) / 2:
            bias.append(rng.randrange(1, 1000) + rng.random())    # the paper's "integer + U(0, 1)"
        else:
            bias.append(rng.uniform(0.01, 3.0))                   # mostly decimal
    return n, src, dst, bias


def test_quantize_matches_oracle():
    b = B()
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(0, 10, 5000), rng.lognormal(0, 4, 5000), rng.uniform(-1, 1, 200),
                        np.array([0.0, -0.0, np.nan, np.inf, -np.inf, 1e-30, 3.4e38, 0.5, 1.0, 0.1, 0.554, 0.726,
                                  0.32, 16777215.0, 16777216.0, 255.99609375])]).astype(np.float32)
    for lam, F in [(1.0, 8), (10.0, 8), (0.001, 16), (3.7, 1), (1e6, 4)]:
        got = b.quantize_biases(torch.from_numpy(x).cuda(), lam, F)
        want = O.quantize(x, lam, F)
        assert np.array_equal(u32(got), want), (lam, F)


@pytest.mark.parametrize("F", [1, 4, 8, 16])
@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("int_share", [0.3, 0.95])
def test_build_and_walks(F, adaptive, int_share):
    n, src, dst, bias = float_graph(F, int_share=int_share)
    lam = {1: 100.0, 4: 10.0, 8: 1.0, 16: 0.01}[F]
    og, gg = qboth(n, src, dst, bias, lam, F, adaptive)
    assert_same_structure(og, gg, "float build F=%d" % F)
    starts = np.array([0, 5, 6, 3, 1, 2, 7, 40, 6, 6] * 40)
    for mode in (0, 1):
        paths, steps = gg.walk(starts, 25, 11, base=3, mode=mode)
        opaths, osteps = og.deepwalk(starts, 25, 11, base=3)
        assert np.array_equal(u32(paths), opaths), mode
        assert int(steps.item()) == osteps


def test_paper_example_walks():
    """Fig. SAMPLING2's vertex 2 (lambda = 10), many one-step walks: the GPU picks what the oracle picks,
    decimal group draws included."""
    og, gg = qboth(6, [2, 2, 2], [1, 4, 5], [0.554, 0.726, 0.320], 10.0, 8)
    starts = np.full(20000, 2)
    paths, _ = gg.walk(starts, 1, 5)
    opaths, _ = og.deepwalk(starts, 1, 5)
    assert np.array_equal(u32(paths), opaths)


@pytest.mark.parametrize("variant,spec,bins", [(0, 1, 1), (1, 2, 0), (1, 4, 1)])
def test_ppr_and_tuning(variant, spec, bins):
    n, src, dst, bias = float_graph(21)
    og, gg = qboth(n, src, dst, bias, 1.0, 8)
    gg.set_tuning(walk_variant=variant, dense_spec=spec, ppr_bins=bins)
    thr = int(0.15 * 2**32)
    sources = np.array([0, 5, 6, 3, 7, 63])
    ooff, ovtx, ocnt, osteps = og.ppr(sources, 200, thr, 200, seed=9)
    for mode in (0, 1):
        off, vtx, cnt, steps = gg.ppr(sources, 200, thr, 200, seed=9, mode=mode)
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and steps == osteps
        paths, _ = gg.walk(np.arange(n).repeat(4), 20, 2, mode=mode)
        opaths, _ = og.deepwalk(np.arange(n).repeat(4), 20, 2)
        assert np.array_equal(u32(paths), opaths)


def test_node2vec():
    n, src, dst, bias = float_graph(5, hub=False)
    og, gg = qboth(n, src, dst, bias, 1.0, 8)
    starts = np.arange(n).repeat(8)
    paths, _ = gg.node2vec(starts, 20, 4, 0.5, 2.0)
    opaths, _ = og.node2vec(starts, 20, 4, 0.5, 2.0)
    assert np.array_equal(u32(paths), opaths)


@pytest.mark.parametrize("split", [0, 64])
def test_update_batches(split):
    F = 8
    n, src, dst, bias = float_graph(33)
    og, gg = qboth(n, src, dst, bias, 4.0, F)
    gg.set_tuning(update_split=split)
    rng = random.Random(split + 1)
    for b in range(10):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ni, nd = rng.randrange(0, 400), rng.randrange(0, 400)
        ins = [(6 if rng.random() < 0.4 else rng.randrange(n), rng.randrange(n)) for _ in range(ni)]
        iw = O.quantize([rng.choice([rng.uniform(0.01, 2.0), float(rng.randrange(1, 200)),
                                     rng.randrange(1, 50) + rng.random()]) for _ in range(ni)], 4.0, F)
        dels = [rng.choice(live) if rng.random() < 0.9 else (rng.randrange(n), rng.randrange(n)) for _ in range(nd)]
        if b == 4:  # every fraction of vertex 0 goes away: its decimal group empties
            dels += [(0, int(t)) for t, w in zip(cur[0]["dst"], cur[0]["w"]) if int(w) % (1 << F)]
        isrc = np.array([a for a, _ in ins], np.int64); idst = np.array([c for _, c in ins], np.int64)
        dsrc = np.array([a for a, _ in dels], np.int64); ddst = np.array([c for _, c in dels], np.int64)
        s2 = og.update(isrc, idst, iw, dsrc, ddst)
        s1 = gg.update(torch.from_numpy(isrc), torch.from_numpy(idst), torch.from_numpy(iw.astype(np.int64)),
                       torch.from_numpy(dsrc), torch.from_numpy(ddst))
        for key in ("inserted", "deleted", "not_found"):
            assert s1[key] == s2[key], (b, key)
        assert np.array_equal(s1["transitions"], s2["transitions"]), b
        assert_same_structure(og, gg, "float batch %d" % b)
        starts = np.arange(n).repeat(3)
        paths, _ = gg.walk(starts, 15, 100 + b)
        opaths, _ = og.deepwalk(starts, 15, 100 + b)
        assert np.array_equal(u32(paths), opaths), b


def test_zero_weight_after_quantization_is_rejected():
    b = B()
    w = O.quantize([1.0, 1e-9], 1.0, 8)
    assert w[1] == 0
    with pytest.raises(b.BingoError) as e:
        b.Graph(4, torch.tensor([0, 1]), torch.tensor([1, 2]), torch.tensor(w.astype(np.int64)), frac_bits=8)
    assert e.value.code == -3

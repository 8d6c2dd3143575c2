"""Parity on inputs shaped like the larger workloads, at sizes the oracle finishes in seconds.

* DeepWalk workload: R-MAT, Zipf(1.5) weights clipped to 2^20 - 1, one length-80 walk per vertex,
  then mixed batches of R-MAT inserts and deletions of existing edges, walks re-run after each.
* Skewed-update workload: R-MAT plus planted hubs (log-uniform extra degree), lognormal(8, 3)
  weights, batches of 10^2 .. 10^5 records (50/50), 80 % of endpoints on hubs.
Structures are compared on the whole dump or on sampled vertex ranges; walks and PPR entirely."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2504_10233_amd as B_
    return B_


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def same_ranges(og, gg, n, ranges):
    for (a, b) in ranges:
        assert np.array_equal(gg.export(a, b), og.dump(a, b)), (a, b)


def sample_ranges(n, k, width, seed):
    rng = np.random.default_rng(seed)
    starts = rng.integers(0, max(n - width, 1), k)
    return [(int(s), int(min(s + width, n))) for s in starts] + [(0, min(width, n)), (max(n - width, 0), n)]


def test_deepwalk_workload_batches():
    scale = 16
    n, m = 1 << scale, 16 << scale
    src, dst = synth.rmat_graph(scale, m, 1002)
    w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, 2002)
    og = O.Graph(n, src.numpy(), dst.numpy(), w.numpy())
    gg = B().Graph(n, src, dst, w)
    assert np.array_equal(gg.export(), og.dump())
    assert np.array_equal(gg.export_index(), og.index_dump())
    starts = np.arange(n)
    mirror = synth.EdgeMirror(src, dst)
    for b in range(3):
        paths, steps = gg.walk(starts, 80, 3002 + b, base=b * n)
        opaths, osteps = og.deepwalk(starts, 80, 3002 + b, base=b * n, threads=8)
        assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps, b
        k = 20_000
        bseed = 4200 + b
        isrc, idst = synth.rmat_graph(scale, k, bseed)
        iw = synth.weights_zipf(k, 1.5, (1 << 20) - 1, bseed)
        pos = mirror.pick_deletions(k, bseed, 30)
        dsrc, ddst = mirror.src[pos], mirror.dst[pos]
        mirror.apply(isrc, idst, pos)
        s1 = gg.update(isrc, idst, iw, dsrc, ddst)
        s2 = og.update(isrc.numpy(), idst.numpy(), iw.numpy(), dsrc.numpy(), ddst.numpy())
        assert (s1["inserted"], s1["deleted"], s1["not_found"]) == (s2["inserted"], s2["deleted"], s2["not_found"])
        assert np.array_equal(s1["transitions"], s2["transitions"])
        assert np.array_equal(gg.export(), og.dump()), b
        assert np.array_equal(gg.export_index(), og.index_dump()), b


@pytest.mark.parametrize("adaptive", [True, False])
def test_skewed_update_workload(adaptive):
    scale = 14
    n = 1 << scale
    src, dst = synth.rmat_graph(scale, 16 << scale, 1004)
    hubs, hsrc, hdst = synth.planted_hubs(n, 12, 3.0, 4.3, 1004)
    src = torch.cat([src, hsrc]); dst = torch.cat([dst, hdst])
    w = synth.weights_lognormal(src.numel(), 8.0, 3.0, 2004)
    og = O.Graph(n, src.numpy(), dst.numpy(), w.numpy(), adaptive=adaptive)
    gg = B().Graph(n, src, dst, w, adaptive=adaptive)
    assert np.array_equal(gg.export(), og.dump())
    assert np.array_equal(gg.export_index(), og.index_dump())
    mirror = synth.EdgeMirror(src, dst)
    for b, size in enumerate([100, 10_000, 100, 100_000]):
        bseed = 4400 + b
        half = size // 2
        isrc = synth.below(bseed, 1, half, n)
        on_hub = synth.below(bseed, 2, half, 10) < 8
        isrc = torch.where(on_hub, hubs[synth.below(bseed, 3, half, hubs.numel())], isrc)
        idst = synth.below(bseed, 4, half, n)
        iw = synth.weights_lognormal(half, 8.0, 3.0, bseed, stream=6)
        pos = mirror.pick_deletions(size - half, bseed, 30, hub_ids=hubs, hub_frac=0.8)
        dsrc, ddst = mirror.src[pos], mirror.dst[pos]
        mirror.apply(isrc, idst, pos)
        s1 = gg.update(isrc, idst, iw, dsrc, ddst)
        s2 = og.update(isrc.numpy(), idst.numpy(), iw.numpy(), dsrc.numpy(), ddst.numpy())
        assert (s1["inserted"], s1["deleted"], s1["not_found"]) == (s2["inserted"], s2["deleted"], s2["not_found"])
        assert np.array_equal(s1["transitions"], s2["transitions"]), b
        same_ranges(og, gg, n, sample_ranges(n, 6, 512, b))
        for h in hubs.tolist()[:4]:
            assert np.array_equal(gg.export(h, h + 1), og.dump(h, h + 1)), (b, h)
    assert np.array_equal(gg.export(), og.dump())
    assert np.array_equal(gg.export_index(), og.index_dump())
    thr = int(0.15 * 2**32)
    srcs = hubs.numpy()
    off, vtx, cnt, st = gg.ppr(srcs, 200, thr, 200, seed=11)
    ooff, ovtx, ocnt, ost = og.ppr(srcs, 200, thr, 200, seed=11, threads=8)
    assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == ost
    mem = gg.memory()
    omem = og.memory()
    assert mem["adjacency_bytes"] == omem["adjacency"]
    ga = omem["adjacency"] + omem["one"] + omem["sparse"] + omem["regular"] + omem["sparse_reduced_lists"]
    assert mem["model_ga_bytes"] == ga
    assert mem["model_bs_bytes"] == omem["adjacency"] + omem["all_regular_groups"]

"""Parity of the HIP path (through the C ABI) with the CPU oracle.  Needs an MI355X.

Everything is integer and the random streams are counter-based, so the bar is bit-exact: the
canonical structure dump, every walk path, every PPR histogram and the update statistics must equal
the oracle's, in both walk forms (persistent and per-step) and with and without group adaption."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU (run them with -m gpu on an MI355X)"


def B():
    _need_gpu()
    import paper_2504_10233_amd as B_
    return B_


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32) if t.dtype == torch.int32 else t.cpu().numpy().astype(np.uint32)


def both(n, src, dst, w, adaptive=True):
    src, dst, w = (np.asarray(x, dtype=np.int64) for x in (src, dst, w))
    og = O.Graph(n, src, dst, w, adaptive=adaptive)
    gg = B().Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), adaptive=adaptive)
    return og, gg


def assert_same_index(og, gg, where=""):
    """The group indexes (inverted index of regular groups, S(u) and the sparse groups' indexes over
    it) equal the oracle's, word for word."""
    a, b = gg.export_index(), og.index_dump()
    if not np.array_equal(a, b):
        n = min(len(a), len(b))
        first = int(np.argmax(a[:n] != b[:n])) if n and np.any(a[:n] != b[:n]) else n
        raise AssertionError("index dumps differ (%s) at word %d of %d/%d" % (where, first, len(a), len(b)))


def assert_same_structure(og, gg, where=""):
    assert_same_index(og, gg, where)
    a, b = gg.export(), og.dump()
    if not np.array_equal(a, b):
        va, vb = O.parse_dump(a, og.n), O.parse_dump(b, og.n)
        for u, (x, y) in enumerate(zip(va, vb)):
            for key in ("d", "next_seq", "mask"):
                assert x[key] == y[key], (where, u, key, x[key], y[key])
            assert np.array_equal(x["dst"], y["dst"]) and np.array_equal(x["w"], y["w"]), (where, u, "adjacency")
            assert np.array_equal(x["seq"], y["seq"]), (where, u, "seq")
            assert x["groups"] == y["groups"], (where, u, x["groups"], y["groups"])
        raise AssertionError("dumps differ (%s)" % where)


def c1():
    c = synth.config_c1()
    return {k: (v.numpy() if isinstance(v, torch.Tensor) else v) for k, v in c.items()}


def skew_edges():
    """Vertex 0 holds every group type; vertex 5 uses all 32 bits; vertex 6 is a hub spanning many
    64-edge chunks; vertex 3 has a self-loop; vertices 7.. are isolated."""
    rng = random.Random(3)
    src, dst, w = [], [], []
    ww = [1] * 40
    for i in range(12):
        ww[i] |= 2
    for i in (5, 9, 17):
        ww[i] |= 4
    ww[33] |= 1 << 9
    for i in range(0, 40, 2):
        ww[i] |= 8
    for i in range(40):
        src.append(0); dst.append(1 + i % 20); w.append(ww[i])
    for k in range(32):
        for r in range(1 + k % 3):
            src.append(5); dst.append(rng.randrange(60)); w.append((1 << k) | rng.randrange(1, 1 << max(k, 1)))
    src.append(5); dst.append(2); w.append(0xFFFFFFFF)
    for i in range(5000):
        src.append(6); dst.append(rng.randrange(60))
        w.append(rng.choice([1, 3, 1 << rng.randrange(32), rng.randrange(1, 1 << 31), 0xF0000000 | i]))
    src += [3, 1, 2]; dst += [3, 0, 5]; w += [7, 9, 1 << 31]
    return 64, src, dst, w


# --------------------------------------------------------------------------- build
@pytest.mark.parametrize("adaptive", [True, False])
def test_build_c1(adaptive):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"], adaptive)
    assert_same_structure(og, gg, "build c1")


@pytest.mark.parametrize("adaptive", [True, False])
def test_build_skew(adaptive):
    og, gg = both(*skew_edges(), adaptive=adaptive)
    assert_same_structure(og, gg, "build skew")


def test_build_degenerate():
    og, gg = both(1, [], [], [])
    assert_same_structure(og, gg, "empty graph")
    og, gg = both(3, [2], [2], [5])
    assert_same_structure(og, gg, "one self-loop")


def test_build_errors():
    b = B()
    with pytest.raises(b.BingoError) as e:
        b.Graph(4, torch.tensor([0, 9]), torch.tensor([1, 1]), torch.tensor([1, 1]))
    assert e.value.code == -2
    with pytest.raises(b.BingoError) as e:
        b.Graph(4, torch.tensor([0, 1]), torch.tensor([1, 1]), torch.tensor([1, 0]))
    assert e.value.code == -3


# --------------------------------------------------------------------------- walks
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("adaptive", [True, False])
def test_walks_c1(mode, adaptive):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"], adaptive)
    paths, steps = gg.walk(c["starts"], c["length"], c["seed"], mode=mode)
    opaths, osteps = og.deepwalk(c["starts"], c["length"], c["seed"])
    assert np.array_equal(u32(paths), opaths)
    assert int(steps.item()) == osteps


def test_walks_skew_sinks_and_bases():
    og, gg = both(*skew_edges())
    starts = np.array([0, 5, 6, 3, 1, 2, 7, 40, 6, 6, 0, 5] * 50)
    for base, seed, L in [(0, 1, 30), (2**40 + 17, 2**63 + 5, 7), (123, 0, 0), (5, 77, 1)]:
        for mode in (0, 1):
            paths, steps = gg.walk(starts, L, seed, base=base, mode=mode)
            opaths, osteps = og.deepwalk(starts, L, seed, base=base)
            assert np.array_equal(u32(paths), opaths), (base, seed, L, mode)
            assert int(steps.item()) == osteps


def test_walk_start_out_of_range():
    b = B()
    og, gg = both(*skew_edges())
    gg.walk(np.array([1, 999]), 4, 1)
    assert gg.status() == -2
    assert gg.status() == 0


# --------------------------------------------------------------------------- PPR
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("p,cap", [(0.15, 200), (1 / 80, 200), (0.15, 3), (0.0, 10)])
def test_ppr_c1(mode, p, cap):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    thr = int(p * 2**32)
    sources = np.array([0, 5, 17, 999, 500, 5])
    off, vtx, cnt, steps = gg.ppr(sources, 64, thr, cap, seed=31, base=7, mode=mode)
    ooff, ovtx, ocnt, osteps = og.ppr(sources, 64, thr, cap, seed=31, base=7)
    assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
    assert np.array_equal(u32(vtx), ovtx)
    assert np.array_equal(u32(cnt), ocnt)
    assert steps == osteps


def test_ppr_skew():
    og, gg = both(*skew_edges())
    sources = np.array([0, 5, 6, 3, 7])
    thr = int(0.15 * 2**32)
    for mode in (0, 1):
        off, vtx, cnt, steps = gg.ppr(sources, 300, thr, 200, seed=3, mode=mode)
        ooff, ovtx, ocnt, osteps = og.ppr(sources, 300, thr, 200, seed=3)
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and steps == osteps


# --------------------------------------------------------------------------- updates
def apply_both(og, gg, ins, dels, where):
    isrc = np.array([a for a, _, _ in ins], np.int64); idst = np.array([b for _, b, _ in ins], np.int64)
    iw = np.array([c for _, _, c in ins], np.int64)
    dsrc = np.array([a for a, _ in dels], np.int64); ddst = np.array([b for _, b in dels], np.int64)
    s2 = og.update(isrc, idst, iw, dsrc, ddst)
    s1 = gg.update(torch.from_numpy(isrc), torch.from_numpy(idst), torch.from_numpy(iw), torch.from_numpy(dsrc),
                   torch.from_numpy(ddst))
    for key in ("inserted", "deleted", "not_found"):
        assert s1[key] == s2[key], (where, key, s1[key], s2[key])
    assert np.array_equal(s1["transitions"], s2["transitions"]), where
    assert_same_structure(og, gg, where)


@pytest.mark.parametrize("adaptive", [True, False])
def test_update_c1(adaptive):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"], adaptive)
    ins = list(zip(c["ins_src"].tolist(), c["ins_dst"].tolist(), c["ins_w"].tolist()))
    dels = list(zip(c["del_src"].tolist(), c["del_dst"].tolist()))
    apply_both(og, gg, ins, dels, "c1 batch")
    for mode in (0, 1):
        paths, steps = gg.walk(c["starts2"], c["length"], c["seed"], base=1000, mode=mode)
        opaths, osteps = og.deepwalk(c["starts2"], c["length"], c["seed"], base=1000)
        assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps


@pytest.mark.parametrize("adaptive", [True, False])
@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("split", [0, 64])
def test_update_random_batches(adaptive, seed, split):
    rng = random.Random(seed)
    n = 40
    src = [rng.randrange(n) for _ in range(400)] + [0] * 300 + [1] * 70
    dst = [rng.randrange(n) for _ in range(400)] + [rng.randrange(6) for _ in range(300)] + \
          [rng.randrange(n) for _ in range(70)]
    w = [rng.choice([1, 2, 3, 7, 64, 1000, rng.randrange(1, 1 << 20), 1 << rng.randrange(32)]) for _ in range(770)]
    og, gg = both(n, src, dst, w, adaptive)
    gg.set_tuning(update_split=split)
    for b in range(14):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        ni, nd = rng.randrange(0, 120), rng.randrange(0, 120)
        hub = rng.random() < 0.6
        ins = [(0 if hub and rng.random() < 0.6 else rng.randrange(n), rng.randrange(n),
                rng.choice([1, 3, 5, 255, 1 << rng.randrange(32), rng.randrange(1, 1 << 32)])) for _ in range(ni)]
        dels = [rng.choice(live) if live and rng.random() < 0.85 else (rng.randrange(n), rng.randrange(n))
                for _ in range(nd)]
        if ins and rng.random() < 0.5:
            dels += [ins[0][:2], ins[-1][:2]]
        if b == 7:  # delete every edge of vertex 1
            dels += [(1, int(t)) for t in cur[1]["dst"]]
        apply_both(og, gg, ins, dels, "batch %d" % b)
        starts = np.arange(n).repeat(3)
        paths, _ = gg.walk(starts, 12, 1000 + b)
        opaths, _ = og.deepwalk(starts, 12, 1000 + b)
        assert np.array_equal(u32(paths), opaths), b


@pytest.mark.parametrize("split", [0, 64, 4096])
def test_update_edge_cases(split):
    """split 0 keeps every vertex in one wave; 64 and the default 4096 hand the hub's passes
    (5000 to 5700 entries, several chunks) to the split kernels."""
    og, gg = both(*skew_edges())
    gg.set_tuning(update_split=split)
    apply_both(og, gg, [], [], "empty batch")
    apply_both(og, gg, [(7, 1, 5)], [], "insert into an isolated vertex")
    apply_both(og, gg, [], [(9, 9), (0, 55)], "deletes of absent edges")
    apply_both(og, gg, [(0, 1, 1 << 30)] * 3, [(0, 1)] * 5, "duplicates inserted and deleted in one batch")
    apply_both(og, gg, [(6, 2, 1 << 31)] * 700, [], "hub grows past its capacity")
    cur = O.parse_dump(og.dump(), og.n)
    apply_both(og, gg, [], [(6, int(t)) for t in cur[6]["dst"][::2]], "hub loses half its edges")
    apply_both(og, gg, [(5, 1, 1)], [(5, int(t)) for t in cur[5]["dst"]], "all old edges of a vertex deleted")


def test_update_rejects_bad_batches():
    b = B()
    og, gg = both(*skew_edges())
    before = gg.export()
    for args in [([0], [1], [0], [], []), ([0], [99], [1], [], []), ([], [], [], [64], [0])]:
        with pytest.raises(b.BingoError):
            gg.update(*[torch.tensor(a, dtype=torch.int64) for a in args])
        assert np.array_equal(gg.export(), before)


def test_update_graph_replays_match_eager():
    """Batches run through the captured graph of their size bucket (replayed many times, with walks,
    exports and a second bucket in between) leave the same structure as the eager launches and the
    oracle."""
    rng = random.Random(11)
    n = 48
    src = [rng.randrange(n) for _ in range(600)] + [0] * 400
    dst = [rng.randrange(n) for _ in range(1000)]
    w = [rng.choice([1, 3, 1 << rng.randrange(32), rng.randrange(1, 1 << 24)]) for _ in range(1000)]
    og, gg = both(n, src, dst, w)
    ge = B().Graph(n, *(torch.tensor(x, dtype=torch.int64) for x in (src, dst, w)))
    ge.set_tuning(update_graphs=0)
    assert gg.get_tuning()["update_graphs"] == 1 and ge.get_tuning()["update_graphs"] == 0
    for b in range(12):
        cur = O.parse_dump(og.dump(), n)
        live = [(u, int(t)) for u, v in enumerate(cur) for t in v["dst"]]
        big = b in (5, 9)  # a second size bucket between replays of the first
        if b == 7:  # a new split threshold makes the captured graphs stale
            gg.set_tuning(update_split=64)
            assert gg.get_tuning()["update_split"] == 64
        ni, nd = (1500, 900) if big else (rng.randrange(1, 300), rng.randrange(1, 300))
        ins = [(rng.randrange(n), rng.randrange(n), rng.randrange(1, 1 << 32)) for _ in range(ni)]
        dels = [rng.choice(live) if rng.random() < 0.9 else (rng.randrange(n), rng.randrange(n)) for _ in range(nd)]
        apply_both(og, gg, ins, dels, "graph batch %d" % b)
        t = [torch.tensor(x, dtype=torch.int64) for x in zip(*ins)] + [torch.tensor(x, dtype=torch.int64)
                                                                        for x in zip(*dels)]
        se = ge.update(*t)
        assert np.array_equal(ge.export(), gg.export()), b
        assert se["touched_vertices"] > 0
        starts = np.arange(n).repeat(2)
        pg, _ = gg.walk(starts, 10, 50 + b)
        pe, _ = ge.walk(starts, 10, 50 + b)
        assert np.array_equal(u32(pg), u32(pe)), b
        torch.cuda.synchronize()


@pytest.mark.parametrize("graphs,split", [(0, 4096), (1, 4096), (1, 0), (0, 64)])
def test_update_candidate_overflow_retries(graphs, split):
    """A small batch whose deletes hit more stored occurrences than the bucket's candidate buffer
    holds is rerun with a larger buffer and still matches the oracle."""
    og, gg = both(*skew_edges())
    gg.set_tuning(update_graphs=graphs, update_split=split)
    rng = random.Random(5)
    ins = [(6, rng.randrange(60), rng.randrange(1, 1 << 32)) for _ in range(80000)]
    apply_both(og, gg, ins, [], "hub grows to 85000 edges")
    apply_both(og, gg, [(6, 1, 3)], [(6, t) for t in range(60)], "60 deletes hit every hub edge")
    apply_both(og, gg, [(6, 2, 5)] * 4, [(6, 2)] * 3, "small batch after the retry")


# --------------------------------------------------------------------------- larger graphs
@pytest.mark.parametrize("weights", ["uniform24", "zipf", "lognormal"])
def test_rmat_scale14(weights):
    scale, ef = 14, 16
    m = ef << scale
    s, d = synth.rmat_graph(scale, m, 1000 + scale)
    if weights == "uniform24":
        w = synth.weights_uniform(m, 1, 1 << 24, 2002)
    elif weights == "zipf":
        w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, 2002)
    else:
        w = synth.weights_lognormal(m, 8.0, 3.0, 2002)
    n = 1 << scale
    og, gg = both(n, s.numpy(), d.numpy(), w.numpy())
    assert_same_structure(og, gg, "rmat build")
    starts = np.arange(n)
    paths, steps = gg.walk(starts, 10, 42)
    opaths, osteps = og.deepwalk(starts, 10, 42, threads=8)
    assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps
    # one mixed batch, 20% on the four largest hubs
    deg = np.bincount(s.numpy(), minlength=n)
    hubs = torch.from_numpy(np.argsort(-deg)[:4].copy())
    mir = synth.EdgeMirror(s, d)
    pos = mir.pick_deletions(3000, 4000, 5, hub_ids=hubs, hub_frac=0.2)
    isrc, idst = synth.rmat_graph(scale, 3000, 4001)
    isrc[:600] = hubs[torch.arange(600) % 4]
    iw = synth.weights_lognormal(3000, 8.0, 3.0, 4002)
    ins = list(zip(isrc.tolist(), idst.tolist(), iw.tolist()))
    dels = list(zip(mir.src[pos].tolist(), mir.dst[pos].tolist()))
    apply_both(og, gg, ins, dels, "rmat batch")
    thr = int(0.15 * 2**32)
    srcs = np.nonzero(deg)[0][:50]
    off, vtx, cnt, st = gg.ppr(srcs, 100, thr, 200, seed=8)
    ooff, ovtx, ocnt, ost = og.ppr(srcs, 100, thr, 200, seed=8, threads=8)
    assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == ost


def test_generators_match_across_devices():
    _need_gpu()
    a = synth.rmat_graph(12, 5000, 7)
    b = synth.rmat_graph(12, 5000, 7, device="cuda")
    assert torch.equal(a[0], b[0].cpu()) and torch.equal(a[1], b[1].cpu())
    assert torch.equal(synth.weights_uniform(999, 1, 1 << 24, 3), synth.weights_uniform(999, 1, 1 << 24, 3, "cuda").cpu())


# --------------------------------------------------------------------------- tuning invariance
@pytest.mark.parametrize("variant,bpc,chunk,spec,bins", [(0, 0, 256, 1, 1), (1, 0, 256, 2, 0), (1, 1, 16, 4, 1),
                                                         (0, 2, 4096, 4, 0), (1, 3, 64, 1, 1), (0, 0, 64, 2, 1)])
def test_results_independent_of_tuning(variant, bpc, chunk, spec, bins):
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    gg.set_tuning(walk_variant=variant, blocks_per_cu=bpc, queue_chunk=chunk, dense_spec=spec, ppr_bins=bins)
    t = gg.get_tuning()
    assert (t["walk_variant"], t["blocks_per_cu"], t["queue_chunk"], t["dense_spec"], t["ppr_bins"]) == \
        (variant, bpc, chunk, spec, bins)
    opaths, osteps = og.deepwalk(c["starts"], c["length"], c["seed"])
    thr = int(0.15 * 2**32)
    sources = np.arange(0, 1000, 37)
    ooff, ovtx, ocnt, ost = og.ppr(sources, 100, thr, 200, seed=4)
    for mode in (0, 1):
        paths, steps = gg.walk(c["starts"], c["length"], c["seed"], mode=mode)
        assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps, mode
        off, vtx, cnt, st = gg.ppr(sources, 100, thr, 200, seed=4, mode=mode)
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == ost, mode


def test_tuning_rejects_bad_values():
    b = B()
    c = c1()
    _, gg = both(c["n"], c["src"], c["dst"], c["w"])
    for kw in [dict(walk_variant=2), dict(queue_chunk=100), dict(queue_chunk=8), dict(blocks_per_cu=65),
               dict(dense_spec=3), dict(dense_spec=8), dict(update_graphs=2), dict(ppr_bins=2),
               dict(update_split=10), dict(update_split=63)]:
        with pytest.raises(b.BingoError):
            gg.set_tuning(**kw)


def test_ppr_histogram_global_path():
    # p = 0 and a cap of 10: each source owns R * 11 > 16384 keys, beyond the per-source LDS
    # histogram, so the query takes the global sort path; both paths must agree with the oracle
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    sources = np.array([3, 4, 900])
    for R in (2000, 64):
        off, vtx, cnt, steps = gg.ppr(sources, R, 0, 10, seed=12, base=5)
        ooff, ovtx, ocnt, osteps = og.ppr(sources, R, 0, 10, seed=12, base=5)
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and steps == osteps


@pytest.mark.parametrize("R,cap", [(40, 9), (100, 9), (200, 9), (300, 12), (500, 15), (1000, 15), (1489, 10)])
@pytest.mark.parametrize("bins", [0, 1])
def test_ppr_histogram_widths(R, cap, bins):
    """p = 0 fixes every per-source key range at R * (cap + 1), so these cases pick each register
    width of the per-source sort (512 to 16384 slots, the last one exactly full), with visits in
    per-source bins (exactly full at p = 0) or in per-walk segments; sinks pad segments."""
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    gg.set_tuning(ppr_bins=bins)
    sources = np.array([0, 3, 4, 900, 17, 17])
    off, vtx, cnt, steps = gg.ppr(sources, R, 0, cap, seed=R, base=3)
    ooff, ovtx, ocnt, osteps = og.ppr(sources, R, 0, cap, seed=R, base=3)
    assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
    assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and steps == osteps


def test_autotune_keeps_results():
    from paper_2504_10233_amd.autotune import tune_ppr
    c = c1()
    og, gg = both(c["n"], c["src"], c["dst"], c["w"])
    thr = int(0.15 * 2**32)
    space = [dict(walk_variant=v, blocks_per_cu=b, queue_chunk=q) for v in (0, 1) for b in (0, 1) for q in (16, 256)]
    res = tune_ppr(gg, np.arange(50), 20, thr, 200, 1, space=space, repeats=1, use_cache=False)
    chosen = dict(res["chosen"])
    assert chosen.pop("wave_degree") in [r["wave_degree"] for r in res["wave_results"]]
    assert chosen in space and len(res["results"]) == len(space)
    assert gg.get_tuning()["wave_degree"] == res["chosen"]["wave_degree"]
    off, vtx, cnt, st = gg.ppr(np.arange(0, 1000, 9), 50, thr, 200, seed=2)
    ooff, ovtx, ocnt, ost = og.ppr(np.arange(0, 1000, 9), 50, thr, 200, seed=2)
    assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == ost

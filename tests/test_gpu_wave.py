"""Wave-per-vertex dense steps (bingo_tuning.wave_degree): a dense step at a vertex of at least the
threshold's degree is served by the whole wave, eight rejection attempts drawn and loaded at once,
the first accepting one in stream order taken by ballot.  At every threshold (every dense step, hubs
only, never) and every dense speculation, DeepWalk paths, step counts and PPR histograms equal the
oracle's, in both PPR forms (per-source bins and per-walk segments) and every selection mode
(integer biases, fixed-point biases, alias rows).  Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_parity import B, c1, skew_edges, u32

pytestmark = pytest.mark.gpu

THR = int(0.15 * 2**32)


def pair(n, src, dst, w, kind="integer"):
    kw = {"fixed": {"frac_bits": 8}, "alias": {"alias_table": True}}.get(kind, {})
    src, dst, w = (np.asarray(x, dtype=np.int64) for x in (src, dst, w))
    og = O.Graph(n, src, dst, w, frac_bits=kw.get("frac_bits", 0), alias=kw.get("alias_table", False))
    gg = B().Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), **kw)
    return og, gg


def check(og, gg, starts, sources, L=40, R=200, seed=11):
    opaths, osteps = og.deepwalk(starts, L, seed=seed, base=7)
    paths, steps = gg.walk(starts, L, seed, base=7)
    assert np.array_equal(u32(paths), opaths) and int(steps.item()) == osteps
    ooff, ovtx, ocnt, ost = og.ppr(sources, R, THR, 200, seed=seed + 1, base=3)
    for bins in (1, 0):
        gg.set_tuning(ppr_bins=bins)
        off, vtx, cnt, st = gg.ppr(sources, R, THR, 200, seed=seed + 1, base=3)
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), ooff), bins
        assert np.array_equal(u32(vtx), ovtx) and np.array_equal(u32(cnt), ocnt) and st == ost, bins


@pytest.mark.parametrize("kind", ["integer", "fixed", "alias"])
@pytest.mark.parametrize("wave_degree", [1, 2, 40, 5000, 0])
@pytest.mark.parametrize("spec", [1, 2, 4])
def test_wave_skew(kind, wave_degree, spec):
    """The skew graph: vertex 0 with dense groups of 40 edges, a hub of 5000 edges (vertex 6), a
    vertex with all 32 bits; thresholds from every dense step to the hub only."""
    n, src, dst, w = skew_edges()
    og, gg = pair(n, src, dst, w, kind)
    gg.set_tuning(walk_variant=1, dense_spec=spec, wave_degree=wave_degree)
    assert gg.get_tuning()["wave_degree"] == wave_degree
    starts = np.array([0, 6, 5, 3, 1, 2, 6, 6, 0] * 60)
    check(og, gg, starts, np.array([0, 6, 5, 3, 6]))


@pytest.mark.parametrize("wave_degree", [1, 16, 300])
def test_wave_c1(wave_degree):
    c = c1()
    og, gg = pair(c["n"], c["src"], c["dst"], c["w"])
    gg.set_tuning(walk_variant=1, wave_degree=wave_degree)
    check(og, gg, c["starts"], np.arange(0, 1000, 37), L=c["length"], R=100)


@pytest.mark.parametrize("weights", ["uniform24", "zipf"])
def test_wave_rmat14(weights):
    """R-MAT 14 (hubs of a few hundred to a few thousand edges) with the bench's weight laws."""
    scale, m = 14, 16 << 14
    src, dst = synth.rmat_graph(scale, m, 1403)
    if weights == "uniform24":
        w = synth.weights_uniform(m, 1, 1 << 24, 1404)
    else:
        w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, 1404)
    og, gg = pair(1 << scale, src.numpy(), dst.numpy(), w.numpy())
    deg = np.bincount(src.numpy(), minlength=1 << scale)
    hubs = np.argsort(-deg)[:8]
    for wd in (1, int(deg[hubs[4]])):
        gg.set_tuning(walk_variant=1, wave_degree=wd)
        starts = np.concatenate([np.repeat(hubs, 40), np.arange(0, 1 << scale, 17)])
        check(og, gg, starts, np.concatenate([hubs, np.arange(1, 1 << scale, 2000)]), L=30, R=150)

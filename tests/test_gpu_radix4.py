"""Radix base 4 (Supplement S.2) on the HIP path: the structure built on the GPU dumps word for word as
the oracle's base-4 structure, and DeepWalk paths and transition counts are bit-equal to the oracle's,
on a vertex with every subgroup type, a hub spanning many 64-edge chunks, the tiny ER workload and
R-MAT 12 with three weight laws, with and without adaption and at both dense speculation widths; the
calls a static base-4 structure does not support are refused.  Needs an MI355X."""
import random

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_parity import B, c1, u32

pytestmark = pytest.mark.gpu


def both4(n, src, dst, w, adaptive=True):
    src, dst, w = (np.asarray(x, dtype=np.int64) for x in (src, dst, w))
    og = O.Graph4(n, src, dst, w, adaptive=adaptive)
    gg = B().Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), adaptive=adaptive,
                   radix_base=4)
    return og, gg


def every_subgroup_edges():
    """Vertex 0: digit 0 of every edge is 1 (dense), digit 1 is 2 on 5 of 40 edges (regular 12.5 %),
    digit 2 is 3 on 2 edges (sparse), digit 5 is 1 on one edge (one element); vertex 1: every weight a
    single digit 3 at position 15 (all 48-bit totals near 2^62); vertex 2: a hub of 3000 edges with
    random weights; vertex 3 has no edges."""
    rng = random.Random(4)
    src, dst, w = [], [], []
    for i in range(40):
        x = 1
        if i < 5:
            x |= 2 << 2
        if i in (7, 30):
            x |= 3 << 4
        if i == 11:
            x |= 1 << 10
        src.append(0); dst.append((i * 3) % 50 + 4); w.append(x)
    for i in range(6):
        src.append(1); dst.append(i + 4); w.append(3 << 30)
    for i in range(3000):
        src.append(2); dst.append(rng.randrange(60)); w.append(rng.randrange(1, 1 << 32))
    for i in range(200):
        src.append(rng.randrange(4, 60)); dst.append(rng.randrange(60)); w.append(rng.choice([1, 3, 12, 48, 1 << 20]))
    return 60, src, dst, w


def check(og, gg, n, starts, length, seed, base=0):
    assert np.array_equal(gg.export(), og.dump())
    for spec in (1, 2):
        gg.set_tuning(dense_spec=spec)
        paths, steps = gg.walk(starts, length, seed, base=base)
        op, os_ = og.deepwalk(np.asarray(starts), length, seed, base=base)
        assert np.array_equal(u32(paths), op), "paths differ (dense_spec %d)" % spec
        assert int(steps.item()) == os_


@pytest.mark.parametrize("adaptive", [True, False])
def test_every_subgroup_type(adaptive):
    n, src, dst, w = every_subgroup_edges()
    og, gg = both4(n, src, dst, w, adaptive=adaptive)
    if adaptive:
        types = {s: t for s, (t, c, m) in O.parse_dump4(og.dump(), n)[0]["subgroups"].items()}
        assert {types[0], types[4], types[8], types[15]} == {O.T_DENSE, O.T_REGULAR, O.T_SPARSE, O.T_ONE}
    starts = np.array([0, 1, 2, 3] * 250)
    check(og, gg, n, starts, 30, 77)
    gg.close()


def test_c1_workload():
    c = c1()
    og, gg = both4(c["n"], c["src"], c["dst"], c["w"])
    check(og, gg, c["n"], np.asarray(c["starts"]), c["length"], c["seed"])
    gg.close()


@pytest.mark.parametrize("kind", ["uniform", "zipf", "lognormal"])
def test_rmat12(kind):
    n = 1 << 12
    src, dst = synth.rmat_graph(12, 16 * n, 61)
    m = src.numel()
    w = {"uniform": lambda: synth.weights_uniform(m, 1, 1 << 24, 62),
         "zipf": lambda: synth.weights_zipf(m, 1.5, (1 << 20) - 1, 62),
         "lognormal": lambda: synth.weights_lognormal(m, 8.0, 3.0, 62)}[kind]()
    og, gg = both4(n, src.numpy(), dst.numpy(), w.numpy())
    starts = synth.below(63, 0, 20000, n).numpy()
    check(og, gg, n, starts, 40, 64, base=1 << 34)
    mem = gg.memory()
    listed = sum(c for v in O.parse_dump4(og.dump(), n) for s, (t, c, mm) in v["subgroups"].items()
                 if t in (O.T_SPARSE, O.T_REGULAR))
    assert mem["list_bytes"] == 4 * listed and mem["edges"] == m
    gg.close()


def test_unsupported_calls_are_refused():
    n, src, dst, w = every_subgroup_edges()
    og, gg = both4(n, src, dst, w)
    b = B()
    lib = b.binding.load()
    e = torch.zeros(1, dtype=torch.int32, device=gg.device)
    with pytest.raises(b.BingoError):
        gg.walk(np.array([0]), 5, 1, mode=b.MODE_PER_STEP)
    with pytest.raises(b.BingoError):
        gg.update(torch.tensor([0]), torch.tensor([1]), torch.tensor([1]), torch.tensor([], dtype=torch.int64),
                  torch.tensor([], dtype=torch.int64))
    with pytest.raises(b.BingoError):
        gg.ppr(np.array([0]), 10, 1 << 30, 20, seed=1)
    with pytest.raises(b.BingoError):
        gg.export_index()
    assert lib.bingo_compact(gg.h, 0, None) == -1
    assert np.array_equal(gg.export(), og.dump())  # unchanged
    gg.close()

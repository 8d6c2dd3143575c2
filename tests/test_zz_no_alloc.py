"""The allocation-free DeepWalk entry point (bingo_walk_noalloc), called through the C ABI: two calls in a
row on one graph, the second with fewer walks and a shorter length, each equal bit for bit to bingo_walk
(persistent form) on the same inputs, and to the oracle; then a walk on a second, larger graph, whose
counters share the same device array.  Needs an MI355X."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_parity import B, c1, u32

pytestmark = pytest.mark.gpu


def _noalloc_vs_walk(og, gg, starts, length, seed, base):
    nw = len(starts)
    paths = torch.full((nw, length + 1), 7, dtype=torch.int32, device=gg.device)
    steps = torch.full((1,), -1, dtype=torch.int64, device=gg.device)
    gg.walk_noalloc(starts, length, seed, paths, steps, base=base)
    ref, rsteps = gg.walk(starts, length, seed, base=base)
    torch.cuda.synchronize()
    assert torch.equal(paths, ref), "paths differ from bingo_walk"
    assert int(steps.item()) == int(rsteps.item())
    op, osteps = og.deepwalk(np.asarray(starts), length, seed, base=base)
    assert np.array_equal(u32(paths), op) and int(steps.item()) == osteps


@pytest.mark.parametrize("spec", [1, 2, 4])
def test_noalloc_walk_twice_equals_bingo_walk(spec):
    c = c1()
    og = O.Graph(c["n"], c["src"], c["dst"], c["w"])
    gg = B().Graph(c["n"], torch.from_numpy(c["src"]), torch.from_numpy(c["dst"]), torch.from_numpy(c["w"]))
    gg.set_tuning(dense_spec=spec)
    starts = np.asarray(c["starts"], dtype=np.int64)
    _noalloc_vs_walk(og, gg, starts, 80, 3001, 0)
    _noalloc_vs_walk(og, gg, starts[:137], 13, 99, 1 << 33)
    gg.close()


def test_noalloc_walk_on_a_second_graph_and_no_walks():
    n = 1 << 12
    src, dst = synth.rmat_graph(12, 8 * n, 41)
    w = synth.weights_zipf(8 * n, 1.5, (1 << 20) - 1, 42)
    og = O.Graph(n, src.numpy(), dst.numpy(), w.numpy())
    gg = B().Graph(n, src, dst, w)
    starts = synth.below(43, 0, 20000, n).numpy()
    _noalloc_vs_walk(og, gg, starts, 40, 5, 0)
    _noalloc_vs_walk(og, gg, starts[:3], 2, 6, 0)
    # no walks: only the transition count (zero) is written
    paths = torch.zeros((0, 5), dtype=torch.int32, device=gg.device)
    steps = torch.full((1,), -1, dtype=torch.int64, device=gg.device)
    gg.walk_noalloc(np.zeros(0, dtype=np.int64), 4, 1, paths, steps)
    torch.cuda.synchronize()
    assert int(steps.item()) == 0
    gg.close()


def test_noalloc_walk_rejects_bad_arguments():
    c = c1()
    gg = B().Graph(c["n"], torch.from_numpy(c["src"]), torch.from_numpy(c["dst"]), torch.from_numpy(c["w"]))
    lib = B().binding.load()
    assert lib.bingo_walk_noalloc(None, 0, None, 0, 1, 0, None, None, None) == -1
    assert lib.bingo_walk_noalloc(gg.h, 4, None, 0, 1, 0, None, None, None) == -1
    gg.close()

"""The random-line read probe (a measurement aid of the library, not part of the method) runs in
both forms and both line widths and reports a positive rate.  Needs an MI355X."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dependent", [0, 1])
@pytest.mark.parametrize("line", [64, 128])
def test_probe_runs(dependent, line):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2504_10233_amd import probe_random_reads
    table = torch.zeros(1 << 18, dtype=torch.int32, device="cuda:0")  # 1 MiB
    r = probe_random_reads(table, 1024, 16, dependent, line)
    assert r["ms"] > 0 and r["GBps"] > 0
    assert r["lanes"] == 1024 and r["line_bytes"] == line


@pytest.mark.parametrize("extra", [0, 1, 3])
def test_replay_probe_counts_its_lines(extra):
    """The visit-stream replay reads one header line per visit plus `extra` adjacency lines per visit
    of a vertex with edges; ids past n are skipped."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import numpy as np
    from paper_2504_10233_amd import Graph
    rng = np.random.default_rng(7)
    n, m = 500, 3000
    src = rng.integers(0, n // 2, m)  # vertices n/2.. have no edges
    dst = rng.integers(0, n, m)
    w = rng.integers(1, 1 << 20, m)
    g = Graph(n, torch.from_numpy(src), torch.from_numpy(dst), torch.from_numpy(w), device="cuda:0")
    visits = rng.integers(0, n + 20, 10007)
    deg = np.bincount(src, minlength=n)
    ok = visits < n
    expect = int(ok.sum()) + extra * int((deg[visits[ok]] > 0).sum())
    for chain, lanes, dep in ((5, 256, True), (1, 512, True), (64, 256, False), (6, 1024, False)):
        r = g.probe_replay(torch.from_numpy(visits), chain, lanes, float(extra), dependent=dep, seed=3)
        assert r["lines"] == expect and r["ms"] > 0
    g.close()

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

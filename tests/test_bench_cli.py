"""The bench's command-line contract on the host: more than one GPU is refused with a message before
anything touches a device, and the result line carries the fixed fields of the contract."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_result_line_fields():
    import bench
    sys.argv = ["bench.py", "--steps", "7", "--warmup", "2"]
    args = bench.parse()
    assert (args.gpus, args.steps, args.warmup, args.workload) == (1, 7, 2, "ppr")
    r = bench.common_fields(args, 1.5e9, "walk-steps/s", 8.5, {"workload": "w"})
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config"):
        assert k in r, k
    assert r["n_gpus"] == 1 and r["vs_baseline"] is None and r["higher_is_better"] is True
    assert r["config"]["workload"] == "w" and r["steps"] == 7 and r["warmup"] == 2

"""Autotuner for the persistent walk kernels.

It sweeps the walk knobs of bingo_set_tuning (walk variant, resident blocks per compute unit,
walk ids per queue atomic, dense-rejection attempts per round) on a probe query and keeps the
fastest setting; then, with that setting, it sweeps the degree threshold above which a dense step
is served by the whole wave instead of its own lane (wave per vertex against thread per walk).
Walks are keyed by (seed, walk id), so every setting returns the same results; only the
walk-kernel time differs.  That time is read from the library's HIP events (bingo_last_phase_ms).
Results are cached as JSON keyed by device and workload signature.
"""
from __future__ import annotations

import json
import os

# The binned PPR kernel has attempt-interleaved lanes whatever walk_variant says; variant 1 is also
# the faster one for the segmented fallback, so the sweep keeps it fixed.
DEFAULT_SPACE = [dict(walk_variant=1, blocks_per_cu=b, queue_chunk=c, dense_spec=s, wave_degree=0)
                 for b in (0, 2, 4, 5, 6, 8) for c in (128, 256, 512) for s in (1, 2, 4)]
# degree thresholds of the wave-per-vertex form (0: every step thread per walk; 1: every dense step
# wave per vertex)
WAVE_DEGREES = (0, 1, 64, 1024, 16384, 262144)


def _cache_path():
    return os.environ.get("BINGO_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "bingo_tune.json"))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune_ppr(g, sources, walks_per_source, thr, max_len, seed, base=0, space=None, repeats=2, signature=None,
             use_cache=True, wave_degrees=WAVE_DEGREES):
    """Pick the fastest tuning for a PPR query shape; returns {"chosen", "results", "wave_results",
    "cached"}."""
    import torch
    dev = torch.cuda.get_device_name(g.device)
    key = json.dumps([dev, signature]) if signature is not None else None
    path = _cache_path()
    cache = _load_cache(path) if use_cache else {}
    if key and key in cache:
        g.set_tuning(**cache[key]["chosen"])
        return dict(cache[key], cached=True)
    results = []
    for cfg in (space or DEFAULT_SPACE):
        g.set_tuning(**cfg)
        best = None
        for _ in range(repeats):
            g.ppr(sources, walks_per_source, thr, max_len, seed, base=base)
            ms = g.last_phase_ms()[1]
            best = ms if best is None else min(best, ms)
        results.append({"tuning": cfg, "walk_kernel_ms": best})
    chosen = dict(min(results, key=lambda r: r["walk_kernel_ms"])["tuning"])
    wave_results = []
    for wd in wave_degrees:
        g.set_tuning(**dict(chosen, wave_degree=wd))
        best = None
        for _ in range(repeats):
            g.ppr(sources, walks_per_source, thr, max_len, seed, base=base)
            ms = g.last_phase_ms()[1]
            best = ms if best is None else min(best, ms)
        wave_results.append({"wave_degree": wd, "walk_kernel_ms": best})
    if wave_results:
        chosen["wave_degree"] = min(wave_results, key=lambda r: r["walk_kernel_ms"])["wave_degree"]
    g.set_tuning(**chosen)
    out = {"chosen": chosen, "results": results, "wave_results": wave_results}
    if key and use_cache:
        cache[key] = out
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return dict(out, cached=False)

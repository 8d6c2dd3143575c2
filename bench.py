"""Benchmark of the radix-group random-walk hot path on one MI355X.

Workload (R-MAT scale 24, edge factor 16: 16,777,216 vertices, 268,435,456 edges, a/b/c/d =
0.57/0.19/0.19/0.05, ids permuted, weights uniform in [1, 2^24)), resident in HBM.  One step is one
pass of the whole hot path over one batch: a batch of 10^6 edge updates (500,000 R-MAT inserts with
uniform weights, 500,000 deletions of existing edges) followed by personalized-PageRank walks from
10,000 distinct non-sink sources x 1,000 walks (termination probability 0.15 before every step,
at most 200 steps), reduced to per-source visit histograms.  The graph build is timed once.

Prints one JSON line.  `value` is walk transitions per second of whole step time (updates + walks +
histograms); the update and walk phases are also reported on their own.  The roofline object covers
the walk kernel, timed with HIP events recorded by the library on the stream it runs on.  The
cpu_baseline object times the CPU oracle on this host on the same workload (the same batches, then
the last step's PPR query) and checks the GPU histograms against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s + edge-updates/s at R-MAT-24 on 1 GPU; p99 query latency"
HBM_PEAK_GBS = 8000.0
LINE = 64  # bytes per random access line counted as algorithmic traffic


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["ppr", "deepwalk", "skewed-updates", "serving"], default="ppr",
                    help="ppr (default): R-MAT 24 PPR with 10^6-record batches; deepwalk: R-MAT 22 Zipf DeepWalk "
                         "with 2x10^6-record batches; skewed-updates: R-MAT 24 + planted hubs, batches 10^2..10^7; "
                         "serving: R-MAT 25 request stream at 50/80/95 %% of saturation")
    ap.add_argument("--serve-count", type=int, default=10_000, help="requests per load level (serving workload)")
    ap.add_argument("--update-sizes", default="100,10000,1000000,10000000",
                    help="batch sizes of the skewed-updates workload (comma-separated; the value is quoted on the "
                         "largest)")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--sources", type=int, default=10_000)
    ap.add_argument("--walks-per-source", type=int, default=1_000)
    ap.add_argument("--batch", type=int, default=1_000_000)
    ap.add_argument("--mode", choices=["persistent", "per_step"], default="persistent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None, help="walk_variant,blocks_per_cu,queue_chunk[,dense_spec[,ppr_bins]] (skips the autotuner)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=1000.0, help="offered requests per second (Poisson)")
    ap.add_argument("--no-insert-delete", action="store_true",
                    help="skip the insert-only / delete-only batch comparison")
    ap.add_argument("--serve-batch", type=int, default=1,
                    help="walk queries the serving loop merges into one launch (1 = none)")
    ap.add_argument("--oracle-threads", type=int, default=16)
    ap.add_argument("--node2vec-walks", type=int, default=1_000_000,
                    help="node2vec walks (length 80, p = 0.5, q = 2) on the final graph; 0 skips")
    ap.add_argument("--stream-records", type=int, default=1_000_000,
                    help="records of the streaming-update measurement on the final graph (0 skips)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the timed steps one at a time (no PPR histogram beside the next update batch)")
    ap.add_argument("--no-random-probe", action="store_true",
                    help="skip the random-line read probe (context for the roofline)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration runs)")
    return ap.parse_args()


def host_cpu():
    """The host the oracle ran on: CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def walk_src_hash():
    h = hashlib.sha256()
    for f in ("walk.hip", "dev.h", "step.h"):
        h.update(open(os.path.join(ROOT, "paper_2504_10233_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


SERVE_TUNING = dict(walk_variant=1, blocks_per_cu=4, queue_chunk=256, dense_spec=2, wave_degree=0)


def serve_phase(g, n, src, dst, args, log):
    """Requests through the serving loop on the resident graph: Poisson arrivals at args.serve_rate,
    4 walk queries per update batch; query start sets log-uniform in [1, 10^4] walks with length
    uniform in 5..80, update batches log-uniform in [1, 10^4] records (half inserts with uniform
    weights, half deletions of input edges).  Latency is submission to result ready.  A warm-up
    stream of 400 requests of the same law comes first: the first batch of each update-size bucket
    builds that bucket's plan and captured graph, which a resident server does once."""
    import numpy as np
    # the server runs with a latency setting (two dense attempts in flight per round, four resident
    # blocks per CU): the PPR throughput setting (one attempt, eight blocks) lengthens each walk's
    # chain of rounds, which a small query waits for; no setting changes a result
    kept = g.get_tuning()
    g.set_tuning(**SERVE_TUNING)
    warm = make_requests(np.random.default_rng(5004), 400, n, src, dst, 4, 4, 1 << 24)
    serve_requests(g, warm, args.serve_rate, max_batch=args.serve_batch)
    rng = np.random.default_rng(5005)
    reqs = make_requests(rng, args.serve_requests, n, src, dst, 4, 4, 1 << 24)
    res = serve_requests(g, reqs, args.serve_rate, max_batch=args.serve_batch)
    g.set_tuning(**kept)
    res.pop("kept")
    res["warmup_requests"] = len(warm)
    res["tuning"] = SERVE_TUNING
    log("serving: query p50 %.3f ms p99 %.3f ms, update p50 %.3f ms p99 %.3f ms" %
        (res["query_p50_ms"], res["query_p99_ms"], res["update_p50_ms"] or -1, res["update_p99_ms"] or -1))
    return res


def random_read_probe(dev, sizes_gib=(0.25, 1, 4, 8, 16)):
    """Random-line read rates on this GPU (bingo_probe_random_reads): uniform random 64-byte lines,
    independent (4 in flight per lane) and dependent (pointer chases), at several table sizes from
    the Infinity Cache's 256 MiB to beyond the walk's working set; the best concurrency of each.
    Context for the walk kernel's roofline: its transitions are short chains of dependent random
    reads, but over a skewed (R-MAT) access distribution rather than a uniform one."""
    import torch
    from paper_2504_10233_amd import probe_random_reads
    out = []
    for gib in sizes_gib:
        table = torch.empty(int(gib * (1 << 28)), dtype=torch.int32, device=dev)
        row = {"table_GiB": gib}
        for name, dep, shapes in [("independent_64B", 0, [(1 << 16, 2048), (1 << 18, 512), (1 << 19, 256)]),
                                  ("dependent_64B", 1, [(1 << 17, 256), (1 << 18, 128), (1 << 19, 64)])]:
            best = None
            for lanes, reads in shapes:
                probe_random_reads(table, lanes, 4, dep, 64)  # warm the code path
                r = probe_random_reads(table, lanes, reads, dep, 64, seed=lanes)
                if best is None or r["GBps"] > best["GBps"]:
                    best = r
            row[name + "_GBps"] = best["GBps"]
            row[name + "_lanes"] = best["lanes"]
        out.append(row)
        del table
        torch.cuda.empty_cache()
    return out


def replay_probe(g, dev, off, vtx, cnt, nwalks, lanes):
    """An achievable rate for the walk kernel's own access pattern (bingo_probe_replay): the visits
    of the query just run (from its per-source histograms, in a seeded random order within each
    source, sources in order) replayed over the same graph at the walk kernel's resident lane
    count, one chain of visits per walk; per visit the header line and 1 or 2 random adjacency
    lines of the vertex; dependent (the next address waits on what was read, as in a walk) at the
    walk's lane count, and independent (only the header-to-adjacency dependency) at the best of 1, 2
    and 4 times that many lanes: the pattern's ceiling."""
    import torch
    nsrc = off.numel() - 1
    seg = torch.repeat_interleave(torch.arange(nsrc, device=dev), off[1:] - off[:-1])
    c = cnt.to(torch.int64)
    visits = torch.repeat_interleave(vtx, c)
    key = torch.repeat_interleave(seg, c) << 32
    gen = torch.Generator(device=dev)
    gen.manual_seed(12345)
    key |= torch.randint(0, 1 << 32, key.shape, device=dev, generator=gen)
    ordered = visits  # each source's visits by vertex, sources in order (the histogram's order)
    visits = visits[torch.argsort(key)].contiguous()
    del seg, c, key
    chain = max(1, int(round(visits.numel() / max(nwalks, 1))))
    out = {"visits": int(visits.numel()), "chain": chain, "lanes": lanes,
           "order": "per-source visits of the query, seeded random order within a source, sources in order; "
                    "'ordered': each source's visits by vertex (repeats of a vertex adjacent, the most cache "
                    "reuse its per-source grouping allows)"}
    for extra in (1, 2):
        best = None
        for mult in (1, 2, 4):
            g.probe_replay(ordered, chain, lanes * mult, float(extra), dependent=False, seed=7)  # warm
            r = g.probe_replay(ordered, chain, lanes * mult, float(extra), dependent=False, seed=7)
            if best is None or r["GBps"] > best["GBps"]:
                best = r
        out["ordered_extra_%d" % extra] = {"ms": best["ms"], "lines": best["lines"], "GBps": best["GBps"],
                                           "lanes": best["lanes"]}
    del ordered
    for dep in (True, False):
        for extra in (1, 2):
            # the walk kernel's resident lanes, and (as the ceiling) the best of 1, 2 and 4 times as many
            best = None
            for mult in ((1,) if dep else (1, 2, 4)):
                g.probe_replay(visits, chain, lanes * mult, float(extra), dependent=dep, seed=7)  # warm
                r = g.probe_replay(visits, chain, lanes * mult, float(extra), dependent=dep, seed=7)
                if best is None or r["GBps"] > best["GBps"]:
                    best = r
            out["%s_extra_%d" % ("dependent" if dep else "independent", extra)] = {
                "ms": best["ms"], "lines": best["lines"], "GBps": best["GBps"], "lanes": best["lanes"]}
    del visits
    torch.cuda.empty_cache()
    return out


def stream_copy_GBps(dev, gib=1):
    """Streaming bandwidth: a 1 GiB device-to-device copy (read + write bytes over the kernel time)."""
    import torch
    a = torch.empty(gib << 28, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(3):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None or ms < best else best
    del a, b
    torch.cuda.empty_cache()
    return 2 * (gib << 30) / (best / 1e3) / 1e9


def update_roofline(rows, mem, edges, r_rand_GBps, r_stream_GBps):
    """Model of the update batch's minimum time (the work the method itself must do): streamed bytes
    (the records, 12 B per insert and 8 B per delete, and about four radix passes reading and writing
    8-byte keys) over the streaming bandwidth, plus random 64-byte lines (an insert touches its adjacency
    slot and, per listed group of the edge, a list slot and its block; a delete the same for the
    deleted edge and for the moved tail edge) over the random-line rate.  Listed groups per edge are
    taken from the structure (live list entries / edges).  Locating deletes is reported beside it, since
    the paper does not say how an edge (src, dst) is found: through the edge locator, one random line per
    delete to find it and, to keep the locator in step, one per delete to retire its slot, two per moved
    edge (its dst and its slot; about one moved edge per delete) and one per insert to claim a slot; with
    the locator off, a scan of the touched adjacencies (8 B per scanned entry)."""
    le = mem["list_bytes"] / 4.0 / max(edges, 1)
    n = len(rows)
    ins = sum(r["inserted"] for r in rows) / n
    dels = sum(r["deleted"] + r["not_found"] for r in rows) / n
    scanned = sum(r["match_scanned"] for r in rows) / n
    ms = sum(r["update_ms"] for r in rows) / n
    b_seq = ins * 12 + dels * 8 + (ins + dels) * 4 * 2 * 8
    lines = ins * (1 + 2 * le) + dels * (1 + 4 * le)
    t_min = b_seq / (r_stream_GBps * 1e9) + lines * 64 / (r_rand_GBps * 1e9)
    located = all(r.get("located", True) for r in rows)
    t_loc = ((4 * dels + ins) * 64 / (r_rand_GBps * 1e9)) if located else scanned * 8 / (r_stream_GBps * 1e9)
    rec = ins + dels
    return {"records_per_batch": rec, "list_entries_per_edge": le, "streamed_bytes": b_seq, "random_lines": lines,
            "R_stream_GBps": r_stream_GBps, "R_rand_GBps": r_rand_GBps, "t_min_ms": t_min * 1e3,
            "locate_scanned_entries": scanned, "locate_by": "locator" if located else "scan",
            "t_locate_ms": t_loc * 1e3, "measured_ms": ms,
            "ceiling_updates_per_s": rec / t_min, "ceiling_with_locate_updates_per_s": rec / (t_min + t_loc),
            "frac": (t_min * 1e3) / ms, "frac_with_locate": ((t_min + t_loc) * 1e3) / ms,
            # the batch's random 64-byte lines (the model's, plus the locator's when it is used) per
            # second of the measured batch, as a fraction of the measured random-line rate and of the
            # 8 TB/s peak: the same denominators the walk's roofline uses
            "random_lines_frac_of_probe": (lines + (4 * dels + ins if located else 0)) * 64 / (ms / 1e3)
            / (r_rand_GBps * 1e9),
            "random_lines_frac_of_peak": (lines + (4 * dels + ins if located else 0)) * 64 / (ms / 1e3) / 8e12}


def torch_index(pos):
    import torch
    return torch.from_numpy(pos).to("cuda:0")


def common_fields(args, metric_value, unit, ms_per_step, config, dtype="u32"):
    return {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def workload_deepwalk(args):
    """R-MAT 22 (4,194,304 vertices, 67,108,864 edges), Zipf(1.5) weights clipped at 2^20 - 1; one DeepWalk
    walk of length 80 per vertex; per step one batch of 10^6 inserts + 10^6 deletions, then the walks again."""
    import numpy as np
    import torch
    import synth
    from paper_2504_10233_amd import Graph
    dev = torch.device("cuda:0")
    scale, ef, c = 22, 16, 2
    n, m = 1 << scale, ef << scale
    src, dst = synth.rmat_graph(scale, m, synth.SEEDS["graph"] + c, device=dev)
    w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, synth.SEEDS["weights"] + c, device=dev)
    torch.cuda.synchronize()
    tb = time.time()
    g = Graph(n, src, dst, w, device=dev)
    torch.cuda.synchronize()
    build_s = time.time() - tb
    nb = args.warmup + args.steps
    mirror = synth.EdgeMirror(src, dst)
    batches = []
    for b in range(nb):
        bseed = synth.SEEDS["batch"] + 100 * c + b
        isrc, idst = synth.rmat_graph(scale, 1_000_000, bseed, device=dev)
        iw = synth.weights_zipf(1_000_000, 1.5, (1 << 20) - 1, bseed, device=dev, stream=7)
        pos = mirror.pick_deletions(1_000_000, bseed, 30)
        dsrc, ddst = mirror.src[pos], mirror.dst[pos]
        mirror.apply(isrc, idst, pos)
        batches.append(tuple(x.to(torch.int32).contiguous() for x in (isrc, idst, iw, dsrc, ddst)))
    del mirror
    starts = torch.arange(n, dtype=torch.int32, device=dev)
    paths = torch.empty((n, 81), dtype=torch.int32, device=dev)
    rows = []
    stream = torch.cuda.current_stream()
    for i in range(nb):
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        st = g.update(*batches[i])
        e1.record(stream)
        _, steps = g.walk(starts, 80, synth.SEEDS["walks"] + c + 10 * i, base=0, out=paths)
        wk = None
        e2.record(stream)
        torch.cuda.synchronize()
        wk = g.last_phase_ms()[0]
        rows.append({"update_ms": e0.elapsed_time(e1), "walk_ms": e1.elapsed_time(e2), "walk_kernel_ms": wk,
                     "steps": int(steps.item()), "records": st["inserted"] + st["deleted"] + st["not_found"]})
        log("deepwalk step %d: update %.2f ms, walks %.2f ms (kernel %.2f), %d transitions" %
            (i, rows[-1]["update_ms"], rows[-1]["walk_ms"], wk, rows[-1]["steps"]))
    timed = rows[args.warmup:]
    tot_ms = sum(r["update_ms"] + r["walk_ms"] for r in timed)
    tot_steps = sum(r["steps"] for r in timed)
    res = common_fields(args, tot_steps / (tot_ms / 1e3), "walk-steps/s", tot_ms / len(timed),
                        {"workload": "rmat22-ef16-zipf1.5-deepwalk80-per-vertex-with-2e6-record-batches",
                         "vertices": n, "edges": m, "walks": n, "length": 80, "update_batch_records": 2_000_000})
    res.update({"walk_steps_per_s": tot_steps / (sum(r["walk_kernel_ms"] for r in timed) / 1e3),
                "edge_updates_per_s": sum(r["records"] for r in timed) / (sum(r["update_ms"] for r in timed) / 1e3),
                "build_s": build_s, "steps_detail": rows})
    # the walks of the first 20000 vertices in the last step (walk ids 0..19999, the ids the oracle gives
    # the same starts; vertex ids are a seeded permutation, so these are a random sample), kept before
    # the comparisons below reuse the path buffer
    sample = np.arange(20000, dtype=np.int64)
    gp = paths[:20000].cpu().numpy().view(np.uint32).copy()
    res["float_bias"] = float_vs_integer(n, src, dst, w, starts, paths, c)
    res["adaption"] = adaption_vs_baseline(n, src, dst, w, starts, paths, c)
    res["alias"] = alias_vs_its(n, src, dst, w, starts, paths, c, batches[:2])
    # sampled parity against the oracle after the same batches
    if not args.no_cpu_baseline:
        import oracle as O
        th = max(1, min(args.oracle_threads, host_cpu()["usable_cpus"] or os.cpu_count() or 1))
        og = O.Graph(n, src.cpu().numpy(), dst.cpu().numpy(), w.cpu().numpy())
        for bt in batches:
            og.update(*[x.cpu().numpy().view(np.uint32) for x in bt])
        t = time.time()
        op, osteps = og.deepwalk(sample, 80, synth.SEEDS["walks"] + c + 10 * (nb - 1), threads=th)
        cpu_s = time.time() - t
        res["parity"] = {"sampled_walks_equal": bool(np.array_equal(gp, op)), "walks": int(len(sample))}
        res["cpu_baseline"] = {"value": osteps / cpu_s, "unit": "walk-steps/s", "cores": th, "kind": "oracle",
                               "sample": "%d DeepWalk walks (the first vertices, a random sample under the id "
                                         "permutation) on the graph after the same batches" % len(sample)}
    return res


def stream_phase(g, n, scale, src, dst, c, count):
    """Streaming updates (one record at a time, Sec. 4.2) on the final graph: count records, half
    R-MAT inserts with uniform weights and half deletes of edges drawn from the initial edge list (some
    already gone: not found), through bingo_update_stream; then 200 records through the batch path
    one record per call (its captured graph of the smallest bucket)."""
    import torch
    import synth
    dev = src.device
    half = count // 2
    bseed = synth.SEEDS["batch"] + 100 * c + 77
    isrc, idst = synth.rmat_graph(scale, half, bseed, device=dev)
    iw = synth.weights_uniform(half, 1, 1 << 24, bseed, device=dev)
    pos = synth.below(bseed, 9, count - half, src.numel(), device=dev)
    dsrc, ddst = src[pos], dst[pos]
    order = torch.argsort(synth.hash_u64(bseed, 10, count, dev))  # inserts and deletes interleaved
    op = torch.cat([torch.zeros(half, dtype=torch.int64, device=dev), torch.ones(count - half, dtype=torch.int64,
                                                                                   device=dev)])[order]
    ss = torch.cat([isrc, dsrc])[order]
    dd = torch.cat([idst, ddst])[order]
    ww = torch.cat([iw, torch.zeros(count - half, dtype=iw.dtype, device=dev)])[order]
    rec = tuple(x.to(torch.int32).contiguous() for x in (op, ss, dd, ww))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.update_stream(*rec)
    t1 = time.perf_counter()
    ph = g.last_phase_ms()
    one = []
    e = torch.empty(0, dtype=torch.int32, device=dev)
    for i in range(200):
        if int(rec[0][i]) == 0:
            a = (rec[1][i:i + 1], rec[2][i:i + 1], rec[3][i:i + 1], e, e)
        else:
            a = (e, e, e, rec[1][i:i + 1], rec[2][i:i + 1])
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        g.update(*a)
        one.append(time.perf_counter() - u0)
    one.sort()
    out = {"records": count, "ms": (t1 - t0) * 1e3, "records_per_s": count / (t1 - t0),
           "apply_kernel_ms": ph[1] if len(ph) > 1 else None, "inserted": st["inserted"], "deleted": st["deleted"],
           "not_found": st["not_found"], "sources": st["touched_vertices"],
           "batch_of_one_median_ms": one[len(one) // 2] * 1e3, "batch_of_one_records_per_s": 1.0 / one[len(one) // 2]}
    log("streaming: %d records in %.1f ms (%.3g records/s; apply kernel %.1f ms, %d sources); batch path with one "
        "record per call: median %.3f ms (%.3g records/s)" %
        (count, out["ms"], out["records_per_s"], out["apply_kernel_ms"] or -1, out["sources"],
         out["batch_of_one_median_ms"], out["batch_of_one_records_per_s"]))
    return out


def float_vs_integer(n, src, dst, w, starts, paths, c):
    """Floating-point vs integer biases (the paper's microbenchmark: the float bias is the integer bias
    plus a uniform value in [0, 1)): the same edges built twice, once with the integer weights and once
    with the float biases (lambda = 1, 8 fraction bits); DeepWalk of length 80 from every vertex on
    each, three runs; walk-kernel time and memory ratios."""
    import torch
    import synth
    from paper_2504_10233_amd import Graph, quantize_biases
    frac = synth.below(synth.SEEDS["weights"] + c, 11, w.numel(), 1 << 24, device=w.device).to(torch.float32) / 2**24
    bias = w.to(torch.float32) + frac
    qw = quantize_biases(bias, 1.0, 8)
    del frac, bias
    out = {}
    for name, graph in (("integer", lambda: Graph(n, src, dst, w, device=w.device)),
                        ("float", lambda: Graph(n, src, dst, qw, device=w.device, frac_bits=8))):
        g = graph()
        ms = []
        for r in range(3):
            g.walk(starts, 80, synth.SEEDS["walks"] + c + 1000 + r, base=0, out=paths)
            torch.cuda.synchronize()
            ms.append(g.last_phase_ms()[0])
        mem = g.memory()
        out[name] = {"walk_kernel_ms": sorted(ms)[1], "pool_used_bytes": mem["pool_used_bytes"],
                     "model_ga_bytes": mem["model_ga_bytes"], "groups_by_type": mem["groups_by_type"]}
        g.close()
        torch.cuda.synchronize()
    out["time_ratio"] = out["float"]["walk_kernel_ms"] / out["integer"]["walk_kernel_ms"]
    out["memory_ratio_pool"] = out["float"]["pool_used_bytes"] / out["integer"]["pool_used_bytes"]
    out["memory_ratio_model"] = out["float"]["model_ga_bytes"] / out["integer"]["model_ga_bytes"]
    log("float biases: walk kernel %.2f ms vs %.2f ms integer (x%.3f), pool memory x%.3f, model memory x%.3f" %
        (out["float"]["walk_kernel_ms"], out["integer"]["walk_kernel_ms"], out["time_ratio"],
         out["memory_ratio_pool"], out["memory_ratio_model"]))
    return out


def adaption_vs_baseline(n, src, dst, w, starts, paths, c):
    """Group adaption (GA, Sec. 5.1) against the all-regular baseline (BS, Sec. 6.2): the same edges
    built both ways, DeepWalk of length 80 from every vertex, three runs each; walk-kernel time,
    pool memory and the paper's memory model."""
    import torch
    import synth
    from paper_2504_10233_amd import Graph
    out = {}
    for name, adaptive in (("ga", True), ("bs", False)):
        g = Graph(n, src, dst, w, device=w.device, adaptive=adaptive)
        ms = []
        for r in range(3):
            g.walk(starts, 80, synth.SEEDS["walks"] + c + 2000 + r, base=0, out=paths)
            torch.cuda.synchronize()
            ms.append(g.last_phase_ms()[0])
        mem = g.memory()
        out[name] = {"walk_kernel_ms": sorted(ms)[1], "pool_used_bytes": mem["pool_used_bytes"],
                     "groups_by_type": mem["groups_by_type"]}
        if adaptive:
            out["model_ga_bytes"], out["model_bs_bytes"] = mem["model_ga_bytes"], mem["model_bs_bytes"]
        g.close()
        torch.cuda.synchronize()
    out["bs_over_ga_time"] = out["bs"]["walk_kernel_ms"] / out["ga"]["walk_kernel_ms"]
    out["bs_over_ga_pool"] = out["bs"]["pool_used_bytes"] / out["ga"]["pool_used_bytes"]
    out["bs_over_ga_model"] = out["model_bs_bytes"] / out["model_ga_bytes"]
    log("adaption: walk kernel %.2f ms (GA) vs %.2f ms (BS, all regular) (x%.3f); pool memory BS/GA x%.3f, "
        "model BS/GA x%.3f" % (out["ga"]["walk_kernel_ms"], out["bs"]["walk_kernel_ms"], out["bs_over_ga_time"],
                               out["bs_over_ga_pool"], out["bs_over_ga_model"]))
    return out


def alias_vs_its(n, src, dst, w, starts, paths, c, batches):
    """Inter-group selection by inverse transform over the group totals (the default) against the
    32-slot alias rows: the same edges built both ways, DeepWalk of length 80 from every vertex, three
    runs each, then the first two 2e6-record update batches of this workload on each; the second
    batch's pipeline time (which includes rebuilding the rows of every touched vertex) is reported, the
    first one's carrying the allocation of the update plan."""
    import torch
    import synth
    from paper_2504_10233_amd import Graph
    out = {}
    for name, alias in (("its", False), ("alias", True)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g = Graph(n, src, dst, w, device=w.device, alias_table=alias)
        torch.cuda.synchronize()
        build = time.perf_counter() - t
        ms = []
        for r in range(3):
            g.walk(starts, 80, synth.SEEDS["walks"] + c + 3000 + r, base=0, out=paths)
            torch.cuda.synchronize()
            ms.append(g.last_phase_ms()[0])
        for b in batches:
            g.update(*b)
            torch.cuda.synchronize()
            upd = g.last_phase_ms()[0]
        mem = g.memory()
        out[name] = {"walk_kernel_ms": sorted(ms)[1], "build_s": build, "update_pipeline_ms": upd,
                     "alias_bytes": mem["alias_bytes"], "header_bytes": mem["header_bytes"]}
        g.close()
        torch.cuda.synchronize()
    out["alias_over_its_time"] = out["alias"]["walk_kernel_ms"] / out["its"]["walk_kernel_ms"]
    out["alias_over_its_update"] = out["alias"]["update_pipeline_ms"] / out["its"]["update_pipeline_ms"]
    log("alias rows: walk kernel %.2f ms vs %.2f ms inverse transform (x%.3f); update batch %.2f ms vs %.2f ms; "
        "rows %.2f GB beside %.2f GB of headers" %
        (out["alias"]["walk_kernel_ms"], out["its"]["walk_kernel_ms"], out["alias_over_its_time"],
         out["alias"]["update_pipeline_ms"], out["its"]["update_pipeline_ms"], out["alias"]["alias_bytes"] / 1e9,
         out["alias"]["header_bytes"] / 1e9))
    return out


def workload_skewed_updates(args):
    """R-MAT 24 plus 1,000 planted hubs with 10^U(5,6) extra edges each, lognormal(8, 3) weights;
    update batches of 10^2, 10^4, 10^6 and 10^7 records (half inserts, half deletions, 80 % of the
    endpoints on hubs), each size several times, with the captured-graph path and the eager path."""
    import numpy as np
    import torch
    import synth
    from paper_2504_10233_amd import Graph
    dev = torch.device("cuda:0")
    scale, c = 24, 4
    n = 1 << scale
    src, dst = synth.rmat_graph(scale, 16 << scale, synth.SEEDS["graph"] + c, device=dev)
    hubs, hsrc, hdst = synth.planted_hubs(n, 1000, 5.0, 6.0, synth.SEEDS["graph"] + c, device=dev)
    src = torch.cat([src, hsrc]); dst = torch.cat([dst, hdst])
    del hsrc, hdst
    m = src.numel()
    w = synth.weights_lognormal(m, 8.0, 3.0, synth.SEEDS["weights"] + c, device=dev)
    torch.cuda.synchronize()
    tb = time.time()
    g = Graph(n, src, dst, w, device=dev)
    torch.cuda.synchronize()
    build_s = time.time() - tb
    log("skewed: %d edges (%d on planted hubs), built in %.2fs" % (m, m - (16 << scale), build_s))
    # Parity at full size on a vertex sample: the batch changes every vertex independently (all its
    # inserts, then its deletes, then its rebuild), so the oracle needs only the edges and records
    # whose source is sampled to reproduce those vertices.  Sample: 20 hubs and 2000 other vertices.
    sample = torch.unique(torch.cat([hubs[:20].to(dev), synth.below(synth.SEEDS["graph"] + c, 40, 2000, n,
                                                                       device=dev)]))
    in_s = torch.zeros(n, dtype=torch.bool, device=dev)
    in_s[sample] = True
    em = in_s[src]
    o_edges = [x[em].cpu().numpy() for x in (src, dst, w)]
    o_batches = []
    mirror = synth.EdgeMirror(src, dst)
    del src, dst, w, em
    reps_for = {100: 40, 10_000: 20, 1_000_000: 4, 10_000_000: 2}
    plan = [(int(x), reps_for.get(int(x), 4)) for x in args.update_sizes.split(",")]
    out = {}
    b = 0
    for size, reps in plan:
        half = size // 2
        res = {}
        for graphs in (1, 0):
            g.set_tuning(update_graphs=graphs)
            times = []
            recs = 0
            for r in range(reps + 1):  # the first batch of each setting is a warm-up (plan build, capture)
                bseed = synth.SEEDS["batch"] + 100 * c + b
                b += 1
                isrc = synth.below(bseed, 1, half, n, device=dev)
                on_hub = synth.below(bseed, 2, half, 10, device=dev) < 8
                isrc = torch.where(on_hub, hubs[synth.below(bseed, 3, half, hubs.numel(), device=dev)], isrc)
                idst = synth.below(bseed, 4, half, n, device=dev)
                iw = synth.weights_lognormal(half, 8.0, 3.0, bseed, device=dev, stream=6)
                pos = mirror.pick_deletions(size - half, bseed, 30, hub_ids=hubs, hub_frac=0.8)
                dsrc, ddst = mirror.src[pos], mirror.dst[pos]
                mirror.apply(isrc, idst, pos)
                bt = tuple(x.to(torch.int32).contiguous() for x in (isrc, idst, iw, dsrc, ddst))
                mi, md = in_s[isrc], in_s[dsrc]
                o_batches.append([isrc[mi].cpu().numpy(), idst[mi].cpu().numpy(), iw[mi].cpu().numpy(),
                                  dsrc[md].cpu().numpy(), ddst[md].cpu().numpy()])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = g.update(*bt)
                t1 = time.perf_counter()
                if r:
                    times.append((t1 - t0) * 1e3)
                    recs += st["inserted"] + st["deleted"] + st["not_found"]
            times.sort()
            res["graph" if graphs else "eager"] = {"median_ms": times[len(times) // 2], "min_ms": times[0],
                                                   "records_per_s": recs / (sum(times) / 1e3), "batches": reps}
        res["graph_speedup"] = res["eager"]["median_ms"] / res["graph"]["median_ms"]
        mem = g.memory()
        res["memory"] = {k: mem[k] for k in ("model_ga_bytes", "model_bs_bytes", "list_bytes", "adjacency_bytes",
                                             "groups_by_type")}
        res["memory"]["bs_over_ga"] = mem["model_bs_bytes"] / max(mem["model_ga_bytes"], 1)
        out[str(size)] = res
        log("skewed: batch %d: graph %.3f ms, eager %.3f ms (x%.2f), %.3g records/s" %
            (size, res["graph"]["median_ms"], res["eager"]["median_ms"], res["graph_speedup"],
             res["graph"]["records_per_s"]))
    g.set_tuning(update_graphs=1)
    parity = None
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle as O
        t = time.time()
        og = O.Graph(n, *o_edges)
        for bb in o_batches:
            og.update(*bb)
        o_s = time.time() - t
        su = sample.cpu().numpy()
        dumps = index = True
        for u in su.tolist():
            dumps &= bool(np.array_equal(g.export(u, u + 1), og.dump(u, u + 1)))
            index &= bool(np.array_equal(g.export_index(u, u + 1), og.index_dump(u, u + 1)))
        hub_d = [int(O.parse_dump(og.dump(int(h), int(h) + 1), 1)[0]["d"]) for h in hubs[:20].tolist()]
        parity = {"sampled_vertices": int(su.size), "sampled_hubs": 20, "hub_degrees_min_max": [min(hub_d), max(hub_d)],
                  "oracle_edges": int(o_edges[0].size), "oracle_records": int(sum(x[0].size + x[3].size for x in o_batches)),
                  "batches_replayed": len(o_batches), "dumps_equal": dumps, "index_dumps_equal": index,
                  "oracle_s": o_s,
                  "method": "the oracle holds only the edges and records whose source is sampled; the batch changes "
                            "each vertex independently, so the sampled vertices' dumps must equal the GPU's"}
        log("skewed: parity on %d sampled vertices (20 hubs of degree %d..%d after the batches): dumps %s, "
            "indexes %s (oracle %.1fs, %d records)" % (su.size, min(hub_d), max(hub_d), dumps, index, o_s,
                                                       parity["oracle_records"]))
    big = out[str(plan[-1][0])]["graph"]
    r = common_fields(args, big["records_per_s"], "edge-updates/s", big["median_ms"],
                      {"workload": "rmat24-ef16-plus-1000-planted-hubs-lognormal-update-batches",
                       "vertices": n, "edges": m, "batch_sizes": [p[0] for p in plan], "hub_endpoint_share": 0.8})
    r.update({"batches": out, "build_s": build_s, "parity": parity,
              "note": "value: edge-updates/s of 10^7-record batches through the captured graph (host clock "
                      "around bingo_update_batch, which synchronizes); the inputs are device-resident"})
    return r


def make_requests(rng, count, n, src, dst, q_max_exp, u_max_exp, w_hi, base_shift=24):
    """4 walk queries per update batch: query start sets floor(10^U(0, q_max_exp)) uniform vertices with
    length uniform in 5..80; update batches floor(10^U(0, u_max_exp)) records, half inserts with uniform
    weights in [1, w_hi), half deletions of input edges."""
    m = src.numel()
    reqs = []
    for i in range(count):
        if rng.random() < 0.2:
            k = max(1, int(10 ** rng.uniform(0, u_max_exp)))
            ki = k // 2
            pos = rng.integers(0, m, k - ki)
            reqs.append(("update", rng.integers(0, n, ki), rng.integers(0, n, ki), rng.integers(1, w_hi, ki),
                         src[torch_index(pos)].cpu().numpy(), dst[torch_index(pos)].cpu().numpy()))
        else:
            nw = max(1, int(10 ** rng.uniform(0, q_max_exp)))
            reqs.append(("walk", rng.integers(0, n, nw), int(rng.integers(5, 81)), int(rng.integers(1 << 62)),
                         i << base_shift))
    return reqs


def serve_requests(g, reqs, rate, max_inflight=8, max_batch=1, keep=()):
    """Submit the requests to the serving loop with Poisson arrivals at `rate` per second (0: all at
    once), collect every result; latency is submission to result ready.  The paths of the walk
    requests whose indices are in `keep` are returned under "kept"."""
    import threading
    import numpy as np
    from paper_2504_10233_amd import Server
    rng = np.random.default_rng(len(reqs))
    gaps = rng.exponential(1.0 / rate, len(reqs)) if rate > 0 else np.zeros(len(reqs))
    srv = Server(g, max_inflight=max_inflight, max_batch=max_batch)
    tickets = [None] * len(reqs)
    infos = [None] * len(reqs)
    kept = {}
    keep = set(keep)
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(len(reqs)):
            ready.acquire()
            paths, infos[i] = srv.wait(tickets[i])
            if i in keep:
                kept[i] = paths

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    due = t0
    for i, r in enumerate(reqs):
        due += gaps[i]
        while time.perf_counter() < due:
            pass
        if r[0] == "walk":
            tickets[i] = srv.submit_walk(r[1], r[2], r[3], r[4])
        else:
            tickets[i] = srv.submit_update(*r[1:])
        ready.release()
    th.join()
    makespan = time.perf_counter() - t0
    srv.close()
    q = np.array([x["latency_us"] for x in infos if x["kind"] == 0]) / 1e3
    u = np.array([x["latency_us"] for x in infos if x["kind"] == 1]) / 1e3
    steps = sum(x["steps"] for x in infos if x["kind"] == 0)
    recs = sum(x["updates_applied"] + x["updates_not_found"] for x in infos if x["kind"] == 1)
    return {"requests": len(reqs), "offered_rate_per_s": rate, "max_inflight": max_inflight, "max_batch": max_batch,
            "achieved_rate_per_s": len(reqs) / makespan,
            "query_p50_ms": float(np.percentile(q, 50)), "query_p99_ms": float(np.percentile(q, 99)),
            "update_p50_ms": float(np.percentile(u, 50)) if u.size else None,
            "update_p99_ms": float(np.percentile(u, 99)) if u.size else None,
            "sustained_walk_steps_per_s": steps / makespan, "sustained_edge_updates_per_s": recs / makespan,
            "makespan_s": makespan, "errors": int(sum(1 for x in infos if x["status"] != 0)), "kept": kept}


def workload_serving(args):
    """R-MAT 25 (33,554,432 vertices, 536,870,912 edges), Zipf(1.5) weights, resident; Poisson
    stream of walk queries (start sets log-uniform in [1, 10^5], length 5..80) and update batches
    (log-uniform in [1, 10^4] records) at 4:1 by count; saturation measured first, then offered
    loads of 50, 80 and 95 % of it."""
    import numpy as np
    import torch
    import synth
    from paper_2504_10233_amd import Graph
    dev = torch.device("cuda:0")
    scale, c = 25, 5
    n, m = 1 << scale, 16 << scale
    src, dst = synth.rmat_graph(scale, m, synth.SEEDS["graph"] + c, device=dev)
    w = synth.weights_zipf(m, 1.5, (1 << 20) - 1, synth.SEEDS["weights"] + c, device=dev)
    torch.cuda.synchronize()
    tb = time.time()
    g = Graph(n, src, dst, w, device=dev)
    torch.cuda.synchronize()
    build_s = time.time() - tb
    w_host = None if args.no_cpu_baseline else w.cpu().numpy()  # for the oracle's replay
    del w
    rng = np.random.default_rng(synth.SEEDS["serving"] if "serving" in synth.SEEDS else 5005)
    nreq = args.serve_count
    # every request in submission order, for the oracle's replay; the server applies the updates in
    # that order and a query sees exactly the updates submitted before it
    history = []
    warm = make_requests(rng, 200, n, src, dst, 5, 4, 1 << 20)
    serve_requests(g, warm, 0, max_batch=args.serve_batch)
    history += warm
    sreqs = make_requests(rng, max(500, nreq // 4), n, src, dst, 5, 4, 1 << 20)
    # a sample of the served queries of the saturation run (every request submitted at once, so the
    # most queries and updates in flight together) is checked against the oracle
    walks = [i for i, q in enumerate(sreqs) if q[0] == "walk"]
    keep = walks[:: max(1, len(walks) // 24)][:24]
    sat = serve_requests(g, sreqs, 0, max_batch=args.serve_batch, keep=keep)
    checked = {len(history) + i: paths for i, paths in sat.pop("kept").items()}
    history += sreqs
    rate_sat = sat["achieved_rate_per_s"]
    log("serving R-MAT 25: saturation %.0f requests/s, %.3g walk steps/s" % (rate_sat, sat["sustained_walk_steps_per_s"]))
    loads = {}
    for frac in (0.5, 0.8, 0.95):
        reqs = make_requests(rng, nreq, n, src, dst, 5, 4, 1 << 20)
        r = serve_requests(g, reqs, frac * rate_sat, max_batch=args.serve_batch)
        r.pop("kept")
        loads["%d%%" % int(frac * 100)] = r
        log("serving at %d%% load: query p50 %.2f ms p99 %.2f ms, update p50 %.2f ms p99 %.2f ms, %.3g steps/s" %
            (frac * 100, r["query_p50_ms"], r["query_p99_ms"], r["update_p50_ms"] or -1, r["update_p99_ms"] or -1,
             r["sustained_walk_steps_per_s"]))
    mid = loads["80%"]
    parity = None
    if not args.no_cpu_baseline and checked:
        import oracle as O
        t = time.time()
        log("serving: oracle: building on the host (%d edges)" % m)
        og = O.Graph(n, src.cpu().numpy(), dst.cpu().numpy(), w_host)
        build_o = time.time() - t
        last = max(checked)
        log("serving: oracle: built in %.1fs; replaying %d requests" % (build_o, last + 1))
        equal, walks_checked, steps_checked, recs = True, 0, 0, 0
        t = time.time()
        for i, q in enumerate(history[:last + 1]):
            if i % 250 == 0:
                log("serving: oracle: request %d of %d" % (i, last + 1))
            if q[0] == "update":
                st = og.update(*q[1:])
                recs += st["inserted"] + st["deleted"] + st["not_found"]
            elif i in checked:
                opaths, osteps = og.deepwalk(q[1], q[2], q[3], base=q[4], threads=args.oracle_threads)
                gp = checked[i]
                equal &= bool(np.array_equal(np.asarray(gp).reshape(-1).view(np.uint32), opaths.reshape(-1)))
                walks_checked += int(q[1].size)
                steps_checked += osteps
        parity = {"queries_checked": len(checked), "walks_checked": walks_checked, "steps_checked": steps_checked,
                  "paths_equal": equal, "updates_replayed": int(sum(1 for q in history[:last + 1] if q[0] == "update")),
                  "records_replayed": recs, "oracle_build_s": build_o, "oracle_replay_s": time.time() - t,
                  "method": "the request stream (warm-up, then the saturation run with every request submitted "
                            "at once) replayed on the oracle in submission order up to the last checked query; "
                            "each checked query (a sample of the saturation run) run at its version and its "
                            "served paths compared word for word"}
        log("serving: parity on %d served queries (%d walks) after %d replayed updates: %s" %
            (len(checked), walks_checked, parity["updates_replayed"], equal))
    res = common_fields(args, mid["sustained_walk_steps_per_s"], "walk-steps/s",
                        mid["makespan_s"] * 1e3 / max(mid["requests"], 1),
                        {"workload": "rmat25-ef16-zipf1.5-serving-4to1-queries-updates", "vertices": n, "edges": m,
                         "query_starts": "log-uniform [1, 1e5]", "query_length": "uniform 5..80",
                         "update_records": "log-uniform [1, 1e4]", "max_inflight": 8,
                         "max_batch": args.serve_batch})
    res.update({"p99_query_latency_ms": mid["query_p99_ms"], "saturation": sat, "loads": loads, "build_s": build_s,
                "parity": parity,
                "note": "value: sustained walk-steps/s at 80 % of the measured saturation rate; ms_per_step is "
                        "makespan per request at that load"})
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the graph would be replicated per "
              "GPU, walk ids range-sharded and each update batch broadcast). Use --gpus 1.", flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2504_10233_amd import Graph, MODE_PER_STEP, MODE_PERSISTENT, ppr_threshold

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload != "ppr":
        fn = {"deepwalk": workload_deepwalk, "skewed-updates": workload_skewed_updates,
              "serving": workload_serving}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    scale, ef = args.scale, args.edge_factor
    n, m = 1 << scale, ef << scale
    c = 3  # seeds of the R-MAT-24 PPR workload
    t0 = time.time()
    src, dst = synth.rmat_graph(scale, m, synth.SEEDS["graph"] + c, device=dev)
    w = synth.weights_uniform(m, 1, 1 << 24, synth.SEEDS["weights"] + c, device=dev)
    torch.cuda.synchronize()
    log("graph generated: n=%d m=%d in %.1fs" % (n, m, time.time() - t0))

    torch.cuda.synchronize()
    tb = time.time()
    g = Graph(n, src, dst, w, device=dev)
    torch.cuda.synchronize()
    build_s = time.time() - tb
    log("built in %.2fs" % build_s)

    # sources: distinct non-sink vertices
    deg = torch.bincount(src, minlength=n)
    nz = torch.nonzero(deg > 0).flatten()
    order = torch.argsort(synth.uniform_u32(synth.SEEDS["walks"] + c, 1, nz.numel(), dev))
    sources = nz[order[: args.sources]].contiguous()
    del deg, nz, order

    # update batches (device resident before timing)
    nb = args.warmup + args.steps
    mirror = synth.EdgeMirror(src, dst)
    batches = []
    half = args.batch // 2
    for b in range(nb):
        bseed = synth.SEEDS["batch"] + 100 * c + b
        isrc, idst = synth.rmat_graph(scale, half, bseed, device=dev)
        iw = synth.weights_uniform(half, 1, 1 << 24, bseed, device=dev, stream=7)
        pos = mirror.pick_deletions(args.batch - half, bseed, 30)
        dsrc, ddst = mirror.src[pos], mirror.dst[pos]
        mirror.apply(isrc, idst, pos)
        batches.append(tuple(x.to(torch.int32).contiguous() for x in (isrc, idst, iw, dsrc, ddst)))
    del mirror
    torch.cuda.synchronize()
    log("%d update batches ready" % nb)

    thr = ppr_threshold(0.15)
    cap = 200
    R = args.walks_per_source
    mode = MODE_PERSISTENT if args.mode == "persistent" else MODE_PER_STEP
    seed = synth.SEEDS["walks"] + c
    stream = torch.cuda.current_stream()
    tune = None
    if args.tuning:
        t_ = [int(x) for x in args.tuning.split(",")]
        g.set_tuning(walk_variant=t_[0], blocks_per_cu=t_[1], queue_chunk=t_[2],
                     dense_spec=t_[3] if len(t_) > 3 else None, ppr_bins=t_[4] if len(t_) > 4 else None)
    elif not args.no_autotune:
        from paper_2504_10233_amd.autotune import tune_ppr
        # tuned on a query of the timed one's size (a tenth of it favours fewer resident blocks: its
        # tail, where few walks are left, weighs more), with other walk ids
        probe_src = sources
        tune = tune_ppr(g, probe_src, R, thr, cap, seed + 1, base=1 << 40,
                        signature=[n, m, args.sources, R, "uniform24"], use_cache=False)
        log("autotune: chose %s" % tune["chosen"])
    rows = []
    last = None
    replay = None
    loc_on = g.get_tuning().get("update_locate", 1) == 1
    # the timed steps run back to back on a stream of their own: each query's visit histogram is
    # left running on a second stream (bingo_ppr_async) beside the next step's update batch, and
    # the K steps are timed as a whole between two device synchronizations; warm-up steps, and
    # every step with --no-overlap or the per-step form, run one at a time
    overlap = mode == MODE_PERSISTENT and not args.no_overlap
    main_st = torch.cuda.Stream() if overlap else stream
    hist_st = torch.cuda.Stream() if overlap else None
    t_timed = None
    pend = []
    for i in range(nb):
        base = i * args.sources * R
        timed_async = overlap and i >= args.warmup
        if not timed_async or i == args.warmup:
            torch.cuda.synchronize()
        if timed_async and i == args.warmup:
            t_timed = time.perf_counter()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        with torch.cuda.stream(main_st):
            e0.record(main_st)
            st = g.update(*batches[i])
            upd_phases = g.last_phase_ms()
            e1.record(main_st)
            if overlap:
                steps = g.ppr_async(sources, R, thr, cap, seed, base=base, hist_stream=hist_st)
                ppr_phases = list(g.last_phase_ms()[:2]) + [None]
                vtx = None
                if not timed_async:  # a warm-up step (first use of both streams) waits for its histogram
                    ne, hms = g.ppr_wait()
                    ppr_phases[2] = hms
            else:
                off, vtx, cnt, steps = g.ppr(sources, R, thr, cap, seed, base=base, mode=mode)
                ppr_phases = g.last_phase_ms()
            e2.record(main_st)
        if not timed_async:
            torch.cuda.synchronize()
        pend.append((e0, e1, e2))
        rows.append({"bound_ms": ppr_phases[0], "walk_kernel_ms": ppr_phases[1],
                     "hist_ms": ppr_phases[2], "update_phases_ms": upd_phases, "steps": steps,
                     "records": st["inserted"] + st["deleted"] + st["not_found"],
                     "entries": int(vtx.numel()) if vtx is not None else (ne if overlap and not timed_async else None),
                     "inserted": st["inserted"], "deleted": st["deleted"], "not_found": st["not_found"],
                     "touched_vertices": st["touched_vertices"], "match_scanned": st["match_scanned"],
                     "match_candidates": st["match_candidates"], "located": loc_on,
                     "histogram_overlapped": timed_async})
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_timed) * 1e3 if t_timed is not None else None
    if overlap:
        ne, hms = g.ppr_wait()
        rows[-1]["hist_ms"], rows[-1]["entries"] = hms, ne
        off, vtx, cnt = g.ppr_result()
    for i, ((e0, e1, e2), r) in enumerate(zip(pend, rows)):
        r["update_ms"], r["ppr_ms"], r["step_ms"] = e0.elapsed_time(e1), e1.elapsed_time(e2), e0.elapsed_time(e2)
        log("step %d: update %.2f ms %s (%d touched, %d entries read to locate deletes), ppr %.2f ms (bound %.2f, walk "
            "kernel %.2f, histogram %s), %d transitions" %
            (i, r["update_ms"], ["%.2f" % x for x in r["update_phases_ms"]], r["touched_vertices"],
             r["match_scanned"], r["ppr_ms"], r["bound_ms"], r["walk_kernel_ms"],
             "%.2f" % r["hist_ms"] if r["hist_ms"] is not None else "beside the next update", r["steps"]))
    steps = rows[-1]["steps"]
    base = (nb - 1) * args.sources * R
    last = (base, off.cpu().numpy(), vtx.cpu().numpy().view(np.uint32), cnt.cpu().numpy().view(np.uint32), steps)
    if not args.no_random_probe:
        tun = g.get_tuning()
        # resident blocks per CU of the walk kernel (0: as many as fit, 8 blocks of 256 threads)
        bpc = tun["blocks_per_cu"] or 8
        lanes = bpc * torch.cuda.get_device_properties(dev).multi_processor_count * 256
        replay = replay_probe(g, dev, off, vtx, cnt, args.sources * R, lanes)
        replay["transitions"] = int(steps)
        log("replay of the last query's %d visits over the graph (%d lanes, chains of %d), 1 / 2 adjacency "
            "lines per visit: dependent %.0f / %.0f GB/s, independent %.0f / %.0f GB/s, ordered %.0f / %.0f "
            "GB/s" % (replay["visits"], lanes, replay["chain"], replay["dependent_extra_1"]["GBps"],
                      replay["dependent_extra_2"]["GBps"], replay["independent_extra_1"]["GBps"],
                      replay["independent_extra_2"]["GBps"], replay["ordered_extra_1"]["GBps"],
                      replay["ordered_extra_2"]["GBps"]))
    timed = rows[args.warmup:]
    # overlapped steps: the wall time of the K steps together; else the sum of the steps' own times
    tot_ms = wall_ms if wall_ms is not None else sum(r["step_ms"] for r in timed)
    tot_steps = sum(r["steps"] for r in timed)
    upd_ms = sum(r["update_ms"] for r in timed)
    walk_ms = sum(r["walk_kernel_ms"] for r in timed)
    ppr_ms = sum(r["ppr_ms"] for r in timed)
    recs = sum(r["records"] for r in timed)

    # host-to-device time of an update batch (the paper copies its batches from the host): the last
    # batch's arrays from freshly allocated pinned host buffers; reported beside value, never in it
    hb = [torch.empty(x.shape, dtype=x.dtype, pin_memory=True) for x in batches[-1]]
    for h, x in zip(hb, batches[-1]):
        h.copy_(x)
    db = [torch.empty_like(x) for x in batches[-1]]
    torch.cuda.synchronize()
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record()
    for d_, h in zip(db, hb):
        d_.copy_(h, non_blocking=True)
    h1.record()
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1)
    h2d_bytes = sum(x.numel() * 4 for x in hb)
    per_batch_ms = upd_ms / len(timed)
    update_h2d = {"bytes_per_batch": h2d_bytes, "h2d_ms": h2d_ms, "h2d_GBps": h2d_bytes / (h2d_ms / 1e3) / 1e9,
                  "edge_updates_per_s_with_h2d": (recs / len(timed)) / ((per_batch_ms + h2d_ms) / 1e3)}
    del hb, db
    log("update batch from pinned host memory: %.3f ms for %.1f MB (%.1f GB/s); %.3g updates/s with the copy" %
        (h2d_ms, h2d_bytes / 1e6, update_h2d["h2d_GBps"], update_h2d["edge_updates_per_s_with_h2d"]))

    # the other walk form on the same (final) graph, for the persistent vs per-step comparison
    other = MODE_PER_STEP if mode == MODE_PERSISTENT else MODE_PERSISTENT
    g.ppr(sources, R, thr, cap, seed, base=last[0], mode=other)
    other_ms = g.last_phase_ms()[1]

    # node2vec (second order, p = 0.5, q = 2, length 80) on the same final graph: the first call
    # rebuilds the neighbour index, the second reuses it
    n2v = None
    if args.node2vec_walks:
        n2v_starts = sources.repeat((args.node2vec_walks + args.sources - 1) // args.sources)[: args.node2vec_walks]
        n2v_starts = n2v_starts.contiguous()
        n2v_seed = synth.SEEDS["walks"] + 40 + c
        g.node2vec(n2v_starts, 80, n2v_seed, 0.5, 2.0)
        idx_ms = g.last_phase_ms()[0]
        n2v_paths, n2v_counts = g.node2vec(n2v_starts, 80, n2v_seed, 0.5, 2.0)
        ph = g.last_phase_ms()
        n2v_steps, n2v_props = (int(x) for x in n2v_counts.tolist())
        n2v = {"walks": args.node2vec_walks, "length": 80, "p": 0.5, "q": 2.0, "starts": "the PPR sources, repeated",
               "index_rebuild_ms": idx_ms, "walk_kernel_ms": ph[1], "transitions": n2v_steps,
               "proposals": n2v_props, "steps_per_s": n2v_steps / (ph[1] / 1e3),
               "proposals_per_transition": n2v_props / max(n2v_steps, 1)}
        n2v_check = (n2v_starts[:2000].cpu().numpy(), n2v_paths[:2000].cpu().numpy().view(np.uint32), n2v_seed)
        del n2v_paths
        log("node2vec: %d walks, %.2f ms kernel (%.3g steps/s, %.2f proposals per step), index rebuild %.2f ms" %
            (args.node2vec_walks, ph[1], n2v["steps_per_s"], n2v["proposals_per_transition"], idx_ms))

    serving = None
    if args.serve_requests:
        serving = serve_phase(g, n, src, dst, args, log)

    # insert-only and delete-only batches of 5e5 records each (the paper finds inserts slower than
    # deletes, Sec. 6.3): the first batch's inserts again, and deletes of input edges, after an
    # untimed insert-only batch of the same size bucket
    kinds = None
    half = batches[0][0].numel()
    pos = None if args.no_insert_delete else synth.below(synth.SEEDS["batch"] + 100 * c + 91, 12, half, m, device=dev)
    if pos is not None:
        dsrc, ddst = src[pos].to(torch.int32).contiguous(), dst[pos].to(torch.int32).contiguous()
        e32 = torch.empty(0, dtype=torch.int32, device=dev)
        kinds = {}
        g.update(*(batches[1][:3] + (e32, e32)))  # untimed: builds and captures this size bucket's plan
        for kind, args5 in (("insert_only", batches[0][:3] + (e32, e32)),
                            ("delete_only", (e32, e32, e32, dsrc, ddst))):
            torch.cuda.synchronize()
            k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            k0.record()
            st_k = g.update(*args5)
            k1.record()
            torch.cuda.synchronize()
            kinds[kind] = {"records": half, "ms": k0.elapsed_time(k1),
                           "applied": st_k["inserted"] + st_k["deleted"], "not_found": st_k["not_found"]}
        kinds["insert_over_delete_time"] = kinds["insert_only"]["ms"] / kinds["delete_only"]["ms"]
        log("insert-only batch %.2f ms, delete-only batch %.2f ms (%d records each; x%.2f)" %
            (kinds["insert_only"]["ms"], kinds["delete_only"]["ms"], half, kinds["insert_over_delete_time"]))

    probe = None
    if not args.no_random_probe:
        probe = random_read_probe(dev)
        for row in probe:
            log("random 64-byte reads over %g GiB: independent %.0f GB/s, dependent %.0f GB/s" %
                (row["table_GiB"], row["independent_64B_GBps"], row["dependent_64B_GBps"]))

    if args.calibrate_copy_mb:
        # a plain streaming kernel of known traffic (read N bytes, write N bytes) under a kernel name
        # used nowhere else in the run, to scale the FETCH_SIZE / WRITE_SIZE counters
        a = torch.empty(args.calibrate_copy_mb << 18, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()

    result = {
        "metric": METRIC,
        "value": tot_steps / (tot_ms / 1e3),
        "unit": "walk-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tot_ms / len(timed),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "rmat%d-ef%d-uniform24-ppr-with-update-batches" % (scale, ef), "vertices": n,
                   "edges": m, "weights": "uniform[1,2^24)", "ppr_sources": args.sources, "walks_per_source": R,
                   "termination_prob": 0.15, "max_len": cap, "update_batch_records": args.batch,
                   "walk_form": args.mode, "group_adaption": True},
        "walk_steps_per_s": tot_steps / (walk_ms / 1e3),
        # the query's walk phase; its histogram runs beside the next update batch (overlapped steps)
        "ppr_query_ms": ppr_ms / len(timed),
        "histogram_overlap": overlap,
        "step_sum_ms": sum(r["step_ms"] for r in timed) / len(timed),
        "edge_updates_per_s": recs / (upd_ms / 1e3),
        "update_batch_ms": upd_ms / len(timed),
        "update_h2d": update_h2d,
        "build_s": build_s,
        "walk_form_compare": {"persistent_ms" if mode == MODE_PERSISTENT else "per_step_ms": walk_ms / len(timed),
                              "per_step_ms" if mode == MODE_PERSISTENT else "persistent_ms": other_ms},
        "p99_query_latency_ms": serving["query_p99_ms"] if serving else None,
        "node2vec": n2v,
        "serving": serving,
        "insert_vs_delete": kinds,
        "tuning": g.get_tuning(),
        "autotune": tune,
        "steps_detail": rows,
    }
    mem = g.memory()
    result["memory"] = {k: mem[k] for k in ("pool_used_bytes", "pool_garbage_bytes", "header_bytes",
                                             "adjacency_bytes", "list_bytes", "model_ga_bytes", "model_bs_bytes",
                                             "groups_by_type")}
    # ---- pool compaction after the batches (wall time: size scan, new arena, copy, old arena freed)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g.compact()
    torch.cuda.synchronize()
    mem2 = g.memory()
    result["compaction"] = {"ms": (time.perf_counter() - t) * 1e3, "garbage_bytes_before": mem["pool_garbage_bytes"],
                            "used_bytes_before": mem["pool_used_bytes"], "used_bytes_after": mem2["pool_used_bytes"],
                            "pool_bytes": mem2["pool_bytes"]}
    log("compaction: %.1f ms, %.2f GB of replaced blocks reclaimed (pool use %.2f -> %.2f GB)" %
        (result["compaction"]["ms"], mem["pool_garbage_bytes"] / 1e9, mem["pool_used_bytes"] / 1e9,
         mem2["pool_used_bytes"] / 1e9))

    # ---- CPU oracle on the host: same batches, then the last step's query; parity of the histograms
    mix = None
    if not args.no_cpu_baseline:
        import oracle as O
        th = max(1, min(args.oracle_threads, host_cpu()["usable_cpus"] or os.cpu_count() or 1))
        log("oracle: building on the host (%d edges)" % m)
        t = time.time()
        og = O.Graph(n, src.cpu().numpy(), dst.cpu().numpy(), w.cpu().numpy())
        log("oracle: built in %.1fs" % (time.time() - t))
        del w  # src and dst stay for the streaming measurement
        t = time.time()
        urecs = 0
        for bt in batches:
            a = [x.cpu().numpy().view(np.uint32) for x in bt]
            s2 = og.update(*a)
            urecs += s2["inserted"] + s2["deleted"] + s2["not_found"]
        oracle_upd_s = time.time() - t
        base, off, vtx, cnt, steps = last
        t = time.time()
        ooff, ovtx, ocnt, osteps, ost = og.ppr(sources.cpu().numpy(), R, thr, cap, seed, base=base, threads=th,
                                               with_stats=True)
        oracle_ppr_s = time.time() - t
        same = (np.array_equal(off.astype(np.uint64), ooff) and np.array_equal(vtx, ovtx)
                and np.array_equal(cnt, ocnt) and steps == osteps)
        result["parity"] = {"last_step_ppr_histograms_equal": bool(same), "sources": args.sources,
                            "entries": int(len(ovtx)), "transitions": int(osteps)}
        if n2v:
            st0, gp, sd = n2v_check
            op, _ = og.node2vec(st0, 80, sd, 0.5, 2.0, threads=th)
            result["parity"]["node2vec_first_2000_walks_equal"] = bool(np.array_equal(gp, op))
            log("oracle: node2vec parity on 2000 walks %s" % result["parity"]["node2vec_first_2000_walks_equal"])
        # the same oracle on one thread, over the first 200 sources of the query
        n1 = min(200, args.sources)
        t = time.time()
        _, _, _, osteps1 = og.ppr(sources[:n1].cpu().numpy(), R, thr, cap, seed, base=base, threads=1)
        one_s = time.time() - t
        result["cpu_baseline"] = {"value": osteps / oracle_ppr_s, "unit": "walk-steps/s", "cores": th,
                                  "kind": "oracle",
                                  "sample": "the last step's full PPR query (%d sources x %d walks, %d transitions) "
                                            "on the graph after the same %d update batches, %d OpenMP threads"
                                            % (args.sources, R, osteps, nb, th),
                                  "host": host_cpu(),
                                  "single_thread": {"value": osteps1 / one_s, "unit": "walk-steps/s",
                                                    "sample": "the first %d sources of the same query x %d walks "
                                                              "(%d transitions, %.1f s)" % (n1, R, osteps1, one_s)},
                                  "update_single_thread": {"value": urecs / oracle_upd_s, "unit": "edge-updates/s",
                                                           "sample": "the same %d batches of %d records replayed "
                                                                     "(%.1f s)" % (nb, args.batch, oracle_upd_s)}}
        log("oracle: single thread %.3g steps/s over %d sources" % (osteps1 / one_s, n1))
        mix = {"steps": int(ost[1] + ost[2] + ost[3] + ost[4]), "one": int(ost[1]), "dense": int(ost[2]),
               "sparse": int(ost[3]), "regular": int(ost[4]), "dense_attempts": int(ost[5])}
        result["selection_mix"] = mix
        log("oracle: ppr %.1fs (%d threads), parity %s" % (oracle_ppr_s, th, same))

    # ---- roofline of the walk kernel: algorithmic random lines per transition from the selection mix
    roof = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "achieved": None, "frac": None, "traffic": None}
    if mix and mix["steps"]:
        lines = 2 * mix["one"] + 3 * (mix["sparse"] + mix["regular"]) + mix["dense"] + mix["dense_attempts"]
        per_step = LINE * lines / mix["steps"] + 8  # + the 8-byte visit record written per transition
        per_walk = LINE + 8  # the start vertex's header line and its visit record
        nwalks = args.sources * R
        byts = per_step * tot_steps / len(timed) + per_walk * nwalks
        ach = byts / (walk_ms / len(timed) / 1e3) / 1e9
        roof.update({"achieved": ach, "frac": ach / HBM_PEAK_GBS, "bytes_per_transition": per_step,
                     "lines_per_transition": lines / mix["steps"]})
    if probe:
        roof["random_read_probe"] = probe
        r_stream = stream_copy_GBps(dev)
        big = max(probe, key=lambda r: r["table_GiB"])
        r_rand = max(big["independent_64B_GBps"], big["dependent_64B_GBps"])
        # the achievable random-access rate over a table at least the walk's working set (headers and adjacency)
        roof["random_probe_GBps"] = r_rand
        roof["random_probe_table_GiB"] = big["table_GiB"]
        if roof["achieved"] is not None:
            roof["frac_of_random_probe"] = roof["achieved"] / r_rand
    if replay is not None:
        roof["replay_probe"] = replay
        if roof["achieved"] is not None:
            # the replay's line rate at the walk's own mix: its lines beyond the header per transition,
            # spread over every visit (the start visits take none), interpolated linearly between the
            # runs with 1 and 2 extra lines per visit
            x = (roof["lines_per_transition"] - 1.0) * replay["transitions"] / replay["visits"]
            x = min(max(x, 1.0), 2.0)
            replay["walk_extra_lines_per_visit"] = x
            for form in ("dependent", "independent", "ordered"):
                r1, r2 = replay[form + "_extra_1"]["GBps"], replay[form + "_extra_2"]["GBps"]
                replay[form + "_GBps_at_walk_mix"] = r1 + (x - 1.0) * (r2 - r1)
            roof["achievable_GBps"] = max(replay[f + "_GBps_at_walk_mix"]
                                          for f in ("dependent", "independent", "ordered"))
            roof["frac_of_achievable"] = roof["achieved"] / roof["achievable_GBps"]
            roof["achievable_note"] = ("the query's own visits replayed over the graph (bingo_probe_replay) at the "
                                       "walk's lines per visit; the best of three orders: shuffled within each "
                                       "source with dependent chains, shuffled with independent visits, and each "
                                       "source's visits by vertex (the most reuse the per-source grouping allows). "
                                       "The walk itself lies between the shuffled and the ordered replays: its "
                                       "wave's lanes walk from one source in step")
            roof["frac_of_shuffled_replay"] = roof["achieved"] / max(replay["independent_GBps_at_walk_mix"],
                                                                     replay["dependent_GBps_at_walk_mix"])
        result["update_roofline"] = update_roofline(timed, mem, m, r_rand, r_stream)
        ur = result["update_roofline"]
        log("update roofline: %.2f ms model (%.2f ms locating deletes) vs %.2f ms measured: %.2f of the model, "
            "%.2f with locating (R_stream %.0f GB/s, R_rand %.0f GB/s over %g GiB)" %
            (ur["t_min_ms"], ur["t_locate_ms"], ur["measured_ms"], ur["frac"], ur["frac_with_locate"], r_stream,
             r_rand, big["table_GiB"]))
    prof = os.path.join(ROOT, "profiles", "walk_kernel_counters.json")
    if os.path.exists(prof):
        pc = json.load(open(prof))
        spec = g.get_tuning()["dense_spec"]
        if pc.get("src_hash") == walk_src_hash() and pc.get("kernel") == "k_ppr_binned<%d, 0>" % spec:
            roof["traffic"] = pc.get("traffic_bytes_per_launch")
    result["roofline"] = roof
    result["walk_src_hash"] = walk_src_hash()
    if args.stream_records:
        result["streaming"] = stream_phase(g, n, scale, src, dst, c, args.stream_records)
    # release the graph (pool, update plans, streams) and the inputs before the result line, so no
    # device work or allocation of the run outlives it
    g.close()
    del g, batches
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

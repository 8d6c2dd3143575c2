"""ctypes binding of libbingo.so: argument marshalling only.

Every function here converts torch device tensors into the plain pointers and sizes of the C ABI
(include/bingo.h) and raises BingoError on a non-zero return code.  No step of the method runs in
Python; if the shared library is missing the first call raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libbingo.so")
_lock = threading.Lock()
_lib = None

MODE_PERSISTENT = 0
MODE_PER_STEP = 1
STOP = 0xFFFFFFFF


class BingoError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().bingo_strerror(code).decode()
        super().__init__("%s: %s (%d)" % (where, msg, code))


class _Config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("adaptive", C.c_uint32), ("alpha_pct", C.c_uint32),
                ("beta_pct", C.c_uint32), ("pool_bytes", C.c_uint64), ("frac_bits", C.c_uint32),
                ("alias_table", C.c_uint32), ("radix_base", C.c_uint32), ("reserved", C.c_uint32)]


class _UpdateStats(C.Structure):
    _fields_ = [("inserted", C.c_uint64), ("deleted", C.c_uint64), ("not_found", C.c_uint64),
                ("touched_vertices", C.c_uint64), ("transitions", C.c_uint64 * 25), ("match_scanned", C.c_uint64),
                ("match_candidates", C.c_uint64)]


class _MemStats(C.Structure):
    _fields_ = [("vertices", C.c_uint64), ("edges", C.c_uint64), ("pool_bytes", C.c_uint64),
                ("pool_used_bytes", C.c_uint64), ("pool_garbage_bytes", C.c_uint64),
                ("header_bytes", C.c_uint64), ("adjacency_bytes", C.c_uint64),
                ("adjacency_reserved_bytes", C.c_uint64), ("list_bytes", C.c_uint64),
                ("list_reserved_bytes", C.c_uint64), ("groups_by_type", C.c_uint64 * 5),
                ("model_ga_bytes", C.c_uint64), ("model_bs_bytes", C.c_uint64), ("alias_bytes", C.c_uint64),
                ("index_bytes", C.c_uint64), ("index_reserved_bytes", C.c_uint64),
                ("locator_bytes", C.c_uint64)]


EXPORTS = ["bingo_build", "bingo_update_batch", "bingo_walk", "bingo_ppr", "bingo_ppr_fetch", "bingo_export",
           "bingo_export_range", "bingo_memory", "bingo_status", "bingo_last_phase_ms", "bingo_set_tuning",
           "bingo_get_tuning", "bingo_num_vertices", "bingo_destroy", "bingo_strerror", "bingo_server_create",
           "bingo_server_submit_walk", "bingo_server_submit_update", "bingo_server_wait", "bingo_server_destroy",
           "bingo_probe_random_reads", "bingo_node2vec", "bingo_quantize_biases", "bingo_update_stream",
           "bingo_compact", "bingo_walk_batch", "bingo_walk_noalloc", "bingo_export_index_range", "bingo_probe_replay",
           "bingo_check_locator", "bingo_ppr_async", "bingo_ppr_wait"]


class _ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("max_inflight", C.c_uint32), ("hbm_budget_bytes", C.c_uint64),
                ("max_batch", C.c_uint32), ("reserved", C.c_uint32)]


class _WalkQuery(C.Structure):
    _fields_ = [("n_walks", C.c_uint64), ("d_starts", C.c_void_p), ("walk_id_base", C.c_uint64),
                ("length", C.c_uint32), ("reserved", C.c_uint32), ("seed", C.c_uint64), ("d_paths", C.c_void_p),
                ("d_steps_taken", C.c_void_p)]


WALK_BATCH_MAX = 32


class _RequestInfo(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("status", C.c_int32), ("epoch", C.c_uint64), ("queue_us", C.c_double),
                ("latency_us", C.c_double), ("steps", C.c_uint64), ("path_words", C.c_uint64),
                ("updates_applied", C.c_uint64), ("updates_not_found", C.c_uint64)]


class _Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("walk_variant", C.c_uint32), ("blocks_per_cu", C.c_uint32),
                ("queue_chunk", C.c_uint32), ("update_graphs", C.c_uint32), ("dense_spec", C.c_uint32),
                ("ppr_bins", C.c_uint32), ("update_split", C.c_uint32), ("wave_degree", C.c_uint32),
                ("update_locate", C.c_uint32)]


def lib_path() -> str:
    return _LIB


def load():
    """Load libbingo.so (built by __graft_entry__.build() / build_lib.py)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB):
            raise RuntimeError("libbingo.so is not built (%s); run __graft_entry__.build()" % _LIB)
        L = C.CDLL(_LIB)
        vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
        L.bingo_build.argtypes = [C.POINTER(_Config), u32, u64, vp, vp, vp, vp, C.POINTER(vp)]
        L.bingo_update_batch.argtypes = [vp, u64, vp, vp, vp, u64, vp, vp, vp, C.POINTER(_UpdateStats)]
        L.bingo_update_stream.argtypes = [vp, u64, vp, vp, vp, vp, vp, C.POINTER(_UpdateStats)]
        L.bingo_walk.argtypes = [vp, u64, vp, u64, u32, u64, vp, vp, u32, vp]
        L.bingo_walk_noalloc.argtypes = [vp, u64, vp, u64, u32, u64, vp, vp, vp]
        L.bingo_node2vec.argtypes = [vp, u64, vp, u64, u32, C.c_double, C.c_double, u64, vp, vp, vp]
        L.bingo_ppr.argtypes = [vp, u32, vp, u32, u32, u32, u64, u64, u32, C.POINTER(u64), C.POINTER(u64), vp]
        L.bingo_ppr_fetch.argtypes = [vp, vp, vp, vp, u64, vp]
        L.bingo_export.argtypes = [vp, vp, u64, C.POINTER(u64), vp]
        L.bingo_export_range.argtypes = [vp, u32, u32, vp, u64, C.POINTER(u64), vp]
        L.bingo_export_index_range.argtypes = [vp, u32, u32, vp, u64, C.POINTER(u64), vp]
        L.bingo_memory.argtypes = [vp, C.POINTER(_MemStats), vp]
        L.bingo_check_locator.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), vp]
        L.bingo_ppr_async.argtypes = [vp, u32, vp, u32, u32, u32, u64, u64, C.POINTER(u64), vp, vp]
        L.bingo_ppr_wait.argtypes = [vp, C.POINTER(u64), C.POINTER(C.c_float)]
        L.bingo_compact.argtypes = [vp, C.c_uint64, vp]
        L.bingo_walk_batch.argtypes = [vp, C.c_uint32, C.POINTER(_WalkQuery), vp]
        L.bingo_status.argtypes = [vp, vp]
        L.bingo_last_phase_ms.argtypes = [vp, C.POINTER(C.c_float), u32, C.POINTER(u32)]
        L.bingo_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.bingo_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.bingo_server_create.argtypes = [vp, C.POINTER(_ServerConfig), C.POINTER(vp)]
        L.bingo_server_submit_walk.argtypes = [vp, u64, vp, u32, u64, u64, C.POINTER(u64)]
        L.bingo_server_submit_update.argtypes = [vp, u64, vp, vp, vp, u64, vp, vp, C.POINTER(u64)]
        L.bingo_server_wait.argtypes = [vp, u64, vp, u64, C.POINTER(_RequestInfo)]
        L.bingo_server_destroy.argtypes = [vp]
        L.bingo_probe_random_reads.argtypes = [vp, u64, u32, u32, u32, u32, u64, vp, C.POINTER(C.c_float), vp]
        L.bingo_probe_replay.argtypes = [vp, vp, u64, u32, u32, u32, u32, u64, vp, C.POINTER(C.c_float), vp]
        L.bingo_quantize_biases.argtypes = [u64, vp, C.c_double, u32, vp, vp]
        L.bingo_num_vertices.argtypes = [vp]
        L.bingo_num_vertices.restype = u32
        L.bingo_destroy.argtypes = [vp]
        L.bingo_destroy.restype = None
        L.bingo_strerror.argtypes = [C.c_int]
        L.bingo_strerror.restype = C.c_char_p
        _lib = L
        return L


def probe_random_reads(table, lanes, reads, dependent, line_bytes=64, seed=1, stream=None) -> dict:
    """Random-line read rate over a device tensor (measurement aid; see bingo_probe_random_reads)."""
    import torch
    sink = torch.empty(lanes, dtype=torch.int32, device=table.device)
    ms = C.c_float(0.0)
    rc = load().bingo_probe_random_reads(C.c_void_p(table.data_ptr()), table.numel() * table.element_size(), lanes,
                                         reads, int(bool(dependent)), line_bytes, seed, _ptr(sink), C.byref(ms),
                                         _stream(stream))
    _check(rc, "bingo_probe_random_reads")
    n = lanes * reads
    return {"ms": ms.value, "lines_per_s": n / (ms.value / 1e3), "GBps": n * line_bytes / (ms.value / 1e3) / 1e9,
            "lanes": lanes, "reads_per_lane": reads, "dependent": bool(dependent), "line_bytes": line_bytes}


def quantize_biases(bias, lam, frac_bits, out=None, stream=None):
    """Float32 device biases -> uint32 fixed-point weights floor(lam * b * 2^F) (bingo_quantize_biases);
    0 marks a bias that gives no weight in [1, 2^32)."""
    import torch
    if not isinstance(bias, torch.Tensor) or bias.dtype != torch.float32 or not bias.is_cuda:
        raise TypeError("bias must be a float32 device tensor")
    b = bias.contiguous()
    w = out if out is not None else torch.empty(b.numel(), dtype=torch.int32, device=b.device)
    _check(load().bingo_quantize_biases(b.numel(), _ptr(b), float(lam), frac_bits, _ptr(w), _stream(stream)),
           "bingo_quantize_biases")
    return w


def ppr_threshold(p: float) -> int:
    """Termination word threshold floor(p * 2^32)."""
    return int(p * 4294967296.0)


def _check(rc, where):
    if rc != 0:
        raise BingoError(rc, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def as_u32(x, device=None) -> torch.Tensor:
    """A contiguous int32 device tensor holding the low 32 bits of x (uint32 bit pattern)."""
    t = torch.as_tensor(x)
    if device is not None:
        t = t.to(device)
    if t.dtype != torch.int32:
        t = t.to(torch.int64) & 0xFFFFFFFF
        t = torch.where(t >= 2**31, t - 2**32, t).to(torch.int32)
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t is not None and t.numel() else None)


class Graph:
    """A dynamic graph with its radix-group sampling space resident in device memory."""

    def __init__(self, n, src, dst, w, adaptive=True, alpha=40, beta=10, pool_bytes=0, device="cuda", stream=None,
                 frac_bits=0, alias_table=False, radix_base=2):
        L = load()
        self.device = torch.device(device)
        s, d, ww = as_u32(src, self.device), as_u32(dst, self.device), as_u32(w, self.device)
        cfg = _Config(C.sizeof(_Config), int(bool(adaptive)), alpha, beta, pool_bytes, frac_bits, int(bool(alias_table)),
                      radix_base, 0)
        h = C.c_void_p()
        rc = L.bingo_build(C.byref(cfg), n, s.numel(), _ptr(s), _ptr(d), _ptr(ww), _stream(stream), C.byref(h))
        _check(rc, "bingo_build")
        self.h = h
        self.n = n
        self.adaptive = bool(adaptive)
        self.frac_bits = frac_bits
        self.alias_table = bool(alias_table)
        self.radix_base = radix_base

    def close(self):
        if getattr(self, "h", None):
            load().bingo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def walk(self, starts, length, seed, base=0, mode=MODE_PERSISTENT, stream=None, out=None):
        """DeepWalk paths (n_walks, length + 1) as int32 bit patterns of uint32; returns (paths, steps)."""
        st = as_u32(starts, self.device)
        nw = st.numel()
        paths = out if out is not None else torch.empty((nw, length + 1), dtype=torch.int32, device=self.device)
        steps = torch.zeros(1, dtype=torch.int64, device=self.device)
        rc = load().bingo_walk(self.h, nw, _ptr(st), base, length, seed, _ptr(paths), _ptr(steps), mode,
                               _stream(stream))
        _check(rc, "bingo_walk")
        return paths, steps

    def walk_noalloc(self, starts, length, seed, paths, steps, base=0, stream=None):
        """bingo_walk_noalloc into caller-owned paths (n_walks, length + 1) int32 and steps (1,) int64."""
        st = as_u32(starts, self.device)
        rc = load().bingo_walk_noalloc(self.h, st.numel(), _ptr(st), base, length, seed, _ptr(paths), _ptr(steps),
                                       _stream(stream))
        _check(rc, "bingo_walk_noalloc")
        return paths, steps

    def walk_batch(self, queries, stream=None):
        """Several DeepWalk queries in one launch; queries = [(starts, length, seed, base), ...].
        Returns [(paths, steps), ...] with the shapes and meaning of walk()."""
        qs = (_WalkQuery * max(len(queries), 1))()
        keep, out = [], []
        for i, (starts, length, seed, base) in enumerate(queries):
            st = as_u32(starts, self.device)
            paths = torch.empty((st.numel(), length + 1), dtype=torch.int32, device=self.device)
            steps = torch.zeros(1, dtype=torch.int64, device=self.device)
            qs[i] = _WalkQuery(st.numel(), _ptr(st).value, base, length, 0, seed, _ptr(paths).value,
                               steps.data_ptr())
            keep.append(st)
            out.append((paths, steps))
        _check(load().bingo_walk_batch(self.h, len(queries), qs, _stream(stream)), "bingo_walk_batch")
        return out

    def node2vec(self, starts, length, seed, p, q, base=0, stream=None, out=None):
        """Second-order node2vec paths (n_walks, length + 1) as int32 bit patterns of uint32; returns
        (paths, counts) with counts = int64 [transitions, proposals] on the device."""
        st = as_u32(starts, self.device)
        nw = st.numel()
        paths = out if out is not None else torch.empty((nw, length + 1), dtype=torch.int32, device=self.device)
        counts = torch.zeros(2, dtype=torch.int64, device=self.device)
        rc = load().bingo_node2vec(self.h, nw, _ptr(st), base, length, float(p), float(q), seed, _ptr(paths),
                                   _ptr(counts), _stream(stream))
        _check(rc, "bingo_node2vec")
        return paths, counts

    def ppr(self, sources, walks_per_source, thr, max_len, seed, base=0, mode=MODE_PERSISTENT, stream=None):
        """Per-source visit histograms: (offsets int64 [n_src+1], vertex int32, count int32, steps)."""
        src = as_u32(sources, self.device)
        L = load()
        ne, ns = C.c_uint64(0), C.c_uint64(0)
        rc = L.bingo_ppr(self.h, src.numel(), _ptr(src), walks_per_source, thr, max_len, seed, base, mode,
                         C.byref(ne), C.byref(ns), _stream(stream))
        _check(rc, "bingo_ppr")
        off = torch.empty(src.numel() + 1, dtype=torch.int64, device=self.device)
        vtx = torch.empty(max(ne.value, 1), dtype=torch.int32, device=self.device)
        cnt = torch.empty(max(ne.value, 1), dtype=torch.int32, device=self.device)
        rc = L.bingo_ppr_fetch(self.h, _ptr(off), _ptr(vtx), _ptr(cnt), vtx.numel(), _stream(stream))
        _check(rc, "bingo_ppr_fetch")
        return off, vtx[: ne.value], cnt[: ne.value], int(ns.value)

    def ppr_async(self, sources, walks_per_source, thr, max_len, seed, base=0, stream=None, hist_stream=None):
        """Walk phase of a persistent PPR query; its histogram is left running on hist_stream
        (see bingo_ppr_async).  Returns the transitions; ppr_result() collects the histograms.
        `sources` must stay alive until then."""
        src = as_u32(sources, self.device)
        self._async_src = src
        ns = C.c_uint64(0)
        rc = load().bingo_ppr_async(self.h, src.numel(), _ptr(src), walks_per_source, thr, max_len, seed, base,
                                    C.byref(ns), _stream(stream), _stream(hist_stream))
        _check(rc, "bingo_ppr_async")
        self._async_nsrc = src.numel()
        return int(ns.value)

    def ppr_wait(self):
        """(entries, histogram ms) of the last query, after waiting for its histogram."""
        ne, ms = C.c_uint64(0), C.c_float(0)
        _check(load().bingo_ppr_wait(self.h, C.byref(ne), C.byref(ms)), "bingo_ppr_wait")
        return int(ne.value), float(ms.value)

    def ppr_result(self, stream=None):
        """(offsets, vertex, count) of the last PPR query (waits for a pending histogram)."""
        ne, _ = self.ppr_wait()
        L = load()
        off = torch.empty(self._async_nsrc + 1, dtype=torch.int64, device=self.device)
        vtx = torch.empty(max(ne, 1), dtype=torch.int32, device=self.device)
        cnt = torch.empty(max(ne, 1), dtype=torch.int32, device=self.device)
        rc = L.bingo_ppr_fetch(self.h, _ptr(off), _ptr(vtx), _ptr(cnt), vtx.numel(), _stream(stream))
        _check(rc, "bingo_ppr_fetch")
        return off, vtx[:ne], cnt[:ne]

    def update(self, ins_src, ins_dst, ins_w, del_src, del_dst, stream=None):
        a, b, c = (as_u32(x, self.device) for x in (ins_src, ins_dst, ins_w))
        d, e = (as_u32(x, self.device) for x in (del_src, del_dst))
        stats = _UpdateStats()
        rc = load().bingo_update_batch(self.h, a.numel(), _ptr(a), _ptr(b), _ptr(c), d.numel(), _ptr(d), _ptr(e),
                                       _stream(stream), C.byref(stats))
        _check(rc, "bingo_update_batch")
        return {"inserted": stats.inserted, "deleted": stats.deleted, "not_found": stats.not_found,
                "touched_vertices": stats.touched_vertices, "match_scanned": stats.match_scanned,
                "match_candidates": stats.match_candidates,
                "transitions": np.array(list(stats.transitions), dtype=np.int64).reshape(5, 5)}

    def update_stream(self, op, src, dst, w, stream=None):
        """Records applied one at a time in order (op 0 insert, 1 delete; see bingo_update_stream)."""
        o, a, b, c = (as_u32(x, self.device) for x in (op, src, dst, w))
        stats = _UpdateStats()
        rc = load().bingo_update_stream(self.h, o.numel(), _ptr(o), _ptr(a), _ptr(b), _ptr(c), _stream(stream),
                                        C.byref(stats))
        _check(rc, "bingo_update_stream")
        return {"inserted": stats.inserted, "deleted": stats.deleted, "not_found": stats.not_found,
                "touched_vertices": stats.touched_vertices, "match_scanned": stats.match_scanned,
                "match_candidates": stats.match_candidates,
                "transitions": np.array(list(stats.transitions), dtype=np.int64).reshape(5, 5)}

    def export(self, u_begin=None, u_end=None, stream=None) -> np.ndarray:
        """Canonical dump as uint32 words (layout in include/bingo.h)."""
        L = load()
        n = C.c_uint64(0)
        ub = 0 if u_begin is None else u_begin
        ue = self.n if u_end is None else u_end
        rc = L.bingo_export_range(self.h, ub, ue, None, 0, C.byref(n), _stream(stream))
        _check(rc, "bingo_export")
        buf = np.zeros(max(n.value, 1), dtype=np.uint32)
        rc = L.bingo_export_range(self.h, ub, ue, C.c_void_p(buf.ctypes.data), buf.size, C.byref(n),
                                  _stream(stream))
        _check(rc, "bingo_export")
        return buf[: n.value]

    def export_index(self, u_begin=None, u_end=None, stream=None) -> np.ndarray:
        """Group index dump as uint32 words (layout in include/bingo.h, bingo_export_index_range)."""
        L = load()
        n = C.c_uint64(0)
        ub = 0 if u_begin is None else u_begin
        ue = self.n if u_end is None else u_end
        rc = L.bingo_export_index_range(self.h, ub, ue, None, 0, C.byref(n), _stream(stream))
        _check(rc, "bingo_export_index_range")
        buf = np.zeros(max(n.value, 1), dtype=np.uint32)
        rc = L.bingo_export_index_range(self.h, ub, ue, C.c_void_p(buf.ctypes.data), buf.size, C.byref(n),
                                        _stream(stream))
        _check(rc, "bingo_export_index_range")
        return buf[: n.value]

    def compact(self, pool_bytes=0, stream=None):
        """Move every live block into a fresh arena (0: of the current size), leaving replaced blocks behind."""
        _check(load().bingo_compact(self.h, int(pool_bytes), _stream(stream)), "bingo_compact")

    def probe_replay(self, visits, chain, lanes, extra_lines, dependent=True, seed=1, stream=None) -> dict:
        """Replay of a visit stream over this graph's headers and adjacency (measurement aid; see
        bingo_probe_replay): lines read, time and the 64-byte line rate."""
        v = as_u32(visits, self.device)
        ctr = torch.zeros(2, dtype=torch.int64, device=self.device)
        ms = C.c_float(0.0)
        rc = load().bingo_probe_replay(self.h, _ptr(v), v.numel(), chain, lanes, int(round(extra_lines * 256)),
                                       int(bool(dependent)), seed, _ptr(ctr), C.byref(ms), _stream(stream))
        _check(rc, "bingo_probe_replay")
        lines = int(ctr[0].item())
        return {"ms": ms.value, "lines": lines, "visits": v.numel(), "chain": chain, "lanes": lanes,
                "extra_lines_per_visit": extra_lines, "dependent": bool(dependent),
                "GBps": lines * 64 / (ms.value / 1e3) / 1e9}

    def check_locator(self, stream=None):
        """(inconsistencies, live slots) of the edge locator; None when no locator is in step."""
        bad, live = C.c_uint64(0), C.c_uint64(0)
        rc = load().bingo_check_locator(self.h, C.byref(bad), C.byref(live), _stream(stream))
        if rc == -1:  # BINGO_E_INVALID
            return None
        _check(rc, "bingo_check_locator")
        return int(bad.value), int(live.value)

    def memory(self, stream=None) -> dict:
        m = _MemStats()
        _check(load().bingo_memory(self.h, C.byref(m), _stream(stream)), "bingo_memory")
        out = {k: getattr(m, k) for k, _ in _MemStats._fields_ if k != "groups_by_type"}
        out["groups_by_type"] = list(m.groups_by_type)
        return out

    def last_phase_ms(self) -> list:
        """Device milliseconds per phase of the last walk / ppr / update call (HIP events on its stream)."""
        L = load()
        buf = (C.c_float * 8)()
        n = C.c_uint32(0)
        _check(L.bingo_last_phase_ms(self.h, buf, 8, C.byref(n)), "bingo_last_phase_ms")
        return [float(buf[i]) for i in range(n.value)]

    def set_tuning(self, walk_variant=None, blocks_per_cu=None, queue_chunk=None, update_graphs=None, dense_spec=None,
                   ppr_bins=None, update_split=None, wave_degree=None, update_locate=None):
        cur = self.get_tuning()
        t = _Tuning(C.sizeof(_Tuning), cur["walk_variant"] if walk_variant is None else walk_variant,
                    cur["blocks_per_cu"] if blocks_per_cu is None else blocks_per_cu,
                    cur["queue_chunk"] if queue_chunk is None else queue_chunk,
                    cur["update_graphs"] if update_graphs is None else update_graphs,
                    cur["dense_spec"] if dense_spec is None else dense_spec,
                    cur["ppr_bins"] if ppr_bins is None else ppr_bins,
                    cur["update_split"] if update_split is None else update_split,
                    cur["wave_degree"] if wave_degree is None else wave_degree,
                    cur["update_locate"] if update_locate is None else update_locate)
        _check(load().bingo_set_tuning(self.h, C.byref(t)), "bingo_set_tuning")

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(load().bingo_get_tuning(self.h, C.byref(t)), "bingo_get_tuning")
        return {"walk_variant": t.walk_variant, "blocks_per_cu": t.blocks_per_cu, "queue_chunk": t.queue_chunk,
                "update_graphs": t.update_graphs, "dense_spec": t.dense_spec, "ppr_bins": t.ppr_bins,
                "update_split": t.update_split, "wave_degree": t.wave_degree, "update_locate": t.update_locate}

    def status(self, stream=None) -> int:
        return load().bingo_status(self.h, _stream(stream))


def _host_u32(x):
    a = x.cpu().numpy() if isinstance(x, torch.Tensor) else np.asarray(x)
    return np.ascontiguousarray((a.astype(np.int64) & 0xFFFFFFFF).astype(np.uint32))


def _hptr(a):
    return C.c_void_p(a.ctypes.data if a.size else None)


class Server:
    """Request loop over a resident graph (see include/bingo.h): walk queries and update batches are
    admitted first-in first-out; queries run concurrently on up to max_inflight streams."""

    def __init__(self, graph: Graph, max_inflight=8, hbm_budget_bytes=0, max_batch=1):
        L = load()
        cfg = _ServerConfig(C.sizeof(_ServerConfig), max_inflight, hbm_budget_bytes, max_batch, 0)
        h = C.c_void_p()
        _check(L.bingo_server_create(graph.h, C.byref(cfg), C.byref(h)), "bingo_server_create")
        self.h = h
        self.graph = graph
        self._shapes = {}

    def submit_walk(self, starts, length, seed, base=0) -> int:
        st = _host_u32(starts)
        t = C.c_uint64(0)
        _check(load().bingo_server_submit_walk(self.h, st.size, _hptr(st), length, seed, base, C.byref(t)),
               "bingo_server_submit_walk")
        self._shapes[t.value] = (st.size, length + 1)
        return t.value

    def submit_update(self, ins_src, ins_dst, ins_w, del_src, del_dst) -> int:
        a, b, c, d, e = (_host_u32(x) for x in (ins_src, ins_dst, ins_w, del_src, del_dst))
        t = C.c_uint64(0)
        _check(load().bingo_server_submit_update(self.h, a.size, _hptr(a), _hptr(b), _hptr(c), d.size, _hptr(d),
                                                 _hptr(e), C.byref(t)), "bingo_server_submit_update")
        self._shapes[t.value] = None
        return t.value

    def wait(self, ticket):
        """Returns (paths as uint32 numpy (n_walks, length + 1) or None, info dict)."""
        shape = self._shapes.pop(ticket)
        info = _RequestInfo()
        out = np.zeros(shape, np.uint32) if shape else None
        rc = load().bingo_server_wait(self.h, ticket, C.c_void_p(out.ctypes.data) if out is not None and out.size
                                      else None, out.size if out is not None else 0, C.byref(info))
        _check(rc, "bingo_server_wait")
        return out, {k: getattr(info, k) for k, _ in _RequestInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().bingo_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""CPU oracle for radix-based bias factorization (Bingo, arXiv 2504.10233).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU product path never does.
It shares no code with the HIP library.

``bingo_oracle.c`` holds the arithmetic (see its header for the paper sections
each part follows); this module compiles it with gcc on first use and wraps it
with ctypes.  ``pyref`` holds a second, pure-Python implementation of the
random-number pieces, written independently, used to cross-check the C code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bingo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

T_EMPTY, T_ONE, T_DENSE, T_SPARSE, T_REGULAR = 0, 1, 2, 3, 4
TYPE_NAMES = ["empty", "one", "dense", "sparse", "regular"]
STOP = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile the oracle shared library (gcc, OpenMP over independent walks)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB_PATH)
            u32p, u64p, u8p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_uint8)
            L.o_philox.argtypes = [u32p, u32p, u32p]
            L.o_stream_words.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, u32p]
            L.o_below_bits_words.argtypes = [C.c_uint64, C.c_int, u64p, C.c_uint64, u64p]
            L.o_below_bits_words.restype = C.c_uint64
            L.o_below_bits_all_words.argtypes = [C.c_uint64, C.c_int, u64p]
            L.o_below_bits_all_words.restype = C.c_uint64
            L.o_below32.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
            L.o_below32.restype = C.c_uint32
            L.o_below64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint64]
            L.o_below64.restype = C.c_uint64
            L.o_type.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_uint32, C.c_uint32]
            L.o_type.restype = C.c_int
            L.o_pick_group.argtypes = [u32p, C.c_uint64]
            L.o_pick_group.restype = C.c_int
            L.o_two_phase.argtypes = [u32p, C.c_uint32, u8p]
            L.o_two_phase.restype = C.c_uint32
            L.o_build.argtypes = [C.c_uint32, C.c_uint64, u32p, u32p, u32p, C.c_int, C.c_uint32, C.c_uint32,
                                  C.c_uint32, C.c_int, C.POINTER(C.c_void_p)]
            L.o_alias_table.argtypes = [u64p, u64p, u32p]
            L.o_alias_pick.argtypes = [u64p, C.c_uint32, C.c_uint64]
            L.o_alias_pick.restype = C.c_int
            L.o_quantize.argtypes = [C.c_uint64, C.POINTER(C.c_float), C.c_double, C.c_uint32, u32p]
            L.o_build.restype = C.c_int
            L.o_free.argtypes = [C.c_void_p]
            L.o_step.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, C.c_uint32]
            L.o_step.restype = C.c_uint32
            L.o_deepwalk.argtypes = [C.c_void_p, C.c_uint64, u32p, C.c_uint64, C.c_uint32, C.c_uint64, u32p,
                                     C.c_int, u64p]
            L.o_deepwalk.restype = C.c_uint64
            L.o_node2vec_thresholds.argtypes = [C.c_double, C.c_double, u64p]
            L.o_node2vec_thresholds.restype = C.c_int
            L.o_node2vec_step.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32,
                                          u64p, u64p]
            L.o_node2vec_step.restype = C.c_uint32
            L.o_node2vec.argtypes = [C.c_void_p, C.c_uint64, u32p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_double,
                                     C.c_double, u32p, C.c_int, u64p]
            L.o_node2vec.restype = C.c_uint64
            L.o_ppr.argtypes = [C.c_void_p, C.c_uint32, u32p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                C.c_uint64, C.c_int]
            L.o_ppr.restype = C.c_void_p
            L.o_ppr_entries.argtypes = [C.c_void_p]
            L.o_ppr_entries.restype = C.c_uint64
            L.o_ppr_steps.argtypes = [C.c_void_p]
            L.o_ppr_steps.restype = C.c_uint64
            L.o_ppr_stats.argtypes = [C.c_void_p, u64p]
            L.o_ppr_fetch.argtypes = [C.c_void_p, u64p, u32p, u32p]
            L.o_ppr_free.argtypes = [C.c_void_p]
            L.o_update.argtypes = [C.c_void_p, C.c_uint64, u32p, u32p, u32p, C.c_uint64, u32p, u32p, u64p]
            L.o_update.restype = C.c_int
            L.o_dump.argtypes = [C.c_void_p, u32p]
            L.o_dump.restype = C.c_uint64
            L.o_dump_range.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, u32p]
            L.o_dump_range.restype = C.c_uint64
            L.o_index_dump_range.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, u32p]
            L.o_index_dump_range.restype = C.c_uint64
            L.o_memory.argtypes = [C.c_void_p, u64p]
            L.o4_build.argtypes = [C.c_uint32, C.c_uint64, u32p, u32p, u32p, C.c_int, C.c_uint32, C.c_uint32,
                                   C.POINTER(C.c_void_p)]
            L.o4_build.restype = C.c_int
            L.o4_free.argtypes = [C.c_void_p]
            L.o4_pick_subgroup.argtypes = [u32p, C.c_uint64]
            L.o4_pick_subgroup.restype = C.c_int
            L.o4_step.argtypes = [C.c_void_p, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32]
            L.o4_step.restype = C.c_uint32
            L.o4_deepwalk.argtypes = [C.c_void_p, C.c_uint64, u32p, C.c_uint64, C.c_uint32, C.c_uint64, u32p,
                                      C.c_int]
            L.o4_deepwalk.restype = C.c_uint64
            L.o4_dump.argtypes = [C.c_void_p, u32p]
            L.o4_dump.restype = C.c_uint64
            _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def philox(ctr, key):
    """Philox-4x32-10 of one counter block (SC'11)."""
    c = _u32(ctr); k = _u32(key); out = np.zeros(4, np.uint32)
    lib().o_philox(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return [int(x) for x in out]


def stream_words(seed, walk, step, nwords):
    out = np.zeros(nwords, np.uint32)
    lib().o_stream_words(seed, walk, step, nwords, _p(out, C.c_uint32))
    return out


def below_words(n, width, words):
    """Lemire draw on [0, n) from supplied ``width``-bit words -> (value, consumed or None)."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    used = C.c_uint64(0)
    v = lib().o_below_bits_words(n, width, _p(w, C.c_uint64), len(w), C.byref(used))
    return int(v), (None if used.value == 2**64 - 1 else int(used.value))


def below_all_words(n, width):
    """Draw once from every single ``width``-bit word -> (accepted counts per value, rejected)."""
    counts = np.zeros(n, np.uint64)
    rej = lib().o_below_bits_all_words(n, width, _p(counts, C.c_uint64))
    return counts, int(rej)


def below32(seed, walk, step, n):
    return int(lib().o_below32(seed, walk, step, n))


def below64(seed, walk, step, n):
    return int(lib().o_below64(seed, walk, step, n))


def type_of(c, d, adaptive=True, alpha=40, beta=10):
    return int(lib().o_type(c, d, int(adaptive), alpha, beta))


def pick_group(counts, r):
    c = np.zeros(32, np.uint32)
    c[: len(counts)] = counts
    return int(lib().o_pick_group(_p(c, C.c_uint32), r))


def two_phase(arr, delete_flags):
    a = _u32(arr).copy()
    d = np.ascontiguousarray(np.asarray(delete_flags, dtype=np.uint8))
    n = lib().o_two_phase(_p(a, C.c_uint32), len(a), _p(d, C.c_uint8))
    return a[:n]


class OracleError(RuntimeError):
    pass



def node2vec_thresholds(p, q):
    """Acceptance thresholds (distance 0, 1, 2) of the node2vec rejection step; 2^32 = always."""
    thr = np.zeros(3, np.uint64)
    if lib().o_node2vec_thresholds(p, q, _p(thr, C.c_uint64)):
        raise ValueError("p and q must be positive")
    return thr

def alias_table(totals):
    """Inter-group alias table (Sec. 4.1) of 32 group totals -> (cut[32], alias[32])."""
    T = np.zeros(32, np.uint64)
    T[: len(totals)] = np.asarray(totals, dtype=np.uint64)
    cut = np.zeros(32, np.uint64)
    al = np.zeros(32, np.uint32)
    lib().o_alias_table(_p(T, C.c_uint64), _p(cut, C.c_uint64), _p(al, C.c_uint32))
    return cut, al


def alias_pick(totals, slot, x):
    T = np.zeros(32, np.uint64)
    T[: len(totals)] = np.asarray(totals, dtype=np.uint64)
    return int(lib().o_alias_pick(_p(T, C.c_uint64), slot, x))


def quantize(bias, lam, frac_bits):
    """Floating-point biases (Sec. 4.3) as stored weights: floor(lam * b * 2^F) for float32 b, the
    product in IEEE double; 0 for a bias that does not give a weight in [1, 2^32)."""
    b = np.ascontiguousarray(np.asarray(bias, dtype=np.float32))
    out = np.zeros(len(b), np.uint32)
    lib().o_quantize(len(b), _p(b, C.c_float), float(lam), frac_bits, _p(out, C.c_uint32))
    return out


class Graph:
    """The oracle's dynamic graph with its radix-group sampling structures.  frac_bits = F > 0
    reads every weight as a fixed-point bias with F fraction bits (Sec. 4.3)."""

    def __init__(self, n, src, dst, w, adaptive=True, alpha=40, beta=10, frac_bits=0, alias=False):
        L = lib()
        self._src = _u32(src); self._dst = _u32(dst); self._w = _u32(w)
        h = C.c_void_p()
        rc = L.o_build(n, len(self._src), _p(self._src, C.c_uint32), _p(self._dst, C.c_uint32),
                       _p(self._w, C.c_uint32), int(adaptive), alpha, beta, frac_bits, int(alias), C.byref(h))
        if rc != 0:
            raise OracleError("o_build failed: %d" % rc)
        self.h = h
        self.n = n
        self.adaptive = adaptive
        self.frac_bits = frac_bits
        self.alias = bool(alias)
        del self._src, self._dst, self._w

    def close(self):
        if self.h:
            lib().o_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, u, seed, walk, step, ppr=False, thr=0):
        return int(lib().o_step(self.h, u, seed, walk, step, int(ppr), thr))

    def deepwalk(self, starts, length, seed, base=0, threads=1, with_stats=False):
        s = _u32(starts)
        paths = np.zeros((len(s), length + 1), np.uint32)
        st = np.zeros(8, np.uint64)
        steps = lib().o_deepwalk(self.h, len(s), _p(s, C.c_uint32), base, length, seed,
                                 _p(paths, C.c_uint32), threads, _p(st, C.c_uint64))
        if with_stats:
            return paths, int(steps), st[:6].copy()
        return paths, int(steps)

    def node2vec(self, starts, length, seed, p, q, base=0, threads=1, with_proposals=False):
        """Second-order walks (Sec. 2.2, Eq. node2vec) by rejection on the first-order sampler."""
        s = _u32(starts)
        paths = np.zeros((len(s), length + 1), np.uint32)
        props = np.zeros(1, np.uint64)
        steps = lib().o_node2vec(self.h, len(s), _p(s, C.c_uint32), base, length, seed, p, q,
                                 _p(paths, C.c_uint32), threads, _p(props, C.c_uint64))
        if with_proposals:
            return paths, int(steps), int(props[0])
        return paths, int(steps)

    def node2vec_step(self, prev, u, seed, walk_id, step, p, q):
        """One second-order transition from u after prev (prev = 0xFFFFFFFF: first step)."""
        thr = node2vec_thresholds(p, q)
        return int(lib().o_node2vec_step(self.h, prev, u, seed, walk_id, step, _p(thr, C.c_uint64), None))

    def ppr(self, sources, walks_per_source, thr, cap, seed, base=0, threads=1, with_stats=False):
        s = _u32(sources)
        L = lib()
        P = L.o_ppr(self.h, len(s), _p(s, C.c_uint32), walks_per_source, thr, cap, seed, base, threads)
        try:
            ne = L.o_ppr_entries(P)
            off = np.zeros(len(s) + 1, np.uint64)
            vtx = np.zeros(max(ne, 1), np.uint32)
            cnt = np.zeros(max(ne, 1), np.uint32)
            L.o_ppr_fetch(P, _p(off, C.c_uint64), _p(vtx, C.c_uint32), _p(cnt, C.c_uint32))
            steps = int(L.o_ppr_steps(P))
            st = np.zeros(6, np.uint64)
            L.o_ppr_stats(P, _p(st, C.c_uint64))
        finally:
            L.o_ppr_free(P)
        res = (off, vtx[:ne], cnt[:ne], steps)
        return res + (st,) if with_stats else res

    def update(self, ins_src, ins_dst, ins_w, del_src, del_dst):
        a, b, c = _u32(ins_src), _u32(ins_dst), _u32(ins_w)
        d, e = _u32(del_src), _u32(del_dst)
        st = np.zeros(28, np.uint64)
        rc = lib().o_update(self.h, len(a), _p(a, C.c_uint32), _p(b, C.c_uint32), _p(c, C.c_uint32),
                            len(d), _p(d, C.c_uint32), _p(e, C.c_uint32), _p(st, C.c_uint64))
        if rc != 0:
            raise OracleError("o_update failed: %d" % rc)
        return {"inserted": int(st[0]), "deleted": int(st[1]), "not_found": int(st[2]),
                "transitions": st[3:].reshape(5, 5).astype(np.int64)}

    def update_stream(self, op, src, dst, w):
        """Streaming updates (Sec. 4.2): every record is its own batch, in order; statistics summed."""
        op, src, dst, w = _u32(op), _u32(src), _u32(dst), _u32(w)
        tot = {"inserted": 0, "deleted": 0, "not_found": 0, "transitions": np.zeros((5, 5), np.int64)}
        for i in range(len(op)):
            if op[i] == 0:
                s = self.update([src[i]], [dst[i]], [w[i]], [], [])
            else:
                s = self.update([], [], [], [src[i]], [dst[i]])
            for k in ("inserted", "deleted", "not_found"):
                tot[k] += s[k]
            tot["transitions"] += s["transitions"]
        return tot

    def dump(self, u_begin=None, u_end=None):
        L = lib()
        if u_begin is None and u_end is None:
            nw = L.o_dump(self.h, None)
            out = np.zeros(max(nw, 1), np.uint32)
            L.o_dump(self.h, _p(out, C.c_uint32))
            return out[:nw]
        ub = 0 if u_begin is None else u_begin
        ue = self.n if u_end is None else u_end
        nw = L.o_dump_range(self.h, ub, ue, None)
        out = np.zeros(max(nw, 1), np.uint32)
        L.o_dump_range(self.h, ub, ue, _p(out, C.c_uint32))
        return out[:nw]

    def index_dump(self, u_begin=None, u_end=None):
        """Group indexes: per vertex |S|, S, then per listed group k, the inverted index at the
        members (regular) or over S (sparse); see o_index_dump_range."""
        L = lib()
        ub = 0 if u_begin is None else u_begin
        ue = self.n if u_end is None else u_end
        nw = L.o_index_dump_range(self.h, ub, ue, None)
        out = np.zeros(max(nw, 1), np.uint32)
        L.o_index_dump_range(self.h, ub, ue, _p(out, C.c_uint32))
        return out[:nw]

    def memory(self):
        out = np.zeros(9, np.uint64)
        lib().o_memory(self.h, _p(out, C.c_uint64))
        keys = ["adjacency", "one", "dense", "sparse", "regular", "reserved", "sparse_reduced_lists",
                "all_regular_groups", "naive_bound"]
        return {k: int(v) for k, v in zip(keys, out)}


def parse_dump(words, n):
    """Parse a canonical dump into per-vertex dicts (for tests and goldens)."""
    words = np.asarray(words, dtype=np.uint32)
    out = []
    o = 0
    for _ in range(n):
        d, nseq, mask = int(words[o]), int(words[o + 1]), int(words[o + 2])
        o += 3
        e = words[o:o + 3 * d].reshape(d, 3)
        o += 3 * d
        groups = {}
        for k in range(32):
            if not (mask >> k) & 1:
                continue
            kk, t, c = int(words[o]), int(words[o + 1]), int(words[o + 2])
            assert kk == k, (kk, k)
            o += 3
            if t == T_ONE:
                members = [int(words[o])]
                o += 1
            elif t in (T_SPARSE, T_REGULAR):
                members = [int(x) for x in words[o:o + c]]
                o += c
            else:
                members = None
            groups[k] = (t, c, members)
        out.append({"d": d, "next_seq": nseq, "mask": mask, "dst": e[:, 0].copy(), "w": e[:, 1].copy(),
                    "seq": e[:, 2].copy(), "groups": groups})
    assert o == len(words), (o, len(words))
    return out


# ---- radix base 4 (Supplement S.2): 48 subgroups s = 3k + v - 1 of the edges whose base-4 digit k is v
def pick_subgroup(c48, r):
    """The subgroup an ascending inverse-transform scan over c_s * v * 4^k selects for r."""
    c = _u32(c48)
    assert c.size == 48
    return lib().o4_pick_subgroup(_p(c, C.c_uint32), int(r))


class Graph4:
    """The oracle's static radix-base-4 structure (build and walks)."""

    def __init__(self, n, src, dst, w, adaptive=True, alpha=40, beta=10):
        s_, d_, w_ = _u32(src), _u32(dst), _u32(w)
        h = C.c_void_p()
        rc = lib().o4_build(n, len(s_), _p(s_, C.c_uint32), _p(d_, C.c_uint32), _p(w_, C.c_uint32), int(adaptive),
                            alpha, beta, C.byref(h))
        if rc != 0:
            raise OracleError("o4_build failed: %d" % rc)
        self.h, self.n = h, n

    def close(self):
        if self.h:
            lib().o4_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, u, seed, walk, step):
        return int(lib().o4_step(self.h, u, seed, walk, step))

    def deepwalk(self, starts, length, seed, base=0, threads=1):
        st = _u32(starts)
        paths = np.zeros((st.size, length + 1), np.uint32)
        total = lib().o4_deepwalk(self.h, st.size, _p(st, C.c_uint32), base, length, seed, _p(paths, C.c_uint32),
                                  threads)
        return paths, int(total)

    def dump(self):
        L = lib()
        nw = L.o4_dump(self.h, None)
        out = np.zeros(max(nw, 1), np.uint32)
        L.o4_dump(self.h, _p(out, C.c_uint32))
        return out[:nw]


def parse_dump4(words, n):
    """Parse a base-4 canonical dump into per-vertex dicts."""
    words = np.asarray(words, dtype=np.uint32)
    out, o = [], 0
    for _ in range(n):
        d = int(words[o]); mask = int(words[o + 1]) | (int(words[o + 2]) << 32)
        o += 3
        e = words[o:o + 2 * d].reshape(d, 2)
        o += 2 * d
        subs = {}
        for s in range(48):
            if not (mask >> s) & 1:
                continue
            ss, t, c = int(words[o]), int(words[o + 1]), int(words[o + 2])
            assert ss == s
            o += 3
            if t == T_ONE:
                members = [int(words[o])]
                o += 1
            elif t in (T_SPARSE, T_REGULAR):
                members = [int(x) for x in words[o:o + c]]
                o += c
            else:
                members = None
            subs[s] = (t, c, members)
        out.append({"d": d, "mask": mask, "dst": e[:, 0].copy(), "w": e[:, 1].copy(), "subgroups": subs})
    assert o == len(words)
    return out

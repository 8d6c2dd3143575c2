"""Graph, weight, query and update-stream generators (see package docstring)."""
from __future__ import annotations

import math

import torch

__all__ = [
    "hash_u64", "uniform_u32", "below", "uniform_f64", "er_graph", "rmat_graph", "permute_ids",
    "weights_uniform", "weights_zipf", "weights_lognormal", "planted_hubs", "EdgeMirror",
    "config_c1", "SEEDS",
]

_I64 = torch.int64


def _s64(c: int) -> int:
    """A 64-bit constant as the signed int64 with the same bits."""
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


_GOLD = _s64(0x9E3779B97F4A7C15)
_MIX1 = _s64(0xBF58476D1CE4E5B9)
_MIX2 = _s64(0x94D049BB133111EB)


def _lsr(z: torch.Tensor, s: int) -> torch.Tensor:
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _MIX1
    z = (z ^ _lsr(z, 27)) * _MIX2
    return z ^ _lsr(z, 31)


def _key(seed: int, stream: int) -> int:
    z = torch.tensor([_s64(seed * 0x100000001B3 + stream * 0x9E3779B1 + 0x632BE59BD9B4E019)], dtype=_I64)
    return int(_mix(_mix(z + _GOLD))[0])


def hash_u64(seed: int, stream: int, n: int, device="cpu", start: int = 0) -> torch.Tensor:
    """n pseudo-random 64-bit words (as int64 bit patterns) for indices start..start+n-1."""
    i = torch.arange(start, start + n, dtype=_I64, device=device)
    return _mix(i * _GOLD + _key(seed, stream))


def uniform_u32(seed, stream, n, device="cpu", start=0) -> torch.Tensor:
    return _lsr(hash_u64(seed, stream, n, device, start), 32)


def below(seed, stream, n, bound, device="cpu", start=0) -> torch.Tensor:
    """Integers in [0, bound) by a 32x32 multiply-shift (inputs only; tiny bias is irrelevant here)."""
    if isinstance(bound, torch.Tensor):
        return _lsr(uniform_u32(seed, stream, n, device, start) * bound, 32)
    assert 0 < bound <= 1 << 32
    return _lsr(uniform_u32(seed, stream, n, device, start) * int(bound), 32)


def uniform_f64(seed, stream, n, device="cpu", start=0) -> torch.Tensor:
    """Doubles in (0, 1] from the top 53 bits."""
    h = _lsr(hash_u64(seed, stream, n, device, start), 11)
    return (h.to(torch.float64) + 1.0) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------
def er_graph(n: int, m: int, seed: int, device="cpu"):
    """Directed Erdos-Renyi multigraph: src uniform, dst uniform over the other n-1 vertices."""
    src = below(seed, 1, m, n, device)
    off = below(seed, 2, m, n - 1, device)
    dst = (src + 1 + off) % n
    return src, dst


def permute_ids(x: torch.Tensor, scale: int, seed: int) -> torch.Tensor:
    """A seeded bijection on [0, 2^scale): rounds of odd multiply, xor-shift and add."""
    mask = (1 << scale) - 1
    y = x.clone()
    for r in range(4):
        k = _key(seed, 100 + r)
        mul = (k | 1) & mask
        add = (k >> 20) & mask
        y = (y * mul) & mask
        y = y ^ (y >> max(1, scale // 2))
        y = (y + add) & mask
    return y


def rmat_graph(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19, device="cpu", permute=True,
               chunk: int = 1 << 26):
    """R-MAT (recursive quadrant choice per level, no noise); ids permuted by a seeded bijection.
    Self-loops and duplicate edges are kept."""
    ta = int(a * 2**32)
    tb = int((a + b) * 2**32)
    tc = int((a + b + c) * 2**32)
    srcs, dsts = [], []
    for s0 in range(0, m, chunk):
        cnt = min(chunk, m - s0)
        src = torch.zeros(cnt, dtype=_I64, device=device)
        dst = torch.zeros(cnt, dtype=_I64, device=device)
        for lev in range(scale):
            u = uniform_u32(seed, 10 + lev, cnt, device, start=s0)
            bit = 1 << (scale - 1 - lev)
            down = u >= tb                      # quadrants c, d: src bit set
            right = ((u >= ta) & (u < tb)) | (u >= tc)   # quadrants b, d: dst bit set
            src |= down.to(_I64) * bit
            dst |= right.to(_I64) * bit
            del u, down, right
        if permute:
            src = permute_ids(src, scale, seed)
            dst = permute_ids(dst, scale, seed)
        srcs.append(src.to(torch.int32))
        dsts.append(dst.to(torch.int32))
    return torch.cat(srcs).to(_I64), torch.cat(dsts).to(_I64)


# ---------------------------------------------------------------------------
# weights (uint32 values >= 1, returned as int64)
# ---------------------------------------------------------------------------
def weights_uniform(n, lo, hi, seed, device="cpu", stream=3):
    return lo + below(seed, stream, n, hi - lo, device)


def weights_zipf(n, s, clip_hi, seed, device="cpu", stream=4):
    """Zipf(s) on {1, 2, ...} by Devroye's rejection method (Non-Uniform Random Variate Generation,
    1986, X.6), clipped to [1, clip_hi]."""
    out = torch.zeros(n, dtype=_I64, device=device)
    todo = torch.arange(n, dtype=_I64, device=device)
    am1 = s - 1.0
    bconst = 2.0 ** am1
    it = 0
    while todo.numel():
        u = uniform_f64(seed, stream * 1000 + 2 * it, n, device)[todo]
        v = uniform_f64(seed, stream * 1000 + 2 * it + 1, n, device)[todo]
        x = torch.floor(u.pow(-1.0 / am1))
        x = torch.clamp(x, max=float(2**62))
        t = (1.0 + 1.0 / x).pow(am1)
        ok = v * x * (t - 1.0) / (bconst - 1.0) <= t / bconst
        sel = todo[ok]
        out[sel] = torch.clamp(x[ok], max=float(clip_hi)).to(_I64)
        todo = todo[~ok]
        it += 1
    return torch.clamp(out, min=1)


def weights_lognormal(n, mu, sigma, seed, device="cpu", stream=5, hi=2**32 - 1):
    """round(exp(mu + sigma z)) with z standard normal (Box-Muller), clipped to [1, hi]."""
    u1 = uniform_f64(seed, stream * 1000, n, device)
    u2 = uniform_f64(seed, stream * 1000 + 1, n, device)
    z = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
    w = torch.round(torch.exp(mu + sigma * z))
    return torch.clamp(w, min=1.0, max=float(hi)).to(_I64)


def planted_hubs(n, n_hubs, lo_exp, hi_exp, seed, device="cpu"):
    """n_hubs distinct hub ids and, per hub, floor(10^U(lo_exp, hi_exp)) extra edges to uniform dst."""
    ids = torch.unique(below(seed, 20, 4 * n_hubs, n, device))
    ids = ids[torch.argsort(_lsr(hash_u64(seed, 21, ids.numel(), device), 1))][:n_hubs]
    e = lo_exp + (hi_exp - lo_exp) * uniform_f64(seed, 22, n_hubs, device)
    deg = torch.floor(torch.pow(10.0, e)).to(_I64)
    src = torch.repeat_interleave(ids, deg)
    dst = below(seed, 23, src.numel(), n, device)
    return ids, src, dst


# ---------------------------------------------------------------------------
# update streams
# ---------------------------------------------------------------------------
class EdgeMirror:
    """The generator's own copy of the current edge multiset (src, dst), used only to pick deletions
    of existing edges.  A deletion names (src, dst); which instance the library removes is the
    library's rule, and the multiset of (src, dst) pairs is the same either way."""

    def __init__(self, src: torch.Tensor, dst: torch.Tensor):
        self.src = src.clone()
        self.dst = dst.clone()

    @property
    def m(self):
        return self.src.numel()

    def pick_deletions(self, k, seed, stream, device=None, hub_ids=None, hub_frac=0.0):
        """k distinct existing instances; with hub_ids, a fraction hub_frac comes from hub sources."""
        dev = self.src.device
        if hub_ids is not None and hub_frac > 0:
            is_hub = torch.isin(self.src, hub_ids.to(dev))
            hub_pos = torch.nonzero(is_hub).flatten()
            oth_pos = torch.nonzero(~is_hub).flatten()
            kh = int(round(k * hub_frac))
            a = self._distinct(hub_pos, kh, seed, stream)
            b = self._distinct(oth_pos, k - kh, seed, stream + 1)
            pos = torch.cat([a, b])
            pos = pos[torch.argsort(_lsr(hash_u64(seed, stream + 2, pos.numel(), dev), 1))]
        else:
            pos = self._distinct(torch.arange(self.m, device=dev), k, seed, stream)
        return pos

    @staticmethod
    def _distinct(pool, k, seed, stream):
        dev = pool.device
        if k >= pool.numel():
            return pool.clone()
        got = torch.empty(0, dtype=_I64, device=dev)
        it = 0
        while got.numel() < k:
            need = 2 * (k - got.numel()) + 16
            cand = below(seed, stream * 97 + it, need, pool.numel(), dev)
            got = torch.unique(torch.cat([got, cand]))
            it += 1
        order = torch.argsort(_lsr(hash_u64(seed, stream * 97 + 1000, got.numel(), dev), 1))
        return pool[got[order][:k]]

    def apply(self, ins_src, ins_dst, del_pos):
        keep = torch.ones(self.m, dtype=torch.bool, device=self.src.device)
        keep[del_pos] = False
        self.src = torch.cat([self.src[keep], ins_src])
        self.dst = torch.cat([self.dst[keep], ins_dst])


SEEDS = {"graph": 1000, "weights": 2000, "walks": 3000, "batch": 4000, "serving": 5005}


def config_c1(device="cpu"):
    """Tiny plain-method case: ER(1000, 10000), w ~ U[1, 2^16), 1000 walks of length 80 from uniform
    starts, one batch of 500 inserts (same edge law) and 500 deletes of existing instances, then
    1000 more walks with ids 1000..1999."""
    n, m = 1000, 10000
    src, dst = er_graph(n, m, SEEDS["graph"] + 1, device)
    w = weights_uniform(m, 1, 1 << 16, SEEDS["weights"] + 1, device)
    starts = below(SEEDS["walks"] + 1, 1, 1000, n, device)
    starts2 = below(SEEDS["walks"] + 1, 2, 1000, n, device)
    bseed = SEEDS["batch"] + 100 + 0
    isrc, idst = er_graph(n, 500, bseed, device)
    iw = weights_uniform(500, 1, 1 << 16, bseed, device, stream=7)
    mir = EdgeMirror(src, dst)
    pos = mir.pick_deletions(500, bseed, 30)
    return {
        "n": n, "src": src, "dst": dst, "w": w, "starts": starts, "starts2": starts2,
        "ins_src": isrc, "ins_dst": idst, "ins_w": iw,
        "del_src": mir.src[pos], "del_dst": mir.dst[pos],
        "length": 80, "seed": 0x5EED0001,
    }

// walk.hip -- random walks on the radix-group sampling space (Sec. 4.1
// hierarchical sampling; Sec. 5.1 dense-group rejection), DeepWalk (Sec. 2.2)
// and personalized PageRank by visit counts (Sec. 1, Sec. 6.1).
//
// One walk per lane.  The persistent form keeps a fixed grid resident; a lane
// whose walk ends takes the next walk id from a device queue (one atomic per
// wave per refill), so uneven walk lengths do not idle the wave.  The per-step
// form launches once per step over the walks still active (the step-by-step
// execution of the paper's Sec. 6).
#include "dev.h"
#include "step.h"
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <mutex>

namespace {

constexpr int TB = 256;
// PPR visits are vertex ids in per-walk segments (the source is implied by the
// segment); a walk stopped early by a vertex without out-edges pads the rest of
// its segment with VPAD, which sorts after every vertex id.
constexpr uint32_t VPAD = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Attempt-interleaved stepping.  A step is split into "begin" (header, group
// choice; one-element and listed groups finish here) and "attempt" (one dense
// rejection try).  In every loop iteration a lane either begins a step and
// makes its first attempt, or makes one more attempt, so the lanes of a wave do
// not wait for the lane with the longest rejection run.
// ---------------------------------------------------------------------------
struct StepState {
    RandStream rs;
    uint64_t adj;
    uint32_t d, sel, tries;
    bool pending;
    bool wave;  // a dense group of a vertex of degree >= the wave threshold: the wave serves it
};

template <int MODE>
__device__ __forceinline__ uint32_t step_begin(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                               uint32_t u, StepState& ss, GroupRule rule, uint32_t wave_deg = 0) {
    GroupPick g;
    if (!pick_group<MODE>(hdr, u, ss.rs, rule, g)) return STOP_VERTEX;
    if (MODE == 1 && g.sel < 0)
        return decimal_pick(hdr + (size_t)u * HDR_WORDS, pool, g.adj, g.d, g.slot0, g.onem, rule, ss.rs);
    if (g.sel < 0) return STOP_VERTEX;  // only on an inconsistent header
    if ((g.onem >> g.sel) & 1u) return g.raw;  // one-element group: the step ends in the header
    const uint32_t t = group_type(g.csel, g.d, rule);
    if (t == GT_DENSE) {
        ss.adj = g.adj; ss.d = g.d; ss.sel = (uint32_t)g.sel; ss.tries = 0; ss.pending = true;
        ss.wave = wave_deg != 0 && g.d >= wave_deg;
        return PENDING;
    }
    const uint32_t info = hdr[(size_t)u * HDR_WORDS + H_INFO + g.sel];
    const uint32_t i = pool[(uint64_t)info * LIST_UNIT_WORDS + rs_below32(ss.rs, g.csel)];
    return pool[g.adj + 2ull * i];
}

template <int SPEC>
__device__ __forceinline__ uint32_t step_attempt(const uint32_t* __restrict__ pool, StepState& ss) {
    const uint32_t v = dense_round<SPEC>(reinterpret_cast<const uint64_t*>(pool + ss.adj), ss.d, ss.sel, ss.rs);
    if (v != PENDING) { ss.pending = false; return v; }
    // bounded only against a corrupted structure (acceptance is above alpha % per try)
    ss.tries += SPEC;
    if (ss.tries >= (1u << 16)) { ss.pending = false; return STOP_VERTEX; }
    return PENDING;
}

// ---------------------------------------------------------------------------
// Wave-per-vertex dense rejection.  The lanes whose step selected a dense group
// of a vertex with at least the wave threshold's degree are served one at a time
// by the whole wave: in a round, lane j < WK takes word j of the served walk's
// stream from where it stands (its own Philox block; the words are those the
// walk itself would draw next), makes it a draw on [0, d) with Lemire's
// rejection, and the draws that are not rejected are the attempts in stream
// order (rank by ballot).  Every attempting lane loads its slot's edge word;
// the first accepting attempt (ballot, lowest lane) is exactly the slot the
// walk's own attempt loop would accept, so results do not depend on the mode.
// Every lane of the wave must call this.
// ---------------------------------------------------------------------------
constexpr int WAVE_ROUND = 8;
constexpr uint32_t DENSE_MAX_ATTEMPTS = 1u << 16;

__device__ __forceinline__ uint32_t wave_dense_serve(const uint32_t* __restrict__ pool, const StepState& ss,
                                                     bool want) {
    uint64_t m = __ballot(want);
    if (!m) return PENDING;
    const uint32_t lane = lane_id();
    uint32_t mine = PENDING;
    while (m) {
        const int ld = __ffsll((long long)m) - 1;
        m &= m - 1;
        const uint64_t adj = ((uint64_t)__shfl((uint32_t)(ss.adj >> 32), ld, 64) << 32) |
                             __shfl((uint32_t)ss.adj, ld, 64);
        const uint32_t d = __shfl(ss.d, ld, 64), sel = __shfl(ss.sel, ld, 64);
        const uint32_t k0 = __shfl(ss.rs.k0, ld, 64), k1 = __shfl(ss.rs.k1, ld, 64);
        const uint32_t w0 = __shfl(ss.rs.w0, ld, 64), w1 = __shfl(ss.rs.w1, ld, 64);
        const uint32_t stp = __shfl(ss.rs.step, ld, 64);
        // position of the next word of the served stream
        uint64_t pos = (uint64_t)__shfl(ss.rs.blk, ld, 64) * 4u - __shfl(ss.rs.left, ld, 64);
        const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + adj);
        const uint32_t zone = (0u - d) % d;
        uint32_t tries = 0, found = PENDING;
        while (found == PENDING) {
            bool valid = false;
            uint32_t i = 0;
            if (lane < (uint32_t)WAVE_ROUND) {
                const uint64_t q = pos + lane;
                uint32_t o[4];
                philox_block(w0, w1, stp, (uint32_t)(q >> 2), k0, k1, o[0], o[1], o[2], o[3]);
                const uint32_t c = (uint32_t)(q & 3u);
                const uint32_t x = c == 0 ? o[0] : c == 1 ? o[1] : c == 2 ? o[2] : o[3];
                const uint64_t mm = (uint64_t)x * d;
                valid = (uint32_t)mm >= zone;
                i = (uint32_t)(mm >> 32);
            }
            const uint64_t vm = __ballot(valid);
            const uint32_t att = tries + (uint32_t)__popcll(vm & lanemask_lt());
            uint64_t e = 0;
            bool acc = false;
            if (valid && att < DENSE_MAX_ATTEMPTS) {
                e = edges[i];
                acc = (e >> (32 + sel)) & 1ull;
            }
            const uint64_t am = __ballot(acc);
            if (am) {
                found = __shfl((uint32_t)e, __ffsll((long long)am) - 1, 64);
            } else {
                tries += (uint32_t)__popcll(vm);
                pos += WAVE_ROUND;
                if (tries >= DENSE_MAX_ATTEMPTS) found = STOP_VERTEX;
            }
        }
        if ((int)lane == ld) mine = found;
    }
    return mine;
}

// ------------------------------------------------------------------ DeepWalk
template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_deepwalk_persistent(const uint32_t* __restrict__ hdr,
                                                            const uint32_t* __restrict__ pool, uint32_t n,
                                                            uint64_t nw, const uint32_t* __restrict__ starts,
                                                            uint64_t base, uint32_t L, uint64_t seed,
                                                            uint32_t* __restrict__ paths, GroupRule rule,
                                                            unsigned long long* __restrict__ ctl,
                                                            uint32_t* __restrict__ err, uint32_t qchunk) {
    // ctl[0] = queue head, ctl[1] = transitions taken
    WaveQueue wq;
    wq.chunk = qchunk;
    uint64_t j = NO_WALK;
    uint32_t u = 0, s = 0;
    uint64_t steps = 0;
    uint32_t* row = nullptr;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                row = paths + j * (uint64_t)(L + 1);
                u = starts[j];
                s = 0;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    row[0] = u;
                    for (uint32_t x = 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                } else {
                    row[0] = u;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        if (j != NO_WALK) {
            if (s < L) {
                RandStream rs;
                rs_init(rs, seed, base + j, s);
                const uint32_t v = walk_step_body<SPEC, MODE>(hdr, pool, u, rs, rule);
                if (v == STOP_VERTEX) {
                    for (uint32_t x = s + 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                } else {
                    row[s + 1] = v;
                    u = v;
                    ++s;
                    ++steps;
                }
            }
            if (j != NO_WALK && s == L) j = NO_WALK;
        }
    }
    wave_add_u64(ctl + 1, steps);
}

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_deepwalk_interleaved(const uint32_t* __restrict__ hdr,
                                                             const uint32_t* __restrict__ pool, uint32_t n,
                                                             uint64_t nw, const uint32_t* __restrict__ starts,
                                                             uint64_t base, uint32_t L, uint64_t seed,
                                                             uint32_t* __restrict__ paths, GroupRule rule,
                                                             unsigned long long* __restrict__ ctl,
                                                             uint32_t* __restrict__ err, uint32_t qchunk,
                                                             uint32_t wave_deg) {
    WaveQueue wq;
    wq.chunk = qchunk;
    StepState ss;
    ss.pending = false;
    ss.wave = false;
    uint64_t j = NO_WALK, steps = 0;
    uint32_t u = 0, s = 0;
    uint32_t* row = nullptr;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                row = paths + j * (uint64_t)(L + 1);
                u = starts[j];
                s = 0;
                ss.pending = false;
                row[0] = u;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    for (uint32_t x = 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                } else if (L == 0) {
                    j = NO_WALK;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        uint32_t v = PENDING;
        if (j != NO_WALK && !ss.pending) {
            rs_init(ss.rs, seed, base + j, s);
            v = step_begin<MODE>(hdr, pool, u, ss, rule, wave_deg);
        }
        if (j != NO_WALK && ss.pending && !ss.wave) v = step_attempt<SPEC>(pool, ss);
        {
            const bool served = j != NO_WALK && ss.pending && ss.wave;
            const uint32_t wv = wave_dense_serve(pool, ss, served);
            if (served) { v = wv; ss.pending = false; }
        }
        if (j != NO_WALK && v != PENDING) {
            if (v == STOP_VERTEX) {
                for (uint32_t x = s + 1; x <= L; ++x) row[x] = STOP_VERTEX;
                j = NO_WALK;
            } else {
                row[s + 1] = v;
                u = v;
                ++s;
                ++steps;
                if (s == L) j = NO_WALK;
            }
        }
    }
    wave_add_u64(ctl + 1, steps);
}

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_deepwalk_step(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                      uint32_t n, uint64_t nw, const uint32_t* __restrict__ starts,
                                                      uint64_t base, uint32_t L, uint32_t s, uint64_t seed,
                                                      uint32_t* __restrict__ paths, GroupRule rule,
                                                      unsigned long long* __restrict__ ctl,
                                                      uint32_t* __restrict__ err) {
    uint64_t steps = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nw; j += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t* row = paths + j * (uint64_t)(L + 1);
        uint32_t u;
        if (s == 0) {
            u = starts[j];
            row[0] = u;
            if (u >= n) { atomicOr(err, ERR_RANGE); u = STOP_VERTEX; }
        } else {
            u = row[s];
        }
        uint32_t v = STOP_VERTEX;
        if (u != STOP_VERTEX) {
            RandStream rs;
            rs_init(rs, seed, base + j, s);
            v = walk_step_body<SPEC, MODE>(hdr, pool, u, rs, rule);
            steps += (v != STOP_VERTEX);
        }
        row[s + 1] = v;
    }
    wave_add_u64(ctl + 1, steps);
}

// ------------------------------------------------------------------ batched DeepWalk queries
// Several queries in one persistent launch (continuous batching in the serving
// loop).  Their walks form one index space, query i holding [first_i, first_i +
// n_i); a lane that takes walk index g finds its query as the last i with
// first_i <= g (an empty query never is: the next one starts at the same index)
// and walks exactly as the single-query kernel does, with that query's seed,
// id base, length and output rows.  Steps taken are added per query: one atomic
// per query among the walks a wave finishes in an iteration.  The table travels
// in the kernel arguments.
struct WalkQueryDev {
    const uint32_t* starts;
    uint32_t* paths;
    unsigned long long* steps;  // may be null
    uint64_t first, base, seed;
    uint32_t L, pad;
};
struct WalkQueryTable {
    WalkQueryDev q[WALK_BATCH_MAX];
};

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_deepwalk_batch(const uint32_t* __restrict__ hdr,
                                                       const uint32_t* __restrict__ pool, uint32_t n,
                                                       const WalkQueryTable tab, uint32_t nq, uint64_t nw,
                                                       GroupRule rule, unsigned long long* __restrict__ ctl,
                                                       uint32_t* __restrict__ err, uint32_t qchunk) {
    const uint32_t lane = lane_id();
    WaveQueue wq;
    wq.chunk = qchunk;
    uint64_t j = NO_WALK, seed = 0, id = 0;
    uint32_t qi = 0, u = 0, s = 0, L = 0;
    uint32_t* row = nullptr;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        bool fin = false;  // a walk ended in this iteration
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                uint32_t lo = 0, hi = nq - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (tab.q[mid].first <= got) lo = mid; else hi = mid - 1;
                }
                qi = lo;
                j = got - tab.q[qi].first;
                L = tab.q[qi].L;
                seed = tab.q[qi].seed;
                id = tab.q[qi].base + j;
                row = tab.q[qi].paths + j * (uint64_t)(L + 1);
                u = tab.q[qi].starts[j];
                s = 0;
                row[0] = u;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    for (uint32_t x = 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                    fin = true;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        if (j != NO_WALK) {
            if (s < L) {
                RandStream rs;
                rs_init(rs, seed, id, s);
                const uint32_t v = walk_step_body<SPEC, MODE>(hdr, pool, u, rs, rule);
                if (v == STOP_VERTEX) {
                    for (uint32_t x = s + 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                    fin = true;
                } else {
                    row[s + 1] = v;
                    u = v;
                    ++s;
                }
            }
            if (j != NO_WALK && s == L) {
                j = NO_WALK;
                fin = true;
            }
        }
        for (uint64_t m = __ballot(fin); m;) {
            const int leader = __ffsll((long long)m) - 1;
            const uint32_t qq = __shfl(qi, leader, 64);
            const uint64_t same = __ballot(fin && qi == qq) & m;
            uint64_t add = ((same >> lane) & 1ull) ? s : 0u;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) add += __shfl_xor(add, o, 64);
            if ((int)lane == leader && tab.q[qq].steps) atomicAdd(tab.q[qq].steps, (unsigned long long)add);
            m &= ~same;
        }
    }
}

__global__ void k_batch_zero(const WalkQueryTable tab, uint32_t nq) {
    const uint32_t i = threadIdx.x;
    if (i < nq && tab.q[i].steps) *tab.q[i].steps = 0ull;
}

// ------------------------------------------------------------------ PPR
// The termination word of step s is the first word of the stream (seed, id, s)
// and depends on nothing else, so a cheap pass finds each walk's last possible
// step B_j (the first s with word < thr, or the cap).  The walk then writes at
// most 1 + B_j visits into its own pre-scanned segment: no atomics on the
// visit path, and the steps s < B_j skip the comparison (their word is known
// to be >= thr).  A walk stopped early by a vertex without out-edges pads the
// rest of its segment with a key that sorts after every real key.
// Termination words come from one Philox block per (walk, step), and walk
// lengths are geometric, so a lane that owned one walk would idle until the
// longest walk of its wave ends (about 4x the mean for 64 lanes at p = 0.15).
// Instead a wave owns BOUND_CHUNK consecutive walks and a lane whose walk ends
// takes the wave's next one, so the wave stays busy until its chunk is drained.
constexpr uint32_t BOUND_CHUNK = 1024;

__global__ void __launch_bounds__(TB) k_ppr_bound(uint64_t nw, uint64_t base, uint64_t seed, uint32_t thr,
                                                  uint32_t cap, uint32_t* __restrict__ len) {
    const uint32_t lane = lane_id();
    const uint64_t nchunks = (nw + BOUND_CHUNK - 1) / BOUND_CHUNK;
    const uint64_t wave0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t c = wave0; c < nchunks; c += nwaves) {
        const uint64_t c0 = c * BOUND_CHUNK;
        const uint64_t c1 = std::min<uint64_t>(c0 + BOUND_CHUNK, nw);
        uint64_t next = c0 + 64;  // identical in every lane
        uint64_t j = c0 + lane;
        uint32_t s = 0;
        while (__ballot(j < c1)) {
            bool fin = false;
            if (j < c1) {
                uint32_t w0, w1, w2, w3;
                const uint64_t id = base + j;
                philox_block((uint32_t)id, (uint32_t)(id >> 32), s, 0, (uint32_t)seed, (uint32_t)(seed >> 32), w0,
                             w1, w2, w3);
                if (w0 < thr || s + 1 >= cap) {
                    // B_j = s when the word stops the walk at s, else the cap
                    len[j] = (w0 < thr ? s : cap) + 1;
                    fin = true;
                } else {
                    ++s;
                }
            }
            const uint64_t b = __ballot(fin);
            if (fin) {
                j = next + __popcll(b & lanemask_lt());
                s = 0;
            }
            next += __popcll(b);
        }
    }
}

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_ppr_persistent(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                       uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                       uint32_t R, uint64_t seed, uint64_t base, GroupRule rule,
                                                       const uint64_t* __restrict__ seg,
                                                       const uint32_t* __restrict__ len,
                                                       unsigned long long* __restrict__ ctl,
                                                       uint32_t* __restrict__ vis, uint32_t* __restrict__ err, uint32_t qchunk) {
    // ctl[0] queue head, ctl[1] transitions
    const uint64_t nw = (uint64_t)nsrc * R;
    WaveQueue wq;
    wq.chunk = qchunk;
    uint64_t j = NO_WALK, pos = 0, lim = 0, steps = 0;
    uint32_t u = 0, s = 0;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                u = sources[j / R];
                s = 0;
                pos = seg[j];
                lim = pos + len[j];
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    for (uint64_t x = pos; x < lim; ++x) vis[x] = VPAD;
                    j = NO_WALK;
                } else {
                    vis[pos++] = u;
                    if (pos == lim) j = NO_WALK;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        if (j != NO_WALK) {
            RandStream rs;
            rs_init(rs, seed, base + j, s);
            rs_next32(rs);  // the termination word, known to be >= thr here
            const uint32_t v = walk_step_body<SPEC, MODE>(hdr, pool, u, rs, rule);
            if (v == STOP_VERTEX) {
                for (uint64_t x = pos; x < lim; ++x) vis[x] = VPAD;
                j = NO_WALK;
            } else {
                vis[pos++] = v;
                u = v;
                ++s;
                ++steps;
                if (pos == lim) j = NO_WALK;
            }
        }
    }
    wave_add_u64(ctl + 1, steps);
}

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_ppr_interleaved(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                        uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                        uint32_t R, uint64_t seed, uint64_t base, GroupRule rule,
                                                        const uint64_t* __restrict__ seg,
                                                        const uint32_t* __restrict__ len,
                                                        unsigned long long* __restrict__ ctl,
                                                        uint32_t* __restrict__ vis, uint32_t* __restrict__ err, uint32_t qchunk,
                                                        uint32_t wave_deg) {
    const uint64_t nw = (uint64_t)nsrc * R;
    WaveQueue wq;
    wq.chunk = qchunk;
    StepState ss;
    ss.pending = false;
    ss.wave = false;
    uint64_t j = NO_WALK, pos = 0, lim = 0, steps = 0;
    uint32_t u = 0, s = 0;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                u = sources[j / R];
                s = 0;
                pos = seg[j];
                lim = pos + len[j];
                ss.pending = false;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    for (uint64_t x = pos; x < lim; ++x) vis[x] = VPAD;
                    j = NO_WALK;
                } else {
                    vis[pos++] = u;
                    if (pos == lim) j = NO_WALK;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        uint32_t v = PENDING;
        if (j != NO_WALK && !ss.pending) {
            rs_init(ss.rs, seed, base + j, s);
            rs_next32(ss.rs);  // the termination word, known to be >= thr here
            v = step_begin<MODE>(hdr, pool, u, ss, rule, wave_deg);
        }
        if (j != NO_WALK && ss.pending && !ss.wave) v = step_attempt<SPEC>(pool, ss);
        {
            const bool served = j != NO_WALK && ss.pending && ss.wave;
            const uint32_t wv = wave_dense_serve(pool, ss, served);
            if (served) { v = wv; ss.pending = false; }
        }
        if (j != NO_WALK && v != PENDING) {
            if (v == STOP_VERTEX) {
                for (uint64_t x = pos; x < lim; ++x) vis[x] = VPAD;
                j = NO_WALK;
            } else {
                vis[pos++] = v;
                u = v;
                ++s;
                ++steps;
                if (pos == lim) j = NO_WALK;
            }
        }
    }
    wave_add_u64(ctl + 1, steps);
}

// Binned PPR: the visits of source q go to bin q (capacity C, fill count
// cnt[q]) in any order, since only their multiset matters.  The termination
// word is tested in the walk itself (no length pass), and in every iteration
// the lanes of a wave that produced a visit append it to their source's bin
// with one atomic per source present in the wave; lanes of a wave hold
// consecutive walk ids, so the appends of an iteration land as one or two
// contiguous runs instead of one partial-sector store per lane.  A bin that
// would overflow sets a flag and the query is rerun with exact per-walk
// segments.  ctl[0] queue head, ctl[1] transitions, ctl[2] overflow.
template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_ppr_binned(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                   uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                   uint32_t R, uint64_t seed, uint64_t base, uint32_t thr,
                                                   uint32_t cap, GroupRule rule, uint64_t C,
                                                   uint32_t* __restrict__ cnt, uint32_t* __restrict__ vis,
                                                   unsigned long long* __restrict__ ctl, uint32_t* __restrict__ err,
                                                   uint32_t qchunk, uint32_t wave_deg) {
    const uint64_t nw = (uint64_t)nsrc * R;
    const uint32_t lane = lane_id();
    WaveQueue wq;
    wq.chunk = qchunk;
    StepState ss;
    ss.pending = false;
    ss.wave = false;
    uint64_t j = NO_WALK, steps = 0;
    uint32_t u = 0, s = 0, q = 0;
    bool done = false, ovf = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take_chunked(need, wq, ctl);
        bool emit = false;
        uint32_t ev = 0;
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                q = (uint32_t)(j / R);
                u = sources[q];
                s = 0;
                ss.pending = false;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    j = NO_WALK;
                } else {
                    emit = true;  // the start counts as a visit; the walk steps from the next iteration
                    ev = u;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        uint32_t v = PENDING;
        if (j != NO_WALK && !emit) {
            if (!ss.pending) {
                // before every transition: the cap, then the termination word
                if (s >= cap) {
                    j = NO_WALK;
                } else {
                    rs_init(ss.rs, seed, base + j, s);
                    if (rs_next32(ss.rs) < thr) j = NO_WALK;
                    else v = step_begin<MODE>(hdr, pool, u, ss, rule, wave_deg);
                }
            }
            if (j != NO_WALK && ss.pending && !ss.wave) v = step_attempt<SPEC>(pool, ss);
        }
        {
            const bool served = j != NO_WALK && !emit && ss.pending && ss.wave;
            const uint32_t wv = wave_dense_serve(pool, ss, served);
            if (served) { v = wv; ss.pending = false; }
        }
        if (j != NO_WALK && !emit) {
            if (v != PENDING) {
                if (v == STOP_VERTEX) {
                    j = NO_WALK;
                } else {
                    emit = true;
                    ev = v;
                    u = v;
                    ++s;
                    ++steps;
                }
            }
        }
        // append this iteration's visits: one atomic per source present in the wave
        uint64_t m = __ballot(emit);
        while (m) {
            const int leader = __ffsll((long long)m) - 1;
            const uint32_t qq = __shfl(q, leader, 64);
            const uint64_t same = __ballot(emit && q == qq) & m;
            uint32_t b = 0;
            if ((int)lane == leader) b = atomicAdd(cnt + qq, (uint32_t)__popcll(same));
            b = __shfl(b, leader, 64);
            if ((same >> lane) & 1ull) {
                const uint64_t pos = (uint64_t)b + __popcll(same & lanemask_lt());
                if (pos < C) vis[(uint64_t)qq * C + pos] = ev;
                else ovf = true;
            }
            m &= ~same;
        }
    }
    wave_add_u64(ctl + 1, steps);
    if (__ballot(ovf) && lane == 0) atomicOr(ctl + 2, 1ull);
}

// Per-step PPR: active walks are (walk id, current vertex) pairs compacted into
// the next list after every step; visits go to the same per-walk segments.
__global__ void __launch_bounds__(TB) k_ppr_start(uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                  uint32_t R,
                                                  const uint64_t* __restrict__ seg, const uint32_t* __restrict__ len,
                                                  uint64_t* __restrict__ act_id, uint32_t* __restrict__ act_v,
                                                  unsigned long long* __restrict__ ctl, uint32_t* __restrict__ vis,
                                                  uint32_t* __restrict__ err) {
    // ctl[3] = size of active list A
    const uint64_t nw = (uint64_t)nsrc * R;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nw; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t q = j / R;
        const uint32_t u = sources[q];
        const uint64_t p = seg[j];
        if (u >= n) {
            atomicOr(err, ERR_RANGE);
            for (uint64_t x = p; x < p + len[j]; ++x) vis[x] = VPAD;
            act_id[j] = NO_WALK;
        } else {
            vis[p] = u;
            act_id[j] = len[j] > 1 ? j : NO_WALK;
        }
        act_v[j] = u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[3] = nw;
}

template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_ppr_step(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                 uint32_t R, uint32_t s, uint64_t seed, uint64_t base,
                                                 GroupRule rule, const uint64_t* __restrict__ seg,
                                                 const uint32_t* __restrict__ len, const uint64_t* __restrict__ in_id,
                                                 const uint32_t* __restrict__ in_v, uint64_t* __restrict__ out_id,
                                                 uint32_t* __restrict__ out_v, unsigned long long* __restrict__ ctl,
                                                 int in_slot, uint32_t* __restrict__ vis) {
    const uint64_t cnt = ctl[3 + in_slot];
    const uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t iters = (cnt + stride - 1) / stride;
    uint64_t steps = 0;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t a = j0 + it * stride;
        bool alive = false;
        uint64_t id = NO_WALK;
        uint32_t v = STOP_VERTEX;
        if (a < cnt) {
            id = in_id[a];
            if (id != NO_WALK) {
                // the walk is active at step s, so s < len - 1 and its termination word is >= thr
                RandStream rs;
                rs_init(rs, seed, base + id, s);
                rs_next32(rs);
                v = walk_step_body<SPEC, MODE>(hdr, pool, in_v[a], rs, rule);
                const uint64_t p0 = seg[id], l = len[id];
                if (v == STOP_VERTEX) {
                    for (uint64_t x = p0 + 1 + s; x < p0 + l; ++x) vis[x] = VPAD;
                } else {
                    vis[p0 + 1 + s] = v;
                    ++steps;
                    alive = (uint64_t)s + 2 < l;
                }
            }
        }
        // compact the walks that continue into the other list
        const uint64_t m = __ballot(alive);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long b = 0;
            if ((int)lane_id() == leader) b = atomicAdd(ctl + 3 + (in_slot ^ 1), (unsigned long long)__popcll(m));
            b = __shfl(b, leader, 64);
            if (alive) {
                const uint64_t pos = b + __popcll(m & lanemask_lt());
                out_id[pos] = id;
                out_v[pos] = v;
            }
        }
    }
    wave_add_u64(ctl + 1, steps);
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

// ------------------------------------------------------------------ histogram
__global__ void k_heads(const uint64_t* __restrict__ keys, uint64_t N, uint32_t* __restrict__ head) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x)
        head[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1u : 0u;
}

__global__ void k_emit(const uint64_t* __restrict__ keys, uint64_t N, const uint32_t* __restrict__ head,
                       const uint64_t* __restrict__ idx, int vbits, uint32_t* __restrict__ vtx,
                       uint64_t* __restrict__ hpos, uint64_t* __restrict__ off) {
    const uint64_t vmask = (1ull << vbits) - 1;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x) {
        if (!head[p]) continue;
        const uint64_t id = idx[p];
        const uint64_t k = keys[p];
        vtx[id] = (uint32_t)(k & vmask);
        hpos[id] = p;
        const uint64_t q = k >> vbits;
        if (p == 0 || (keys[p - 1] >> vbits) != q) off[q] = id;
    }
}

__global__ void k_counts(const uint64_t* __restrict__ hpos, uint64_t U, uint64_t N, uint32_t* __restrict__ cnt,
                         uint64_t* __restrict__ off, uint32_t nsrc) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < U; i += (uint64_t)gridDim.x * blockDim.x)
        cnt[i] = (uint32_t)((i + 1 < U ? hpos[i + 1] : N) - hpos[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) off[nsrc] = U;
}

// ------------------------------------------------------------------ per-source histogram
// The visits of source q are the contiguous key range [seg[q R], seg[(q+1) R]).
// One block of HSB threads per source sorts that range (bitonic network over
// N = HSB * E slots, the vertex id only: the source is implied by the block),
// run-length encodes it and writes the vertices back over the start of the same
// range and their counts to the same positions of a count array; a compaction
// then builds the CSR.  Thread t holds slots
// [t E, t E + E) in registers: partners closer than E slots are exchanged in
// registers, partners in the same wave by lane shuffles, and only the stages
// that cross waves go through LDS (6 of the 91 stages at N = 8192), so the
// block synchronizes a handful of times instead of once per stage.  E is chosen
// per query from the longest range; ranges above HCAP take the global sort.
constexpr int HSB = 512;
constexpr uint32_t HCAP = 16384;
static_assert(HSB * 32 == HCAP, "the widest histogram instantiation covers HCAP");

// x of lane (lane ^ D).  Distances 1, 2, 4 and 8 stay inside a row of 16 lanes
// and are DPP moves on the vector ALU: quad permutations give ^1, ^2 and ^3, the
// half-row mirror ^7 and the row mirror ^15, and ^4 = ^3 then ^7, ^8 = ^7 then
// ^15.  Longer distances go through the LDS crossbar.  Every lane of the wave
// must be active.
template <uint32_t D>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x) {
    constexpr int QP_X1 = 0xB1, QP_X2 = 0x4E, QP_X3 = 0x1B, ROW_MIRROR = 0x140, ROW_HALF_MIRROR = 0x141;
    if constexpr (D == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, QP_X1, 0xF, 0xF, false);
    } else if constexpr (D == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, QP_X2, 0xF, 0xF, false);
    } else if constexpr (D == 4) {
        const int y = __builtin_amdgcn_update_dpp(0, (int)x, QP_X3, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, y, ROW_HALF_MIRROR, 0xF, 0xF, false);
    } else if constexpr (D == 8) {
        const int y = __builtin_amdgcn_update_dpp(0, (int)x, ROW_HALF_MIRROR, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, y, ROW_MIRROR, 0xF, 0xF, false);
    } else {
        return __shfl_xor(x, (int)D, 64);
    }
}

__device__ __forceinline__ void cmp_keep(uint32_t& a, uint32_t b, bool takemin) {
    a = takemin ? min(a, b) : max(a, b);
}

// One stage (KK, J) of the bitonic network over N = HSB * E slots held E per
// thread: slot i is ordered against slot i ^ J, ascending where i & KK == 0.
template <int E, uint32_t KK, uint32_t J>
__device__ __forceinline__ void bitonic_stage(uint32_t (&x)[E], uint32_t t, uint32_t lane, uint32_t* buf) {
    if constexpr (J < (uint32_t)E) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = e ^ (int)J;
            if (p > e) {
                const bool up = ((t * E + e) & KK) == 0;
                const uint32_t a = x[e], b = x[p];
                x[e] = up ? min(a, b) : max(a, b);
                x[p] = up ? max(a, b) : min(a, b);
            }
        }
    } else if constexpr (J < 64u * E) {
        constexpr uint32_t D = J / E;  // partner lane distance
        const bool lower = (lane & D) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t y = lane_xor<D>(x[e]);
            const bool up = ((t * E + e) & KK) == 0;
            cmp_keep(x[e], y, lower == up);
        }
    } else {
        constexpr uint32_t DT = J / E;  // partner thread distance, across waves
        __syncthreads();  // earlier readers of buf are done
#pragma unroll
        for (int e = 0; e < E; ++e) buf[t * E + e] = x[e];
        __syncthreads();
        const uint32_t pt = t ^ DT;
        const bool lower = (t & DT) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool up = ((t * E + e) & KK) == 0;
            cmp_keep(x[e], buf[pt * E + e], lower == up);
        }
    }
}

// Stages (KK, J), (KK, J / 2), ..., (KK, 1), then (2 KK, KK), ... up to KK = N.
template <int E, uint32_t N, uint32_t KK, uint32_t J>
__device__ __forceinline__ void bitonic_from(uint32_t (&x)[E], uint32_t t, uint32_t lane, uint32_t* buf) {
    bitonic_stage<E, KK, J>(x, t, lane, buf);
    if constexpr (J > 1) bitonic_from<E, N, KK, J / 2>(x, t, lane, buf);
    else if constexpr (KK < N) bitonic_from<E, N, 2 * KK, KK>(x, t, lane, buf);
}

template <int E>
__global__ void __launch_bounds__(HSB) k_hist_seg(uint32_t* __restrict__ vis, uint32_t* __restrict__ hcnt,
                                                  const uint64_t* __restrict__ seg, uint32_t R, uint32_t nsrc,
                                                  uint64_t total, uint64_t C, const uint32_t* __restrict__ bin_cnt,
                                                  uint32_t* __restrict__ ucount,
                                                  unsigned long long* __restrict__ too_big) {
    constexpr uint32_t N = HSB * E;
    constexpr int NW = HSB / 64;
    __shared__ uint32_t buf[N];
    __shared__ uint32_t wred[2][NW];
    const uint32_t q = blockIdx.x, t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    // the source's range: its bin, or the segments of its R walks
    const uint64_t S0 = C ? (uint64_t)q * C : seg[(uint64_t)q * R];
    const uint64_t S1 = C ? S0 + bin_cnt[q] : ((q + 1 < nsrc) ? seg[(uint64_t)(q + 1) * R] : total);
    if (S1 - S0 > N) {
        if (t == 0) { ucount[q] = 0; atomicOr(too_big, 1ull); }
        return;
    }
    const uint32_t L = (uint32_t)(S1 - S0);
    uint32_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = t * E + e;
        x[e] = i < L ? vis[S0 + i] : VPAD;
    }
    bitonic_from<E, N, 2, 1>(x, t, lane, buf);
    // run heads: slot i is a head if it holds a vertex different from slot i - 1
    uint32_t prev = __shfl_up(x[E - 1], 1, 64);
    __syncthreads();  // the last cross-wave stage has read buf
    if (lane == 63) wred[0][wave] = x[E - 1];
    __syncthreads();
    if (lane == 0) prev = wave ? wred[0][wave - 1] : VPAD;
    uint32_t hmask = 0, nh = 0, nvalid = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t pv = e ? x[e - 1] : prev;
        const bool valid = x[e] != VPAD;
        const bool head = valid && (t * E + e == 0 || x[e] != pv);
        hmask |= (uint32_t)head << e;
        nh += head;
        nvalid += valid;
    }
    // block-wide exclusive scan of head counts; total heads and valid slots
    uint32_t inc = nh, vs = nvalid;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc += y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) vs += __shfl_xor(vs, o, 64);
    __syncthreads();  // wred[0] reads above are done
    if (lane == 63) wred[0][wave] = inc;
    if (lane == 0) wred[1][wave] = vs;
    __syncthreads();
    uint32_t before = 0, U = 0, V = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < (int)wave) before += wred[0][w];
        U += wred[0][w];
        V += wred[1][w];
    }
    // head positions by rank, then each head's count is the gap to the next head
    uint32_t r = before + inc - nh;
#pragma unroll
    for (int e = 0; e < E; ++e)
        if ((hmask >> e) & 1u) buf[r++] = t * E + e;
    __syncthreads();
    r = before + inc - nh;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if ((hmask >> e) & 1u) {
            const uint32_t next = r + 1 < U ? buf[r + 1] : V;
            vis[S0 + r] = x[e];
            hcnt[S0 + r] = next - (t * E + e);
            ++r;
        }
    }
    if (t == 0) ucount[q] = U;
}

__global__ void __launch_bounds__(256) k_hist_compact(const uint32_t* __restrict__ vis,
                                                      const uint32_t* __restrict__ hcnt,
                                                      const uint64_t* __restrict__ seg, uint32_t R, uint64_t C,
                                                      const uint32_t* __restrict__ ucount,
                                                      const uint64_t* __restrict__ off, uint32_t* __restrict__ vtx,
                                                      uint32_t* __restrict__ cnt) {
    const uint32_t q = blockIdx.x;
    const uint64_t S0 = C ? (uint64_t)q * C : seg[(uint64_t)q * R], o = off[q];
    const uint32_t U = ucount[q];
    for (uint32_t k = threadIdx.x; k < U; k += 256) {
        vtx[o + k] = vis[S0 + k];
        cnt[o + k] = hcnt[S0 + k];
    }
}

// Global path: (source, vertex) keys from the visit segments; padding becomes
// `pad`, above every key.  The source of position p is the last q whose first
// walk's segment starts at or before p.
__global__ void k_vis_keys(const uint32_t* __restrict__ vis, const uint64_t* __restrict__ seg, uint32_t R,
                           uint32_t nsrc, uint64_t total, int vbits, uint64_t pad, uint64_t* __restrict__ keys) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = vis[p];
        uint32_t lo = 0, hi = nsrc - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (seg[(uint64_t)mid * R] <= p) lo = mid; else hi = mid - 1;
        }
        keys[p] = v == VPAD ? pad : (((uint64_t)lo << vbits) | v);
    }
}

__global__ void k_set_last_off(uint64_t* off, uint32_t nsrc, const unsigned long long* total) { off[nsrc] = *total; }

// Largest bin fill, reduced per block then one atomic per block.
__global__ void __launch_bounds__(256) k_bin_max(const uint32_t* __restrict__ cnt, uint32_t nsrc,
                                                 unsigned long long* __restrict__ out) {
    __shared__ unsigned long long m[4];
    unsigned long long best = 0;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nsrc; q += (uint64_t)gridDim.x * blockDim.x)
        best = std::max<unsigned long long>(best, cnt[q]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = std::max<unsigned long long>(best, __shfl_xor(best, o));
    if (lane_id() == 0) m[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) best = std::max<unsigned long long>(best, m[w]);
        atomicMax(out, best);
    }
}

// Largest per-source key range (visits plus padding), reduced per block then one atomic per block.
__global__ void __launch_bounds__(256) k_seg_maxlen(const uint64_t* __restrict__ seg, uint32_t R, uint32_t nsrc,
                                                    const unsigned long long* __restrict__ total,
                                                    unsigned long long* __restrict__ out) {
    __shared__ unsigned long long m[4];
    unsigned long long best = 0;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nsrc; q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t S0 = seg[q * R];
        const uint64_t S1 = (q + 1 < nsrc) ? seg[(q + 1) * R] : *total;
        best = std::max<unsigned long long>(best, S1 - S0);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = std::max<unsigned long long>(best, __shfl_xor(best, o));
    if (lane_id() == 0) m[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) best = std::max<unsigned long long>(best, m[w]);
        atomicMax(out, best);
    }
}

inline uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n + TB - 1) / TB, 1), 1u << 20);
}

int resident_grid(const void* kernel, uint32_t blocks_per_cu) {
    static int cus = 0;
    static const void* seen[32] = {};
    static int occ[32] = {};
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    int per_cu = 0;
    for (int i = 0; i < 32; ++i)
        if (seen[i] == kernel) per_cu = occ[i];
    if (!per_cu) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, TB, 0) != hipSuccess || per_cu <= 0)
            per_cu = 4;
        for (int i = 0; i < 32; ++i)
            if (!seen[i]) { seen[i] = kernel; occ[i] = per_cu; break; }
    }
    if (blocks_per_cu && (int)blocks_per_cu < per_cu) per_cu = (int)blocks_per_cu;
    return cus * per_cu;
}

int bits_for(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

template <int SPEC, int MODE>
void deepwalk_kernels(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, uint64_t seed,
                      uint32_t* paths, uint32_t mode, unsigned long long* ctl, hipStream_t st) {
    if (mode == BINGO_WALK_PER_STEP) {
        const uint32_t grid = grid_for(nw);
        if (L == 0) {
            // only the start entries
            hipLaunchKernelGGL((k_deepwalk_persistent<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts,
                               base, L, seed, paths, g->rule, ctl, g->d_err, g->queue_chunk);
        }
        for (uint32_t s = 0; s < L; ++s)
            hipLaunchKernelGGL((k_deepwalk_step<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts, base,
                               L, s, seed, paths, g->rule, ctl, g->d_err);
    } else {
        const void* kern = g->walk_variant ? (const void*)k_deepwalk_interleaved<SPEC, MODE> : (const void*)k_deepwalk_persistent<SPEC, MODE>;
        const int rg = resident_grid(kern, g->blocks_per_cu);
        const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)rg, (nw + TB - 1) / TB);
        if (g->walk_variant)
            hipLaunchKernelGGL((k_deepwalk_interleaved<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts,
                               base, L, seed, paths, g->rule, ctl, g->d_err, g->queue_chunk, g->wave_degree);
        else
            hipLaunchKernelGGL((k_deepwalk_persistent<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts,
                               base, L, seed, paths, g->rule, ctl, g->d_err, g->queue_chunk);
    }
}

template <int SPEC, int MODE>
void ppr_kernels(bingo_graph* g, uint32_t nsrc, const uint32_t* sources, uint32_t R, uint32_t cap, uint64_t seed,
                 uint64_t base, const uint64_t* seg, const uint32_t* len, uint32_t mode,
                 uint64_t* idA, uint32_t* vA, uint64_t* idB, uint32_t* vB, unsigned long long* ctl, uint32_t* vis,
                 hipStream_t st) {
    const uint64_t nw = (uint64_t)nsrc * R;
    if (mode == BINGO_WALK_PER_STEP) {
        const uint32_t grid = grid_for(nw);
        hipLaunchKernelGGL(k_ppr_start, dim3(grid), dim3(TB), 0, st, g->n, nsrc, sources, R, seg, len, idA, vA, ctl,
                           vis, g->d_err);
        for (uint32_t s = 0; s < cap; ++s) {
            const int in_slot = s & 1;
            hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, ctl + 3 + (in_slot ^ 1), 0ull);
            hipLaunchKernelGGL((k_ppr_step<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, R, s, seed, base,
                               g->rule, seg, len, in_slot ? idB : idA, in_slot ? vB : vA, in_slot ? idA : idB,
                               in_slot ? vA : vB, ctl, in_slot, vis);
        }
    } else {
        const void* kern = g->walk_variant ? (const void*)k_ppr_interleaved<SPEC, MODE> : (const void*)k_ppr_persistent<SPEC, MODE>;
        const int rg = resident_grid(kern, g->blocks_per_cu);
        const uint32_t grid = std::max<uint32_t>((uint32_t)std::min<uint64_t>((uint64_t)rg, (nw + TB - 1) / TB), 1);
        if (g->walk_variant)
            hipLaunchKernelGGL((k_ppr_interleaved<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nsrc, sources, R,
                               seed, base, g->rule, seg, len, ctl, vis, g->d_err, g->queue_chunk, g->wave_degree);
        else
            hipLaunchKernelGGL((k_ppr_persistent<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nsrc, sources, R,
                               seed, base, g->rule, seg, len, ctl, vis, g->d_err, g->queue_chunk);
    }
}

}  // namespace

namespace {
template <int SPEC, int MODE>
void deepwalk_batch_kernel(bingo_graph* g, const WalkQueryTable& tab, uint32_t nq, uint64_t nw,
                           unsigned long long* ctl, hipStream_t st) {
    const int rg = resident_grid((const void*)k_deepwalk_batch<SPEC, MODE>, g->blocks_per_cu);
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)rg, (nw + TB - 1) / TB));
    hipLaunchKernelGGL((k_deepwalk_batch<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, tab, nq, nw,
                       g->rule, ctl, g->d_err, g->queue_chunk);
}
}  // namespace

int walk_slot_take(bingo_graph* g, hipStream_t st, uint32_t* slot) {
    const uint32_t i = g->walk_slot++ % WALK_SLOTS;
    if (!g->slot_ev[i]) HIPCHK(hipEventCreateWithFlags(&g->slot_ev[i], hipEventDisableTiming));
    else if (g->slot_st[i] != st) {
        // a call still in flight on another stream owns these counters until its event
        const hipError_t q = hipEventQuery(g->slot_ev[i]);
        if (q == hipErrorNotReady) HIPCHK(hipStreamWaitEvent(st, g->slot_ev[i], 0));
        else if (q != hipSuccess) HIPCHK(q);
    }
    g->slot_st[i] = st;
    HIPCHK(hipMemsetAsync(g->d_ctl + CTL_WALK0 + 2 * i, 0, 16, st));
    *slot = i;
    return BINGO_OK;
}

int walk_slot_release(bingo_graph* g, uint32_t slot, hipStream_t st) {
    HIPCHK(hipEventRecord(g->slot_ev[slot], st));
    return BINGO_OK;
}

int launch_walk_batch(bingo_graph* g, uint32_t nq, const bingo_walk_query* hq, hipStream_t st) {
    if (nq == 0) return BINGO_OK;
    WalkQueryTable tab;
    memset(&tab, 0, sizeof tab);
    uint64_t nw = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        tab.q[i] = WalkQueryDev{hq[i].d_starts, hq[i].d_paths, (unsigned long long*)hq[i].d_steps_taken, nw,
                                hq[i].walk_id_base, hq[i].seed, hq[i].length, 0u};
        nw += hq[i].n_walks;
    }
    uint32_t slot = 0;
    if (int rc = walk_slot_take(g, st, &slot)) return rc;
    unsigned long long* ctl = g->d_ctl + CTL_WALK0 + 2 * slot;
    phase_mark(g, st, true);
    hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(WALK_BATCH_MAX), 0, st, tab, nq);
    if (nw) {
        switch (g->dense_spec) {
#define DWB(S) (walk_mode(g) == 1 ? deepwalk_batch_kernel<S, 1> : walk_mode(g) == 2 ? deepwalk_batch_kernel<S, 2> : deepwalk_batch_kernel<S, 0>)
            case 1: DWB(1)(g, tab, nq, nw, ctl, st); break;
            case 4: DWB(4)(g, tab, nq, nw, ctl, st); break;
            default: DWB(2)(g, tab, nq, nw, ctl, st); break;
#undef DWB
        }
    }
    phase_mark(g, st, false);
    if (int rc = walk_slot_release(g, slot, st)) return rc;
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

int launch_walk(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, uint64_t seed,
                uint32_t* paths, uint64_t* steps, uint32_t mode, hipStream_t st) {
    // per-call queue head and transition counter from a ring of slots, so that
    // walks on different streams do not share counters
    uint32_t slot = 0;
    if (int rc = walk_slot_take(g, st, &slot)) return rc;
    unsigned long long* ctl = g->d_ctl + CTL_WALK0 + 2 * slot;
    phase_mark(g, st, true);
    if (nw == 0) {
        if (steps) HIPCHK(hipMemsetAsync(steps, 0, 8, st));
        return walk_slot_release(g, slot, st);
    }
    switch (g->dense_spec) {
#define DWK(S) (walk_mode(g) == 1 ? deepwalk_kernels<S, 1> : walk_mode(g) == 2 ? deepwalk_kernels<S, 2> : deepwalk_kernels<S, 0>)
        case 1: DWK(1)(g, nw, starts, base, L, seed, paths, mode, ctl, st); break;
        case 4: DWK(4)(g, nw, starts, base, L, seed, paths, mode, ctl, st); break;
        default: DWK(2)(g, nw, starts, base, L, seed, paths, mode, ctl, st); break;
#undef DWK
    }
    phase_mark(g, st, false);
    if (steps) HIPCHK(hipMemcpyAsync(steps, ctl + 1, 8, hipMemcpyDeviceToDevice, st));
    if (int rc = walk_slot_release(g, slot, st)) return rc;
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

static int ensure_ppr_off(bingo_graph* g, uint32_t nsrc) {
    if (g->ppr_off_cap < nsrc + 1 || !g->ppr_off) {
        hipFree(g->ppr_off);
        g->ppr_off_cap = nsrc + 1;
        if (hipMalloc(&g->ppr_off, (uint64_t)(nsrc + 1) * 8) != hipSuccess) {
            g->ppr_off = nullptr; g->ppr_off_cap = 0;
            return BINGO_E_OOM;
        }
    }
    return BINGO_OK;
}

// Per-source histograms in one block per source (ranges of at most HCAP keys:
// the sources' bins when C != 0, else their walks' segments), then the CSR.
// Ends the histogram phase and synchronizes.
static int finish_lds_hist(bingo_graph* g, uint32_t* vis, uint32_t* hcnt, uint32_t* ucount, const uint64_t* seg,
                           uint32_t R, uint64_t C, const uint32_t* bin_cnt, uint32_t nsrc, uint64_t total,
                           uint64_t maxlen, void* tmp, unsigned long long* ctl, uint64_t steps, uint64_t* h_entries,
                           uint64_t* h_steps, hipStream_t st) {
    const int rc = ensure_ppr_off(g, nsrc);
    if (rc != BINGO_OK) return rc;
    HIPCHK(hipMemsetAsync(ctl, 0, 8, st));
#define BINGO_HIST(E_)                                                                                     \
    hipLaunchKernelGGL((k_hist_seg<E_>), dim3(nsrc), dim3(HSB), 0, st, vis, hcnt, seg, R, nsrc, total, C, bin_cnt, \
                       ucount, ctl)
    if (maxlen <= HSB * 1) BINGO_HIST(1);
    else if (maxlen <= HSB * 2) BINGO_HIST(2);
    else if (maxlen <= HSB * 4) BINGO_HIST(4);
    else if (maxlen <= HSB * 8) BINGO_HIST(8);
    else if (maxlen <= HSB * 16) BINGO_HIST(16);
    else BINGO_HIST(32);
#undef BINGO_HIST
    scan_u32_to_u64(ucount, g->ppr_off, nsrc, tmp, ctl + 1, st);
    unsigned long long hv[2];
    HIPCHK(hipMemcpyAsync(hv, ctl, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hv[0]) return BINGO_E_HIP;  // unreachable: every range was checked against the width before
    const uint64_t U = hv[1];
    if (g->ppr_cap < U || !g->ppr_vtx) {
        hipFree(g->ppr_vtx); hipFree(g->ppr_cnt);
        // sized for every visit a distinct vertex (as the asynchronous form needs), so that a
        // later query of the same shape, synchronous or not, allocates nothing
        g->ppr_cap = std::max<uint64_t>(std::max(U, total), 1024);
        if (hipMalloc(&g->ppr_vtx, g->ppr_cap * 4) != hipSuccess || hipMalloc(&g->ppr_cnt, g->ppr_cap * 4) != hipSuccess) {
            g->ppr_vtx = g->ppr_cnt = nullptr; g->ppr_cap = 0;
            return BINGO_E_OOM;
        }
    }
    hipLaunchKernelGGL(k_set_last_off, dim3(1), dim3(1), 0, st, g->ppr_off, nsrc, (const unsigned long long*)(ctl + 1));
    hipLaunchKernelGGL(k_hist_compact, dim3(nsrc), dim3(256), 0, st, vis, hcnt, seg, R, C, ucount, g->ppr_off,
                       g->ppr_vtx, g->ppr_cnt);
    phase_mark(g, st, false);
    HIPCHK(hipStreamSynchronize(st));
    g->ppr_entries = U;
    g->ppr_nsrc = nsrc;
    if (h_entries) *h_entries = U;
    if (h_steps) *h_steps = steps;
    return BINGO_OK;
}

// The same histogram enqueued on hs after the walk phase on st, without waiting:
// the outputs are sized for every visit being a distinct vertex, so no count is
// needed before the compaction; the count lands in d_ctl[CTL_PPR_U] for ppr_wait.
static int finish_lds_hist_async(bingo_graph* g, uint32_t* vis, uint32_t* hcnt, uint32_t* ucount, uint32_t R,
                                 uint64_t C, const uint32_t* bin_cnt, uint32_t nsrc, uint64_t total, uint64_t maxlen,
                                 void* tmp, unsigned long long* ctl, uint64_t steps, uint64_t* h_steps, hipStream_t st,
                                 hipStream_t hs) {
    int rc = ensure_ppr_off(g, nsrc);
    if (rc != BINGO_OK) return rc;
    if (g->ppr_cap < total || !g->ppr_vtx) {
        hipFree(g->ppr_vtx); hipFree(g->ppr_cnt);
        g->ppr_cap = std::max<uint64_t>(total, 1024);
        if (hipMalloc(&g->ppr_vtx, g->ppr_cap * 4) != hipSuccess || hipMalloc(&g->ppr_cnt, g->ppr_cap * 4) != hipSuccess) {
            g->ppr_vtx = g->ppr_cnt = nullptr; g->ppr_cap = 0;
            return BINGO_E_OOM;
        }
    }
    for (hipEvent_t* e : {&g->ppr_done, &g->ppr_h0, &g->ppr_h1})
        if (!*e) HIPCHK(hipEventCreate(e));
    HIPCHK(hipEventRecord(g->ppr_done, st));  // the walk phase
    HIPCHK(hipStreamWaitEvent(hs, g->ppr_done, 0));
    HIPCHK(hipEventRecord(g->ppr_h0, hs));
    HIPCHK(hipMemsetAsync(ctl, 0, 8, hs));
#define BINGO_HIST(E_)                                                                                            \
    hipLaunchKernelGGL((k_hist_seg<E_>), dim3(nsrc), dim3(HSB), 0, hs, vis, hcnt, (const uint64_t*)nullptr, R, nsrc, \
                       total, C, bin_cnt, ucount, ctl)
    if (maxlen <= HSB * 1) BINGO_HIST(1);
    else if (maxlen <= HSB * 2) BINGO_HIST(2);
    else if (maxlen <= HSB * 4) BINGO_HIST(4);
    else if (maxlen <= HSB * 8) BINGO_HIST(8);
    else if (maxlen <= HSB * 16) BINGO_HIST(16);
    else BINGO_HIST(32);
#undef BINGO_HIST
    scan_u32_to_u64(ucount, g->ppr_off, nsrc, tmp, ctl + 1, hs);
    hipLaunchKernelGGL(k_set_last_off, dim3(1), dim3(1), 0, hs, g->ppr_off, nsrc, (const unsigned long long*)(ctl + 1));
    hipLaunchKernelGGL(k_hist_compact, dim3(nsrc), dim3(256), 0, hs, vis, hcnt, (const uint64_t*)nullptr, R, C, ucount,
                       g->ppr_off, g->ppr_vtx, g->ppr_cnt);
    HIPCHK(hipMemcpyAsync(g->d_ctl + CTL_PPR_U, ctl + 1, 8, hipMemcpyDeviceToDevice, hs));
    HIPCHK(hipEventRecord(g->ppr_h1, hs));
    HIPCHK(hipEventRecord(g->ppr_done, hs));
    g->ppr_pending = true;
    g->ppr_entries = 0;
    g->ppr_nsrc = nsrc;
    if (h_steps) *h_steps = steps;
    return BINGO_OK;
}

int ppr_wait(bingo_graph* g, uint64_t* h_entries, float* h_hist_ms) {
    if (!g->ppr_pending) {
        if (h_entries) *h_entries = g->ppr_entries;
        if (h_hist_ms) *h_hist_ms = 0.f;
        return BINGO_OK;
    }
    g->ppr_pending = false;
    HIPCHK(hipEventSynchronize(g->ppr_done));
    unsigned long long u = 0;
    HIPCHK(hipMemcpy(&u, g->d_ctl + CTL_PPR_U, 8, hipMemcpyDeviceToHost));
    g->ppr_entries = u;
    if (h_entries) *h_entries = u;
    if (h_hist_ms) HIPCHK(hipEventElapsedTime(h_hist_ms, g->ppr_h0, g->ppr_h1));
    return BINGO_OK;
}

constexpr int PPR_RETRY = 1;

// Persistent PPR into per-source bins (k_ppr_binned).  Returns PPR_RETRY when a
// bin overflowed or a source has more visits than the per-source histogram
// holds; the caller then reruns the query with exact per-walk segments.
static int run_ppr_binned(bingo_graph* g, uint32_t nsrc, const uint32_t* sources, uint32_t R, uint32_t thr,
                          uint32_t cap, uint64_t seed, uint64_t base, uint64_t* h_entries, uint64_t* h_steps,
                          hipStream_t st, hipStream_t hs) {
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    // bin capacity: 1.25 x the expected visits of R walks plus slack, at most the worst case R (cap + 1)
    const double keep = 1.0 - (double)thr / 4294967296.0;
    double mean = 1.0, term = 1.0;
    for (uint32_t i = 0; i < cap && term > 1e-12; ++i) { term *= keep; mean += term; }
    const uint64_t worst = (uint64_t)R * ((uint64_t)cap + 1);
    const uint64_t C = std::min<uint64_t>(worst, (uint64_t)(1.25 * mean * R) + 1024);
    const uint64_t cells = (uint64_t)nsrc * C;
    char* ws = (char*)ws_get(g, 2 * al(cells * 4) + 2 * al((uint64_t)nsrc * 4) + scan_temp_bytes(nsrc) + 1024);
    if (!ws) return BINGO_E_OOM;
    uint32_t* vis = (uint32_t*)ws;      ws += al(cells * 4);
    uint32_t* hcnt = (uint32_t*)ws;     ws += al(cells * 4);
    uint32_t* bin_cnt = (uint32_t*)ws;  ws += al((uint64_t)nsrc * 4);
    uint32_t* ucount = (uint32_t*)ws;   ws += al((uint64_t)nsrc * 4);
    void* tmp = ws;
    unsigned long long* ctl = g->d_ctl + 2;  // [0] queue, [1] transitions, [2] overflow, [3] largest bin
    HIPCHK(hipMemsetAsync(ctl, 0, 32, st));
    HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
    phase_mark(g, st, true);
    HIPCHK(hipMemsetAsync(bin_cnt, 0, (uint64_t)nsrc * 4, st));
    phase_mark(g, st, false);
#define BINGO_BINNED(S_, M_)                                                                                          \
    do {                                                                                                           \
        const int rg = resident_grid((const void*)k_ppr_binned<S_, M_>, g->blocks_per_cu);                             \
        const uint64_t nw = (uint64_t)nsrc * R;                                                                    \
        const uint32_t grid = std::max<uint32_t>((uint32_t)std::min<uint64_t>((uint64_t)rg, (nw + TB - 1) / TB), 1); \
        hipLaunchKernelGGL((k_ppr_binned<S_, M_>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nsrc, sources, R, \
                           seed, base, thr, cap, g->rule, C, bin_cnt, vis, ctl, g->d_err, g->queue_chunk,         \
                           g->wave_degree);                                                                         \
    } while (0)
    switch (g->dense_spec) {
        case 1: if (walk_mode(g) == 1) BINGO_BINNED(1, 1); else if (walk_mode(g) == 2) BINGO_BINNED(1, 2); else BINGO_BINNED(1, 0); break;
        case 4: if (walk_mode(g) == 1) BINGO_BINNED(4, 1); else if (walk_mode(g) == 2) BINGO_BINNED(4, 2); else BINGO_BINNED(4, 0); break;
        default: if (walk_mode(g) == 1) BINGO_BINNED(2, 1); else if (walk_mode(g) == 2) BINGO_BINNED(2, 2); else BINGO_BINNED(2, 0); break;
    }
#undef BINGO_BINNED
    phase_mark(g, st, false);
    hipLaunchKernelGGL(k_bin_max, dim3((uint32_t)std::min<uint64_t>((nsrc + 255) / 256, 1024)), dim3(256), 0, st,
                       bin_cnt, nsrc, ctl + 3);
    unsigned long long c4[4];
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(c4, ctl, 32, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (err) return err_to_code(err);
    if (c4[2] || c4[3] > C || c4[3] > HCAP) return PPR_RETRY;
    if (hs)
        return finish_lds_hist_async(g, vis, hcnt, ucount, R, C, bin_cnt, nsrc, cells, c4[3], tmp, ctl + 2, c4[1],
                                     h_steps, st, hs);
    return finish_lds_hist(g, vis, hcnt, ucount, nullptr, R, C, bin_cnt, nsrc, cells, c4[3], tmp, ctl + 2, c4[1],
                           h_entries, h_steps, st);
}

int run_ppr(bingo_graph* g, uint32_t nsrc, const uint32_t* sources, uint32_t R, uint32_t thr, uint32_t cap,
            uint64_t seed, uint64_t base, uint32_t mode, uint64_t* h_entries, uint64_t* h_steps, hipStream_t st,
            hipStream_t hist_st) {
    if (g->ppr_pending) {
        // the previous query's histogram still reads the visit bins this query is about to
        // overwrite: st waits for it on the device; its result gives way to this query's
        HIPCHK(hipStreamWaitEvent(st, g->ppr_done, 0));
        g->ppr_pending = false;
    }
    if (mode == BINGO_WALK_PERSISTENT && g->ppr_bins) {
        const int rc = run_ppr_binned(g, nsrc, sources, R, thr, cap, seed, base, h_entries, h_steps, st, hist_st);
        if (rc != PPR_RETRY) return rc;
    }
    // the exact-segment form below finishes its histogram before returning, asynchronous call or not
    const uint64_t nw = (uint64_t)nsrc * R;
    const int vbits = std::max(1, bits_for((uint64_t)g->n - 1));
    const int qbits = std::max(1, bits_for(nsrc));  // q < nsrc < 2^qbits
    if (vbits + qbits > 63) return BINGO_E_INVALID;
    const uint64_t pad = (1ull << (vbits + qbits)) - 1;  // above every (q, v) key
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    unsigned long long* ctl = g->d_ctl + 2;  // [0] queue, [1] transitions, [2] scan total, [3..4] active counts
    // per-walk arrays (lengths, segment offsets, active lists) live in the handle's aux buffer so
    // that the workspace can grow once the total is known
    const uint64_t act_bytes = mode == BINGO_WALK_PER_STEP ? 2 * (al(nw * 8) + al(nw * 4)) : 0;
    const size_t aux_need = al(nw * 4) + al(nw * 8) + act_bytes + scan_temp_bytes(nw) + 512;
    if (aux_need > g->aux_bytes) {
        HIPCHK(hipStreamSynchronize(st));
        hipFree(g->aux);
        g->aux = nullptr;
        g->aux_bytes = 0;
        if (hipMalloc(&g->aux, aux_need + aux_need / 4) != hipSuccess) { g->aux = nullptr; return BINGO_E_OOM; }
        g->aux_bytes = aux_need + aux_need / 4;
    }
    char* a = (char*)g->aux;
    uint32_t* len = (uint32_t*)a;  a += al(nw * 4);
    uint64_t* seg = (uint64_t*)a;  a += al(nw * 8);
    char* act = a;                 a += act_bytes;
    void* atmp = a;
    HIPCHK(hipMemsetAsync(ctl, 0, 40, st));
    HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
    phase_mark(g, st, true);
    hipLaunchKernelGGL(k_ppr_bound, dim3((uint32_t)std::min<uint64_t>((nw + BOUND_CHUNK * 4 - 1) / (BOUND_CHUNK * 4), 8192)),
                       dim3(TB), 0, st, nw, base, seed, thr, cap, len);
    scan_u32_to_u64(len, seg, nw, atmp, ctl + 2, st);
    hipLaunchKernelGGL(k_seg_maxlen, dim3((uint32_t)std::min<uint64_t>((nsrc + 255) / 256, 1024)), dim3(256), 0, st, seg,
                       R, nsrc, (const unsigned long long*)(ctl + 2), ctl + 3);
    unsigned long long tm[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(tm, ctl + 2, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const unsigned long long total = tm[0];
    const bool lds_hist = tm[1] <= HCAP;
    const uint64_t TT = std::max<uint64_t>(total, 1);
    // visits (u32 per position); then the LDS path's count array and per-source
    // entry counts, or the global path's keys, sorted keys, heads and positions
    const size_t part = lds_hist ? al(TT * 4) + al((uint64_t)nsrc * 4) : 4 * al(TT * 8) + al(TT * 4);
    char* ws = (char*)ws_get(g, al(TT * 4) + part + std::max(sort_temp_bytes(TT, true), scan_temp_bytes(TT)) + 1024);
    if (!ws) return BINGO_E_OOM;
    uint32_t* vis = (uint32_t*)ws;     ws += al(TT * 4);
    uint32_t *hcnt = nullptr, *ucount = nullptr, *head = nullptr;
    uint64_t *keys = nullptr, *sorted = nullptr, *idx = nullptr, *hpos = nullptr;
    if (lds_hist) {
        hcnt = (uint32_t*)ws;    ws += al(TT * 4);
        ucount = (uint32_t*)ws;  ws += al((uint64_t)nsrc * 4);
    } else {
        keys = (uint64_t*)ws;    ws += al(TT * 8);
        sorted = (uint64_t*)ws;  ws += al(TT * 8);
        head = (uint32_t*)ws;    ws += al(TT * 4);
        idx = (uint64_t*)ws;     ws += al(TT * 8);
        hpos = (uint64_t*)ws;    ws += al(TT * 8);
    }
    void* tmp = ws;
    phase_mark(g, st, false);
    uint64_t *idA = nullptr, *idB = nullptr;
    uint32_t *vA = nullptr, *vB = nullptr;
    if (mode == BINGO_WALK_PER_STEP) {
        idA = (uint64_t*)act;
        vA = (uint32_t*)(act + al(nw * 8));
        idB = (uint64_t*)(act + al(nw * 8) + al(nw * 4));
        vB = (uint32_t*)(act + 2 * al(nw * 8) + al(nw * 4));
    }
    switch (g->dense_spec) {
#define PPK(S) (walk_mode(g) == 1 ? ppr_kernels<S, 1> : walk_mode(g) == 2 ? ppr_kernels<S, 2> : ppr_kernels<S, 0>)
        case 1: PPK(1)(g, nsrc, sources, R, cap, seed, base, seg, len, mode, idA, vA, idB, vB, ctl, vis, st); break;
        case 4: PPK(4)(g, nsrc, sources, R, cap, seed, base, seg, len, mode, idA, vA, idB, vB, ctl, vis, st); break;
        default: PPK(2)(g, nsrc, sources, R, cap, seed, base, seg, len, mode, idA, vA, idB, vB, ctl, vis, st); break;
#undef PPK
    }
    phase_mark(g, st, false);
    unsigned long long steps = 0;
    HIPCHK(hipMemcpyAsync(&steps, ctl + 1, 8, hipMemcpyDeviceToHost, st));
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (err) return err_to_code(err);
    const uint64_t N = nw + steps;  // visits: every start and every transition
    if (lds_hist)
        return finish_lds_hist(g, vis, hcnt, ucount, seg, R, 0, nullptr, nsrc, total, tm[1], tmp, ctl + 3, steps,
                               h_entries, h_steps, st);
    {
        const int rc = ensure_ppr_off(g, nsrc);
        if (rc != BINGO_OK) return rc;
    }
    // histogram: sort (source, vertex) keys (padding sorts last), then run-length encode
    hipLaunchKernelGGL(k_vis_keys, dim3(grid_for(total)), dim3(TB), 0, st, vis, seg, R, nsrc, (uint64_t)total, vbits,
                       pad, keys);
    sort_keys_u64(keys, sorted, total, vbits + qbits, tmp, st);
    hipLaunchKernelGGL(k_heads, dim3(grid_for(N)), dim3(TB), 0, st, sorted, N, head);
    scan_u32_to_u64(head, idx, N, tmp, ctl + 2, st);
    unsigned long long U = 0;
    HIPCHK(hipMemcpyAsync(&U, ctl + 2, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (g->ppr_cap < U || !g->ppr_vtx) {
        hipFree(g->ppr_vtx); hipFree(g->ppr_cnt);
        g->ppr_cap = std::max<uint64_t>(U, 1024) * 5 / 4;
        if (hipMalloc(&g->ppr_vtx, g->ppr_cap * 4) != hipSuccess ||
            hipMalloc(&g->ppr_cnt, g->ppr_cap * 4) != hipSuccess) {
            g->ppr_vtx = g->ppr_cnt = nullptr; g->ppr_cap = 0;
            return BINGO_E_OOM;
        }
    }
    hipLaunchKernelGGL(k_emit, dim3(grid_for(N)), dim3(TB), 0, st, sorted, N, head, idx, vbits, g->ppr_vtx, hpos,
                       g->ppr_off);
    hipLaunchKernelGGL(k_counts, dim3(grid_for(U)), dim3(TB), 0, st, hpos, (uint64_t)U, N, g->ppr_cnt, g->ppr_off,
                       nsrc);
    phase_mark(g, st, false);
    HIPCHK(hipStreamSynchronize(st));
    g->ppr_entries = U;
    g->ppr_nsrc = nsrc;
    if (h_entries) *h_entries = U;
    if (h_steps) *h_steps = steps;
    return BINGO_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free DeepWalk entry point.  bingo_walk takes its per-call counters
// (the persistent kernel's work-queue head and its transition count) from the
// handle's slot ring, whose events it creates on first use.  This variant keeps
// them in a fixed device array instead and creates nothing: no device memory,
// no events.  The array is one per device, holds the counters of one call at a
// time, and is cleared by a fill kernel at the start of every call (no memset,
// so the call can be captured into a graph).
// ---------------------------------------------------------------------------
namespace {

constexpr uint32_t NOALLOC_WORDS = 32;  // 256 bytes per device: [0] queue head, [1] transitions
static __device__ __align__(256) unsigned long long scratch[NOALLOC_WORDS];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
unsigned long long* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

__global__ void k_noalloc_begin(unsigned long long* __restrict__ s) {
    if (threadIdx.x < NOALLOC_WORDS) s[threadIdx.x] = 0ull;
}
__global__ void k_noalloc_end(const unsigned long long* __restrict__ s, unsigned long long* __restrict__ steps) {
    *steps = s[1];
}

// Device address of this device's copy of the array, looked up once per device
// with that device current (the array's host-side name is not a device address).
int noalloc_scratch(unsigned long long** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return BINGO_E_INVALID;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        noalloc_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    *out = noalloc_ptr[dev];
    return BINGO_OK;
}

}  // namespace

extern "C" int bingo_walk_noalloc(const bingo_graph* gc, uint64_t n_walks, const uint32_t* d_starts,
                                  uint64_t walk_id_base, uint32_t length, uint64_t seed, uint32_t* d_paths,
                                  uint64_t* d_steps_taken, void* stream) {
    if (!gc || gc->radix_base != 2 || (n_walks && (!d_starts || !d_paths)) || length == 0xFFFFFFFFu)
        return BINGO_E_INVALID;
    bingo_graph* g = const_cast<bingo_graph*>(gc);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long* ctl = nullptr;
    if (int rc = noalloc_scratch(&ctl)) return rc;
    hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(NOALLOC_WORDS), 0, st, ctl);
    if (n_walks) {
        switch (g->dense_spec) {
#define DWN(S) (walk_mode(g) == 1 ? deepwalk_kernels<S, 1> : walk_mode(g) == 2 ? deepwalk_kernels<S, 2> : deepwalk_kernels<S, 0>)
            case 1: DWN(1)(g, n_walks, d_starts, walk_id_base, length, seed, d_paths, BINGO_WALK_PERSISTENT, ctl, st); break;
            case 4: DWN(4)(g, n_walks, d_starts, walk_id_base, length, seed, d_paths, BINGO_WALK_PERSISTENT, ctl, st); break;
            default: DWN(2)(g, n_walks, d_starts, walk_id_base, length, seed, d_paths, BINGO_WALK_PERSISTENT, ctl, st); break;
#undef DWN
        }
    }
    if (d_steps_taken)
        hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(1), 0, st, ctl, (unsigned long long*)d_steps_taken);
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

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
#include <stdio.h>
#include <algorithm>

namespace {

constexpr int TB = 256;
constexpr uint64_t NO_WALK = ~0ull;

// One transition from u.  Returns the next vertex or STOP_VERTEX.
template <bool PPR>
__device__ __forceinline__ uint32_t walk_step(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                              uint32_t u, RandStream& rs, uint32_t thr, GroupRule rule) {
    const uint4* h4 = reinterpret_cast<const uint4*>(hdr + (size_t)u * HDR_WORDS);
    // line 0 of the header in one go: mask, d, W, adjacency offset, c_0..c_25
    const uint4 q0 = h4[0], q1 = h4[1], q2 = h4[2], q3 = h4[3], q4 = h4[4], q5 = h4[5], q6 = h4[6], q7 = h4[7];
    const uint32_t d = q0.y;
    if (d == 0) return STOP_VERTEX;
    if (PPR) {
        if (rs_next32(rs) < thr) return STOP_VERTEX;
    }
    const uint64_t W = ((uint64_t)q0.w << 32) | q0.z;
    const uint64_t r = rs_below64(rs, W);
    const uint32_t c[26] = {q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z,
                            q4.w, q5.x, q5.y, q5.z, q5.w, q6.x, q6.y, q6.z, q6.w, q7.x, q7.y, q7.z, q7.w};
    uint64_t acc = 0;
    int sel = -1;
    uint32_t csel = 0;
#pragma unroll
    for (int k = 0; k < 26; ++k) {
        acc += (uint64_t)c[k] << k;
        if (sel < 0 && r < acc) { sel = k; csel = c[k]; }
    }
    if (sel < 0) {
        const uint4 a = h4[8], b = h4[9];
        const uint32_t hc[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            acc += (uint64_t)hc[k] << (26 + k);
            if (sel < 0 && r < acc) { sel = 26 + k; csel = hc[k]; }
        }
    }
    const uint64_t adj = ((uint64_t)q1.y << 32) | q1.x;
    const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + adj);
    const uint32_t t = group_type(csel, d, rule);
    if (t == GT_DENSE) {
        // rejection on the whole neighbor list: accept a slot whose weight has
        // bit sel.  Acceptance is above alpha % per attempt, so the bound is
        // never reached on a consistent structure; it only keeps a corrupted
        // one from spinning forever.
        for (uint32_t att = 0; att < (1u << 16); ++att) {
            const uint32_t i = rs_below32(rs, d);
            const uint64_t e = edges[i];
            if ((e >> (32 + sel)) & 1ull) return (uint32_t)e;
        }
        return STOP_VERTEX;
    }
    const uint32_t info = hdr[(size_t)u * HDR_WORDS + H_INFO + sel];
    uint32_t i;
    if (t == GT_ONE) {
        i = info;
    } else {
        i = pool[(uint64_t)info * LIST_UNIT_WORDS + rs_below32(rs, csel)];
    }
    return pool[adj + 2ull * i];
}

__device__ __forceinline__ void wave_add_u64(unsigned long long* p, uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0 && v) atomicAdd(p, (unsigned long long)v);
}

// Take one walk id per lane that asked for one (ballot + one atomic per wave).
__device__ __forceinline__ uint64_t wave_take(bool need, unsigned long long* queue) {
    const uint64_t want = __ballot(need);
    if (!want) return NO_WALK;
    const int leader = __ffsll((long long)want) - 1;
    unsigned long long basew = 0;
    if ((int)lane_id() == leader) basew = atomicAdd(queue, (unsigned long long)__popcll(want));
    basew = __shfl(basew, leader, 64);
    return need ? basew + __popcll(want & lanemask_lt()) : NO_WALK;
}

// ------------------------------------------------------------------ DeepWalk
__global__ void __launch_bounds__(TB) k_deepwalk_persistent(const uint32_t* __restrict__ hdr,
                                                            const uint32_t* __restrict__ pool, uint32_t n,
                                                            uint64_t nw, const uint32_t* __restrict__ starts,
                                                            uint64_t base, uint32_t L, uint64_t seed,
                                                            uint32_t* __restrict__ paths, GroupRule rule,
                                                            unsigned long long* __restrict__ ctl,
                                                            uint32_t* __restrict__ err) {
    // ctl[0] = queue head, ctl[1] = transitions taken
    uint64_t j = NO_WALK;
    uint32_t u = 0, s = 0;
    uint64_t steps = 0;
    uint32_t* row = nullptr;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take(need, ctl);
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
                const uint32_t v = walk_step<false>(hdr, pool, u, rs, 0, rule);
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
            v = walk_step<false>(hdr, pool, u, rs, 0, rule);
            steps += (v != STOP_VERTEX);
        }
        row[s + 1] = v;
    }
    wave_add_u64(ctl + 1, steps);
}

// ------------------------------------------------------------------ PPR
// Visits are appended as keys (source index << vbits | vertex) to a buffer of
// capacity cap_visits; the count keeps growing past the capacity so the host
// can size a retry exactly.
__device__ __forceinline__ void wave_append(bool has, uint64_t key, unsigned long long* counter,
                                            uint64_t* __restrict__ out, uint64_t capv) {
    const uint64_t m = __ballot(has);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long b = 0;
    if ((int)lane_id() == leader) b = atomicAdd(counter, (unsigned long long)__popcll(m));
    b = __shfl(b, leader, 64);
    if (has) {
        const uint64_t pos = b + __popcll(m & lanemask_lt());
        if (pos < capv) out[pos] = key;
    }
}

__global__ void __launch_bounds__(TB) k_ppr_persistent(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                       uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                       uint32_t R, uint32_t thr, uint32_t cap, uint64_t seed,
                                                       uint64_t base, int vbits, GroupRule rule,
                                                       unsigned long long* __restrict__ ctl,
                                                       uint64_t* __restrict__ visits, uint64_t capv,
                                                       uint32_t* __restrict__ err) {
    // ctl[0] queue head, ctl[1] transitions, ctl[2] visits appended
    const uint64_t nw = (uint64_t)nsrc * R;
    uint64_t j = NO_WALK;
    uint32_t u = 0, s = 0;
    uint64_t q = 0, steps = 0;
    bool done = false;
    for (;;) {
        const bool need = !done && j == NO_WALK;
        const uint64_t got = wave_take(need, ctl);
        bool has = false;
        uint64_t key = 0;
        if (need) {
            if (got >= nw) {
                done = true;
            } else {
                j = got;
                q = j / R;
                u = sources[q];
                s = 0;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    j = NO_WALK;
                } else {
                    has = true;
                    key = (q << vbits) | u;
                }
            }
        }
        wave_append(has, key, ctl + 2, visits, capv);
        if (__ballot(!done) == 0) break;
        has = false;
        if (j != NO_WALK) {
            uint32_t v = STOP_VERTEX;
            if (s < cap) {
                RandStream rs;
                rs_init(rs, seed, base + j, s);
                v = walk_step<true>(hdr, pool, u, rs, thr, rule);
            }
            if (v == STOP_VERTEX) {
                j = NO_WALK;
            } else {
                has = true;
                key = (q << vbits) | v;
                u = v;
                ++s;
                ++steps;
            }
        }
        wave_append(has, key, ctl + 2, visits, capv);
    }
    wave_add_u64(ctl + 1, steps);
}

// Per-step PPR: active walks are (walk id, current vertex) pairs compacted into
// the next list after every step.
__global__ void __launch_bounds__(TB) k_ppr_start(uint32_t n, uint32_t nsrc, const uint32_t* __restrict__ sources,
                                                  uint32_t R, int vbits, uint64_t* __restrict__ act_id,
                                                  uint32_t* __restrict__ act_v, unsigned long long* __restrict__ ctl,
                                                  uint64_t* __restrict__ visits, uint64_t capv,
                                                  uint32_t* __restrict__ err) {
    // ctl[2] visits, ctl[3] active count of list A
    const uint64_t nw = (uint64_t)nsrc * R;
    const uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t iters = (nw + stride - 1) / stride;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t j = j0 + it * stride;
        bool has = false;
        uint64_t key = 0;
        uint32_t u = 0;
        if (j < nw) {
            const uint64_t q = j / R;
            u = sources[q];
            if (u >= n) atomicOr(err, ERR_RANGE);
            else { has = true; key = (q << vbits) | u; }
        }
        wave_append(has, key, ctl + 2, visits, capv);
        // the initial active list is the walks themselves, in id order
        if (j < nw) { act_id[j] = has ? j : NO_WALK; act_v[j] = has ? u : STOP_VERTEX; }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[3] = nw;
}

__global__ void __launch_bounds__(TB) k_ppr_step(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                 uint32_t R, uint32_t thr, uint32_t s, uint64_t seed, uint64_t base,
                                                 int vbits, GroupRule rule, const uint64_t* __restrict__ in_id,
                                                 const uint32_t* __restrict__ in_v, uint64_t* __restrict__ out_id,
                                                 uint32_t* __restrict__ out_v, unsigned long long* __restrict__ ctl,
                                                 int in_slot, uint64_t* __restrict__ visits, uint64_t capv) {
    const uint64_t cnt = ctl[3 + in_slot];
    const uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t iters = (cnt + stride - 1) / stride;
    uint64_t steps = 0;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t a = j0 + it * stride;
        bool alive = false;
        uint64_t key = 0, id = NO_WALK;
        uint32_t v = STOP_VERTEX;
        if (a < cnt) {
            id = in_id[a];
            if (id != NO_WALK) {
                RandStream rs;
                rs_init(rs, seed, base + id, s);
                v = walk_step<true>(hdr, pool, in_v[a], rs, thr, rule);
                if (v != STOP_VERTEX) {
                    alive = true;
                    key = ((id / R) << vbits) | v;
                    ++steps;
                }
            }
        }
        wave_append(alive, key, ctl + 2, visits, capv);
        // compact survivors into the other list
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

inline uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n + TB - 1) / TB, 1), 1u << 20);
}

int resident_grid(const void* kernel) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, TB, 0) != hipSuccess || per_cu <= 0) per_cu = 4;
    return cus * per_cu;
}

int bits_for(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

}  // namespace

int launch_walk(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, uint64_t seed,
                uint32_t* paths, uint64_t* steps, uint32_t mode, hipStream_t st) {
    // per-call queue head and transition counter from a ring of slots, so that
    // walks on different streams do not share counters
    unsigned long long* ctl = g->d_ctl + CTL_WALK0 + 2 * (g->walk_slot++ % WALK_SLOTS);
    HIPCHK(hipMemsetAsync(ctl, 0, 16, st));
    phase_mark(g, st, true);
    if (nw == 0) {
        if (steps) HIPCHK(hipMemsetAsync(steps, 0, 8, st));
        return BINGO_OK;
    }
    if (mode == BINGO_WALK_PER_STEP) {
        const uint32_t grid = grid_for(nw);
        if (L == 0) {
            // only the start entries
            hipLaunchKernelGGL(k_deepwalk_persistent, dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts,
                               base, L, seed, paths, g->rule, ctl, g->d_err);
        }
        for (uint32_t s = 0; s < L; ++s)
            hipLaunchKernelGGL(k_deepwalk_step, dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts, base,
                               L, s, seed, paths, g->rule, ctl, g->d_err);
    } else {
        static int rgrid = 0;
        if (!rgrid) rgrid = resident_grid((const void*)k_deepwalk_persistent);
        const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)rgrid, (nw + TB - 1) / TB);
        hipLaunchKernelGGL(k_deepwalk_persistent, dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n, nw, starts,
                           base, L, seed, paths, g->rule, ctl, g->d_err);
    }
    phase_mark(g, st, false);
    if (steps) HIPCHK(hipMemcpyAsync(steps, ctl + 1, 8, hipMemcpyDeviceToDevice, st));
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

int run_ppr(bingo_graph* g, uint32_t nsrc, const uint32_t* sources, uint32_t R, uint32_t thr, uint32_t cap,
            uint64_t seed, uint64_t base, uint32_t mode, uint64_t* h_entries, uint64_t* h_steps, hipStream_t st) {
    const uint64_t nw = (uint64_t)nsrc * R;
    const int vbits = std::max(1, bits_for((uint64_t)g->n - 1));
    const int qbits = std::max(1, bits_for(nsrc));  // q < nsrc < 2^qbits, so the pad key is above every key
    if (vbits + qbits > 63) return BINGO_E_INVALID;
    // expected visits per walk without sinks: 1 + sum_{s=1..cap} (1-p)^s
    const double p = (double)thr / 4294967296.0;
    double ev = 1.0, a = 1.0;
    for (uint32_t s = 0; s < cap; ++s) { a *= (1.0 - p); ev += a; if (a < 1e-12) break; }
    uint64_t capv = (uint64_t)((double)nw * ev * 1.15) + 4096;
    capv = std::min<uint64_t>(capv, nw * ((uint64_t)cap + 1));
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    unsigned long long* ctl = g->d_ctl + 2;  // [2] queue, [3] transitions, [4] visits, [5..6] active counts
    for (int attempt = 0; attempt < 2; ++attempt) {
        const uint64_t act_bytes = mode == BINGO_WALK_PER_STEP ? 2 * (al(nw * 8) + al(nw * 4)) : 0;
        const size_t need = al(capv * 8) * 2 + act_bytes + 1024;
        char* ws = (char*)ws_get(g, need + std::max(sort_temp_bytes(capv, true), scan_temp_bytes(capv)) +
                                        al(capv * 4) + al(capv * 8) * 2);
        if (!ws) return BINGO_E_OOM;
        uint64_t* visits = (uint64_t*)ws;  ws += al(capv * 8);
        uint64_t* sorted = (uint64_t*)ws;  ws += al(capv * 8);
        char* act = ws;                    ws += act_bytes;
        uint32_t* head = (uint32_t*)ws;    ws += al(capv * 4);
        uint64_t* idx = (uint64_t*)ws;     ws += al(capv * 8);
        uint64_t* hpos = (uint64_t*)ws;    ws += al(capv * 8);
        void* tmp = ws;
        HIPCHK(hipMemsetAsync(ctl, 0, 40, st));
        HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
        phase_mark(g, st, true);
        if (mode == BINGO_WALK_PER_STEP) {
            uint64_t* idA = (uint64_t*)act;
            uint32_t* vA = (uint32_t*)(act + al(nw * 8));
            uint64_t* idB = (uint64_t*)(act + al(nw * 8) + al(nw * 4));
            uint32_t* vB = (uint32_t*)(act + 2 * al(nw * 8) + al(nw * 4));
            const uint32_t grid = grid_for(nw);
            hipLaunchKernelGGL(k_ppr_start, dim3(grid), dim3(TB), 0, st, g->n, nsrc, sources, R, vbits, idA, vA, ctl,
                               visits, capv, g->d_err);
            for (uint32_t s = 0; s < cap; ++s) {
                const int in_slot = s & 1;
                hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, ctl + 3 + (in_slot ^ 1), 0ull);
                hipLaunchKernelGGL(k_ppr_step, dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, R, thr, s, seed, base,
                                   vbits, g->rule, in_slot ? idB : idA, in_slot ? vB : vA, in_slot ? idA : idB,
                                   in_slot ? vA : vB, ctl, in_slot, visits, capv);
            }
        } else {
            static int rgrid = 0;
            if (!rgrid) rgrid = resident_grid((const void*)k_ppr_persistent);
            const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)rgrid, (nw + TB - 1) / TB);
            hipLaunchKernelGGL(k_ppr_persistent, dim3(std::max<uint32_t>(grid, 1)), dim3(TB), 0, st, g->hdr, g->pool,
                               g->n, nsrc, sources, R, thr, cap, seed, base, vbits, g->rule, ctl, visits, capv,
                               g->d_err);
        }
        phase_mark(g, st, false);
        unsigned long long c[3];
        HIPCHK(hipMemcpyAsync(c, ctl + 1, 24, hipMemcpyDeviceToHost, st));
        uint32_t err = 0;
        HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (err) return err_to_code(err);
        const uint64_t N = c[1];
        if (N > capv) {  // more visits than the estimate: retry with the exact size
            capv = N;
            continue;
        }
        // histogram: sort (source, vertex) keys, then run-length encode
        sort_keys_u64(visits, sorted, N, vbits + qbits, tmp, st);
        hipLaunchKernelGGL(k_heads, dim3(grid_for(N)), dim3(TB), 0, st, sorted, N, head);
        scan_u32_to_u64(head, idx, N, tmp, ctl + 4, st);
        unsigned long long U = 0;
        HIPCHK(hipMemcpyAsync(&U, ctl + 4, 8, hipMemcpyDeviceToHost, st));
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
        if (g->ppr_off_cap < nsrc + 1 || !g->ppr_off) {
            hipFree(g->ppr_off);
            g->ppr_off_cap = nsrc + 1;
            if (hipMalloc(&g->ppr_off, (uint64_t)(nsrc + 1) * 8) != hipSuccess) {
                g->ppr_off = nullptr; g->ppr_off_cap = 0;
                return BINGO_E_OOM;
            }
        }
        hipLaunchKernelGGL(k_emit, dim3(grid_for(N)), dim3(TB), 0, st, sorted, N, head, idx, vbits, g->ppr_vtx, hpos,
                           g->ppr_off);
        hipLaunchKernelGGL(k_counts, dim3(grid_for(U)), dim3(TB), 0, st, hpos, (uint64_t)U, N, g->ppr_cnt,
                           g->ppr_off, nsrc);
        phase_mark(g, st, false);
        HIPCHK(hipStreamSynchronize(st));
        g->ppr_entries = U;
        g->ppr_nsrc = nsrc;
        if (h_entries) *h_entries = U;
        if (h_steps) *h_steps = c[0];
        return BINGO_OK;
    }
    return BINGO_E_CAPACITY;
}

// node2vec.hip -- second-order walks (Sec. 2.2, Eq. node2vec) by rejection on
// the first-order radix-group sampler, the approach the paper adopts from
// KnightKing (Sec. 8): at u, coming from w, propose v with the first-order
// step and accept it with probability f(w, v) / max(1/p, 1, 1/q), where
// f = 1/p for v = w, 1 when w has an edge to v, 1/q otherwise.
//
// Stream layout: proposal t of step s of walk id draws its first-order step
// from (seed, id, s) starting at block t * 2^16 (proposal 0 is exactly the
// DeepWalk step), and its acceptance word is word 0 of block t * 2^16 + 0xFFFF,
// so the result does not depend on how many words a proposal over-draws
// (dense speculation).  Acceptance is the integer test word < thr_c, with
// thr_c = 2^32 (no draw) for the largest factor.
//
// "w has an edge to v" is a search (interpolation, then bisection) in a
// per-vertex sorted copy of the destinations, rebuilt from the adjacency (one
// global radix sort of (vertex, dst) keys) at the first node2vec call after the
// graph changed.
#include "dev.h"
#include "step.h"
#include <math.h>
#include <algorithm>

namespace {

constexpr int TB = 256;
constexpr uint32_t MAX_PROPOSALS = 1u << 15;
constexpr uint32_t ACCEPT_BLOCK = 0xFFFFu;

inline uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n + TB - 1) / TB, 1), 1u << 20);
}

__global__ void k_n2v_deg(const uint32_t* __restrict__ hdr, uint32_t n, uint32_t* __restrict__ deg) {
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (uint64_t)gridDim.x * blockDim.x)
        deg[u] = hdr[u * HDR_WORDS + H_DEG];
}

// (u << 32 | dst) for every live edge, one wave per vertex
__global__ void __launch_bounds__(TB) k_n2v_keys(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                 uint32_t n, const uint64_t* __restrict__ off,
                                                 uint64_t* __restrict__ keys) {
    const uint32_t lane = lane_id();
    for (uint64_t u = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < n;
         u += ((uint64_t)gridDim.x * blockDim.x) >> 6) {
        const uint32_t* h = hdr + u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        const uint64_t adj = hdr_adj(h);
        const uint64_t o = off[u];
        for (uint32_t i = lane; i < d; i += 64) keys[o + i] = (u << 32) | pool[adj + 2ull * i];
    }
}

__global__ void k_n2v_low(const uint64_t* __restrict__ keys, uint64_t m, uint32_t* __restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)keys[i];
}

// Membership of v in w's sorted destinations.  Vertex ids are a seeded
// permutation, so a vertex's destinations spread over the id range and the
// position of v is well guessed from its value between two known entries
// (interpolation: about log log d probes instead of log d); at most four
// guesses, then bisection.  Invariant: nidx[L] = a < v < b = nidx[H], v can only
// sit strictly between L and H.
__device__ __forceinline__ bool has_edge(const uint32_t* __restrict__ nidx, const uint64_t* __restrict__ off,
                                         uint32_t w, uint32_t v) {
    const uint64_t lo = off[w], hi = off[w + 1];
    if (lo == hi) return false;
    uint64_t L = lo, H = hi - 1;
    uint32_t a = nidx[L], b = nidx[H];
    if (v <= a) return v == a;
    if (v >= b) return v == b;
    for (int it = 0; it < 4 && H - L > 16; ++it) {
        const uint64_t inner = H - L - 1;  // candidate positions L+1 .. H-1
        uint64_t g = L + 1 + ((uint64_t)(v - a) * inner) / (uint64_t)(b - a);
        if (g > H - 1) g = H - 1;
        const uint32_t x = nidx[g];
        if (x == v) return true;
        if (x < v) { L = g; a = x; } else { H = g; b = x; }
    }
    uint64_t l = L + 1, h = H;  // bisection over [L+1, H)
    while (l < h) {
        const uint64_t mid = (l + h) >> 1;
        if (nidx[mid] < v) l = mid + 1; else h = mid;
    }
    return l < H && nidx[l] == v;
}

// One lane per walk from the chunked device queue (as the DeepWalk kernel); in
// every iteration a lane makes one proposal, so a rejected lane retries while
// the others move on.  ctl[0] queue head, ctl[1] transitions, ctl[2] proposals.
template <int SPEC, int MODE>
__global__ void __launch_bounds__(TB) k_node2vec(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                 const uint32_t* __restrict__ nidx,
                                                 const uint64_t* __restrict__ noff, uint32_t n, uint64_t nw,
                                                 const uint32_t* __restrict__ starts, uint64_t base, uint32_t L,
                                                 uint64_t seed, uint32_t thr0, uint32_t thr1, uint32_t thr2,
                                                 uint32_t full, uint32_t* __restrict__ paths, GroupRule rule,
                                                 unsigned long long* __restrict__ ctl, uint32_t* __restrict__ err,
                                                 uint32_t qchunk) {
    WaveQueue wq;
    wq.chunk = qchunk;
    uint64_t j = NO_WALK, steps = 0, props = 0;
    uint32_t u = 0, prev = STOP_VERTEX, s = 0, t = 0;
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
                prev = STOP_VERTEX;
                s = 0;
                t = 0;
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
        if (j != NO_WALK) {
            const uint64_t id = base + j;
            RandStream rs;
            rs_init_blk(rs, seed, id, s, t << 16);
            uint32_t v = walk_step_body<SPEC, MODE>(hdr, pool, u, rs, rule);
            ++props;
            bool accept = true;
            if (v != STOP_VERTEX && prev != STOP_VERTEX) {
                const uint32_t c = v == prev ? 0u : (has_edge(nidx, noff, prev, v) ? 1u : 2u);
                if (!((full >> c) & 1u)) {
                    uint32_t a0, a1, a2, a3;
                    philox_block((uint32_t)id, (uint32_t)(id >> 32), s, (t << 16) | ACCEPT_BLOCK, (uint32_t)seed,
                                 (uint32_t)(seed >> 32), a0, a1, a2, a3);
                    accept = a0 < (c == 0 ? thr0 : (c == 1 ? thr1 : thr2));
                }
            }
            if (!accept && ++t >= MAX_PROPOSALS) {
                v = STOP_VERTEX;
                accept = true;
            }
            if (accept) {
                if (v == STOP_VERTEX) {
                    for (uint32_t x = s + 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                } else {
                    row[s + 1] = v;
                    prev = u;
                    u = v;
                    ++s;
                    t = 0;
                    ++steps;
                    if (s == L) j = NO_WALK;
                }
            }
        }
    }
    wave_add_u64(ctl + 1, steps);
    wave_add_u64(ctl + 2, props);
}

int resident_blocks(const void* kernel) {
    int dev = 0, cus = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, TB, 0) != hipSuccess || per <= 0) per = 4;
    return std::max(cus, 1) * per;
}

int build_index(bingo_graph* g, hipStream_t st) {
    const uint32_t n = g->n;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    if (!g->n2v_off) {
        if (hipMalloc(&g->n2v_off, ((uint64_t)n + 1) * 8) != hipSuccess) { g->n2v_off = nullptr; return BINGO_E_OOM; }
    }
    char* w = (char*)ws_get(g, al((uint64_t)n * 4) + scan_temp_bytes((uint64_t)n + 1) + 512);
    if (!w) return BINGO_E_OOM;
    uint32_t* deg = (uint32_t*)w;
    void* tmp = w + al((uint64_t)n * 4);
    unsigned long long* tot = g->d_ctl + CTL_N2V + 3;
    hipLaunchKernelGGL(k_n2v_deg, dim3(grid_for(n)), dim3(TB), 0, st, g->hdr, n, deg);
    scan_u32_to_u64(deg, g->n2v_off, n, tmp, tot, st);
    unsigned long long m = 0;
    HIPCHK(hipMemcpyAsync(&m, tot, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(g->n2v_off + n, tot, 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    if (m > g->n2v_cap || !g->n2v_idx) {
        hipFree(g->n2v_idx);
        g->n2v_cap = std::max<uint64_t>(m, 1024) + m / 8;
        if (hipMalloc(&g->n2v_idx, g->n2v_cap * 4) != hipSuccess) {
            g->n2v_idx = nullptr;
            g->n2v_cap = 0;
            return BINGO_E_OOM;
        }
    }
    if (m) {
        const int vb = std::max(1, (int)(64 - __builtin_clzll((uint64_t)n - 1 | 1)));
        char* w2 = (char*)ws_get(g, 2 * al(m * 8) + sort_temp_bytes(m, true) + 512);
        if (!w2) return BINGO_E_OOM;
        uint64_t* keys = (uint64_t*)w2;
        uint64_t* sorted = (uint64_t*)(w2 + al(m * 8));
        void* stmp = w2 + 2 * al(m * 8);
        const uint32_t kgrid = (uint32_t)std::min<uint64_t>(((uint64_t)n * 64 + TB - 1) / TB, 1u << 16);
        hipLaunchKernelGGL(k_n2v_keys, dim3(kgrid), dim3(TB), 0, st, g->hdr, g->pool, n, g->n2v_off, keys);
        sort_keys_u64(keys, sorted, m, 32 + vb, stmp, st);
        hipLaunchKernelGGL(k_n2v_low, dim3(grid_for(m)), dim3(TB), 0, st, sorted, m, g->n2v_idx);
    }
    HIPCHK(hipGetLastError());
    g->n2v_version = g->version;
    return BINGO_OK;
}

template <int SPEC, int MODE>
void launch_n2v(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, uint64_t seed,
                const uint32_t thr[3], uint32_t full, uint32_t* paths, unsigned long long* ctl, hipStream_t st) {
    const int rg = resident_blocks((const void*)k_node2vec<SPEC, MODE>);
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)rg, (nw + TB - 1) / TB));
    hipLaunchKernelGGL((k_node2vec<SPEC, MODE>), dim3(grid), dim3(TB), 0, st, g->hdr, g->pool, g->n2v_idx, g->n2v_off,
                       g->n, nw, starts, base, L, seed, thr[0], thr[1], thr[2], full, paths, g->rule, ctl, g->d_err,
                       g->queue_chunk);
}

}  // namespace

// Acceptance thresholds of the three distance classes (index 0: v = w, 1: edge
// w -> v, 2: otherwise): bit c of *full set when f_c is the largest factor.
static int node2vec_thresholds(double p, double q, uint32_t thr[3], uint32_t* full) {
    if (!(p > 0.0) || !(q > 0.0) || !std::isfinite(p) || !std::isfinite(q)) return BINGO_E_INVALID;
    const double f[3] = {1.0 / p, 1.0, 1.0 / q};
    const double fmax = std::max(f[0], std::max(f[1], f[2]));
    *full = 0;
    for (int c = 0; c < 3; ++c) {
        if (f[c] == fmax) {
            *full |= 1u << c;
            thr[c] = 0;
        } else {
            thr[c] = (uint32_t)((f[c] / fmax) * 4294967296.0);
        }
    }
    return BINGO_OK;
}

int run_node2vec(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, double p, double q,
                 uint64_t seed, uint32_t* paths, uint64_t* d_counts, hipStream_t st) {
    uint32_t thr[3], full = 0;
    if (node2vec_thresholds(p, q, thr, &full) != BINGO_OK) return BINGO_E_INVALID;
    phase_mark(g, st, true);
    if (g->n2v_version != g->version || !g->n2v_off) {
        const int rc = build_index(g, st);
        if (rc != BINGO_OK) return rc;
    }
    phase_mark(g, st, false);
    unsigned long long* ctl = g->d_ctl + CTL_N2V;
    HIPCHK(hipMemsetAsync(ctl, 0, 24, st));
    if (nw) {
        switch (g->dense_spec) {
            case 1: (walk_mode(g) == 1 ? launch_n2v<1, 1> : walk_mode(g) == 2 ? launch_n2v<1, 2> : launch_n2v<1, 0>)(g, nw, starts, base, L, seed, thr, full, paths, ctl, st); break;
            case 4: (walk_mode(g) == 1 ? launch_n2v<4, 1> : walk_mode(g) == 2 ? launch_n2v<4, 2> : launch_n2v<4, 0>)(g, nw, starts, base, L, seed, thr, full, paths, ctl, st); break;
            default: (walk_mode(g) == 1 ? launch_n2v<2, 1> : walk_mode(g) == 2 ? launch_n2v<2, 2> : launch_n2v<2, 0>)(g, nw, starts, base, L, seed, thr, full, paths, ctl, st); break;
        }
    }
    phase_mark(g, st, false);
    if (d_counts) HIPCHK(hipMemcpyAsync(d_counts, ctl + 1, 16, hipMemcpyDeviceToDevice, st));
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

// locate.hip -- building, sizing and checking the edge locator (locate.h).
// The batch pipeline (update.hip) keeps it in step with the adjacency; the
// streaming path marks it stale and the next batch that uses it rebuilds it.
#include "locate.h"
#include <stdio.h>
#include <algorithm>

namespace {

constexpr int WB = 256;

__global__ void k_loc_clear(uint64_t* __restrict__ tab, uint64_t cap) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x)
        *reinterpret_cast<ulonglong2*>(tab + 2 * i) = make_ulonglong2(LOC_EMPTY, 0ull);
}

// One wave per vertex: every live edge claims a slot.  cnt[0] += edges, cnt[1] += failed claims.
__global__ void __launch_bounds__(WB) k_loc_build(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                  uint32_t n, LocView L, unsigned long long* __restrict__ cnt) {
    const uint32_t lane = lane_id();
    uint32_t edges = 0, fail = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * (WB / 64) + (threadIdx.x >> 6); u < n; u += (uint64_t)gridDim.x * (WB / 64)) {
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        const uint64_t adj = hdr_adj(h);
        for (uint32_t i = lane; i < d; i += 64) {
            ++edges;
            if (!loc_claim(L, loc_key((uint32_t)u, pool[adj + 2ull * i]), i)) ++fail;
        }
    }
    edges = loc_wave_sum(edges);
    fail = loc_wave_sum(fail);
    if (lane == 0) {
        atomicAdd(cnt, (unsigned long long)edges);
        if (fail) atomicAdd(cnt + 1, (unsigned long long)fail);
    }
}

// Consistency: every live edge finds its own slot (cnt[0] counts those that do not),
// and the table holds no other live slot (cnt[1] counts live slots).
__global__ void __launch_bounds__(WB) k_loc_check_edges(const uint32_t* __restrict__ hdr,
                                                        const uint32_t* __restrict__ pool, uint32_t n, LocView L,
                                                        unsigned long long* __restrict__ cnt) {
    const uint32_t lane = lane_id();
    uint32_t bad = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * (WB / 64) + (threadIdx.x >> 6); u < n; u += (uint64_t)gridDim.x * (WB / 64)) {
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        const uint64_t adj = hdr_adj(h);
        for (uint32_t i = lane; i < d; i += 64)
            if (loc_find(L, loc_key((uint32_t)u, pool[adj + 2ull * i]), i) == LOC_EMPTY) ++bad;
    }
    bad = loc_wave_sum(bad);
    if (lane == 0 && bad) atomicAdd(cnt, (unsigned long long)bad);
}

__global__ void k_loc_count_live(LocView L, unsigned long long* __restrict__ cnt) {
    uint32_t live = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= L.mask; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = L.tab[2 * i];
        if (k != LOC_EMPTY && k != LOC_TOMB) ++live;
    }
    live = loc_wave_sum(live);
    if (lane_id() == 0 && live) atomicAdd(cnt + 1, (unsigned long long)live);
}

uint32_t grid_of(uint64_t items, uint32_t per_block) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((items + per_block - 1) / per_block, 1u << 16));
}

// Rebuild into a table of `cap` slots (reallocated when the capacity changes).
bool loc_build(bingo_graph* g, uint64_t cap, hipStream_t st) {
    g->loc_valid = false;
    if (cap != g->loc_cap || !g->loc_tab) {
        // the captured update graphs hold the old table's address
        update_drop_graphs(g);
        hipFree(g->loc_tab);
        g->loc_tab = nullptr;
        g->loc_cap = 0;
        if (hipMalloc(&g->loc_tab, cap * 16) != hipSuccess) {
            (void)hipGetLastError();
            g->loc_tab = nullptr;
            return false;
        }
        g->loc_cap = cap;
    }
    const LocView L{g->loc_tab, cap - 1};
    unsigned long long* cnt = g->d_ctl + CTL_LOC;
    if (hipMemsetAsync(cnt, 0, 16, st) != hipSuccess) return false;
    hipLaunchKernelGGL(k_loc_clear, dim3(grid_of(cap, 256)), dim3(256), 0, st, g->loc_tab, cap);
    hipLaunchKernelGGL(k_loc_build, dim3(grid_of(g->n, WB / 64)), dim3(WB), 0, st, (const uint32_t*)g->hdr,
                       (const uint32_t*)g->pool, g->n, L, cnt);
    unsigned long long c[2] = {0, 0};
    if (hipMemcpyAsync(c, cnt, 16, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return false;
    if (c[1]) return false;  // unreachable: the capacity is at least 1.6 times the edges
    g->loc_live = g->loc_used = c[0];
    g->loc_valid = true;
    return true;
}

uint64_t pow2_ge(uint64_t x) {
    uint64_t c = 1ull << 16;
    while (c < x) c <<= 1;
    return c;
}

// live edges of the structure (one pass over the headers)
__global__ void k_loc_edges(const uint32_t* __restrict__ hdr, uint32_t n, unsigned long long* __restrict__ cnt) {
    uint64_t s = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (uint64_t)gridDim.x * blockDim.x)
        s += hdr[(size_t)u * HDR_WORDS + H_DEG];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane_id() == 0 && s) atomicAdd(cnt, (unsigned long long)s);
}

}  // namespace

LocView locator_view(const bingo_graph* g) {
    if (!g->update_locate || !g->loc_valid) return LocView{nullptr, 0};
    return LocView{g->loc_tab, g->loc_cap - 1};
}

bool locator_prepare(bingo_graph* g, uint64_t n_ins, hipStream_t st) {
    if (!g->update_locate || g->radix_base != 2) return false;
    // load limits: at most 0.8 of the slots taken (live + TOMB) after the batch's claims; a
    // rebuild sizes the table to at least 1.6 times the live edges plus the batch
    if (g->loc_valid && (double)(g->loc_used + n_ins) <= 0.8 * (double)g->loc_cap) return true;
    uint64_t live = g->loc_live;
    if (!g->loc_valid) {
        unsigned long long* cnt = g->d_ctl + CTL_LOC;
        unsigned long long c = 0;
        if (hipMemsetAsync(cnt, 0, 8, st) != hipSuccess) return false;
        hipLaunchKernelGGL(k_loc_edges, dim3(grid_of(g->n, 256)), dim3(256), 0, st, (const uint32_t*)g->hdr, g->n, cnt);
        if (hipMemcpyAsync(&c, cnt, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return false;
        live = c;
    }
    const uint64_t want = pow2_ge((uint64_t)(1.6 * (double)(live + n_ins)) + 1);
    // keep a larger table that still fits the limit rather than shrinking it
    const uint64_t cap = (g->loc_cap >= want && (double)(live + n_ins) <= 0.5 * (double)g->loc_cap) ? g->loc_cap : want;
    return loc_build(g, cap, st);
}

void locator_after_batch(bingo_graph* g, uint64_t kills, uint64_t claims, uint64_t fresh, uint64_t bad) {
    if (!g->loc_valid) return;
    if (bad) {
        fprintf(stderr, "libbingo: edge locator out of step (%llu lookups failed); it will be rebuilt\n",
                (unsigned long long)bad);
        g->loc_valid = false;
        return;
    }
    g->loc_live = g->loc_live + claims - kills;
    g->loc_used += fresh;
}

void locator_invalidate(bingo_graph* g) { g->loc_valid = false; }

void locator_release(bingo_graph* g) {
    hipFree(g->loc_tab);
    g->loc_tab = nullptr;
    g->loc_cap = g->loc_live = g->loc_used = 0;
    g->loc_valid = false;
}

extern "C" int bingo_check_locator(bingo_graph* g, uint64_t* h_bad, uint64_t* h_live, void* stream) {
    if (!g || !h_bad || g->radix_base != 2) return BINGO_E_INVALID;
    if (!g->loc_valid) return BINGO_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const LocView L{g->loc_tab, g->loc_cap - 1};
    unsigned long long* cnt = g->d_ctl + CTL_LOC;
    HIPCHK(hipMemsetAsync(cnt, 0, 16, st));
    hipLaunchKernelGGL(k_loc_check_edges, dim3(grid_of(g->n, WB / 64)), dim3(WB), 0, st, (const uint32_t*)g->hdr,
                       (const uint32_t*)g->pool, g->n, L, cnt);
    hipLaunchKernelGGL(k_loc_count_live, dim3(grid_of(g->loc_cap, 256)), dim3(256), 0, st, L, cnt);
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, cnt, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // edges without their slot, plus live slots beyond the edges (or edges beyond the live slots)
    unsigned long long edges = 0;
    {
        HIPCHK(hipMemsetAsync(cnt, 0, 8, st));
        hipLaunchKernelGGL(k_loc_edges, dim3(grid_of(g->n, 256)), dim3(256), 0, st, (const uint32_t*)g->hdr, g->n, cnt);
        HIPCHK(hipMemcpyAsync(&edges, cnt, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    *h_bad = c[0] + (c[1] > edges ? c[1] - edges : edges - c[1]) + (c[1] != g->loc_live ? 1 : 0);
    if (h_live) *h_live = c[1];
    return BINGO_OK;
}

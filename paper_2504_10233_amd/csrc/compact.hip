// compact.hip -- pool compaction.  Every live block (a vertex's adjacency block
// at its capacity, one list block per listed group at its capacity; Sec. 5.2
// dynamic arrays; each with its group index, Sec. 4.2; the reduced list S(u),
// Sec. 5.1) is copied into a fresh arena in vertex order and the headers
// take the new offsets; the blocks that earlier batches replaced by larger ones
// (the pool's garbage) stay behind.  Block sizes and contents do not change, so
// neither does the canonical dump nor any walk: only where blocks live.
#include "dev.h"
#include <algorithm>

namespace {

constexpr int WB = 256;

// Lane k < 32: the block words (list and index) of group k if it is listed;
// lane 32: the S(u) block; other lanes 0.
__device__ __forceinline__ uint64_t lane_list_words(const uint32_t* __restrict__ h, uint32_t d, uint32_t mask,
                                                    uint32_t lane, GroupRule rule) {
    if (lane == 32) return h[H_SCAP];
    if (lane >= 32 || !((mask >> lane) & 1u)) return 0ull;
    const uint32_t c = slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane);
    const uint32_t t = group_type(c, d, rule);
    if (!type_listed(t)) return 0ull;
    const uint32_t lcap = 1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu);
    return list_block_words(lcap, index_cap_for(t, h[H_ACAP], h[H_SCAP]));
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Pool words vertex u holds.  One wave per vertex.
__global__ void __launch_bounds__(WB) k_cmp_size(const uint32_t* __restrict__ hdr, uint32_t n, GroupRule rule,
                                                 uint64_t* __restrict__ need) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint64_t u = (uint64_t)blockIdx.x * (WB / 64) + wave; u < n; u += (uint64_t)gridDim.x * (WB / 64)) {
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint64_t w = wave_sum64(lane_list_words(h, h[H_DEG], h[H_MASK], lane, rule));
        if (lane == 0) need[u] = w + adj_block_words(h[H_ACAP]);
    }
}

// Copy words [0, words) of src to dst, 16 bytes per lane and step (both 32-byte aligned).
__device__ __forceinline__ void wave_copy(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, uint64_t words,
                                          uint32_t lane) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* t = reinterpret_cast<uint4*>(dst);
    for (uint64_t i = lane; i < words / 4; i += 64) t[i] = s[i];
}

// Vertex u's blocks from the old arena to the new one at off[u]: the adjacency
// block first, then the list blocks (list and index) in ascending k, then the
// S(u) block; the header takes the new offsets.  One wave per vertex.
__global__ void __launch_bounds__(WB) k_cmp_copy(uint32_t* __restrict__ hdr, const uint32_t* __restrict__ src,
                                                 uint32_t* __restrict__ dst, uint32_t n, GroupRule rule,
                                                 const uint64_t* __restrict__ off) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint64_t u = (uint64_t)blockIdx.x * (WB / 64) + wave; u < n; u += (uint64_t)gridDim.x * (WB / 64)) {
        uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG], mask = h[H_MASK], cap = h[H_ACAP];
        const uint64_t adj = hdr_adj(h);
        const uint64_t lw = lane_list_words(h, d, mask, lane, rule);
        const uint32_t info = lane < 32 ? h[H_INFO + lane] : (lane == 32 ? h[H_SBLK] : 0u);
        uint64_t o = off[u];
        if (cap) {
            const uint64_t words = adj_block_words(cap);
            wave_copy(src + adj, dst + o, words, lane);
            if (lane == 0) {
                h[H_ADJLO] = (uint32_t)o;
                h[H_ADJHI] = adjhi_word(o, hdr_hi(h));
            }
            o += words;
        }
        // each listed group's new offset: exclusive prefix of the capacities over lanes
        uint64_t x = lw;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const uint64_t y = __shfl_up(x, s, 64);
            if (lane >= (uint32_t)s) x += y;
        }
        const uint64_t mine = o + (x - lw);
        for (uint64_t lm = __ballot(lw != 0); lm; lm &= lm - 1) {
            const int k = __ffsll((long long)lm) - 1;
            const uint64_t from = (uint64_t)__shfl(info, k, 64) * LIST_UNIT_WORDS;
            const uint64_t to = __shfl(mine, k, 64);
            wave_copy(src + from, dst + to, __shfl(lw, k, 64), lane);
        }
        if (lw && lane < 32) h[H_INFO + lane] = (uint32_t)(mine / LIST_UNIT_WORDS);
        if (lw && lane == 32) h[H_SBLK] = (uint32_t)(mine / LIST_UNIT_WORDS);
    }
}

__global__ void k_cmp_ctl(unsigned long long* __restrict__ ctl, const unsigned long long* __restrict__ total) {
    ctl[0] = *total;  // words in use
    ctl[1] = 0;       // garbage
}

uint32_t vertex_grid(uint32_t n) { return (uint32_t)std::min<uint64_t>(((uint64_t)n + 3) / 4, 4096); }

}  // namespace

int compact_pool(bingo_graph* g, uint64_t pool_words, hipStream_t st) {
    const uint32_t n = g->n;
    if (pool_words == 0) pool_words = g->pool_words;
    if (pool_words > (1ull << 35)) return BINGO_E_INVALID;  // list offsets are 32-bit counts of 32-byte units
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    char* ws = (char*)ws_get(g, al(((uint64_t)n + 1) * 8) * 2 + al(8) + scan_temp_bytes((uint64_t)n + 1) + 256);
    if (!ws) return BINGO_E_OOM;
    uint64_t* need = (uint64_t*)ws;                       ws += al(((uint64_t)n + 1) * 8);
    uint64_t* off = (uint64_t*)ws;                        ws += al(((uint64_t)n + 1) * 8);
    unsigned long long* total = (unsigned long long*)ws;  ws += al(8);
    void* tmp = ws;
    hipLaunchKernelGGL(k_cmp_size, dim3(vertex_grid(n)), dim3(WB), 0, st, (const uint32_t*)g->hdr, n, g->rule, need);
    scan_u64(need, off, n, tmp, total, st);
    unsigned long long live = 0;
    HIPCHK(hipMemcpyAsync(&live, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (live > pool_words) return BINGO_E_OOM;
    uint32_t* fresh = nullptr;
    if (hipMalloc(&fresh, pool_words * 4) != hipSuccess) {
        (void)hipGetLastError();
        return BINGO_E_OOM;
    }
    hipLaunchKernelGGL(k_cmp_copy, dim3(vertex_grid(n)), dim3(WB), 0, st, g->hdr, (const uint32_t*)g->pool, fresh, n,
                       g->rule, (const uint64_t*)off);
    hipLaunchKernelGGL(k_cmp_ctl, dim3(1), dim3(1), 0, st, g->d_ctl, (const unsigned long long*)total);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(g->pool));
    g->pool = fresh;
    g->pool_words = pool_words;
    // captured update graphs hold the old arena's address
    update_drop_graphs(g);
    return BINGO_OK;
}

// export.hip -- canonical dump of the structure (the layout is defined in
// bingo.h) and memory statistics, including the paper's memory model with and
// without group adaption (Sec. 4.4 space complexity, Sec. 6.2).
#include "dev.h"
#include <stdio.h>
#include <algorithm>
#include <vector>

namespace {

constexpr int WB = 256;

__device__ __forceinline__ uint32_t stored_words(uint32_t t, uint32_t c) {
    return t == GT_ONE ? 1u : (type_listed(t) ? c : 0u);
}

__global__ void k_dump_size(const uint32_t* __restrict__ hdr, uint32_t u0, uint32_t u1, GroupRule rule,
                            uint64_t* __restrict__ sz) {
    const uint32_t u = u0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= u1) return;
    const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    const uint32_t d = h[H_DEG], mask = h[H_MASK], onem = h[H_ONEMASK], hi = hdr_hi(h);
    uint64_t s = 3 + 3ull * d;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
        const int k = __ffs(mm) - 1;
        const uint32_t c = slot_count(hdr_slot(h, k, hi), onem, k);
        s += 3 + stored_words(group_type(c, d, rule), c);
    }
    sz[u - u0] = s;
}

__global__ void __launch_bounds__(WB) k_dump_write(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                   uint32_t u0, uint32_t u1, GroupRule rule,
                                                   const uint64_t* __restrict__ off, uint32_t* __restrict__ out) {
    const uint32_t u = u0 + blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= u1) return;
    const uint32_t lane = lane_id();
    const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    const uint32_t d = h[H_DEG], mask = h[H_MASK];
    uint32_t* o = out + off[u - u0];
    if (lane == 0) { o[0] = d; o[1] = h[H_NSEQ]; o[2] = mask; }
    const uint64_t adj = hdr_adj(h);
    const uint32_t cap = h[H_ACAP];
    const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + adj);
    const uint32_t* seqs = pool + adj + 2ull * cap;
    for (uint32_t i = lane; i < d; i += 64) {
        const uint64_t e = edges[i];
        o[3 + 3 * (uint64_t)i] = (uint32_t)e;
        o[4 + 3 * (uint64_t)i] = (uint32_t)(e >> 32);
        o[5 + 3 * (uint64_t)i] = seqs[i];
    }
    // group records in ascending k: lane k computes its record's size and start
    const bool ne = lane < 32 && ((mask >> lane) & 1u);
    const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane) : 0u;
    const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
    const uint64_t sz = ne ? 3ull + stored_words(t, c) : 0ull;
    uint64_t x = sz;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint64_t y = __shfl_up(x, s, 64);
        if (lane >= (uint32_t)s) x += y;
    }
    const uint64_t my = 3 + 3ull * d + (x - sz);
    const uint32_t info = ne ? h[H_INFO + lane] : 0u;
    if (ne) {
        o[my] = lane;
        o[my + 1] = t;
        o[my + 2] = c;
        if (t == GT_ONE) o[my + 3] = info;
    }
    uint32_t lm = (uint32_t)(__ballot(ne && type_listed(t)) & 0xFFFFFFFFull);
    while (lm) {
        const int k = __ffs(lm) - 1;
        lm &= lm - 1;
        const uint64_t dst0 = __shfl(my, k, 64) + 3;
        const uint32_t ck = __shfl(c, k, 64);
        const uint64_t src0 = (uint64_t)__shfl(info, k, 64) * LIST_UNIT_WORDS;
        for (uint32_t i = lane; i < ck; i += 64) o[dst0 + i] = pool[src0 + i];
    }
}

// ---------------------------------------------------------------------------
// Group index dump (Sec. 4.2 inverted index, Sec. 5.1 reduced list S(u)), per
// vertex u: |S|, S in stored order; then for each listed group k ascending: k,
// then for a regular group its index read at the list's members in list order
// (index[L[p]], p < c), for a sparse group, for every s < |S|, the position of
// S[s] in the list, or 0xFFFFFFFF when S[s] is not a member (an index entry
// is a member's position when it is below c and the list holds S[s] there).
// ---------------------------------------------------------------------------
__global__ void k_idx_size(const uint32_t* __restrict__ hdr, uint32_t u0, uint32_t u1, GroupRule rule,
                           uint64_t* __restrict__ sz) {
    const uint32_t u = u0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= u1) return;
    const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    const uint32_t d = h[H_DEG], mask = h[H_MASK], onem = h[H_ONEMASK], hi = hdr_hi(h);
    const uint32_t slen = h[H_SCAP] ? h[H_SLEN] : 0u;
    uint64_t s = 1 + (uint64_t)slen;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
        const int k = __ffs(mm) - 1;
        const uint32_t c = slot_count(hdr_slot(h, k, hi), onem, k);
        const uint32_t t = group_type(c, d, rule);
        if (t == GT_REGULAR) s += 1 + (uint64_t)c;
        else if (t == GT_SPARSE) s += 1 + (uint64_t)slen;
    }
    sz[u - u0] = s;
}

__global__ void __launch_bounds__(WB) k_idx_write(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                  uint32_t u0, uint32_t u1, GroupRule rule,
                                                  const uint64_t* __restrict__ off, uint32_t* __restrict__ out) {
    const uint32_t u = u0 + blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= u1) return;
    const uint32_t lane = lane_id();
    const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    const uint32_t d = h[H_DEG], mask = h[H_MASK];
    const uint32_t slen = h[H_SCAP] ? h[H_SLEN] : 0u;
    const uint32_t* S = pool + (uint64_t)h[H_SBLK] * LIST_UNIT_WORDS;
    uint32_t* o = out + off[u - u0];
    if (lane == 0) o[0] = slen;
    for (uint32_t i = lane; i < slen; i += 64) o[1 + i] = S[i];
    const bool ne = lane < 32 && ((mask >> lane) & 1u);
    const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane) : 0u;
    const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
    const uint64_t sz = t == GT_REGULAR ? 1ull + c : (t == GT_SPARSE ? 1ull + slen : 0ull);
    uint64_t x = sz;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint64_t y = __shfl_up(x, s, 64);
        if (lane >= (uint32_t)s) x += y;
    }
    const uint64_t my = 1 + (uint64_t)slen + (x - sz);
    if (sz) o[my] = lane;
    const uint32_t info = ne ? h[H_INFO + lane] : 0u;
    const uint32_t lcap = ne ? (1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu)) : 0u;
    for (uint32_t lm = (uint32_t)(__ballot(sz != 0) & 0xFFFFFFFFull); lm; lm &= lm - 1) {
        const int k = __ffs(lm) - 1;
        const uint64_t dst0 = __shfl(my, k, 64) + 1;
        const uint32_t ck = __shfl(c, k, 64);
        const uint32_t* L = pool + (uint64_t)__shfl(info, k, 64) * LIST_UNIT_WORDS;
        const uint32_t* I = L + __shfl(lcap, k, 64);
        if (__shfl(t, k, 64) == GT_REGULAR) {
            for (uint32_t p = lane; p < ck; p += 64) o[dst0 + p] = I[L[p]];
        } else {
            for (uint32_t s = lane; s < slen; s += 64) {
                const uint32_t q = I[s];
                o[dst0 + s] = (q < ck && L[q] == S[s]) ? q : 0xFFFFFFFFu;
            }
        }
    }
}

// memory statistics: [0] groups by type (5), [5] list live bytes, [6] list reserved bytes,
// [10] adjacency reserved bytes, [11] GA model bytes, [12] BS model bytes, [13] edges,
// [14] index live bytes, [15] index reserved bytes
// Totals are kept per wave in registers over a grid-stride loop and reduced per
// block; one atomic per counter per block (per-vertex atomics on a dozen
// addresses would serialize in L2 over 10^7 vertices).
constexpr uint32_t MEM_GRID = 2048;
constexpr int MEM_CTRS = 16;  // [14] index live bytes, [15] index reserved bytes

__global__ void __launch_bounds__(WB) k_mem(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                            uint32_t n, GroupRule rule, unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long red[WB / 64][MEM_CTRS];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint64_t tot[MEM_CTRS];  // identical in every lane of the wave
#pragma unroll
    for (int i = 0; i < MEM_CTRS; ++i) tot[i] = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * (WB / 64) + wave; u < n; u += (uint64_t)gridDim.x * (WB / 64)) {
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG], mask = h[H_MASK];
        const bool ne = lane < 32 && ((mask >> lane) & 1u);
        const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane) : 0u;
        const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
        const uint32_t capb = lane < 32 ? ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu) : 0u;
        const uint32_t smask = (uint32_t)(__ballot(ne && t == GT_SPARSE) & 0xFFFFFFFFull);
        // |S(u)|: edges in at least one sparse group
        uint64_t S = 0;
        if (smask) {
            const uint64_t adj = hdr_adj(h);
            const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + adj);
            for (uint32_t i0 = 0; i0 < d; i0 += 64) {
                const uint32_t i = i0 + lane;
                const bool in = i < d && (member_word((uint32_t)(edges[i] >> 32), rule.fbits) & smask);
                S += __popcll(__ballot(in));
            }
        }
        // stored index structures: a regular group's inverted index (d live entries in a block
        // of the adjacency capacity), a sparse group's index over S(u) (|S(u)| entries, capacity
        // of S(u)), and S(u) itself
        const uint32_t acap = h[H_ACAP], scap = h[H_SCAP], slen = scap ? h[H_SLEN] : 0u;
        uint64_t v[6] = {0, 0, 0, 0, 0, 0};  // live list, reserved list, ga, bs, live index, reserved index
        if (ne) {
            if (type_listed(t)) {
                v[0] = 4ull * c;
                v[1] = 4ull << capb;
                v[4] = t == GT_REGULAR ? 4ull * d : 4ull * slen;
                v[5] = list_block_words(1u << capb, index_cap_for(t, acap, scap)) * 4ull - (4ull << capb);
            }
            v[2] = t == GT_ONE ? 4ull : (t == GT_SPARSE ? 4ull * c + 4ull * S : (t == GT_REGULAR ? 4ull * (c + (uint64_t)d) : 0));
            v[3] = 4ull * (c + (uint64_t)d);
        }
        if (lane == 32) { v[4] = 4ull * slen; v[5] = 4ull * scap; }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o);
#pragma unroll
        for (int tt = 1; tt < 5; ++tt) tot[tt] += __popcll(__ballot(ne && t == (uint32_t)tt));
        tot[5] += v[0];
        tot[6] += v[1];
        tot[10] += 12ull * h[H_ACAP];
        tot[11] += v[2] + 4ull * S + 12ull * d;
        tot[12] += v[3] + 12ull * d;
        tot[13] += d;
        tot[14] += v[4];
        tot[15] += v[5];
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < MEM_CTRS; ++i) red[wave][i] = tot[i];
    __syncthreads();
    if (threadIdx.x < MEM_CTRS) {
        unsigned long long x = 0;
#pragma unroll
        for (int w = 0; w < WB / 64; ++w) x += red[w][threadIdx.x];
        if (x) atomicAdd(acc + threadIdx.x, x);
    }
}

}  // namespace

int export_graph(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
                 hipStream_t st) {
    if (u1 > g->n || u0 > u1) return BINGO_E_INVALID;
    const uint32_t nv = u1 - u0;
    if (nv == 0) { *h_len = 0; return BINGO_OK; }
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    char* ws = (char*)ws_get(g, 2 * al((uint64_t)nv * 8) + scan_temp_bytes(nv) + 512);
    if (!ws) return BINGO_E_OOM;
    uint64_t* sz = (uint64_t*)ws;
    uint64_t* off = (uint64_t*)(ws + al((uint64_t)nv * 8));
    unsigned long long* total = (unsigned long long*)(ws + 2 * al((uint64_t)nv * 8));
    void* tmp = ws + 2 * al((uint64_t)nv * 8) + 256;
    hipLaunchKernelGGL(k_dump_size, dim3((nv + 255) / 256), dim3(256), 0, st, g->hdr, u0, u1, g->rule, sz);
    scan_u64(sz, off, nv, tmp, total, st);
    unsigned long long T = 0;
    HIPCHK(hipMemcpyAsync(&T, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *h_len = T;
    if (!h_buf) return BINGO_OK;
    if (cap < T) return BINGO_E_CAPACITY;
    uint32_t* dbuf = nullptr;
    if (hipMalloc(&dbuf, std::max<uint64_t>(T, 1) * 4) != hipSuccess) return BINGO_E_OOM;
    hipLaunchKernelGGL(k_dump_write, dim3((nv + 3) / 4), dim3(WB), 0, st, g->hdr, g->pool, u0, u1, g->rule,
                       (const uint64_t*)off, dbuf);
    hipError_t e1 = hipMemcpyAsync(h_buf, dbuf, T * 4, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(dbuf);
    return (e1 == hipSuccess && e2 == hipSuccess) ? BINGO_OK : BINGO_E_HIP;
}

int export_index(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
                 hipStream_t st) {
    if (u1 > g->n || u0 > u1) return BINGO_E_INVALID;
    const uint32_t nv = u1 - u0;
    if (nv == 0) { *h_len = 0; return BINGO_OK; }
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    char* ws = (char*)ws_get(g, 2 * al((uint64_t)nv * 8) + scan_temp_bytes(nv) + 512);
    if (!ws) return BINGO_E_OOM;
    uint64_t* sz = (uint64_t*)ws;
    uint64_t* off = (uint64_t*)(ws + al((uint64_t)nv * 8));
    unsigned long long* total = (unsigned long long*)(ws + 2 * al((uint64_t)nv * 8));
    void* tmp = ws + 2 * al((uint64_t)nv * 8) + 256;
    hipLaunchKernelGGL(k_idx_size, dim3((nv + 255) / 256), dim3(256), 0, st, g->hdr, u0, u1, g->rule, sz);
    scan_u64(sz, off, nv, tmp, total, st);
    unsigned long long T = 0;
    HIPCHK(hipMemcpyAsync(&T, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *h_len = T;
    if (!h_buf) return BINGO_OK;
    if (cap < T) return BINGO_E_CAPACITY;
    uint32_t* dbuf = nullptr;
    if (hipMalloc(&dbuf, std::max<uint64_t>(T, 1) * 4) != hipSuccess) return BINGO_E_OOM;
    hipLaunchKernelGGL(k_idx_write, dim3((nv + 3) / 4), dim3(WB), 0, st, g->hdr, g->pool, u0, u1, g->rule,
                       (const uint64_t*)off, dbuf);
    hipError_t e1 = hipMemcpyAsync(h_buf, dbuf, T * 4, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(dbuf);
    return (e1 == hipSuccess && e2 == hipSuccess) ? BINGO_OK : BINGO_E_HIP;
}

int memory_stats(bingo_graph* g, bingo_mem_stats* out, hipStream_t st) {
    unsigned long long* acc = (unsigned long long*)ws_get(g, 16 * 8);
    if (!acc) return BINGO_E_OOM;
    HIPCHK(hipMemsetAsync(acc, 0, 16 * 8, st));
    hipLaunchKernelGGL(k_mem, dim3(std::min<uint32_t>(MEM_GRID, (g->n + 3) / 4)), dim3(WB), 0, st, g->hdr, g->pool, g->n,
                       g->rule, acc);
    unsigned long long a[16], ctl[2];
    HIPCHK(hipMemcpyAsync(a, acc, sizeof a, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out->vertices = g->n;
    out->edges = a[13];
    out->pool_bytes = g->pool_words * 4;
    out->pool_used_bytes = ctl[0] * 4;
    out->pool_garbage_bytes = ctl[1] * 4;
    out->header_bytes = (uint64_t)g->n * HDR_WORDS * 4;
    out->adjacency_bytes = 12ull * a[13];
    out->adjacency_reserved_bytes = a[10];
    out->list_bytes = a[5];
    out->list_reserved_bytes = a[6];
    for (int t = 0; t < 5; ++t) out->groups_by_type[t] = t ? a[t] : 0;
    out->model_ga_bytes = a[11];
    out->model_bs_bytes = a[12];
    out->alias_bytes = g->alias ? (uint64_t)g->n * ALIAS_ENTRIES * sizeof(uint4) : 0;
    out->index_bytes = a[14];
    out->index_reserved_bytes = a[15];
    out->locator_bytes = g->loc_tab ? g->loc_cap * 16 : 0;
    return BINGO_OK;
}

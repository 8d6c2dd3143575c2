// radix4.hip -- walks, canonical dump and memory statistics of the radix-base-4
// structure (Supplement S.2).  Every weight is read as base-4 digits; subgroup
// s = 3k + v - 1 (v = 1..3) holds the edges whose digit k is v and carries
// c_s v 4^k in total.  A step draws r = below64(W), takes the first subgroup
// in ascending s whose running total exceeds r (the group is chosen by its
// total and the subgroup inside it by c_s v, which is the same single scan),
// then a member: a one-element subgroup's destination from the header, a
// listed subgroup's list entry L_s[below32(c_s)], or for a dense subgroup
// i = below32(d) until digit k of w_i is v (Sec. 5.1 rejection).  The stream of
// a step is the Philox stream keyed by (seed, walk id, step), as for base 2.
#include "dev.h"
#include "step.h"
#include <algorithm>
#include <string.h>

namespace {

constexpr int TB4 = 256;

// One round of SPEC dense attempts: indices come from the stream alone, so the
// loads are issued together; the first accepting attempt in stream order is
// the sequential result.
template <int SPEC>
__device__ __forceinline__ uint32_t dense_round4(const uint64_t* __restrict__ edges, uint32_t d, uint32_t k,
                                                 uint32_t v, RandStream& rs) {
    uint64_t e[SPEC];
#pragma unroll
    for (int a = 0; a < SPEC; ++a) e[a] = edges[rs_below32(rs, d)];
    uint32_t out = PENDING;
#pragma unroll
    for (int a = SPEC - 1; a >= 0; --a)
        if (r4_digit((uint32_t)(e[a] >> 32), k) == v) out = (uint32_t)e[a];
    return out;
}

template <int SPEC>
__device__ __forceinline__ uint32_t step4(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                          uint32_t u, RandStream& rs, GroupRule rule) {
    const uint32_t* h = hdr + (size_t)u * H4_WORDS;
    const uint4* h4 = reinterpret_cast<const uint4*>(h);
    uint32_t w[60];  // header words 0..59: fields and the 48 slots
#pragma unroll
    for (int q = 0; q < 15; ++q) {
        const uint4 x = h4[q];
        w[4 * q] = x.x; w[4 * q + 1] = x.y; w[4 * q + 2] = x.z; w[4 * q + 3] = x.w;
    }
    const uint32_t d = w[H4_DEG];
    if (d == 0) return STOP_VERTEX;
    const uint64_t W = ((uint64_t)w[H4_WHI] << 32) | w[H4_WLO];
    const uint64_t adj = ((uint64_t)w[H4_ADJHI] << 32) | w[H4_ADJLO];
    const uint64_t onem = ((uint64_t)w[H4_ONEHI] << 32) | w[H4_ONELO];
    const uint64_t r = rs_below64(rs, W);
    uint64_t acc = 0;
    int sel = -1;
    uint32_t csel = 0, raw = 0;
#pragma unroll
    for (int s = 0; s < R4_SUB; ++s) {
        const uint32_t slot = w[H4_SLOT + s];
        const uint32_t c = ((onem >> s) & 1ull) ? 1u : slot;
        acc += ((uint64_t)c * (uint64_t)(s % 3 + 1)) << (2 * (s / 3));
        if (sel < 0 && r < acc) { sel = s; csel = c; raw = slot; }
    }
    if (sel < 0) return STOP_VERTEX;  // only on an inconsistent header
    if ((onem >> sel) & 1ull) return raw;
    const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + adj);
    if (group_type(csel, d, rule) == GT_DENSE) {
        const uint32_t k = (uint32_t)sel / 3, v = (uint32_t)sel % 3 + 1;
        for (uint32_t att = 0; att < (1u << 16); att += SPEC) {
            const uint32_t x = dense_round4<SPEC>(edges, d, k, v, rs);
            if (x != PENDING) return x;
        }
        return STOP_VERTEX;
    }
    const uint32_t info = h[H4_INFO + sel];
    const uint32_t i = pool[(uint64_t)info * LIST_UNIT_WORDS + rs_below32(rs, csel)];
    return (uint32_t)edges[i];
}

// Persistent DeepWalk on the base-4 structure: walk ids from a chunked device
// queue, one lane per walk until it ends; ctl[0] queue head, ctl[1] transitions.
template <int SPEC>
__global__ void __launch_bounds__(TB4) k_deepwalk4(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                   uint32_t n, uint64_t nw, const uint32_t* __restrict__ starts,
                                                   uint64_t base, uint32_t L, uint64_t seed,
                                                   uint32_t* __restrict__ paths, GroupRule rule,
                                                   unsigned long long* __restrict__ ctl, uint32_t* __restrict__ err,
                                                   uint32_t qchunk) {
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
                row[0] = u;
                if (u >= n) {
                    atomicOr(err, ERR_RANGE);
                    for (uint32_t x = 1; x <= L; ++x) row[x] = STOP_VERTEX;
                    j = NO_WALK;
                }
            }
        }
        if (__ballot(!done) == 0) break;
        if (j != NO_WALK) {
            if (s < L) {
                RandStream rs;
                rs_init(rs, seed, base + j, s);
                const uint32_t v = step4<SPEC>(hdr, pool, u, rs, rule);
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

__global__ void k_copy_steps(const unsigned long long* __restrict__ c, unsigned long long* __restrict__ steps) {
    *steps = c[1];
}

// ---------------------------------------------------------------------------
// Canonical dump of the base-4 structure, per vertex u ascending: d, the mask
// of non-empty subgroups (subgroups 0..31, then 32..47), (dst, w) per index,
// then for each non-empty subgroup s ascending: s, type, c, followed by the
// member index (one-element) or the list (sparse and regular).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t stored4(uint32_t t, uint32_t c) {
    return t == GT_ONE ? 1u : (type_listed(t) ? c : 0u);
}

__global__ void k_dump4_size(const uint32_t* __restrict__ hdr, uint32_t u0, uint32_t u1, GroupRule rule,
                             uint64_t* __restrict__ sz) {
    const uint32_t u = u0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= u1) return;
    const uint32_t* h = hdr + (size_t)u * H4_WORDS;
    const uint32_t d = h[H4_DEG];
    const uint64_t mask = ((uint64_t)h[H4_MASKHI] << 32) | h[H4_MASKLO];
    const uint64_t onem = ((uint64_t)h[H4_ONEHI] << 32) | h[H4_ONELO];
    uint64_t s = 3 + 2ull * d;
    for (uint64_t mm = mask; mm; mm &= mm - 1) {
        const int sg = __ffsll((long long)mm) - 1;
        const uint32_t c = ((onem >> sg) & 1ull) ? 1u : h[H4_SLOT + sg];
        s += 3 + stored4(group_type(c, d, rule), c);
    }
    sz[u - u0] = s;
}

__global__ void __launch_bounds__(TB4) k_dump4_write(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                     uint32_t u0, uint32_t u1, GroupRule rule,
                                                     const uint64_t* __restrict__ off, uint32_t* __restrict__ out) {
    const uint32_t u = u0 + blockIdx.x * (TB4 / 64) + (threadIdx.x >> 6);
    if (u >= u1) return;
    const uint32_t lane = lane_id();
    const uint32_t* h = hdr + (size_t)u * H4_WORDS;
    const uint32_t d = h[H4_DEG];
    const uint64_t mask = ((uint64_t)h[H4_MASKHI] << 32) | h[H4_MASKLO];
    const uint64_t onem = ((uint64_t)h[H4_ONEHI] << 32) | h[H4_ONELO];
    uint32_t* o = out + off[u - u0];
    if (lane == 0) { o[0] = d; o[1] = (uint32_t)mask; o[2] = (uint32_t)(mask >> 32); }
    const uint64_t adj = ((uint64_t)h[H4_ADJHI] << 32) | h[H4_ADJLO];
    const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + adj);
    for (uint32_t i = lane; i < d; i += 64) {
        const uint64_t e = edges[i];
        o[3 + 2 * (uint64_t)i] = (uint32_t)e;
        o[4 + 2 * (uint64_t)i] = (uint32_t)(e >> 32);
    }
    const bool ne = lane < R4_SUB && ((mask >> lane) & 1ull);
    const uint32_t c = ne ? (((onem >> lane) & 1ull) ? 1u : h[H4_SLOT + lane]) : 0u;
    const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
    const uint64_t sz = ne ? 3ull + stored4(t, c) : 0ull;
    uint64_t x = sz;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint64_t y = __shfl_up(x, s, 64);
        if (lane >= (uint32_t)s) x += y;
    }
    const uint64_t my = 3 + 2ull * d + (x - sz);
    const uint32_t info = ne ? h[H4_INFO + lane] : 0u;
    if (ne) {
        o[my] = lane;
        o[my + 1] = t;
        o[my + 2] = c;
        if (t == GT_ONE) o[my + 3] = info;
    }
    for (uint64_t lm = __ballot(ne && type_listed(t)); lm; lm &= lm - 1) {
        const int sg = __ffsll((long long)lm) - 1;
        const uint64_t dst0 = __shfl(my, sg, 64) + 3;
        const uint32_t cs = __shfl(c, sg, 64);
        const uint64_t src0 = (uint64_t)__shfl(info, sg, 64) * LIST_UNIT_WORDS;
        for (uint32_t i = lane; i < cs; i += 64) o[dst0 + i] = pool[src0 + i];
    }
}

// Memory statistics of the base-4 structure: [0..4] subgroups by type, [5] live
// list bytes, [6] reserved list bytes, [7] adjacency reserved bytes, [8] edges.
constexpr int MEM4_CTRS = 9;
__global__ void __launch_bounds__(TB4) k_mem4(const uint32_t* __restrict__ hdr, uint32_t n, GroupRule rule,
                                              unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long red[TB4 / 64][MEM4_CTRS];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint64_t tot[MEM4_CTRS];
#pragma unroll
    for (int i = 0; i < MEM4_CTRS; ++i) tot[i] = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * (TB4 / 64) + wave; u < n; u += (uint64_t)gridDim.x * (TB4 / 64)) {
        const uint32_t* h = hdr + (size_t)u * H4_WORDS;
        const uint32_t d = h[H4_DEG];
        const uint64_t mask = ((uint64_t)h[H4_MASKHI] << 32) | h[H4_MASKLO];
        const uint64_t onem = ((uint64_t)h[H4_ONEHI] << 32) | h[H4_ONELO];
        const bool ne = lane < R4_SUB && ((mask >> lane) & 1ull);
        const uint32_t c = ne ? (((onem >> lane) & 1ull) ? 1u : h[H4_SLOT + lane]) : 0u;
        const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
        const uint32_t capb = lane < R4_SUB ? ((h[H4_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu) : 0u;
        uint64_t v0 = type_listed(t) ? 4ull * c : 0ull, v1 = type_listed(t) ? (4ull << capb) : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            v0 += __shfl_xor(v0, o);
            v1 += __shfl_xor(v1, o);
        }
#pragma unroll
        for (int tt = 1; tt < 5; ++tt) tot[tt] += __popcll(__ballot(ne && t == (uint32_t)tt));
        tot[5] += v0;
        tot[6] += v1;
        tot[7] += 8ull * h[H4_ACAP];
        tot[8] += d;
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < MEM4_CTRS; ++i) red[wave][i] = tot[i];
    __syncthreads();
    if (threadIdx.x < MEM4_CTRS) {
        unsigned long long x = 0;
#pragma unroll
        for (int w = 0; w < TB4 / 64; ++w) x += red[w][threadIdx.x];
        if (x) atomicAdd(acc + threadIdx.x, x);
    }
}

}  // namespace

int launch_walk4(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t L, uint64_t seed,
                 uint32_t* paths, uint64_t* steps, hipStream_t st) {
    uint32_t slot = 0;
    if (int rc = walk_slot_take(g, st, &slot)) return rc;
    unsigned long long* ctl = g->d_ctl + CTL_WALK0 + 2 * slot;
    phase_mark(g, st, true);
    if (nw) {
        int dev = 0, cus = 0, per = 0;
        HIPCHK(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        const void* kern = g->dense_spec == 1 ? (const void*)k_deepwalk4<1> : (const void*)k_deepwalk4<2>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, TB4, 0) != hipSuccess || per <= 0) per = 4;
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * per, (nw + TB4 - 1) / TB4));
        if (g->dense_spec == 1)
            hipLaunchKernelGGL(k_deepwalk4<1>, dim3(grid), dim3(TB4), 0, st, g->hdr, g->pool, g->n, nw, starts, base, L,
                               seed, paths, g->rule, ctl, g->d_err, g->queue_chunk);
        else
            hipLaunchKernelGGL(k_deepwalk4<2>, dim3(grid), dim3(TB4), 0, st, g->hdr, g->pool, g->n, nw, starts, base, L,
                               seed, paths, g->rule, ctl, g->d_err, g->queue_chunk);
    }
    phase_mark(g, st, false);
    if (steps) hipLaunchKernelGGL(k_copy_steps, dim3(1), dim3(1), 0, st, (const unsigned long long*)ctl,
                                  (unsigned long long*)steps);
    if (int rc = walk_slot_release(g, slot, st)) return rc;
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

int export_graph4(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
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
    hipLaunchKernelGGL(k_dump4_size, dim3((nv + 255) / 256), dim3(256), 0, st, g->hdr, u0, u1, g->rule, sz);
    scan_u64(sz, off, nv, tmp, total, st);
    unsigned long long T = 0;
    HIPCHK(hipMemcpyAsync(&T, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *h_len = T;
    if (!h_buf) return BINGO_OK;
    if (cap < T) return BINGO_E_CAPACITY;
    uint32_t* dbuf = nullptr;
    if (hipMalloc(&dbuf, std::max<uint64_t>(T, 1) * 4) != hipSuccess) return BINGO_E_OOM;
    hipLaunchKernelGGL(k_dump4_write, dim3((nv + 3) / 4), dim3(TB4), 0, st, g->hdr, g->pool, u0, u1, g->rule,
                       (const uint64_t*)off, dbuf);
    hipError_t e1 = hipMemcpyAsync(h_buf, dbuf, T * 4, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    hipFree(dbuf);
    return (e1 == hipSuccess && e2 == hipSuccess) ? BINGO_OK : BINGO_E_HIP;
}

int memory_stats4(bingo_graph* g, bingo_mem_stats* out, hipStream_t st) {
    unsigned long long* acc = (unsigned long long*)ws_get(g, 16 * 8);
    if (!acc) return BINGO_E_OOM;
    HIPCHK(hipMemsetAsync(acc, 0, 16 * 8, st));
    hipLaunchKernelGGL(k_mem4, dim3(std::min<uint32_t>(2048, (g->n + 3) / 4)), dim3(TB4), 0, st, g->hdr, g->n, g->rule,
                       acc);
    unsigned long long a[16], ctl[2];
    HIPCHK(hipMemcpyAsync(a, acc, sizeof a, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memset(out, 0, sizeof *out);
    out->vertices = g->n;
    out->edges = a[8];
    out->pool_bytes = g->pool_words * 4;
    out->pool_used_bytes = ctl[0] * 4;
    out->header_bytes = (uint64_t)g->n * H4_WORDS * 4;
    out->adjacency_bytes = 8ull * a[8];
    out->adjacency_reserved_bytes = a[7];
    out->list_bytes = a[5];
    out->list_reserved_bytes = a[6];
    for (int t = 1; t < 5; ++t) out->groups_by_type[t] = a[t];
    return BINGO_OK;
}

// build.hip -- sampling-space construction (Sec. 4.1: decomposition of every
// weight into its set bits, Eq. eq:dwi, and per-group totals c_k 2^k,
// Eq. eq:wpk; Sec. 5.1: group adaption).  One wave per vertex: for every
// 64-edge chunk, one ballot per bit position gives that bit's members in the
// chunk; popcounts give the counts and prefix popcounts the list positions.
#include "dev.h"
#include <stdio.h>
#include <algorithm>

namespace {

constexpr int WB = 256;  // block of 4 waves, one vertex per wave

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

__global__ void k_validate(uint64_t m, uint32_t n, const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                           const uint32_t* __restrict__ w, uint32_t* __restrict__ err) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        if (src[i] >= n || dst[i] >= n) bad |= ERR_RANGE;
        if (w[i] == 0) bad |= ERR_WEIGHT;
    }
    // combine in the wave first; one atomic per wave that saw a problem
    bad |= __shfl_xor(bad, 1); bad |= __shfl_xor(bad, 2); bad |= __shfl_xor(bad, 4);
    bad |= __shfl_xor(bad, 8); bad |= __shfl_xor(bad, 16); bad |= __shfl_xor(bad, 32);
    if (bad && lane_id() == 0) atomicOr(err, bad);
}

__global__ void k_iota(uint32_t* __restrict__ v, uint64_t m) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        v[i] = (uint32_t)i;
}

__global__ void k_gather(uint64_t m, const uint32_t* __restrict__ ids, const uint32_t* __restrict__ dst,
                         const uint32_t* __restrict__ w, uint32_t* __restrict__ cdst, uint32_t* __restrict__ cw) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = ids[i];
        cdst[i] = dst[e];
        cw[i] = w[e];
    }
}

// start[u] = first position of key u in the sorted keys (u = 0..n).
__global__ void k_row_start(const uint32_t* __restrict__ keys, uint64_t m, uint32_t n, uint32_t* __restrict__ start) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < u) lo = mid + 1; else hi = mid;
    }
    start[u] = (uint32_t)lo;
}

// Pass 1: counts, totals, one-element members, types; block sizes.
__global__ void __launch_bounds__(WB) k_header(uint32_t n, const uint32_t* __restrict__ start,
                                               const uint32_t* __restrict__ cw, uint32_t* __restrict__ hdr,
                                               uint64_t* __restrict__ adjw, uint64_t* __restrict__ listw,
                                               GroupRule rule) {
    const uint32_t u = blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t b = start[u], d = start[u + 1] - b;
    uint32_t cnt = 0, last = 0;  // lane k < 32 owns bit k
    uint64_t wraw = 0;           // this lane's share of sum(weights)
    for (uint32_t c0 = 0; c0 < d; c0 += 64) {
        const uint32_t i = c0 + lane;
        const uint32_t w = i < d ? cw[b + i] : 0u;
        wraw += w;
        const uint32_t wv = member_word(w, rule.fbits);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const uint64_t bal = __ballot((wv >> k) & 1u);
            if (lane == (uint32_t)k && bal) {
                cnt += __popcll(bal);
                last = c0 + 63 - __clzll(bal);
            }
        }
    }
    const uint32_t t = lane < 32 ? group_type(cnt, d, rule) : GT_EMPTY;
    // |S(u)|: the edges in at least one sparse group (Sec. 5.1)
    const uint32_t smask = (uint32_t)(__ballot(t == GT_SPARSE) & 0xFFFFFFFFull);
    uint32_t slen = 0;
    for (uint32_t c0 = 0; smask && c0 < d; c0 += 64) {
        const uint32_t i = c0 + lane;
        const bool in = i < d && (member_word(cw[b + i], rule.fbits) & smask);
        slen += __popcll(__ballot(in));
    }
    const uint32_t cap = adj_cap_for(d), scap = s_cap_for(slen);
    // W = sum of the weights (= sum_k c_k 2^k for integer biases)
    uint64_t wsum = wraw;
    // pool words: each listed group's block (list, then index), then the S(u) block
    uint64_t lw = type_listed(t) ? list_block_words(list_cap_for(cnt), index_cap_for(t, cap, scap)) : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        wsum += __shfl_xor(wsum, o);
        lw += __shfl_xor(lw, o);
    }
    const uint64_t mask = __ballot(cnt > 0) & 0xFFFFFFFFull;
    const uint32_t hi = mask_hi((uint32_t)mask);
    uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    if (lane < 32) {
        if (lane <= hi) h[H_CNT + (hi - lane)] = cnt;
        h[H_INFO + lane] = (t == GT_ONE) ? last : 0u;
    }
    if (lane == 0) {
        h[H_MASK] = (uint32_t)mask;
        h[H_DEG] = d;
        h[H_WLO] = (uint32_t)wsum;
        h[H_WHI] = (uint32_t)(wsum >> 32);
        h[H_ACAP] = cap;
        h[H_NSEQ] = d;
        h[H_SLEN] = slen;
        h[H_SCAP] = scap;
        h[H_SBLK] = 0;
        adjw[u] = adj_block_words(cap);
        listw[u] = lw + scap;
    }
}

// Pass 2: adjacency blocks (edge words and sequence numbers), listed-group
// lists (ascending neighbor indices) with their indexes, and S(u).
__global__ void __launch_bounds__(WB) k_fill(uint32_t n, const uint32_t* __restrict__ start,
                                             const uint32_t* __restrict__ cdst, const uint32_t* __restrict__ cw,
                                             const uint64_t* __restrict__ adj_off, const uint64_t* __restrict__ list_off,
                                             uint64_t list_base, uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                             GroupRule rule) {
    const uint32_t u = blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t b = start[u], d = start[u + 1] - b;
    uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    if (d == 0) {
        if (lane == 0) { h[H_ADJLO] = 0; h[H_ADJHI] = 0; }
        if (lane < 8) h[H_LCAPLOG + lane] = 0;
        return;
    }
    const uint32_t cap = h[H_ACAP];
    const uint64_t ao = adj_off[u];
    const uint32_t hi = mask_hi(h[H_MASK]);
    if (lane == 0) { h[H_ADJLO] = (uint32_t)ao; h[H_ADJHI] = adjhi_word(ao, hi); }
    uint64_t* edges = (uint64_t*)(pool + ao);
    uint32_t* seqs = pool + ao + 2ull * cap;
    // list blocks of the listed groups, in ascending k
    const uint32_t cnt = lane < 32 ? hdr_slot(h, lane, hi) : 0u;
    const uint32_t t = lane < 32 ? group_type(cnt, d, rule) : GT_EMPTY;
    const bool lst = type_listed(t);
    const uint32_t lcap = lst ? list_cap_for(cnt) : 0u;
    const uint32_t scap = h[H_SCAP];
    // lanes 0..31: the group blocks (list, then index); lane 32: the S(u) block
    const uint64_t bw = lst ? list_block_words(lcap, index_cap_for(t, cap, scap)) : (lane == 32 ? scap : 0ull);
    uint64_t x = bw;  // inclusive scan over lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    const uint64_t my_block = list_base + list_off[u] + (x - bw);  // words
    if (lane < 32 && lst) h[H_INFO + lane] = (uint32_t)(my_block / LIST_UNIT_WORDS);
    if (lane == 32) h[H_SBLK] = (uint32_t)(my_block / LIST_UNIT_WORDS);
    const uint64_t sblk = __shfl(my_block, 32, 64);
    const uint32_t smask = (uint32_t)(__ballot(t == GT_SPARSE) & 0xFFFFFFFFull);
    // one-element groups: the member's destination in the count slot
    const bool one = lane < 32 && t == GT_ONE;
    if (one) h[H_CNT + (hi - lane)] = cdst[b + h[H_INFO + lane]];
    const uint32_t onemask = (uint32_t)(__ballot(one) & 0xFFFFFFFFull);
    if (lane == 0) h[H_ONEMASK] = onemask;
    // list capacity exponents, one byte per group, packed four per word
    const uint32_t lg = lst ? (31 - __clz(lcap)) : 0u;
    const uint32_t byte = lg << (8 * (lane & 3));
    uint32_t packed = byte;
    packed |= __shfl_xor(packed, 1);
    packed |= __shfl_xor(packed, 2);
    if (lane < 32 && (lane & 3) == 0) h[H_LCAPLOG + (lane >> 2)] = packed;
    const uint32_t lmask = (uint32_t)(__ballot(lst) & 0xFFFFFFFFull);
    uint32_t fill = 0;   // lane k: entries written so far into group k
    uint32_t sfill = 0;  // entries written so far into S(u) (uniform)
    for (uint32_t c0 = 0; c0 < d; c0 += 64) {
        const uint32_t i = c0 + lane;
        uint32_t wv = 0;
        if (i < d) {
            const uint32_t w = cw[b + i];
            edges[i] = (uint64_t)cdst[b + i] | ((uint64_t)w << 32);
            seqs[i] = i;
            wv = member_word(w, rule.fbits);
        }
        // S(u) in ascending index order; spos is this edge's position in it
        const bool sb = (wv & smask) != 0u;
        const uint64_t sbal = __ballot(sb);
        const uint32_t spos = sfill + __popcll(sbal & lanemask_lt());
        if (sb) pool[sblk + spos] = i;
        sfill += __popcll(sbal);
        uint32_t mm = lmask;
        while (mm) {
            const int k = __ffs(mm) - 1;
            mm &= mm - 1;
            const bool bit = (wv >> k) & 1u;
            const uint64_t bal = __ballot(bit);
            const uint64_t blk = __shfl(my_block, k, 64);
            const uint32_t f = __shfl(fill, k, 64);
            const uint32_t lk = __shfl(lcap, k, 64);
            const bool reg = ((smask >> k) & 1u) == 0u;  // a listed group that is not sparse is regular
            if (bit) {
                const uint32_t pos = f + __popcll(bal & lanemask_lt());
                pool[blk + pos] = i;
                pool[blk + lk + (reg ? i : spos)] = pos;  // the group's index entry
            }
            if (lane == (uint32_t)k) fill += __popcll(bal);
        }
    }
}

// ---------------------------------------------------------------------------
// Radix base 4 (Supplement S.2).  Pass 1: per subgroup s = 3k + v - 1 (lane s)
// the count c_s of edges whose base-4 digit k is v (one ballot per subgroup per
// 64 edges), the one-element member (the first such edge), types by the rule of
// Sec. 5.1, W and the block sizes.  Pass 2: adjacency words, one-element
// destinations, and each listed subgroup's ascending list.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WB) k_header4(uint32_t n, const uint32_t* __restrict__ start,
                                                const uint32_t* __restrict__ cw, uint32_t* __restrict__ hdr,
                                                uint64_t* __restrict__ adjw, uint64_t* __restrict__ listw,
                                                GroupRule rule) {
    const uint32_t u = blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t b = start[u], d = start[u + 1] - b;
    uint32_t cnt = 0, first = 0xFFFFFFFFu;  // lane s < 48 owns subgroup s
    uint64_t wraw = 0;
    for (uint32_t c0 = 0; c0 < d; c0 += 64) {
        const uint32_t i = c0 + lane;
        const uint32_t w = i < d ? cw[b + i] : 0u;
        wraw += w;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t dg = i < d ? r4_digit(w, (uint32_t)k) : 0u;
#pragma unroll
            for (int v = 1; v <= 3; ++v) {
                const uint64_t bal = __ballot(dg == (uint32_t)v);
                if (lane == (uint32_t)(3 * k + v - 1) && bal) {
                    cnt += __popcll(bal);
                    if (first == 0xFFFFFFFFu) first = c0 + (uint32_t)(__ffsll((long long)bal) - 1);
                }
            }
        }
    }
    const uint32_t t = lane < R4_SUB ? group_type(cnt, d, rule) : GT_EMPTY;
    uint64_t wsum = wraw;
    uint64_t lw = type_listed(t) ? (uint64_t)list_cap_for(cnt) : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        wsum += __shfl_xor(wsum, o);
        lw += __shfl_xor(lw, o);
    }
    const uint64_t mask = __ballot(cnt > 0), onem = __ballot(t == GT_ONE);
    uint32_t* h = hdr + (size_t)u * H4_WORDS;
    if (lane < R4_SUB) {
        h[H4_SLOT + lane] = cnt;
        h[H4_INFO + lane] = t == GT_ONE ? first : 0u;
    }
    if (lane == 0) {
        const uint32_t cap = adj_cap_for(d);
        h[H4_DEG] = d;
        h[H4_ACAP] = cap;
        h[H4_WLO] = (uint32_t)wsum;
        h[H4_WHI] = (uint32_t)(wsum >> 32);
        h[H4_ONELO] = (uint32_t)onem;
        h[H4_ONEHI] = (uint32_t)(onem >> 32);
        h[H4_MASKLO] = (uint32_t)mask;
        h[H4_MASKHI] = (uint32_t)(mask >> 32);
        adjw[u] = cap ? r4_adj_words(cap) : 0ull;
        listw[u] = lw;
    }
}

__global__ void __launch_bounds__(WB) k_fill4(uint32_t n, const uint32_t* __restrict__ start,
                                              const uint32_t* __restrict__ cdst, const uint32_t* __restrict__ cw,
                                              const uint64_t* __restrict__ adj_off, const uint64_t* __restrict__ list_off,
                                              uint64_t list_base, uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                              GroupRule rule) {
    const uint32_t u = blockIdx.x * (WB / 64) + (threadIdx.x >> 6);
    if (u >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t b = start[u], d = start[u + 1] - b;
    uint32_t* h = hdr + (size_t)u * H4_WORDS;
    const uint64_t ao = d ? adj_off[u] : 0ull;
    if (lane == 0) { h[H4_ADJLO] = (uint32_t)ao; h[H4_ADJHI] = (uint32_t)(ao >> 32); }
    uint64_t* edges = reinterpret_cast<uint64_t*>(pool + ao);
    const uint32_t cnt = lane < R4_SUB ? h[H4_SLOT + lane] : 0u;
    const uint32_t t = lane < R4_SUB ? group_type(cnt, d, rule) : GT_EMPTY;
    const bool lst = type_listed(t);
    const uint32_t lcap = lst ? list_cap_for(cnt) : 0u;
    uint64_t x = lcap;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    const uint64_t my_block = list_base + list_off[u] + (x - lcap);
    if (lst) h[H4_INFO + lane] = (uint32_t)(my_block / LIST_UNIT_WORDS);
    if (lane < R4_SUB && t == GT_ONE) h[H4_SLOT + lane] = cdst[b + h[H4_INFO + lane]];
    const uint32_t lg = lst ? (31 - __clz(lcap)) : 0u;
    uint32_t packed = lg << (8 * (lane & 3));
    packed |= __shfl_xor(packed, 1);
    packed |= __shfl_xor(packed, 2);
    if (lane < R4_SUB && (lane & 3) == 0) h[H4_LCAPLOG + (lane >> 2)] = packed;
    const uint64_t lmask = __ballot(lst);
    uint32_t fill = 0;
    for (uint32_t c0 = 0; c0 < d; c0 += 64) {
        const uint32_t i = c0 + lane;
        uint32_t w = 0;
        if (i < d) {
            w = cw[b + i];
            edges[i] = (uint64_t)cdst[b + i] | ((uint64_t)w << 32);
        }
        for (uint64_t mm = lmask; mm; mm &= mm - 1) {
            const int sg = __ffsll((long long)mm) - 1;
            const bool bit = i < d && r4_digit(w, (uint32_t)sg / 3) == (uint32_t)(sg % 3) + 1;
            const uint64_t bal = __ballot(bit);
            const uint64_t blk = __shfl(my_block, sg, 64);
            const uint32_t f = __shfl(fill, sg, 64);
            if (bit) pool[blk + f + __popcll(bal & lanemask_lt())] = i;
            if (lane == (uint32_t)sg) fill += __popcll(bal);
        }
    }
}

inline uint32_t grid_for(uint64_t n, uint32_t block) {
    uint64_t g = (n + block - 1) / block;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(g, 1), 1u << 20);
}

// Floating-point biases as fixed-point weights (Sec. 4.3): floor(lambda * b * 2^F)
// with lambda * b one IEEE double product (round to nearest) and an exact
// scaling by 2^F; 0 where the result is not a number in [1, 2^32).
__global__ void k_quantize(uint64_t m, const float* __restrict__ b, double lambda, uint32_t F,
                           uint32_t* __restrict__ w) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        const double s = (double)b[i] * lambda;
        uint32_t q = 0;
        if (s >= 0.0 && !isinf(s)) {
            const double t = s * (double)(1u << F);
            if (t < 4294967296.0) q = (uint32_t)t;
        }
        w[i] = q;
    }
}

// Inter-group alias rows (alias-table mode; Sec. 4.1), exact in integers: the
// 32 slots are the 32 groups, every slot holds W units and group k owns
// 32 c_k 2^k of them.  Small groups (32 T_k < W) and large ones are two
// first-in first-out queues in ascending k; the front small slot keeps its own
// units and takes the rest from the front large group, which joins the back of
// the small queue once its remainder drops below W; leftover slots keep all W
// units.  Entry j = {cut lo, cut hi, alias, 0}: a draw (j, x < W) selects j when
// x < cut, else alias.  One thread per vertex.
constexpr int ALIAS_TB = 128;
__global__ void __launch_bounds__(ALIAS_TB) k_alias_rows(const uint32_t* __restrict__ hdr, uint32_t n,
                                                          const uint32_t* __restrict__ list,
                                                          const unsigned long long* __restrict__ dcount, uint64_t maxc,
                                                          uint4* __restrict__ alias) {
    // per thread, one column: the slot counts and the remainders of large slots that fell below W
    __shared__ uint32_t cnt[ALIAS_ENTRIES][ALIAS_TB];
    __shared__ uint64_t rem[ALIAS_ENTRIES][ALIAS_TB];
    const uint32_t tx = threadIdx.x;
    const uint64_t total = dcount ? std::min<uint64_t>(*dcount, maxc) : maxc;
    for (uint64_t i = (uint64_t)blockIdx.x * ALIAS_TB + tx; i < total; i += (uint64_t)gridDim.x * ALIAS_TB) {
        const uint32_t u = list ? list[i] : (uint32_t)i;
        if (u >= n) continue;  // a rejected stream's bad source id
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        uint4* row = alias + (size_t)u * ALIAS_ENTRIES;
        const uint32_t onem = h[H_ONEMASK], hi = hdr_hi(h);
        uint64_t W = 0;
        for (int k = 0; k < ALIAS_ENTRIES; ++k) {
            const uint32_t c = slot_count(hdr_slot(h, (uint32_t)k, hi), onem, (uint32_t)k);
            cnt[k][tx] = c;
            W += (uint64_t)c << k;
        }
        // slot k holds 32 T_k = c_k 2^(k+5) units (below 2^69); it is small when that is below W
        uint32_t S = 0, L = 0;
        for (int k = 0; k < ALIAS_ENTRIES; ++k) {
            if (((unsigned __int128)cnt[k][tx] << (k + 5)) < W) S |= 1u << k;
            else L |= 1u << k;
        }
        // The small queue is the initial small slots in ascending k, then the large
        // slots in the order they fall below W; large slots are taken in ascending k,
        // so both parts are in ascending k and each is a bit mask.
        uint32_t P = 0, done = 0;
        int cur = L ? __ffs(L) - 1 : -1;
        unsigned __int128 R = cur >= 0 ? (unsigned __int128)cnt[cur][tx] << (cur + 5) : 0;
        while ((S | P) != 0 && cur >= 0) {
            int sm;
            uint64_t us;
            if (S) {
                sm = __ffs(S) - 1;
                S &= S - 1;
                us = (uint64_t)((unsigned __int128)cnt[sm][tx] << (sm + 5));
            } else {
                sm = __ffs(P) - 1;
                P &= P - 1;
                us = rem[sm][tx];
            }
            row[sm] = make_uint4((uint32_t)us, (uint32_t)(us >> 32), (uint32_t)cur, 0u);
            done |= 1u << sm;
            R -= W - us;
            if (R < W) {
                rem[cur][tx] = (uint64_t)R;
                P |= 1u << cur;
                L &= L - 1;
                cur = L ? __ffs(L) - 1 : -1;
                R = cur >= 0 ? (unsigned __int128)cnt[cur][tx] << (cur + 5) : 0;
            }
        }
        // every slot not taken as small keeps exactly W units (the units sum to 32 W)
        for (int k = 0; k < ALIAS_ENTRIES; ++k)
            if (!((done >> k) & 1u)) row[k] = make_uint4((uint32_t)W, (uint32_t)(W >> 32), (uint32_t)k, 0u);
    }
}

// ---------------------------------------------------------------------------
// S(u) rebuild (Sec. 5.1 sparse groups): after an update, S(u) = the ascending
// neighbor indices i < d whose membership word meets the sparse mask, written
// into the vertex's S(u) block; then every sparse group's index over S(u):
// entry s = the position of S[s] in the group's list.  k_sr_compact gathers the
// flagged vertices, so every one of them gets a block of its own (a batch on a
// few hubs would otherwise rebuild them one after another); k_srebuild runs
// one block per vertex of more than SR_WAVE edges, k_srebuild_wave one wave per
// smaller one.  Pass 1 ranks the flagged entries of each tile of
// SR_TB * SR_TPT indices by ballots (rows of SR_TB consecutive indices, waves
// in order); pass 2 finds each list member's position in S(u) by a search
// that starts in LDS samples of S(u) (every 2^sh-th entry) and ends with at
// most sh steps in global memory.
// ---------------------------------------------------------------------------
constexpr int SR_TB = 256;
constexpr uint32_t SR_TPT = 16;     // adjacency words in flight per thread in pass 1
constexpr uint32_t SR_XL = 8192;    // LDS samples of S(u) (32 KB)
constexpr uint32_t SR_ILV = 4;      // list members searched together per thread in pass 2
constexpr uint32_t SR_LIST0 = 64;
// Vertices of more than SR_BIG edges are split into chunks of SR_CHUNK adjacency
// entries, each handled by a block of its own; vertices of at most SR_WAVE edges
// (most of them) take one wave each, with S(u) staged in the wave's LDS.  Work
// buffer (u32): [0] block vertices, [1] large vertices, [2] chunks, [3] wave
// vertices; the block list grows up from SR_LIST0 and the wave list down from
// SR_LIST0 + mc - 1 (a vertex is in one of them); the large list (vertex, first
// chunk, chunks) after them; then the chunk owners and counts.
constexpr uint32_t SR_BIG = 1u << 15;
constexpr uint32_t SR_CHUNK = 1u << 14;
constexpr uint32_t SR_NO_OWNER = 0xFFFFFFFFu;
constexpr uint32_t SR_WAVE = 1024;  // largest degree rebuilt by one wave
constexpr int SRW_TB = 256;         // blocks of the wave kernel
__host__ __device__ inline uint64_t sr_chunk_cap(uint64_t mc) { return 4 * mc + 65536; }
__host__ __device__ inline uint64_t sr_big_off(uint64_t mc) { return SR_LIST0 + mc; }
__host__ __device__ inline uint64_t sr_owner_off(uint64_t mc) { return sr_big_off(mc) + 3 * mc; }
__host__ __device__ inline uint64_t sr_cnt_off(uint64_t mc) { return sr_owner_off(mc) + sr_chunk_cap(mc); }

__global__ void k_sr_zero(uint32_t* __restrict__ work) {
    if (threadIdx.x < 4) work[threadIdx.x] = 0;
}

__global__ void k_sr_compact(uint32_t n, const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ list,
                             const unsigned long long* __restrict__ dcount, uint64_t maxc,
                             const uint32_t* __restrict__ dirty, uint32_t* __restrict__ work) {
    const uint64_t total = dcount ? std::min<uint64_t>(*dcount, maxc) : maxc;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (uint64_t)gridDim.x * blockDim.x) {
        if (dirty && !dirty[it]) continue;
        const uint32_t u = list ? list[it] : (uint32_t)it;
        if (u >= n) continue;
        const uint32_t d = hdr[(size_t)u * HDR_WORDS + H_DEG];
        bool small = d <= SR_BIG;
        if (!small) {
            const uint32_t nch = (d + SR_CHUNK - 1) / SR_CHUNK;
            const uint32_t cb = atomicAdd(work + 2, nch);
            if ((uint64_t)cb + nch <= sr_chunk_cap(maxc)) {
                const uint32_t b = atomicAdd(work + 1, 1u);
                uint32_t* e = work + sr_big_off(maxc) + 3ull * b;
                e[0] = u; e[1] = cb; e[2] = nch;
                for (uint32_t j = 0; j < nch; ++j) work[sr_owner_off(maxc) + cb + j] = b;
            } else {
                // no room in the chunk table: one block does it; the reserved ids below the
                // table's end get no owner
                for (uint64_t q = cb; q < (uint64_t)cb + nch && q < sr_chunk_cap(maxc); ++q)
                    work[sr_owner_off(maxc) + q] = SR_NO_OWNER;
                small = true;
            }
        }
        // one atomic per wave and list: the lanes of a list take consecutive slots
        const bool to_wave = small && d <= SR_WAVE, to_block = small && !to_wave;
        const uint64_t bw = __ballot(to_wave), bb = __ballot(to_block);
        const uint32_t lane = lane_id(), leader = __ffsll((long long)(bw | bb)) - 1;
        uint32_t basew = 0, baseb = 0;
        if (lane == leader) {
            if (bw) basew = atomicAdd(work + 3, (uint32_t)__popcll(bw));
            if (bb) baseb = atomicAdd(work, (uint32_t)__popcll(bb));
        }
        basew = __shfl(basew, leader, 64);
        baseb = __shfl(baseb, leader, 64);
        const uint64_t lt = lanemask_lt();
        if (to_wave) work[SR_LIST0 + maxc - 1 - (basew + (uint32_t)__popcll(bw & lt))] = u;
        if (to_block) work[SR_LIST0 + baseb + (uint32_t)__popcll(bb & lt)] = u;
    }
}

// The sparse mask of vertex u and, in LDS, each group's count, list block and
// capacity (wave 0 of the block; the caller synchronizes).
__device__ __forceinline__ void sr_groups(const uint32_t* __restrict__ h, uint32_t d, GroupRule rule,
                                          uint32_t* g_c, uint32_t* g_info, uint32_t* g_lcap, uint32_t* s_smask) {
    const uint32_t lane = lane_id();
    const uint32_t mask = h[H_MASK], onem = h[H_ONEMASK];
    const bool ne = lane < 32 && ((mask >> lane) & 1u);
    const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), onem, lane) : 0u;
    const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
    const uint32_t sm = (uint32_t)(__ballot(t == GT_SPARSE) & 0xFFFFFFFFull);
    if (lane < 32) {
        g_c[lane] = c;
        g_info[lane] = h[H_INFO + lane];
        g_lcap[lane] = 1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu);
    }
    if (lane == 0) *s_smask = sm;
}

constexpr int SRC_TB = 256;       // blocks of the chunked kernels
constexpr uint32_t SRC_ROWS = 8;  // rows of SRC_TB adjacency words per step (loads in flight)

// Large vertices, pass 1: the members of S(u) in each chunk.
__global__ void __launch_bounds__(SRC_TB) k_sr_count(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                     GroupRule rule, uint64_t maxc, uint32_t* __restrict__ work) {
    __shared__ uint32_t red[SRC_TB / 64];
    const uint32_t nchunks = min(work[2], (uint32_t)sr_chunk_cap(maxc));
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t b = work[sr_owner_off(maxc) + c];
        if (b == SR_NO_OWNER) continue;
        const uint32_t* e = work + sr_big_off(maxc) + 3ull * b;
        const uint32_t u = e[0], j = c - e[1];
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        // sparse mask from the final header (every lane of a wave computes it)
        const uint32_t mask = h[H_MASK], onem = h[H_ONEMASK], hi = hdr_hi(h);
        const bool ne = lane < 32 && ((mask >> lane) & 1u);
        const uint32_t cc = ne ? slot_count(hdr_slot(h, lane, hi), onem, lane) : 0u;
        const uint32_t smask = (uint32_t)(__ballot(ne && group_type(cc, d, rule) == GT_SPARSE) & 0xFFFFFFFFull);
        const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + hdr_adj(h));
        const uint32_t i0 = j * SR_CHUNK, i1 = min(i0 + SR_CHUNK, d);
        uint32_t cnt = 0;
        for (uint32_t r0 = i0; r0 < i1; r0 += SRC_TB * SRC_ROWS) {
            uint64_t x[SRC_ROWS];
#pragma unroll
            for (uint32_t q = 0; q < SRC_ROWS; ++q) {
                const uint32_t i = r0 + q * SRC_TB + threadIdx.x;
                x[q] = i < i1 ? edges[i] : 0ull;
            }
#pragma unroll
            for (uint32_t q = 0; q < SRC_ROWS; ++q)
                cnt += (member_word((uint32_t)(x[q] >> 32), rule.fbits) & smask) != 0u;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        __syncthreads();
        if (lane == 0) red[wave] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) work[sr_cnt_off(maxc) + c] = red[0] + red[1] + red[2] + red[3];
    }
}

// Large vertices, pass 2: each chunk writes its members at the chunk's offset in
// S(u) (the counts of the vertex's earlier chunks), in index order (rows of
// SRC_TB consecutive indices ranked by ballots); the last chunk sets |S(u)|.
__global__ void __launch_bounds__(SRC_TB) k_sr_write(uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                                     GroupRule rule, uint64_t maxc, const uint32_t* __restrict__ work) {
    __shared__ uint32_t wc[SRC_ROWS][SRC_TB / 64], s_base;
    const uint32_t nchunks = min(work[2], (uint32_t)sr_chunk_cap(maxc));
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t b = work[sr_owner_off(maxc) + c];
        if (b == SR_NO_OWNER) continue;
        const uint32_t* e = work + sr_big_off(maxc) + 3ull * b;
        const uint32_t u = e[0], cb = e[1], nch = e[2], j = c - cb;
        uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        const uint32_t mask = h[H_MASK], onem = h[H_ONEMASK], hi = hdr_hi(h);
        const bool ne = lane < 32 && ((mask >> lane) & 1u);
        const uint32_t cc = ne ? slot_count(hdr_slot(h, lane, hi), onem, lane) : 0u;
        const uint32_t smask = (uint32_t)(__ballot(ne && group_type(cc, d, rule) == GT_SPARSE) & 0xFFFFFFFFull);
        __syncthreads();
        if (wave == 0) {
            uint32_t x = 0;
            for (uint32_t q = lane; q < j; q += 64) x += work[sr_cnt_off(maxc) + cb + q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) s_base = x;
        }
        __syncthreads();
        uint32_t base = s_base;
        const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + hdr_adj(h));
        uint32_t* S = pool + (uint64_t)h[H_SBLK] * LIST_UNIT_WORDS;
        const uint32_t i0 = j * SR_CHUNK, i1 = min(i0 + SR_CHUNK, d);
        for (uint32_t r0 = i0; r0 < i1; r0 += SRC_TB * SRC_ROWS) {
            uint64_t x[SRC_ROWS];
#pragma unroll
            for (uint32_t q = 0; q < SRC_ROWS; ++q) {
                const uint32_t i = r0 + q * SRC_TB + threadIdx.x;
                x[q] = i < i1 ? edges[i] : 0ull;
            }
            uint64_t bal[SRC_ROWS];
#pragma unroll
            for (uint32_t q = 0; q < SRC_ROWS; ++q) {
                const uint32_t i = r0 + q * SRC_TB + threadIdx.x;
                bal[q] = __ballot(i < i1 && (member_word((uint32_t)(x[q] >> 32), rule.fbits) & smask) != 0u);
                if (lane == 0) wc[q][wave] = (uint32_t)__popcll(bal[q]);
            }
            __syncthreads();
#pragma unroll
            for (uint32_t q = 0; q < SRC_ROWS; ++q) {
                uint32_t rk = base + (uint32_t)__popcll(bal[q] & lanemask_lt());
                for (uint32_t w = 0; w < wave; ++w) rk += wc[q][w];
                if ((bal[q] >> lane) & 1ull) S[rk] = r0 + q * SRC_TB + threadIdx.x;
                base += wc[q][0] + wc[q][1] + wc[q][2] + wc[q][3];
            }
            __syncthreads();  // wc is rewritten by the next step
        }
        if (j == nch - 1 && threadIdx.x == 0) h[H_SLEN] = base;
    }
}

// Large vertices, pass 3: chunk j of a vertex with nch chunks fills the index entries of the
// members in [c_k j / nch, c_k (j + 1) / nch) of every sparse group k (LDS samples of S(u), then
// at most sh steps in global memory per member).
constexpr uint32_t SRI_XL = 4096;  // LDS samples of S(u) per chunk block (16 KB)
__global__ void __launch_bounds__(SRC_TB) k_sr_index(const uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                                     GroupRule rule, uint64_t maxc, const uint32_t* __restrict__ work) {
    __shared__ uint32_t smp[SRI_XL];
    __shared__ uint32_t g_c[32], g_info[32], g_lcap[32], s_smask;
    const uint32_t nchunks = min(work[2], (uint32_t)sr_chunk_cap(maxc));
    const uint32_t tid = threadIdx.x;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t b = work[sr_owner_off(maxc) + c];
        if (b == SR_NO_OWNER) continue;
        const uint32_t* e = work + sr_big_off(maxc) + 3ull * b;
        const uint32_t u = e[0], nch = e[2], j = c - e[1];
        const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        __syncthreads();  // the previous chunk is done with the shared arrays
        if ((tid >> 6) == 0) sr_groups(h, d, rule, g_c, g_info, g_lcap, &s_smask);
        const uint32_t sfill = h[H_SLEN];
        const uint32_t* S = pool + (uint64_t)h[H_SBLK] * LIST_UNIT_WORDS;
        uint32_t sh = 0;
        while ((sfill >> sh) >= SRI_XL) ++sh;
        const uint32_t nl = (sfill + (1u << sh) - 1) >> sh;
        for (uint32_t q = tid; q < nl; q += SRC_TB) smp[q] = S[(uint64_t)q << sh];
        __syncthreads();
        for (uint32_t mm = s_smask; mm; mm &= mm - 1) {
            const int k = __ffs(mm) - 1;
            const uint32_t ck = g_c[k];
            uint32_t* L = pool + (uint64_t)g_info[k] * LIST_UNIT_WORDS;
            uint32_t* I = L + g_lcap[k];
            const uint32_t p0 = (uint32_t)((uint64_t)ck * j / nch), p1 = (uint32_t)((uint64_t)ck * (j + 1) / nch);
            // SR_ILV members per thread at a time, their global search steps interleaved
            for (uint32_t pb = p0 + tid; pb < p1; pb += SRC_TB * SR_ILV) {
                uint32_t v[SR_ILV], a[SR_ILV], bb[SR_ILV];
#pragma unroll
                for (uint32_t x = 0; x < SR_ILV; ++x) {
                    const uint32_t p = pb + x * SRC_TB;
                    v[x] = p < p1 ? L[p] : 0u;
                }
#pragma unroll
                for (uint32_t x = 0; x < SR_ILV; ++x) {
                    uint32_t lo = 0, hi = nl;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (smp[mid] < v[x]) lo = mid + 1; else hi = mid;
                    }
                    a[x] = lo > 0 ? ((lo - 1) << sh) + 1 : 0u;
                    bb[x] = lo > 0 ? min(lo << sh, sfill) : 0u;
                }
                for (uint32_t step = 0; step <= sh; ++step) {
#pragma unroll
                    for (uint32_t x = 0; x < SR_ILV; ++x) {
                        if (a[x] < bb[x]) {
                            const uint32_t mid = (a[x] + bb[x]) >> 1;
                            if (S[mid] < v[x]) a[x] = mid + 1; else bb[x] = mid;
                        }
                    }
                }
#pragma unroll
                for (uint32_t x = 0; x < SR_ILV; ++x) {
                    const uint32_t p = pb + x * SRC_TB;
                    if (p < p1) I[a[x]] = p;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(SR_TB) k_srebuild(uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                                    GroupRule rule, const uint32_t* __restrict__ work) {
    __shared__ uint32_t smp[SR_XL];
    __shared__ uint32_t g_c[32], g_info[32], g_lcap[32];
    __shared__ uint32_t wcnt[SR_TPT][SR_TB / 64];
    __shared__ uint32_t s_smask;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t nt = work[0];
    for (uint32_t q = blockIdx.x; q < nt; q += gridDim.x) {
        const uint32_t u = work[SR_LIST0 + q];
        uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        __syncthreads();  // the previous vertex is done with the shared arrays
        if (wave == 0) {
            const uint32_t mask = h[H_MASK], onem = h[H_ONEMASK];
            const bool ne = lane < 32 && ((mask >> lane) & 1u);
            const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), onem, lane) : 0u;
            const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
            const uint32_t sm = (uint32_t)(__ballot(t == GT_SPARSE) & 0xFFFFFFFFull);
            if (lane < 32) {
                g_c[lane] = c;
                g_info[lane] = h[H_INFO + lane];
                g_lcap[lane] = 1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu);
            }
            if (lane == 0) s_smask = sm;
        }
        __syncthreads();
        const uint32_t smask = s_smask;
        if (!smask) {
            if (tid == 0) h[H_SLEN] = 0;
            continue;
        }
        const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + hdr_adj(h));
        uint32_t* S = pool + (uint64_t)h[H_SBLK] * LIST_UNIT_WORDS;
        uint32_t sfill = 0;
        for (uint32_t q0 = 0; q0 < d; q0 += SR_TB * SR_TPT) {
            uint64_t bal[SR_TPT];
            bool in[SR_TPT];
#pragma unroll
            for (uint32_t j = 0; j < SR_TPT; ++j) {
                const uint32_t i = q0 + j * SR_TB + tid;
                in[j] = i < d && (member_word((uint32_t)(edges[i] >> 32), rule.fbits) & smask) != 0u;
            }
#pragma unroll
            for (uint32_t j = 0; j < SR_TPT; ++j) {
                bal[j] = __ballot(in[j]);
                if (lane == 0) wcnt[j][wave] = (uint32_t)__popcll(bal[j]);
            }
            __syncthreads();
#pragma unroll
            for (uint32_t j = 0; j < SR_TPT; ++j) {
                uint32_t rk = sfill + (uint32_t)__popcll(bal[j] & lanemask_lt()), row = 0;
                for (uint32_t w = 0; w < SR_TB / 64; ++w) {
                    const uint32_t x = wcnt[j][w];
                    if (w < wave) rk += x;
                    row += x;
                }
                if (in[j]) S[rk] = q0 + j * SR_TB + tid;
                sfill += row;
            }
            __syncthreads();  // wcnt is rewritten by the next tile
        }
        if (tid == 0) h[H_SLEN] = sfill;
        __threadfence_block();
        __syncthreads();  // S(u) complete and visible to the block
        uint32_t sh = 0;
        while ((sfill >> sh) >= SR_XL) ++sh;
        const uint32_t nl = (sfill + (1u << sh) - 1) >> sh;
        for (uint32_t j = tid; j < nl; j += SR_TB) smp[j] = S[(uint64_t)j << sh];
        __syncthreads();
        for (uint32_t mm = smask; mm; mm &= mm - 1) {
            const int k = __ffs(mm) - 1;
            const uint32_t c = g_c[k];
            uint32_t* L = pool + (uint64_t)g_info[k] * LIST_UNIT_WORDS;
            uint32_t* I = L + g_lcap[k];
            // SR_ILV members per thread at a time, their global search steps interleaved
            for (uint32_t p0 = tid; p0 < c; p0 += SR_TB * SR_ILV) {
                uint32_t v[SR_ILV], a[SR_ILV], b[SR_ILV];
#pragma unroll
                for (uint32_t j = 0; j < SR_ILV; ++j) {
                    const uint32_t p = p0 + j * SR_TB;
                    v[j] = p < c ? L[p] : 0u;
                }
#pragma unroll
                for (uint32_t j = 0; j < SR_ILV; ++j) {
                    uint32_t lo = 0, hi = nl;  // samples below v
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (smp[mid] < v[j]) lo = mid + 1; else hi = mid;
                    }
                    a[j] = lo > 0 ? ((lo - 1) << sh) + 1 : 0u;
                    b[j] = lo > 0 ? min(lo << sh, sfill) : 0u;
                }
                for (uint32_t step = 0; step <= sh; ++step) {
#pragma unroll
                    for (uint32_t j = 0; j < SR_ILV; ++j) {
                        if (a[j] < b[j]) {
                            const uint32_t mid = (a[j] + b[j]) >> 1;
                            if (S[mid] < v[j]) a[j] = mid + 1; else b[j] = mid;
                        }
                    }
                }
#pragma unroll
                for (uint32_t j = 0; j < SR_ILV; ++j) {
                    const uint32_t p = p0 + j * SR_TB;
                    if (p < c) I[a[j]] = p;
                }
            }
        }
    }
}

// Vertices of at most SR_WAVE edges, one wave each: S(u) by ballots over rows of
// 64 indices (written to its block and to the wave's LDS), then every sparse
// group's index by a binary search of each list member in the LDS copy.
__global__ void __launch_bounds__(SRW_TB) k_srebuild_wave(uint32_t* __restrict__ hdr, uint32_t* __restrict__ pool,
                                                          GroupRule rule, uint64_t maxc,
                                                          const uint32_t* __restrict__ work) {
    __shared__ uint32_t sl[SRW_TB / 64][SR_WAVE];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t* S_l = sl[wave];
    const uint32_t nt = work[3];
    for (uint64_t q = (uint64_t)blockIdx.x * (SRW_TB / 64) + wave; q < nt; q += (uint64_t)gridDim.x * (SRW_TB / 64)) {
        const uint32_t u = work[SR_LIST0 + maxc - 1 - q];
        uint32_t* h = hdr + (size_t)u * HDR_WORDS;
        const uint32_t d = h[H_DEG];
        const uint32_t mask = h[H_MASK], onem = h[H_ONEMASK];
        const bool ne = lane < 32 && ((mask >> lane) & 1u);
        const uint32_t c = ne ? slot_count(hdr_slot(h, lane, hdr_hi(h)), onem, lane) : 0u;
        const uint32_t t = ne ? group_type(c, d, rule) : GT_EMPTY;
        const uint32_t smask = (uint32_t)(__ballot(t == GT_SPARSE) & 0xFFFFFFFFull);
        const uint32_t info = lane < 32 ? h[H_INFO + lane] : 0u;
        const uint32_t lcap = lane < 32 ? 1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu) : 0u;
        if (!smask) {
            if (lane == 0) h[H_SLEN] = 0;
            continue;
        }
        const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + hdr_adj(h));
        uint32_t* S = pool + (uint64_t)h[H_SBLK] * LIST_UNIT_WORDS;
        uint32_t sfill = 0;
        constexpr uint32_t ROWS = 8;  // rows of 64 indices whose weights are loaded together
        for (uint32_t i0 = 0; i0 < d; i0 += 64 * ROWS) {
            uint32_t wr[ROWS];
#pragma unroll
            for (uint32_t j = 0; j < ROWS; ++j) {
                const uint32_t i = i0 + j * 64 + lane;
                wr[j] = i < d ? (uint32_t)(edges[i] >> 32) : 0u;
            }
#pragma unroll
            for (uint32_t j = 0; j < ROWS; ++j) {
                const uint32_t i = i0 + j * 64 + lane;
                const bool in = i < d && (member_word(wr[j], rule.fbits) & smask) != 0u;
                const uint64_t b = __ballot(in);
                const uint32_t rk = sfill + (uint32_t)__popcll(b & lanemask_lt());
                if (in) {
                    S[rk] = i;
                    S_l[rk] = i;
                }
                sfill += (uint32_t)__popcll(b);
            }
        }
        if (lane == 0) h[H_SLEN] = sfill;
        __builtin_amdgcn_wave_barrier();  // S_l written by the wave before any lane searches it
        for (uint32_t mm = smask; mm; mm &= mm - 1) {
            const int k = __ffs(mm) - 1;
            const uint32_t ck = __shfl(c, k, 64);
            uint32_t* L = pool + (uint64_t)__shfl(info, k, 64) * LIST_UNIT_WORDS;
            uint32_t* I = L + __shfl(lcap, k, 64);
            for (uint32_t p = lane; p < ck; p += 64) {
                const uint32_t v = L[p];
                uint32_t lo = 0, hi = sfill;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (S_l[mid] < v) lo = mid + 1; else hi = mid;
                }
                I[lo] = p;
            }
        }
        __builtin_amdgcn_wave_barrier();  // the next vertex overwrites S_l
    }
}

int bits_for(uint64_t v) {  // bits needed to hold values in [0, v]
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

}  // namespace

void alias_rows(bingo_graph* g, const uint32_t* list, const unsigned long long* count, uint64_t max_count,
                hipStream_t st) {
    if (!g->alias || max_count == 0) return;
    hipLaunchKernelGGL(k_alias_rows, dim3(grid_for(max_count, ALIAS_TB)), dim3(ALIAS_TB), 0, st,
                       (const uint32_t*)g->hdr, g->n, list, count, max_count, g->alias);
}

void sparse_rebuild(bingo_graph* g, const uint32_t* list, const unsigned long long* count, uint64_t max_count,
                    const uint32_t* dirty, uint32_t* work, hipStream_t st) {
    if (max_count == 0 || !g->rule.adaptive) return;  // without adaption no group is sparse
    hipLaunchKernelGGL(k_sr_zero, dim3(1), dim3(64), 0, st, work);
    hipLaunchKernelGGL(k_sr_compact, dim3(grid_for(max_count, 256)), dim3(256), 0, st, g->n, (const uint32_t*)g->hdr,
                       list, count, max_count, dirty, work);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(max_count, 2048);
    hipLaunchKernelGGL(k_srebuild, dim3(grid), dim3(SR_TB), 0, st, g->hdr, g->pool, g->rule, (const uint32_t*)work);
    const uint32_t wgrid = (uint32_t)std::min<uint64_t>((max_count + SRW_TB / 64 - 1) / (SRW_TB / 64), 4096);
    hipLaunchKernelGGL(k_srebuild_wave, dim3(wgrid), dim3(SRW_TB), 0, st, g->hdr, g->pool, g->rule, max_count,
                       (const uint32_t*)work);
    hipLaunchKernelGGL(k_sr_count, dim3(2048), dim3(SRC_TB), 0, st, (const uint32_t*)g->hdr, (const uint32_t*)g->pool,
                       g->rule, max_count, work);
    hipLaunchKernelGGL(k_sr_write, dim3(2048), dim3(SRC_TB), 0, st, g->hdr, g->pool, g->rule, max_count,
                       (const uint32_t*)work);
    hipLaunchKernelGGL(k_sr_index, dim3(2048), dim3(SRC_TB), 0, st, (const uint32_t*)g->hdr, g->pool, g->rule,
                       max_count, (const uint32_t*)work);
}

int quantize_biases(uint64_t m, const float* b, double lambda, uint32_t F, uint32_t* w, hipStream_t st) {
    if (m == 0) return BINGO_OK;
    hipLaunchKernelGGL(k_quantize, dim3(grid_for(m, 256)), dim3(256), 0, st, m, b, lambda, F, w);
    return hipGetLastError() == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

int build_graph(bingo_graph* g, uint64_t m, const uint32_t* src, const uint32_t* dst, const uint32_t* w,
                hipStream_t st) {
    const uint32_t n = g->n;
    HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
    if (m) hipLaunchKernelGGL(k_validate, dim3(grid_for(m, 256)), dim3(256), 0, st, m, n, src, dst, w, g->d_err);
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (err) return err_to_code(err);

    // scratch layout
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t mm = m ? m : 1;
    const size_t sort_tmp = sort_temp_bytes(mm, false);
    const size_t scan_tmp = scan_temp_bytes((uint64_t)n + 1);
    const size_t need = al(mm * 4) * 4 + al(((uint64_t)n + 1) * 4) + 2 * al(((uint64_t)n + 1) * 8) * 2 +
                        std::max(sort_tmp, scan_tmp) + 1024;
    char* ws = (char*)ws_get(g, need);
    if (!ws) return BINGO_E_OOM;
    uint32_t* ids = (uint32_t*)ws;            ws += al(mm * 4);
    uint32_t* skeys = (uint32_t*)ws;          ws += al(mm * 4);
    uint32_t* sids = (uint32_t*)ws;           ws += al(mm * 4);
    uint32_t* cdst = ids;                     // ids are dead after the sort
    uint32_t* cw = (uint32_t*)ws;             ws += al(mm * 4);
    uint32_t* start = (uint32_t*)ws;          ws += al(((uint64_t)n + 1) * 4);
    uint64_t* adjw = (uint64_t*)ws;           ws += al(((uint64_t)n + 1) * 8);
    uint64_t* listw = (uint64_t*)ws;          ws += al(((uint64_t)n + 1) * 8);
    uint64_t* adj_off = (uint64_t*)ws;        ws += al(((uint64_t)n + 1) * 8);
    uint64_t* list_off = (uint64_t*)ws;       ws += al(((uint64_t)n + 1) * 8);
    unsigned long long* totals = (unsigned long long*)ws;  ws += 256;
    void* tmp = ws;

    if (m) {
        hipLaunchKernelGGL(k_iota, dim3(grid_for(m, 256)), dim3(256), 0, st, ids, m);
        sort_pairs_u32(src, ids, skeys, sids, m, bits_for(n - 1), tmp, st);
        hipLaunchKernelGGL(k_gather, dim3(grid_for(m, 256)), dim3(256), 0, st, m, sids, dst, w, cdst, cw);
    }
    hipLaunchKernelGGL(k_row_start, dim3(((uint64_t)n + 1 + 255) / 256), dim3(256), 0, st, skeys, m, n, start);
    const uint32_t vgrid = (uint32_t)(((uint64_t)n + 3) / 4);
    const bool r4 = g->radix_base == 4;
    if (r4) hipLaunchKernelGGL(k_header4, dim3(vgrid), dim3(WB), 0, st, n, start, cw, g->hdr, adjw, listw, g->rule);
    else hipLaunchKernelGGL(k_header, dim3(vgrid), dim3(WB), 0, st, n, start, cw, g->hdr, adjw, listw, g->rule);
    scan_u64(adjw, adj_off, n, tmp, totals, st);
    scan_u64(listw, list_off, n, tmp, totals + 1, st);
    unsigned long long tot[2];
    HIPCHK(hipMemcpyAsync(tot, totals, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint64_t used = tot[0] + tot[1];
    uint64_t pool_words = g->pool_words;  // requested size (words), 0 = automatic
    if (pool_words == 0) pool_words = used * 2 + (4ull << 20);  // twice the input plus 16 MB; grows on demand
    if (pool_words < used + 1024) return BINGO_E_OOM;
    if (pool_words > (1ull << 35)) pool_words = std::max<uint64_t>(1ull << 35, used + 1024);
    if (used + 1024 > (1ull << 35)) return BINGO_E_OOM;  // list offsets are 32-bit in 32-byte units
    if (hipMalloc(&g->pool, pool_words * 4) != hipSuccess) {
        g->pool = nullptr;
        return BINGO_E_OOM;
    }
    g->pool_words = pool_words;
    if (r4)
        hipLaunchKernelGGL(k_fill4, dim3(vgrid), dim3(WB), 0, st, n, start, cdst, cw, adj_off, list_off,
                           (uint64_t)tot[0], g->hdr, g->pool, g->rule);
    else
        hipLaunchKernelGGL(k_fill, dim3(vgrid), dim3(WB), 0, st, n, start, cdst, cw, adj_off, list_off,
                           (uint64_t)tot[0], g->hdr, g->pool, g->rule);
    if (g->alias_mode) {
        if (hipMalloc(&g->alias, (size_t)n * ALIAS_ENTRIES * sizeof(uint4)) != hipSuccess) {
            g->alias = nullptr;
            return BINGO_E_OOM;
        }
        g->rule.alias = g->alias;
        alias_rows(g, nullptr, nullptr, n, st);
    }
    unsigned long long ctl[2] = {(unsigned long long)used, 0ull};
    HIPCHK(hipMemcpyAsync(g->d_ctl, ctl, 16, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return BINGO_OK;
}

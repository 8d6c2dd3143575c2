// step.h -- one first-order transition on the radix-group sampling space
// (Sec. 4.1 hierarchical sampling: group by inverse transform over
// c_k 2^k, Eq. eq:group_prob; member uniformly, Eq. eq:pvp; rejection on
// the adjacency for dense groups, Sec. 5.1), and the chunked walk-id queue
// of the persistent kernels.  Shared by the walk kernels.
#pragma once
#include "dev.h"

namespace {

constexpr uint32_t PENDING = 0xFFFFFFFEu;
constexpr uint64_t NO_WALK = ~0ull;

// One round of SPEC dense-rejection attempts.  The attempt indices depend only
// on the random stream, not on the loaded words, so the SPEC loads are issued
// together and the dependent chain of a step shrinks from one load per attempt
// to one per round.  The accepted slot is the first accepting attempt in stream
// order, exactly as with one attempt at a time; words drawn for attempts after
// it are never used (every step, and every node2vec proposal, starts a fresh
// stream).  Returns PENDING when no
// attempt of the round accepts.
template <int SPEC>
__device__ __forceinline__ uint32_t dense_round(const uint64_t* __restrict__ edges, uint32_t d, uint32_t sel,
                                                RandStream& rs) {
    uint64_t e[SPEC];
#pragma unroll
    for (int a = 0; a < SPEC; ++a) e[a] = edges[rs_below32(rs, d)];
    uint32_t v = PENDING;
#pragma unroll
    for (int a = SPEC - 1; a >= 0; --a)
        if ((e[a] >> (32 + sel)) & 1ull) v = (uint32_t)e[a];
    return v;
}

// The decimal group of fixed-point biases (slot 0; Sec. 4.3): its members weigh
// their fractions q = weight mod 2^F.  A one-element group returns its member;
// otherwise a candidate is drawn uniformly from the group's list (listed types)
// or from the whole adjacency (dense) and accepted when the top F bits of the
// next random word are below its q.  Every member has q >= 1, so an attempt
// accepts with probability at least 2^-F (at least alpha % of that for the
// dense form); the attempt bound (2^24, with F <= 16) is never reached on a
// consistent structure and only keeps a corrupted one from spinning.
constexpr uint32_t DEC_MAX_ATTEMPTS = 1u << 24;

__device__ __forceinline__ uint32_t decimal_pick(const uint32_t* __restrict__ h, const uint32_t* __restrict__ pool,
                                                 uint64_t adj, uint32_t d, uint32_t slot0, uint32_t onem,
                                                 GroupRule rule, RandStream& rs) {
    if (onem & 1u) return slot0;  // one member: its destination sits in the slot
    const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + adj);
    const uint32_t c0 = slot0;
    const uint32_t t = group_type(c0, d, rule);
    const uint32_t info = h[H_INFO];
    const uint32_t fm = (1u << rule.fbits) - 1u;
    const uint64_t lst = (uint64_t)info * LIST_UNIT_WORDS;
    for (uint32_t att = 0; att < DEC_MAX_ATTEMPTS; ++att) {
        const uint32_t i = type_listed(t) ? pool[lst + rs_below32(rs, c0)] : rs_below32(rs, d);
        const uint32_t x = rs_next32(rs) >> (32 - rule.fbits);
        const uint64_t e = edges[i];
        if (x < ((uint32_t)(e >> 32) & fm)) return (uint32_t)e;
    }
    return STOP_VERTEX;
}

// The group choice of a step at u (Sec. 4.1: group k with probability
// c_k 2^k / W, Eq. eq:group_prob).  Returns false at a vertex without out-edges.
// MODE 0 (integer biases, inverse transform): the ascending scan picks the k
// with prefix(k-1) <= r < prefix(k); with t = W - r that is the k with
// suffix(k+1) < t <= suffix(k), found from the top.  The header's first 64
// bytes hold the ten highest groups, so a step reads the rest of the slots
// only when t exceeds their total.  MODE 1 (fixed-point biases): integer
// groups F..31 ascending, the decimal group (slot 0) last, over all slots.
// MODE 2: the alias table picks the group; its slot comes from the first 64
// bytes when it is among the ten highest.
struct GroupPick {
    int sel;         // the group; -1: the decimal group (MODE 1), or an inconsistent header
    uint32_t csel;   // its count
    uint32_t raw;    // its slot word (a one-element group's destination)
    uint32_t d, onem, hi;
    uint32_t slot0;  // MODE 1: slot of group 0, the decimal group's count
    uint64_t adj;
};

template <int MODE>
__device__ __forceinline__ bool pick_group(const uint32_t* __restrict__ hdr, uint32_t u, RandStream& rs,
                                           GroupRule rule, GroupPick& g) {
    const uint32_t* __restrict__ h = hdr + (size_t)u * HDR_WORDS;
    const uint4* h4 = reinterpret_cast<const uint4*>(h);
    const uint4 q0 = h4[0], q1 = h4[1], q2 = h4[2], q3 = h4[3];
    g.d = q0.y;
    if (g.d == 0) return false;
    const uint64_t W = ((uint64_t)q0.w << 32) | q0.z;
    g.onem = q0.x;
    g.hi = q1.y >> H_HI_SHIFT;
    g.adj = ((uint64_t)(q1.y & H_ADJHI_MASK) << 32) | q1.x;
    g.sel = -1;
    g.csel = g.raw = g.slot0 = 0;
    uint32_t sl[32];  // sl[r]: slot of group hi - r
    sl[0] = q1.z; sl[1] = q1.w;
    sl[2] = q2.x; sl[3] = q2.y; sl[4] = q2.z; sl[5] = q2.w;
    sl[6] = q3.x; sl[7] = q3.y; sl[8] = q3.z; sl[9] = q3.w;
    if constexpr (MODE == 2) {
        // alias table: slot j from the top 5 bits of a word, then x < W against the slot's cut
        const uint32_t j = rs_next32(rs) >> 27;
        const uint4 e = rule.alias[(size_t)u * ALIAS_ENTRIES + j];
        const uint64_t x = rs_below64(rs, W);
        const uint32_t k = x < (((uint64_t)e.y << 32) | e.x) ? j : e.z;
        if (k > g.hi) return true;  // an empty group: only on an inconsistent structure
        const uint32_t r = g.hi - k;
        uint32_t raw = 0;
        if (r < 10) {
#pragma unroll
            for (int q = 0; q < 10; ++q)
                if ((uint32_t)q == r) raw = sl[q];
        } else {
            raw = h[H_CNT + r];
        }
        g.sel = (int)k;
        g.raw = raw;
        g.csel = ((g.onem >> k) & 1u) ? 1u : raw;
    } else if constexpr (MODE == 1) {
        const uint4 q4 = h4[4], q5 = h4[5], q6 = h4[6], q7 = h4[7], q8 = h4[8], q9 = h4[9];
        sl[10] = q4.x; sl[11] = q4.y; sl[12] = q4.z; sl[13] = q4.w;
        sl[14] = q5.x; sl[15] = q5.y; sl[16] = q5.z; sl[17] = q5.w;
        sl[18] = q6.x; sl[19] = q6.y; sl[20] = q6.z; sl[21] = q6.w;
        sl[22] = q7.x; sl[23] = q7.y; sl[24] = q7.z; sl[25] = q7.w;
        sl[26] = q8.x; sl[27] = q8.y; sl[28] = q8.z; sl[29] = q8.w;
        sl[30] = q9.x; sl[31] = q9.y;
        // integer groups F..31 ascending (ranks descending), the decimal group last
        const uint64_t r = rs_below64(rs, W);
        uint64_t acc = 0;
#pragma unroll
        for (int q = 31; q >= 0; --q) {
            if ((uint32_t)q <= g.hi) {
                const uint32_t k = g.hi - (uint32_t)q;
                const uint32_t ck = ((g.onem >> k) & 1u) ? 1u : sl[q];
                if (k == 0) g.slot0 = sl[q];
                if (k >= rule.fbits) acc += (uint64_t)ck << k;
                if (g.sel < 0 && r < acc) { g.sel = (int)k; g.csel = ck; g.raw = sl[q]; }
            }
        }
    } else {
        const uint64_t t = W - rs_below64(rs, W);  // in [1, W]
        uint64_t acc = 0;
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            if (g.sel < 0 && (uint32_t)q <= g.hi) {
                const uint32_t k = g.hi - (uint32_t)q;
                const uint32_t ck = ((g.onem >> k) & 1u) ? 1u : sl[q];
                acc += (uint64_t)ck << k;
                if (acc >= t) { g.sel = (int)k; g.csel = ck; g.raw = sl[q]; }
            }
        }
        if (g.sel < 0 && g.hi >= 10) {
            const uint4 q4 = h4[4], q5 = h4[5], q6 = h4[6], q7 = h4[7];
            sl[10] = q4.x; sl[11] = q4.y; sl[12] = q4.z; sl[13] = q4.w;
            sl[14] = q5.x; sl[15] = q5.y; sl[16] = q5.z; sl[17] = q5.w;
            sl[18] = q6.x; sl[19] = q6.y; sl[20] = q6.z; sl[21] = q6.w;
            sl[22] = q7.x; sl[23] = q7.y; sl[24] = q7.z; sl[25] = q7.w;
#pragma unroll
            for (int q = 10; q < 26; ++q) {
                if (g.sel < 0 && (uint32_t)q <= g.hi) {
                    const uint32_t k = g.hi - (uint32_t)q;
                    const uint32_t ck = ((g.onem >> k) & 1u) ? 1u : sl[q];
                    acc += (uint64_t)ck << k;
                    if (acc >= t) { g.sel = (int)k; g.csel = ck; g.raw = sl[q]; }
                }
            }
            if (g.sel < 0 && g.hi >= 26) {
                const uint4 q8 = h4[8], q9 = h4[9];
                sl[26] = q8.x; sl[27] = q8.y; sl[28] = q8.z; sl[29] = q8.w;
                sl[30] = q9.x; sl[31] = q9.y;
#pragma unroll
                for (int q = 26; q < 32; ++q) {
                    if (g.sel < 0 && (uint32_t)q <= g.hi) {
                        const uint32_t k = g.hi - (uint32_t)q;
                        const uint32_t ck = ((g.onem >> k) & 1u) ? 1u : sl[q];
                        acc += (uint64_t)ck << k;
                        if (acc >= t) { g.sel = (int)k; g.csel = ck; g.raw = sl[q]; }
                    }
                }
            }
        }
    }
    return true;
}

// One transition from u (no termination test).  Returns the next vertex or
// STOP_VERTEX for a vertex without out-edges.  MODE 0: integer biases, inverse
// transform over the groups; 1: fixed-point biases (rule.fbits > 0, decimal
// group taken last); 2: integer biases, alias table (rule.alias).  Each
// instance carries only its own selection code.
template <int SPEC, int MODE>
__device__ __forceinline__ uint32_t walk_step_body(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                   uint32_t u, RandStream& rs, GroupRule rule) {
    GroupPick g;
    if (!pick_group<MODE>(hdr, u, rs, rule, g)) return STOP_VERTEX;
    if (MODE == 1 && g.sel < 0)
        return decimal_pick(hdr + (size_t)u * HDR_WORDS, pool, g.adj, g.d, g.slot0, g.onem, rule, rs);
    if (g.sel < 0) return STOP_VERTEX;  // only on an inconsistent header
    if ((g.onem >> g.sel) & 1u) return g.raw;  // one-element group: the step ends in the header
    const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + g.adj);
    const uint32_t t = group_type(g.csel, g.d, rule);
    if (t == GT_DENSE) {
        // rejection on the whole neighbor list: accept a slot whose weight has
        // bit sel.  Acceptance is above alpha % per attempt, so the bound is
        // never reached on a consistent structure; it only keeps a corrupted
        // one from spinning forever.
        for (uint32_t att = 0; att < (1u << 16); att += SPEC) {
            const uint32_t v = dense_round<SPEC>(edges, g.d, (uint32_t)g.sel, rs);
            if (v != PENDING) return v;
        }
        return STOP_VERTEX;
    }
    const uint32_t info = hdr[(size_t)u * HDR_WORDS + H_INFO + g.sel];
    const uint32_t i = pool[(uint64_t)info * LIST_UNIT_WORDS + rs_below32(rs, g.csel)];
    return pool[g.adj + 2ull * i];
}

// Walk ids are handed to waves in chunks: one atomic per QCHUNK ids, and the
// lanes of a wave that need a walk take consecutive ids from the chunk.
struct WaveQueue {
    uint64_t next = 0, end = 0;  // identical in every lane of the wave
    uint32_t chunk = 256;
};

__device__ __forceinline__ uint64_t wave_take_chunked(bool need, WaveQueue& q, unsigned long long* head) {
    const uint64_t want = __ballot(need);
    if (!want) return NO_WALK;
    const uint32_t cnt = __popcll(want);
    const uint32_t rank = __popcll(want & lanemask_lt());
    const uint64_t avail = q.end - q.next;
    uint64_t id;
    if (avail >= cnt) {
        id = q.next + rank;
        q.next += cnt;
    } else {
        // reserve enough whole chunks for every lane that is still short
        const uint64_t chunks = (cnt - avail + q.chunk - 1) / q.chunk;
        unsigned long long nb = 0;
        if (lane_id() == 0) nb = atomicAdd(head, (unsigned long long)(chunks * q.chunk));
        nb = __shfl(nb, 0, 64);
        id = rank < avail ? q.next + rank : nb + (rank - avail);
        q.next = nb + (cnt - avail);
        q.end = nb + chunks * q.chunk;
    }
    return need ? id : NO_WALK;
}

__device__ __forceinline__ void wave_add_u64(unsigned long long* p, uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0 && v) atomicAdd(p, (unsigned long long)v);
}

}  // namespace

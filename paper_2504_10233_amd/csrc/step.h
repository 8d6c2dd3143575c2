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

// One transition from u (no termination test).  Returns the next vertex or
// STOP_VERTEX for a vertex without out-edges.  MODE 0: integer biases, inverse
// transform over the groups; 1: fixed-point biases (rule.fbits > 0, decimal
// group taken last); 2: integer biases, alias table (rule.alias).  Each
// instance carries only its own selection code.
template <int SPEC, int MODE>
__device__ __forceinline__ uint32_t walk_step_body(const uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                                                   uint32_t u, RandStream& rs, GroupRule rule) {
    const uint4* h4 = reinterpret_cast<const uint4*>(hdr + (size_t)u * HDR_WORDS);
    // line 0 of the header in one go: mask, d, W, adjacency offset, c_0..c_25
    const uint4 q0 = h4[0], q1 = h4[1], q2 = h4[2], q3 = h4[3], q4 = h4[4], q5 = h4[5], q6 = h4[6], q7 = h4[7];
    const uint32_t d = q0.y;
    if (d == 0) return STOP_VERTEX;
    const uint64_t W = ((uint64_t)q0.w << 32) | q0.z;
    const uint32_t c[26] = {q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z,
                            q4.w, q5.x, q5.y, q5.z, q5.w, q6.x, q6.y, q6.z, q6.w, q7.x, q7.y, q7.z, q7.w};
    // groups in ascending k; fixed-point biases skip the slots below F (slot 0
    // is their decimal group, taken last)
    // (a one-element group's slot holds its member's destination; its count is 1)
    const uint32_t fb = (MODE == 1) ? rule.fbits : 0u;
    const uint32_t onem = q0.x;
    uint64_t acc = 0;
    int sel = -1;
    uint32_t csel = 0, raw = 0;
    if constexpr (MODE == 2) {
        // alias table: slot j from the top 5 bits of a word, then x < W against the slot's cut
        const uint32_t j = rs_next32(rs) >> 27;
        const uint4 e = rule.alias[(size_t)u * ALIAS_ENTRIES + j];
        const uint64_t x = rs_below64(rs, W);
        sel = x < (((uint64_t)e.y << 32) | e.x) ? (int)j : (int)e.z;
        if (sel < 26) {
#pragma unroll
            for (int k = 0; k < 26; ++k)
                if (k == sel) raw = c[k];
        } else {
            raw = hdr[(size_t)u * HDR_WORDS + H_CNT + sel];
        }
        csel = ((onem >> sel) & 1u) ? 1u : raw;
    } else {
        const uint64_t r = rs_below64(rs, W);
#pragma unroll
        for (int k = 0; k < 26; ++k) {
            const uint32_t ck = ((onem >> k) & 1u) ? 1u : c[k];
            if ((uint32_t)k >= fb) acc += (uint64_t)ck << k;
            if (sel < 0 && r < acc) { sel = k; csel = ck; raw = c[k]; }
        }
        if (sel < 0) {
            const uint4 a = h4[8], b = h4[9];
            const uint32_t hc[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const uint32_t ck = ((onem >> (26 + k)) & 1u) ? 1u : hc[k];
                acc += (uint64_t)ck << (26 + k);
                if (sel < 0 && r < acc) { sel = 26 + k; csel = ck; raw = hc[k]; }
            }
        }
    }
    const uint64_t adj = ((uint64_t)q1.y << 32) | q1.x;
    if (MODE == 1 && sel < 0) return decimal_pick(hdr + (size_t)u * HDR_WORDS, pool, adj, d, c[0], onem, rule, rs);
    if (sel < 0) return STOP_VERTEX;  // only on an inconsistent header
    if ((onem >> sel) & 1u) return raw;  // one-element group: the step ends on line 0
    const uint64_t* __restrict__ edges = reinterpret_cast<const uint64_t*>(pool + adj);
    const uint32_t t = group_type(csel, d, rule);
    if (t == GT_DENSE) {
        // rejection on the whole neighbor list: accept a slot whose weight has
        // bit sel.  Acceptance is above alpha % per attempt, so the bound is
        // never reached on a consistent structure; it only keeps a corrupted
        // one from spinning forever.
        for (uint32_t att = 0; att < (1u << 16); att += SPEC) {
            const uint32_t v = dense_round<SPEC>(edges, d, (uint32_t)sel, rs);
            if (v != PENDING) return v;
        }
        return STOP_VERTEX;
    }
    const uint32_t info = hdr[(size_t)u * HDR_WORDS + H_INFO + sel];
    const uint32_t i = pool[(uint64_t)info * LIST_UNIT_WORDS + rs_below32(rs, csel)];
    return pool[adj + 2ull * i];
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

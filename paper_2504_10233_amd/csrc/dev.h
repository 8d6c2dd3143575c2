// dev.h -- device data layout and device helpers shared by the HIP kernels of
// libbingo (radix-based bias factorization, arXiv 2504.10233), gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "bingo.h"

// ---------------------------------------------------------------------------
// Per-vertex header: the inter-group sampling space of Sec. 3 / Sec. 4.1, one
// fixed 384-byte slot (three 128-byte lines) per vertex, 128-byte aligned.
//   words 0..5: mask of one-element groups, degree d, W = sum_k c_k 2^k (u64),
//           adjacency block offset (u64, in pool words; bits 24..28 of its
//           high word hold hi, the highest non-empty group)
//   words 6..37: the group slots by rank from the top: word 6 + r holds the
//           slot of group hi - r (r = 0..hi)
//   words 38..69: info_k, k = 0..31
//   line 2: adjacency capacity, next sequence number, log2 of each listed
//           group's list capacity (bytes), mask of non-empty groups, the
//           reduced list S(u) (block offset, length, capacity), spare
// Slot k holds c_k, except for a one-element group (c_k = 1), whose slot holds
// its member's destination vertex: a step that selects such a group ends in
// the header without touching the adjacency.  info_k is the member index of a
// one-element group, or the offset of a listed group's list block in 32-byte
// units of the pool.  Dense and empty groups have no info.  The first 64 bytes
// hold W, d, the offset and the ten highest groups, which carry all but a
// fraction 2^-10 or less of W's mass when the top group is full; a walk step
// picks its group from the top (suffix sums) and reads further only when the
// draw falls below them.
// ---------------------------------------------------------------------------
#define HDR_WORDS 96
#define H_ONEMASK 0
#define H_MASK 80
#define H_DEG 1
#define H_WLO 2
#define H_WHI 3
#define H_ADJLO 4
#define H_ADJHI 5
#define H_CNT 6        // 32 words
#define H_INFO 38      // 32 words
#define H_ACAP 70
#define H_NSEQ 71
#define H_LCAPLOG 72   // 32 bytes = 8 words
#define H_SBLK 81      // S(u) block offset in 32-byte units (valid when H_SCAP > 0)
#define H_SLEN 82      // |S(u)|
#define H_SCAP 83      // S(u) capacity in entries (0: the vertex has no sparse group)
#define H_HI_SHIFT 24  // hi in the high word of the adjacency offset
#define H_ADJHI_MASK 0x00FFFFFFu
#define STOP_VERTEX 0xFFFFFFFFu

// ---------------------------------------------------------------------------
// Radix base 4 (Supplement S.2): a weight is read as base-4 digits d_k, k = 0..15;
// subgroup s = 3k + v - 1 (v = 1..3) holds the edges whose digit k is v, each
// carrying v 4^k, so its total is c_s v 4^k.  Static structure (build and walks).
// Per-vertex header of 128 words (512 bytes):
//   degree, adjacency capacity, W (u64), adjacency offset (u64), mask of
//   one-element subgroups (u64), mask of non-empty subgroups (u64), slot s for
//   s = 0..47 (c_s, or a one-element subgroup's destination), info s (member
//   index, or list block offset in 32-byte units), log2 of the list capacities
//   (one byte per subgroup).  Adjacency block: cap 64-bit words dst | w << 32.
// ---------------------------------------------------------------------------
#define R4_SUB 48
#define H4_WORDS 128
#define H4_DEG 0
#define H4_ACAP 1
#define H4_WLO 2
#define H4_WHI 3
#define H4_ADJLO 4
#define H4_ADJHI 5
#define H4_ONELO 6
#define H4_ONEHI 7
#define H4_MASKLO 8
#define H4_MASKHI 9
#define H4_SLOT 10
#define H4_INFO 58
#define H4_LCAPLOG 106  // 12 words
__host__ __device__ inline uint32_t r4_digit(uint32_t w, uint32_t k) { return (w >> (2 * k)) & 3u; }
__host__ __device__ inline uint64_t r4_adj_words(uint32_t cap) { return ((uint64_t)cap * 2 + 7) & ~7ull; }

// c_k from slot k (one-element groups keep their member's destination there)
__host__ __device__ inline uint32_t slot_count(uint32_t slot, uint32_t onemask, uint32_t k) {
    return ((onemask >> k) & 1u) ? 1u : slot;
}
// the highest non-empty group of a mask (0 for an empty one)
__host__ __device__ inline uint32_t mask_hi(uint32_t mask) { return mask ? 31u - (uint32_t)__builtin_clz(mask) : 0u; }
// header fields: adjacency offset, hi, and the slot of group k (0 above hi: those groups are empty)
__host__ __device__ inline uint64_t hdr_adj(const uint32_t* h) {
    return ((uint64_t)(h[H_ADJHI] & H_ADJHI_MASK) << 32) | h[H_ADJLO];
}
__host__ __device__ inline uint32_t hdr_hi(const uint32_t* h) { return h[H_ADJHI] >> H_HI_SHIFT; }
__host__ __device__ inline uint32_t hdr_slot(const uint32_t* h, uint32_t k, uint32_t hi) {
    return k <= hi ? h[H_CNT + (hi - k)] : 0u;
}
// the high word of the adjacency offset with hi
__host__ __device__ inline uint32_t adjhi_word(uint64_t adj, uint32_t hi) {
    return (uint32_t)(adj >> 32) | (hi << H_HI_SHIFT);
}

// Adjacency block of capacity cap (words): cap edge words of 64 bits
// (dst | weight << 32) followed by cap sequence numbers (u32).
// List block of a listed group (Sec. 4.2 intra-group neighbor index list and
// inverted index; Sec. 5.1 sparse and regular groups), 32-byte aligned:
//   [0, lcap)              the list L: neighbor indices
//   [lcap, lcap + icap)    the group's index.  Regular: icap = the adjacency
//                          capacity, entry i = position of neighbor index i in
//                          L.  Sparse: icap = the capacity of the vertex's
//                          reduced list S(u), entry s = position of S[s] in L.
// Only the entries of members are kept: an entry is valid when it is below c
// and L at that position holds the index (resp. S[s]), so no index needs
// clearing.  S(u) block: the neighbor indices, ascending, of the edges that
// belong to at least one sparse group of u (capacity H_SCAP entries).
#define LIST_UNIT_WORDS 8u

enum { GT_EMPTY = 0, GT_ONE = 1, GT_DENSE = 2, GT_SPARSE = 3, GT_REGULAR = 4 };

// Sticky device error bits (mapped to BINGO_E_* on the host).
#define ERR_RANGE 1u
#define ERR_WEIGHT 2u
#define ERR_OOM 4u
#define ERR_INTERNAL 8u

#define PHASE_EVENTS 8

struct GroupRule {
    uint32_t adaptive, alpha, beta;
    uint32_t fbits;  // 0: integer biases; F: fixed-point biases with F fraction bits (Sec. 4.3)
    // alias-table inter-group choice: ALIAS_ENTRIES entries {cut lo, cut hi, alias, 0} per vertex;
    // nullptr: inverse transform
    const uint4* alias;
};
#define ALIAS_ENTRIES 32

// Group membership word of a stored weight: bit k set = member of group k.
// Integer biases: the weight itself.  Fixed-point biases with F fraction bits:
// bits F..31 (the integer part's radix groups) and bit 0 for the decimal group
// (a nonzero fraction); bits 1..F-1 are never set.
__host__ __device__ inline uint32_t member_word(uint32_t w, uint32_t fbits) {
    if (!fbits) return w;
    const uint32_t fm = (1u << fbits) - 1u;
    return (w & ~fm) | ((w & fm) != 0u ? 1u : 0u);
}

// Group type from (count, degree): empty, one element, dense above alpha %,
// sparse below beta %, regular otherwise, in that order (Sec. 5.1).
__host__ __device__ inline uint32_t group_type(uint32_t c, uint32_t d, GroupRule r) {
    if (c == 0) return GT_EMPTY;
    if (!r.adaptive) return GT_REGULAR;
    if (c == 1) return GT_ONE;
    uint64_t c100 = (uint64_t)c * 100u;
    if (c100 > (uint64_t)r.alpha * d) return GT_DENSE;
    if (c100 < (uint64_t)r.beta * d) return GT_SPARSE;
    return GT_REGULAR;
}
__host__ __device__ inline bool type_listed(uint32_t t) { return t == GT_SPARSE || t == GT_REGULAR; }

// Pool block sizes (the dynamic arrays of Sec. 5.2; the pool is bump-allocated in
// 32-byte units).  A vertex of d edges has an adjacency block of capacity
// 2^ceil(log2 d), at least 2 (none for d = 0): cap 64-bit edge words, then cap
// sequence numbers, rounded up to 8 words.  A listed group of c members has a
// list of max(8, 2^ceil(log2 c)) entries.  Every path that allocates or frees
// blocks (build, batched and streaming updates, compaction) uses these sizes.
__host__ __device__ inline uint32_t adj_cap_for(uint32_t d) {
    if (d == 0) return 0;
    uint32_t c = 2;
    while (c < d) c <<= 1;
    return c;
}
__host__ __device__ inline uint64_t adj_block_words(uint32_t cap) { return ((uint64_t)cap * 3 + 7) & ~7ull; }
__host__ __device__ inline uint32_t list_cap_for(uint32_t c) {
    uint32_t x = 8;
    while (x < c) x <<= 1;
    return x;
}
// index capacity of a listed group of type t: the adjacency capacity (regular)
// or the S(u) capacity (sparse)
__host__ __device__ inline uint32_t index_cap_for(uint32_t t, uint32_t acap, uint32_t scap) {
    return t == GT_REGULAR ? acap : (t == GT_SPARSE ? scap : 0u);
}
// words of a list block: the list, then the index, rounded to the 32-byte unit
__host__ __device__ inline uint64_t list_block_words(uint32_t lcap, uint32_t icap) {
    return ((uint64_t)lcap + icap + 7) & ~7ull;
}
// S(u) capacity for an upper bound on |S(u)| (0: no sparse group)
__host__ __device__ inline uint32_t s_cap_for(uint32_t n) { return n ? list_cap_for(n) : 0u; }

// ---------------------------------------------------------------------------
// Counter-based random stream (Philox-4x32-10, Salmon et al. SC'11).  The
// stream of a walk step is keyed by the 64-bit seed; its counter holds the
// 64-bit walk id, the step and a block index.  Words are consumed in block
// order; a 64-bit draw takes the first word as its high half.
// ---------------------------------------------------------------------------
struct RandStream {
    uint32_t k0, k1, w0, w1, step, blk;
    uint32_t b0, b1, b2, b3;
    uint32_t left;
};

__device__ __forceinline__ void philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1, uint32_t& o0, uint32_t& o1,
                                             uint32_t& o2, uint32_t& o3) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo_a = 0xD2511F53u * c0;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

__device__ __forceinline__ void rs_init(RandStream& s, uint64_t seed, uint64_t walk, uint32_t step) {
    s.k0 = (uint32_t)seed; s.k1 = (uint32_t)(seed >> 32);
    s.w0 = (uint32_t)walk; s.w1 = (uint32_t)(walk >> 32);
    s.step = step; s.blk = 0; s.left = 0;
}

// The same stream starting at block blk0 (node2vec proposals use disjoint block ranges of a step's stream).
__device__ __forceinline__ void rs_init_blk(RandStream& s, uint64_t seed, uint64_t walk, uint32_t step, uint32_t blk0) {
    rs_init(s, seed, walk, step);
    s.blk = blk0;
}

__device__ __forceinline__ uint32_t rs_next32(RandStream& s) {
    if (s.left == 0) {
        philox_block(s.w0, s.w1, s.step, s.blk, s.k0, s.k1, s.b0, s.b1, s.b2, s.b3);
        s.blk++;
        s.left = 4;
    }
    const uint32_t v = s.b0;
    s.b0 = s.b1; s.b1 = s.b2; s.b2 = s.b3;
    s.left--;
    return v;
}

__device__ __forceinline__ uint64_t rs_next64(RandStream& s) {
    const uint64_t hi = rs_next32(s);
    return (hi << 32) | rs_next32(s);
}

// Exact uniform draw on [0, n), n >= 1: multiply the word by n, keep the high
// half, and redraw while the low half falls in the biased zone below
// (2^32 - n) mod n (Lemire, ACM TOMACS 2019).
__device__ __forceinline__ uint32_t rs_below32(RandStream& s, uint32_t n) {
    uint64_t m = (uint64_t)rs_next32(s) * n;
    uint32_t low = (uint32_t)m;
    if (low < n) {
        const uint32_t zone = (0u - n) % n;
        while (low < zone) {
            m = (uint64_t)rs_next32(s) * n;
            low = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

__device__ __forceinline__ uint64_t rs_below64(RandStream& s, uint64_t n) {
    uint64_t x = rs_next64(s);
    uint64_t low = x * n;
    uint64_t high = __umul64hi(x, n);
    if (low < n) {
        const uint64_t zone = (0ull - n) % n;
        while (low < zone) {
            x = rs_next64(s);
            low = x * n;
            high = __umul64hi(x, n);
        }
    }
    return high;
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ---------------------------------------------------------------------------
// Host-side graph handle.
// ---------------------------------------------------------------------------
#define WALK_SLOTS 64
struct bingo_graph {
    uint32_t n;
    GroupRule rule;
    uint32_t* hdr;          // n * HDR_WORDS
    uint4* alias = nullptr;  // alias-table mode: n * ALIAS_ENTRIES entries
    uint32_t alias_mode = 0;
    uint32_t* pool;         // device arena, pool_words u32
    uint64_t pool_words;
    bool pool_auto;  // sized by the library (bingo_config.pool_bytes = 0): may grow
    unsigned long long* d_ctl;  // [0] words used, [1] garbage words
    uint32_t* d_err;        // sticky error bits
    // last PPR result
    uint64_t* ppr_off = nullptr;
    uint32_t* ppr_vtx = nullptr;
    uint32_t* ppr_cnt = nullptr;
    uint64_t ppr_entries = 0, ppr_cap = 0;
    uint32_t ppr_nsrc = 0, ppr_off_cap = 0;
    // bingo_ppr_async: the histogram of the last query still running on another stream until
    // ppr_done; ppr_h0..ppr_h1 time it; its entry count lands in d_ctl[CTL_PPR_U]
    bool ppr_pending = false;
    hipEvent_t ppr_done = nullptr, ppr_h0 = nullptr, ppr_h1 = nullptr;
    // grow-only scratch for sorts, scans and temporaries
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // grow-only per-walk arrays of PPR calls (lengths, segments, active lists)
    void* aux = nullptr;
    size_t aux_bytes = 0;
    // ring of per-call counter slots for walks (queue head, transitions); slot_ev[i] is
    // recorded on the stream of the call that last held slot i, after its last use of it
    uint32_t walk_slot = 0;
    hipEvent_t slot_ev[WALK_SLOTS] = {};
    hipStream_t slot_st[WALK_SLOTS] = {};
    // persistent walk kernel: 0 = step-synchronous lanes, 1 = attempt-interleaved lanes
    uint32_t walk_variant = 1;
    uint32_t blocks_per_cu = 0;   // 0 = occupancy limit
    uint32_t queue_chunk = 256;
    // update pipeline: 1 = capture one hipGraph per batch-size bucket and replay it
    uint32_t update_graphs = 1;
    uint32_t dense_spec = 2;
    // persistent PPR: 1 = visits appended to per-source bins (rerun with segments on overflow), 0 = segments
    uint32_t ppr_bins = 1;
    // update pipeline: passes of a touched vertex over more than this many entries are split
    // into chunks processed over the whole GPU (0 = never)
    uint32_t update_split = 4096;
    // attempt-interleaved walks: dense steps at vertices of at least this degree are served by
    // the whole wave (0 = never)
    uint32_t wave_degree = 0;
    // update pipeline: 1 = deletes located through the edge locator (locate.h), 0 = by scanning
    // their source's adjacency
    uint32_t update_locate = 1;
    // edge locator: 16-byte slots (key, neighbour index; capacity loc_cap, a power of two); live
    // slots and slots ever taken (live + TOMB); valid = in step with the adjacency
    uint64_t* loc_tab = nullptr;
    uint64_t loc_cap = 0, loc_live = 0, loc_used = 0;
    bool loc_valid = false;
    struct UpdPlans* upd = nullptr;  // per-bucket workspaces and graphs (update.hip)
    // structure version: bumped by every applied update batch
    uint64_t version = 0;
    // node2vec neighbour index: per-vertex sorted destinations (node2vec.hip)
    uint32_t* n2v_idx = nullptr;
    uint64_t* n2v_off = nullptr;
    uint64_t n2v_cap = 0;
    uint64_t n2v_version = ~0ull;
    // radix base of the structure: 2 (the method) or 4 (Supplement S.2; hdr then holds
    // n * H4_WORDS words, and only walks, dumps and memory statistics are supported)
    uint32_t radix_base = 2;
    // per-phase timing of the last walk / PPR / update call (events on its stream)
    hipEvent_t ev[PHASE_EVENTS] = {};
    uint32_t nev = 0;
};
void phase_mark(bingo_graph* g, hipStream_t st, bool first);
// d_ctl layout (u64): [0] pool words used, [1] garbage words, [2..6] PPR
// counters, [7] asynchronous PPR entry count (CTL_PPR_U), [8..11] node2vec counters (CTL_N2V), [12..13] edge locator
// counters (CTL_LOC), [16 + 2*i .. 17 + 2*i] walk
// call slot i (WALK_SLOTS slots).
#define CTL_PPR_U 7  // entry count of the last asynchronous PPR histogram
#define CTL_N2V 8
#define CTL_LOC 12  // [12..13] edge locator counters (locate.hip)
#define CTL_WALK0 16
#define CTL_WORDS (CTL_WALK0 + 2 * WALK_SLOTS)

#define HIPCHK(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "libbingo: %s failed: %s (%s:%d)\n", #x,              \
                    hipGetErrorString(e_), __FILE__, __LINE__);                    \
            return BINGO_E_HIP;                                                    \
        }                                                                          \
    } while (0)

// Selection code of the walk kernels: 0 integer biases by inverse transform,
// 1 fixed-point biases, 2 integer biases by the alias table.
inline int walk_mode(const bingo_graph* g) { return g->rule.fbits ? 1 : (g->rule.alias ? 2 : 0); }

// ---------------------------------------------------------------------------
// Host launchers implemented in the .hip files.
// ---------------------------------------------------------------------------
// prim.hip: scans and LSD radix sort (stable), all on `stream`.
size_t scan_temp_bytes(uint64_t n);
// exclusive scan of n u32 or u64 values into u64 out; out may alias nothing; writes total to *d_total if non-null
void scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, void* temp, unsigned long long* d_total,
                     hipStream_t st);
void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, void* temp, unsigned long long* d_total,
              hipStream_t st);
size_t sort_temp_bytes(uint64_t n, bool wide_keys);
// stable sort of (keys, vals) by bits [0, bits) of the key; results in keys_out/vals_out
void sort_pairs_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                    uint64_t n, int bits, void* temp, hipStream_t st);
void sort_pairs_u64(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
                    uint64_t n, int bits, void* temp, hipStream_t st);
void sort_keys_u64(const uint64_t* keys_in, uint64_t* keys_out, uint64_t n, int bits, void* temp,
                   hipStream_t st);
// the same on the first min(nmax, *dn) entries, with launches sized by nmax (capturable)
void sort_pairs_u64_dn(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
                       uint64_t nmax, const unsigned long long* dn, int bits, void* temp, hipStream_t st);

// build.hip
// alias rows of the vertices list[0 .. *count) (list == nullptr: vertices 0 .. *count)
void alias_rows(bingo_graph* g, const uint32_t* list, const unsigned long long* count, uint64_t max_count,
                hipStream_t st);
// S(u) (Sec. 5.1) and every sparse group's index over it, rebuilt for the vertices
// list[0 .. *count) (list == nullptr: vertices 0 .. *count) whose dirty flag is set
// (dirty == nullptr: all of them), from the final adjacency, types and lists; work
// holds SPARSE_WORK_WORDS(max_count) u32 of scratch
#define SPARSE_WORK_WORDS(mc) (64 + 4 * (uint64_t)(mc) + 2 * (4 * (uint64_t)(mc) + 65536))
void sparse_rebuild(bingo_graph* g, const uint32_t* list, const unsigned long long* count, uint64_t max_count,
                    const uint32_t* dirty, uint32_t* work, hipStream_t st);
int quantize_biases(uint64_t m, const float* b, double lambda, uint32_t F, uint32_t* w, hipStream_t st);
int build_graph(bingo_graph* g, uint64_t m, const uint32_t* src, const uint32_t* dst, const uint32_t* w,
                hipStream_t st);
// radix4.hip
int launch_walk4(bingo_graph* g, uint64_t n_walks, const uint32_t* starts, uint64_t base, uint32_t len,
                 uint64_t seed, uint32_t* paths, uint64_t* steps, hipStream_t st);
int export_graph4(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
                  hipStream_t st);
int memory_stats4(bingo_graph* g, bingo_mem_stats* out, hipStream_t st);
// walk.hip
#define WALK_BATCH_MAX BINGO_WALK_BATCH_MAX
// the next walk counter slot for a call on st: if the call that held it last ran on another
// stream and may still be running, st first waits for it; the slot's words are cleared on st
int walk_slot_take(bingo_graph* g, hipStream_t st, uint32_t* slot);
// after the call's last use of the slot
int walk_slot_release(bingo_graph* g, uint32_t slot, hipStream_t st);
int launch_walk_batch(bingo_graph* g, uint32_t nq, const bingo_walk_query* hq, hipStream_t st);
int launch_walk(bingo_graph* g, uint64_t n_walks, const uint32_t* starts, uint64_t base, uint32_t len,
                uint64_t seed, uint32_t* paths, uint64_t* steps, uint32_t mode, hipStream_t st);
// hist_st: run the visit histogram there and return without waiting for it (nullptr: wait)
int run_ppr(bingo_graph* g, uint32_t nsrc, const uint32_t* sources, uint32_t R, uint32_t thr, uint32_t cap,
            uint64_t seed, uint64_t base, uint32_t mode, uint64_t* h_entries, uint64_t* h_steps,
            hipStream_t st, hipStream_t hist_st = nullptr);
// Finish a pending asynchronous histogram: wait for it, take its entry count (and its time).
int ppr_wait(bingo_graph* g, uint64_t* h_entries, float* h_hist_ms);
inline int ppr_drain(bingo_graph* g) { return g && g->ppr_pending ? ppr_wait(g, nullptr, nullptr) : BINGO_OK; }
// export.hip
int export_graph(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
                 hipStream_t st);
int export_index(bingo_graph* g, uint32_t u0, uint32_t u1, uint32_t* h_buf, uint64_t cap, uint64_t* h_len,
                 hipStream_t st);
int memory_stats(bingo_graph* g, bingo_mem_stats* out, hipStream_t st);
// update.hip
void update_release(bingo_graph* g);
void update_drop_graphs(bingo_graph* g);  // after the pool moves: captured graphs hold its old address
// compact.hip
int compact_pool(bingo_graph* g, uint64_t pool_words, hipStream_t st);
int run_node2vec(bingo_graph* g, uint64_t nw, const uint32_t* starts, uint64_t base, uint32_t len, double p,
                 double q, uint64_t seed, uint32_t* paths, uint64_t* d_counts, hipStream_t st);
int update_batch(bingo_graph* g, uint64_t n_ins, const uint32_t* is, const uint32_t* id, const uint32_t* iw,
                 uint64_t n_del, const uint32_t* ds, const uint32_t* dd, bingo_update_stats* h_stats,
                 hipStream_t st);
// stream.hip
int update_stream(bingo_graph* g, uint64_t m, const uint32_t* op, const uint32_t* src, const uint32_t* dst,
                  const uint32_t* w, bingo_update_stats* h_stats, hipStream_t st);
// api.hip
void* ws_get(bingo_graph* g, size_t bytes);  // grow-only scratch (synchronizes when it grows)
int err_to_code(uint32_t bits);

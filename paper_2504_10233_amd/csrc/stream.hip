// stream.hip -- streaming updates (Sec. 4.2 insertion and deletion): edge
// records applied one at a time in their given order, each with exactly the
// meaning of a bingo_update_batch call that holds that one record.
//
// Records of different source vertices commute, so a stable sort by source
// gives every touched vertex its own records in order; one wave then applies
// them one by one (vertices in parallel), keeping the vertex's header state in
// registers (lane k holds group k) between records.  An insert appends at index
// d and adds the edge to the lists of its groups; a delete removes the live
// occurrence with the smallest sequence number, moves the tail entry into its
// slot, and fixes every list it touched: the deleted member's position takes
// the list's last entry, and the moved entry is renamed.  A group whose type
// changes gets a fresh ascending list or its one member, as in the batch.
// A regular group finds a member's position through its inverted index
// (Sec. 4.2) and keeps the index in step; a sparse group's list is short (below
// beta % of d) and is scanned, and S(u) with the sparse indexes is rebuilt for
// the touched sources after the stream.
#include "dev.h"
#include "locate.h"
#include <algorithm>
#include <string.h>

namespace {

constexpr int TB = 256;
constexpr uint32_t NF = 0xFFFFFFFFu;
constexpr uint32_t ST_GRID = 2048;
constexpr uint32_t ST_BIG_GRID = 1024;
constexpr int ST_CTRS = 32;  // 0 inserted, 1 deleted, 2 not found, 3..27 transitions, 28 scanned, 29 matches

enum { OP_INSERT = 0, OP_DELETE = 1 };


__global__ void k_st_validate(uint64_t m, uint32_t n, const uint32_t* __restrict__ op,
                              const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                              const uint32_t* __restrict__ w, uint32_t* __restrict__ err) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        if (op[i] > OP_DELETE || src[i] >= n || dst[i] >= n) bad |= ERR_RANGE;
        else if (op[i] == OP_INSERT && w[i] == 0) bad |= ERR_WEIGHT;
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_st_iota(uint32_t* __restrict__ a, uint64_t m) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = (uint32_t)i;
}

// head[p] = 1 where a new source starts in the sorted keys
__global__ void k_st_heads(const uint32_t* __restrict__ sk, uint64_t m, uint32_t* __restrict__ head) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (uint64_t)gridDim.x * blockDim.x)
        head[p] = (p == 0 || sk[p] != sk[p - 1]) ? 1u : 0u;
}

// seg_start[segment] = first sorted position of each source, seg_src[segment] = the source
__global__ void k_st_starts(const uint32_t* __restrict__ head, const uint64_t* __restrict__ hx, uint64_t m,
                            const uint32_t* __restrict__ sk, uint32_t* __restrict__ seg_start,
                            uint32_t* __restrict__ seg_src) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (uint64_t)gridDim.x * blockDim.x)
        if (head[p]) { seg_start[hx[p]] = (uint32_t)p; seg_src[hx[p]] = sk[p]; }
}

// Pool words for the current record.  Each wave takes the pool in chunks of ST_CHUNK words (or
// the request, if larger) from the bump counter (ctl[0]) by compare-and-swap, so that a failed
// reservation leaves the counter unchanged, and serves its records from the chunk; one global
// operation per chunk instead of per record keeps thousands of waves from contending on the
// counter.  The unused tail of a chunk is garbage (counted in `waste`, reclaimed by compaction).
// Near the end of the pool a chunk that does not fit falls back to the exact request.  Every
// lane calls with the same values; the result (NF64 on failure) is uniform.
constexpr uint64_t NF64 = ~0ull;
constexpr uint64_t ST_CHUNK = 1u << 14;
struct StChunk {
    uint64_t cur = 0, end = 0;
};
__device__ uint64_t st_reserve(unsigned long long* ctl, uint64_t pool_words, uint64_t words) {
    unsigned long long got = 0;
    if (lane_id() == 0) {
        unsigned long long cur = *reinterpret_cast<volatile unsigned long long*>(ctl);
        for (;;) {
            if (cur + words > pool_words) { got = NF64; break; }
            const unsigned long long prev = atomicCAS(ctl, cur, cur + words);
            if (prev == cur) { got = cur; break; }
            cur = prev;
        }
    }
    return __shfl(got, 0, 64);
}
__device__ uint64_t st_alloc(StChunk& ch, unsigned long long* ctl, uint64_t pool_words, uint64_t words,
                             uint64_t& waste) {
    if (!words) return 0;
    if (ch.cur + words <= ch.end) {
        const uint64_t r = ch.cur;
        ch.cur += words;
        return r;
    }
    const uint64_t take = words > ST_CHUNK ? words : ST_CHUNK;
    uint64_t got = st_reserve(ctl, pool_words, take);
    uint64_t end = got + take;
    if (got == NF64 && take > words) {
        got = st_reserve(ctl, pool_words, words);
        end = got + words;
    }
    if (got == NF64) return NF64;  // the current chunk stays for smaller requests
    if (lane_id() == 0) waste += ch.end - ch.cur;  // the old chunk's unused tail
    ch.cur = got + words;
    ch.end = end;
    return got;
}

__device__ __forceinline__ uint64_t st_wave_min(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}

// position of val in L[0, len) (it occurs once), by a wave scan with eight
// loads per lane in flight
constexpr uint32_t ST_UNROLL = 8;
constexpr uint32_t ST_SCAN = 32;  // loads per lane in flight in a delete's adjacency scan
constexpr uint32_t ST_BIG_D = 1u << 14;  // sources of at least this degree take a block each
constexpr int STB = 512;                 // threads of k_st_apply_big
__device__ uint32_t st_find(const uint32_t* __restrict__ L, uint32_t len, uint32_t val) {
    const uint32_t lane = lane_id();
    for (uint32_t p0 = 0; p0 < len; p0 += 64 * ST_UNROLL) {
        uint32_t v[ST_UNROLL];
#pragma unroll
        for (uint32_t j = 0; j < ST_UNROLL; ++j) {
            const uint32_t p = p0 + j * 64 + lane;
            v[j] = p < len ? L[p] : ~val;
        }
#pragma unroll
        for (uint32_t j = 0; j < ST_UNROLL; ++j) {
            const uint64_t b = __ballot(v[j] == val);
            if (b) return p0 + j * 64 + (uint32_t)(__ffsll((long long)b) - 1);
        }
    }
    return NF;
}

// Per-vertex state between records; lane k < 32 holds group k.  sblk / scap:
// the S(u) block (Sec. 5.1); sdirty: a record touched a vertex with sparse
// groups, so S(u) and the sparse indexes are rebuilt after the stream.
struct SV {
    uint32_t u, d, cap, nseq;
    uint64_t adj, W;
    uint32_t sblk, scap;
    bool sdirty;
    uint32_t c, info, lcap;
};

// The S(u) capacity after a record: an upper bound on |S(u)| (the sum of the
// sparse groups' counts, at most d), kept when the current capacity holds it.
__device__ __forceinline__ uint32_t st_scap(uint32_t tnew, uint32_t cn, uint32_t d1, uint32_t scap, uint32_t& smn) {
    smn = (uint32_t)(__ballot(tnew == GT_SPARSE) & 0xFFFFFFFFull);
    uint64_t sub = tnew == GT_SPARSE ? cn : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sub += __shfl_xor(sub, o);
    sub = sub < d1 ? sub : d1;
    return smn ? (sub > scap ? s_cap_for((uint32_t)sub) : scap) : 0u;
}

// Group-k lists that need writing after an adjacency change: every group in
// `todo` gets a fresh ascending list of the indices in [0, d) whose membership
// word has bit k, in the block `blk` (lane k's value); a regular group's
// inverted index follows at iofs (lane k's value; 0 for a sparse group, whose
// index is rebuilt with S(u)).
__device__ void st_fresh_lists(uint32_t todo, const uint64_t* __restrict__ edges, uint32_t d, uint32_t fb,
                               uint64_t blk, uint32_t iofs, uint32_t* __restrict__ pool) {
    const uint32_t lane = lane_id();
    uint32_t fill = 0;  // lane k: entries written to group k
    for (uint32_t i0 = 0; i0 < d && todo; i0 += 64) {
        const uint32_t i = i0 + lane;
        const uint32_t mw = i < d ? member_word((uint32_t)(edges[i] >> 32), fb) : 0u;
        uint32_t mm = todo;
        while (mm) {
            const int k = __ffs(mm) - 1;
            mm &= mm - 1;
            const bool bit = (mw >> k) & 1u;
            const uint64_t b = __ballot(bit);
            const uint64_t kb = __shfl(blk, k, 64);
            const uint32_t f = __shfl(fill, k, 64);
            const uint32_t io = __shfl(iofs, k, 64);
            if (bit) {
                const uint32_t pos = f + __popcll(b & lanemask_lt());
                pool[kb + pos] = i;
                if (io) pool[kb + io + i] = pos;
            }
            if (lane == (uint32_t)k) fill += __popcll(b);
        }
    }
}

// first index in [0, d) whose membership word has bit k, for every k in `todo` (lane k's result)
__device__ uint32_t st_first_members(uint32_t todo, const uint64_t* __restrict__ edges, uint32_t d, uint32_t fb) {
    const uint32_t lane = lane_id();
    uint32_t first = NF;
    for (uint32_t i0 = 0; i0 < d && todo; i0 += 64) {
        const uint32_t i = i0 + lane;
        const uint32_t mw = i < d ? member_word((uint32_t)(edges[i] >> 32), fb) : 0u;
        uint32_t mm = todo;
        while (mm) {
            const int k = __ffs(mm) - 1;
            mm &= mm - 1;
            const uint64_t b = __ballot((mw >> k) & 1u);
            if (b) {
                if (lane == (uint32_t)k) first = i0 + (uint32_t)(__ffsll((long long)b) - 1);
                todo &= ~(1u << k);
            }
        }
    }
    return first;
}

// Copy the live part of every list in `todo` to its new block (lane k: old and
// new block offsets, length); a regular group's inverted index is written anew
// at iofs (lane k's value, 0 for a sparse group).
__device__ void st_move_lists(uint32_t todo, uint64_t oblk, uint64_t nblk, uint32_t len, uint32_t iofs,
                              uint32_t* __restrict__ pool) {
    const uint32_t lane = lane_id();
    while (todo) {
        const int k = __ffs(todo) - 1;
        todo &= todo - 1;
        const uint64_t o = __shfl(oblk, k, 64), nb = __shfl(nblk, k, 64);
        const uint32_t L = __shfl(len, k, 64), io = __shfl(iofs, k, 64);
        for (uint32_t p = lane; p < L; p += 64) {
            const uint32_t e = pool[o + p];
            pool[nb + p] = e;
            if (io) pool[nb + io + e] = p;
        }
    }
}

// Statistics of one record (one batch of one record): lane 0 adds to the
// wave's counters in LDS; the type transition of group k is lane k's code.
__device__ void st_count(uint32_t code, unsigned long long* acc) {
#pragma unroll
    for (int c = 0; c < 25; ++c) {
        const uint32_t k = (uint32_t)__popcll(__ballot(code == (uint32_t)c));
        if (lane_id() == 0 && k) acc[3 + c] += k;
    }
}

// One insert record.  Returns false when the pool cannot hold what it needs
// (nothing changed then).  `freed` is per lane (summed over the wave later).
// Blocks move when a list outgrows its capacity or an index outgrows its block
// (a regular group's inverted index spans the adjacency capacity, a sparse
// group's index the S(u) capacity).
__device__ bool st_insert(SV& s, uint32_t v, uint32_t w, GroupRule rule, uint32_t* __restrict__ pool,
                          unsigned long long* ctl, uint64_t pool_words, StChunk& ch, uint64_t& freed,
                          unsigned long long* acc) {
    const uint32_t lane = lane_id();
    const uint32_t fb = rule.fbits;
    const uint32_t mw = member_word(w, fb);
    const uint32_t d1 = s.d + 1;
    const bool g = lane < 32;
    const bool bit = g && ((mw >> lane) & 1u);
    const uint32_t cn = s.c + (bit ? 1u : 0u);
    const uint32_t told = g ? group_type(s.c, s.d, rule) : GT_EMPTY;
    const uint32_t tnew = g ? group_type(cn, d1, rule) : GT_EMPTY;
    const bool kept = type_listed(told) && tnew == told;
    const bool fresh = type_listed(tnew) && !kept;
    const bool grow = d1 > s.cap;
    const uint32_t ncap = grow ? adj_cap_for(d1) : s.cap;
    const uint32_t smo = (uint32_t)(__ballot(told == GT_SPARSE) & 0xFFFFFFFFull);
    uint32_t smn = 0;
    const uint32_t scapn = st_scap(tnew, cn, d1, s.scap, smn);
    const uint32_t ico = index_cap_for(told, s.cap, s.scap), icn = index_cap_for(tnew, ncap, scapn);
    const bool relist = kept && ((bit && cn > s.lcap) || icn != ico);
    const uint32_t nlc = fresh ? list_cap_for(cn) : (relist && cn > s.lcap ? list_cap_for(cn) : s.lcap);
    const uint32_t iofs = tnew == GT_REGULAR ? nlc : 0u;
    // pool words: a larger adjacency block, moved or fresh lists, a larger S(u) block (lane 32)
    const uint64_t aw = grow ? adj_block_words(ncap) : 0ull;
    uint64_t lw = (relist || fresh) ? list_block_words(nlc, icn) : 0ull;
    if (lane == 32 && scapn && scapn != s.scap) lw = scapn;
    uint64_t x = lw;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    const uint64_t total = aw + __shfl(x, 63, 64);
    const uint64_t base = st_alloc(ch, ctl, pool_words, total, freed);
    if (base == NF64) return false;
    const uint64_t myblk = base + aw + (x - lw);
    // adjacency
    if (grow) {
        const uint64_t nadj = base;
        const uint64_t* eo = reinterpret_cast<const uint64_t*>(pool + s.adj);
        const uint32_t* qo = pool + s.adj + 2ull * s.cap;
        uint64_t* en = reinterpret_cast<uint64_t*>(pool + nadj);
        uint32_t* qn = pool + nadj + 2ull * ncap;
        for (uint32_t i = lane; i < s.d; i += 64) { en[i] = eo[i]; qn[i] = qo[i]; }
        if (s.cap && lane == 0) freed += adj_block_words(s.cap);
        s.adj = nadj;
        s.cap = ncap;
    }
    uint64_t* edges = reinterpret_cast<uint64_t*>(pool + s.adj);
    if (lane == 0) {
        edges[s.d] = (uint64_t)v | ((uint64_t)w << 32);
        pool[s.adj + 2ull * s.cap + s.d] = s.nseq;
    }
    __threadfence_block();
    // kept lists: move the ones whose list or index outgrows its block, then append index d
    // (at position c; a regular group's inverted index maps d to c)
    const uint64_t oblk = (uint64_t)s.info * LIST_UNIT_WORDS;
    const uint32_t rmask = (uint32_t)(__ballot(relist) & 0xFFFFFFFFull);
    st_move_lists(rmask, oblk, myblk, s.c, iofs, pool);
    if (relist) {
        freed += list_block_words(s.lcap, ico);
        s.info = (uint32_t)(myblk / LIST_UNIT_WORDS);
        s.lcap = nlc;
    }
    if (kept && bit) {
        uint32_t* L = pool + (uint64_t)s.info * LIST_UNIT_WORDS;
        L[s.c] = s.d;
        if (tnew == GT_REGULAR) L[s.lcap + s.d] = s.c;
    }
    // lists of groups that became listed or switched between sparse and regular
    if (g && type_listed(told) && !kept) freed += list_block_words(s.lcap, ico);
    const uint32_t fmask = (uint32_t)(__ballot(fresh) & 0xFFFFFFFFull);
    if (fresh) {
        s.info = (uint32_t)(myblk / LIST_UNIT_WORDS);
        s.lcap = nlc;
    }
    __threadfence_block();
    st_fresh_lists(fmask, edges, d1, fb, myblk, iofs, pool);
    // S(u): a new block when its capacity grows (rebuilt with the sparse indexes after the stream)
    const uint64_t nsblk = __shfl(myblk, 32, 64);
    if (lane == 32 && s.scap && scapn != s.scap) freed += s.scap;
    if (scapn && scapn != s.scap) s.sblk = (uint32_t)(nsblk / LIST_UNIT_WORDS);
    s.scap = scapn;
    s.sdirty |= (smo | smn) != 0u;
    // one-element groups: an old member stays; a new one is the inserted edge
    if (tnew == GT_ONE && told != GT_ONE) s.info = s.d;
    if (g && !type_listed(tnew) && tnew != GT_ONE) s.info = 0;
    // statistics: one batch with one record
    if (lane == 0) acc[0] += 1;
    st_count(g ? told * 5 + tnew : 31u, acc);
    s.c = cn;
    s.d = d1;
    s.nseq += 1;
    s.W += w;
    return true;
}

// Position of neighbor index i in a kept listed group (lane k's group, every
// lane calls for the same k): through the inverted index for a regular group
// (Sec. 4.2, O(1)), by a wave scan of the list for a sparse one.  NF when the
// index does not hold i at a valid position (an inconsistent structure).
__device__ __forceinline__ uint32_t st_pos(const uint32_t* __restrict__ L, uint32_t c, uint32_t lcap, bool regular,
                                           uint32_t i) {
    if (!regular) return st_find(L, c, i);
    const uint32_t p = L[lcap + i];
    return (p < c && L[p] == i) ? p : NF;
}

// One delete record.
// The live occurrence of v with the smallest sequence number among adjacency
// entries [lo, hi): (seq << 32 | index), ~0 if none, and the number of
// occurrences; the wave's result in every lane.  A hub's records are a
// sequential chain, so the scan keeps ST_SCAN loads per lane in flight.
__device__ uint64_t st_scan_oldest(const uint64_t* __restrict__ edges, const uint32_t* __restrict__ seqs, uint32_t lo,
                                   uint32_t hi, uint32_t v, uint32_t& hits) {
    const uint32_t lane = lane_id();
    uint64_t best = ~0ull;
    hits = 0;
    for (uint32_t i0 = lo; i0 < hi; i0 += 64 * ST_SCAN) {
        uint32_t e[ST_SCAN];
#pragma unroll
        for (uint32_t j = 0; j < ST_SCAN; ++j) {
            const uint32_t i = i0 + j * 64 + lane;
            e[j] = i < hi ? (uint32_t)edges[i] : ~v;
        }
#pragma unroll
        for (uint32_t j = 0; j < ST_SCAN; ++j) {
            const uint32_t i = i0 + j * 64 + lane;
            const bool m = e[j] == v;
            hits += __popcll(__ballot(m));
            if (m) {
                const uint64_t key = ((uint64_t)seqs[i] << 32) | i;
                best = key < best ? key : best;
            }
        }
    }
    return st_wave_min(best);
}

// One delete record whose oldest occurrence (best, from st_scan_oldest over the whole adjacency)
// and occurrence count are known.
__device__ bool st_delete_at(SV& s, uint32_t v, uint64_t best, uint32_t hits, GroupRule rule,
                             uint32_t* __restrict__ pool, unsigned long long* ctl, uint64_t pool_words, StChunk& ch,
                             uint64_t& freed, unsigned long long* acc, uint32_t* __restrict__ errw) {
    const uint32_t lane = lane_id();
    const uint32_t fb = rule.fbits;
    const bool g = lane < 32;
    uint64_t* edges = reinterpret_cast<uint64_t*>(pool + s.adj);
    uint32_t* seqs = pool + s.adj + 2ull * s.cap;
    if (lane == 0) { acc[28] += s.d; acc[29] += hits; }
    const uint32_t told = g ? group_type(s.c, s.d, rule) : GT_EMPTY;
    if (best == ~0ull) {
        if (lane == 0) acc[2] += 1;
        st_count(g ? told * 5 + told : 31u, acc);
        return true;
    }
    const uint32_t i = (uint32_t)best;
    const uint32_t last = s.d - 1;
    const bool moved = i != last;
    const uint64_t ei = edges[i], el = edges[last];
    const uint32_t wi = (uint32_t)(ei >> 32);
    const uint32_t mw = member_word(wi, fb);
    const uint32_t mwl = member_word((uint32_t)(el >> 32), fb);
    const uint32_t d1 = s.d - 1;
    const bool bit = g && ((mw >> lane) & 1u);
    const uint32_t cn = s.c - (bit ? 1u : 0u);
    const uint32_t tnew = g ? group_type(cn, d1, rule) : GT_EMPTY;
    const bool kept = type_listed(told) && tnew == told;
    const bool fresh = type_listed(tnew) && !kept;
    const uint32_t smo = (uint32_t)(__ballot(told == GT_SPARSE) & 0xFFFFFFFFull);
    uint32_t smn = 0;
    const uint32_t scapn = st_scap(tnew, cn, d1, s.scap, smn);
    // the adjacency capacity stays, so only a sparse group's index can outgrow its block
    const uint32_t ico = index_cap_for(told, s.cap, s.scap), icn = index_cap_for(tnew, s.cap, scapn);
    const bool relist = kept && icn != ico;
    const uint32_t nlc = fresh ? list_cap_for(cn) : s.lcap;
    const uint32_t iofs = tnew == GT_REGULAR ? nlc : 0u;
    uint64_t lw = (relist || fresh) ? list_block_words(nlc, icn) : 0ull;
    if (lane == 32 && scapn && scapn != s.scap) lw = scapn;
    uint64_t x = lw;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    const uint64_t total = __shfl(x, 63, 64);
    const uint64_t base = st_alloc(ch, ctl, pool_words, total, freed);
    if (base == NF64) return false;
    const uint64_t myblk = base + (x - lw);
    // adjacency: the tail entry takes the deleted slot
    if (moved && lane == 0) {
        edges[i] = el;
        seqs[i] = seqs[last];
    }
    // kept lists whose index outgrows the block move first (sparse groups; indexes rebuilt later)
    const uint32_t rmask = (uint32_t)(__ballot(relist) & 0xFFFFFFFFull);
    st_move_lists(rmask, (uint64_t)s.info * LIST_UNIT_WORDS, myblk, s.c, 0u, pool);
    if (relist) {
        freed += list_block_words(s.lcap, ico);
        s.info = (uint32_t)(myblk / LIST_UNIT_WORDS);
    }
    __threadfence_block();
    // kept lists: the deleted member's position takes the last entry, then the moved entry is
    // renamed; a regular group finds both positions through its inverted index and updates it
    uint32_t km = (uint32_t)(__ballot(kept && bit) & 0xFFFFFFFFull);
    while (km) {
        const int k = __ffs(km) - 1;
        km &= km - 1;
        uint32_t* L = pool + (uint64_t)__shfl(s.info, k, 64) * LIST_UNIT_WORDS;
        const uint32_t ck = __shfl(s.c, k, 64), lk = __shfl(s.lcap, k, 64);
        const bool reg = __shfl(told, k, 64) == GT_REGULAR;
        const uint32_t p = st_pos(L, ck, lk, reg, i);
        if (lane == 0) {
            if (p == NF) {
                atomicOr(errw, ERR_INTERNAL);
            } else if (p != ck - 1) {
                const uint32_t e = L[ck - 1];
                L[p] = e;
                if (reg) L[lk + e] = p;
            }
        }
        __threadfence_block();
    }
    if (moved) {
        uint32_t rm = (uint32_t)(__ballot(kept && ((mwl >> lane) & 1u)) & 0xFFFFFFFFull);
        while (rm) {
            const int k = __ffs(rm) - 1;
            rm &= rm - 1;
            uint32_t* L = pool + (uint64_t)__shfl(s.info, k, 64) * LIST_UNIT_WORDS;
            const uint32_t len = __shfl(cn, k, 64), lk = __shfl(s.lcap, k, 64);
            const bool reg = __shfl(told, k, 64) == GT_REGULAR;
            const uint32_t q = st_pos(L, len, lk, reg, last);
            if (lane == 0) {
                if (q == NF) {
                    atomicOr(errw, ERR_INTERNAL);
                } else {
                    L[q] = i;
                    if (reg) L[lk + i] = q;
                }
            }
            __threadfence_block();
        }
    }
    // fresh lists and one-element members from the final adjacency
    if (g && type_listed(told) && !kept) freed += list_block_words(s.lcap, ico);
    const uint32_t fmask = (uint32_t)(__ballot(fresh) & 0xFFFFFFFFull);
    if (fresh) {
        s.info = (uint32_t)(myblk / LIST_UNIT_WORDS);
        s.lcap = nlc;
    }
    st_fresh_lists(fmask, edges, d1, fb, myblk, iofs, pool);
    const bool one = tnew == GT_ONE;
    uint32_t member = NF;
    if (one && told == GT_ONE) member = (moved && s.info == last) ? i : s.info;
    const uint32_t scan = (uint32_t)(__ballot(one && member == NF) & 0xFFFFFFFFull);
    const uint32_t first = st_first_members(scan, edges, d1, fb);
    if (one) s.info = member != NF ? member : first;
    if (g && !type_listed(tnew) && tnew != GT_ONE) s.info = 0;
    // S(u)
    const uint64_t nsblk = __shfl(myblk, 32, 64);
    if (lane == 32 && s.scap && scapn != s.scap) freed += s.scap;
    if (scapn && scapn != s.scap) s.sblk = (uint32_t)(nsblk / LIST_UNIT_WORDS);
    s.scap = scapn;
    s.sdirty |= (smo | smn) != 0u;
    if (lane == 0) acc[1] += 1;
    st_count(g ? told * 5 + tnew : 31u, acc);
    s.c = cn;
    s.d = d1;
    s.W -= wi;
    return true;
}

// One delete record, the whole adjacency scanned by the wave.
__device__ bool st_delete(SV& s, uint32_t v, GroupRule rule, uint32_t* __restrict__ pool, unsigned long long* ctl,
                          uint64_t pool_words, StChunk& ch, uint64_t& freed, unsigned long long* acc,
                          uint32_t* __restrict__ errw) {
    const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + s.adj);
    const uint32_t* seqs = pool + s.adj + 2ull * s.cap;
    uint32_t hits;
    const uint64_t best = st_scan_oldest(edges, seqs, 0, s.d, v, hits);
    return st_delete_at(s, v, best, hits, rule, pool, ctl, pool_words, ch, freed, acc, errw);
}

// The state of source u's vertex from its header (lane k < 32: group k).
__device__ __forceinline__ void st_load(SV& s, uint32_t u, const uint32_t* __restrict__ hdr) {
    const uint32_t lane = lane_id();
    s.u = u;
    const uint32_t* h = hdr + (size_t)u * HDR_WORDS;
    s.d = h[H_DEG]; s.cap = h[H_ACAP]; s.nseq = h[H_NSEQ];
    s.adj = hdr_adj(h);
    s.W = ((uint64_t)h[H_WHI] << 32) | h[H_WLO];
    s.c = lane < 32 ? slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane) : 0u;
    s.info = lane < 32 ? h[H_INFO + lane] : 0u;
    s.lcap = lane < 32 ? (1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu)) : 0u;
    s.sblk = h[H_SBLK];
    s.scap = h[H_SCAP];
    s.sdirty = false;
}

// After a source's records: the records not applied (an out-of-pool stop at record `stop`) are
// flagged in `left`, and the vertex's header is rewritten from the state (the wave's lanes).
__device__ void st_store(const SV& s, bool ok, uint32_t stop, uint32_t e, const uint32_t* __restrict__ sv,
                         uint64_t sg, GroupRule rule, uint32_t* __restrict__ hdr, const uint32_t* __restrict__ pool,
                         uint32_t* __restrict__ errw, uint32_t* __restrict__ left, uint32_t* __restrict__ sdirty) {
    const uint32_t lane = lane_id();
    if (!ok) {
        if (lane == 0) atomicOr(errw, ERR_OOM);
        for (uint32_t q = stop + lane; q < e; q += 64) left[sv[q]] = 1u;  // this source's records not applied
    }
    uint32_t* h = hdr + (size_t)s.u * HDR_WORDS;
    const bool ne = lane < 32 && s.c > 0;
    const uint32_t nmask = (uint32_t)(__ballot(ne) & 0xFFFFFFFFull);
    const uint32_t t = lane < 32 ? group_type(s.c, s.d, rule) : GT_EMPTY;
    // one-element groups: the member's destination in the count slot
    const bool onek = lane < 32 && t == GT_ONE;
    const uint32_t onemask = (uint32_t)(__ballot(onek) & 0xFFFFFFFFull);
    const uint32_t nhi = mask_hi(nmask);
    if (lane < 32) {
        if (lane <= nhi)
            h[H_CNT + (nhi - lane)] = onek ? (uint32_t)reinterpret_cast<const uint64_t*>(pool + s.adj)[s.info] : s.c;
        h[H_INFO + lane] = (type_listed(t) || t == GT_ONE) ? s.info : 0u;
    }
    const uint32_t lg = (lane < 32 && type_listed(t)) ? (31 - __clz(s.lcap)) : 0u;
    uint32_t packed = lg << (8 * (lane & 3));
    packed |= __shfl_xor(packed, 1);
    packed |= __shfl_xor(packed, 2);
    if (lane < 32 && (lane & 3) == 0) h[H_LCAPLOG + (lane >> 2)] = packed;
    if (lane == 0) {
        h[H_MASK] = nmask;
        h[H_ONEMASK] = onemask;
        h[H_DEG] = s.d;
        h[H_WLO] = (uint32_t)s.W;
        h[H_WHI] = (uint32_t)(s.W >> 32);
        h[H_ADJLO] = (uint32_t)s.adj;
        h[H_ADJHI] = adjhi_word(s.adj, nhi);
        h[H_ACAP] = s.cap;
        h[H_NSEQ] = s.nseq;
        h[H_SBLK] = s.sblk;
        h[H_SCAP] = s.scap;
        if (!s.scap) h[H_SLEN] = 0;
        sdirty[sg] = (s.scap && s.sdirty) ? 1u : 0u;
    }
}

// One wave per touched source vertex: its records in order.  Sources of at least ST_BIG_D
// edges are listed in `big` instead, for k_st_apply_big.
__global__ void __launch_bounds__(TB) k_st_apply(const uint32_t* __restrict__ err, const unsigned long long* nseg_p,
                                                 uint64_t m, const uint32_t* __restrict__ sk,
                                                 const uint32_t* __restrict__ sv, const uint32_t* __restrict__ seg_start,
                                                 const uint32_t* __restrict__ op, const uint32_t* __restrict__ dst,
                                                 const uint32_t* __restrict__ w, uint32_t* __restrict__ hdr,
                                                 uint32_t* __restrict__ pool, unsigned long long* ctl,
                                                 uint64_t pool_words, GroupRule rule, uint32_t* __restrict__ errw,
                                                 unsigned long long* __restrict__ out, uint32_t* __restrict__ left,
                                                 uint32_t* __restrict__ sdirty, uint32_t* __restrict__ big,
                                                 unsigned long long* __restrict__ nbig) {
    __shared__ unsigned long long red[TB / 64][ST_CTRS];  // per-wave counters, written by lane 0
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    // only the validation bits gate the kernel: waves of this same kernel set ERR_OOM in the same
    // word, and a block that starts after such a stop still owns its segments
    const uint64_t nseg = (*err & (ERR_RANGE | ERR_WEIGHT)) ? 0 : *nseg_p;
    unsigned long long* acc = red[wave];
    if (lane < ST_CTRS) acc[lane] = 0;
    __threadfence_block();
    uint64_t freed = 0;  // per lane
    StChunk ch;          // the wave's pool chunk
    for (uint64_t sg = (uint64_t)blockIdx.x * (TB / 64) + wave; sg < nseg; sg += (uint64_t)gridDim.x * (TB / 64)) {
        const uint32_t b = seg_start[sg];
        const uint32_t e = sg + 1 < nseg ? seg_start[sg + 1] : (uint32_t)m;
        const uint32_t u = sk[b];
        if (hdr[(size_t)u * HDR_WORDS + H_DEG] >= ST_BIG_D) {
            if (lane == 0) big[atomicAdd(nbig, 1ull)] = (uint32_t)sg;
            continue;
        }
        SV s;
        st_load(s, u, hdr);
        bool ok = true;
        uint32_t stop = e;  // first record not applied
        for (uint32_t p = b; p < e && ok; ++p) {
            const uint32_t r = sv[p];
            if (op[r] == OP_INSERT) ok = st_insert(s, dst[r], w[r], rule, pool, ctl, pool_words, ch, freed, acc);
            else ok = st_delete(s, dst[r], rule, pool, ctl, pool_words, ch, freed, acc, errw);
            if (!ok) stop = p;
            __threadfence_block();
        }
        st_store(s, ok, stop, e, sv, sg, rule, hdr, pool, errw, left, sdirty);
    }
    // garbage words of the wave (with its last chunk's unused tail), then the block's counters
    if (lane == 0) freed += ch.end - ch.cur;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) freed += __shfl_xor(freed, o);
    if (lane == 0 && freed) atomicAdd(ctl + 1, (unsigned long long)freed);
    __syncthreads();
    if (threadIdx.x < ST_CTRS) {
        unsigned long long v = 0;
        for (int wv = 0; wv < TB / 64; ++wv) v += red[wv][threadIdx.x];
        if (v) atomicAdd(out + threadIdx.x, v);
    }
}

// The listed sources of at least ST_BIG_D edges, one block of STB threads per source: wave 0
// holds the state and applies the records in order; for a delete every wave scans its share of
// the adjacency for the oldest occurrence first, so a hub's chain of deletes runs STB / 64 times
// as many loads in flight as one wave would.
__global__ void __launch_bounds__(STB) k_st_apply_big(const uint32_t* __restrict__ err,
                                                      const unsigned long long* nseg_p, uint64_t m,
                                                      const uint32_t* __restrict__ sk, const uint32_t* __restrict__ sv,
                                                      const uint32_t* __restrict__ seg_start,
                                                      const uint32_t* __restrict__ op, const uint32_t* __restrict__ dst,
                                                      const uint32_t* __restrict__ w, uint32_t* __restrict__ hdr,
                                                      uint32_t* __restrict__ pool, unsigned long long* ctl,
                                                      uint64_t pool_words, GroupRule rule, uint32_t* __restrict__ errw,
                                                      unsigned long long* __restrict__ out,
                                                      uint32_t* __restrict__ left, uint32_t* __restrict__ sdirty,
                                                      const uint32_t* __restrict__ big,
                                                      const unsigned long long* __restrict__ nbig) {
    constexpr int NW = STB / 64;
    __shared__ unsigned long long acc[ST_CTRS];  // wave 0's counters
    __shared__ uint64_t w_best[NW];
    __shared__ uint32_t w_hits[NW];
    __shared__ uint64_t s_adj;
    __shared__ uint32_t s_d, s_cap, s_ok;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint64_t nseg = (*err & (ERR_RANGE | ERR_WEIGHT)) ? 0 : *nseg_p;
    const uint64_t nb = nseg ? *nbig : 0;
    if (threadIdx.x < ST_CTRS) acc[threadIdx.x] = 0;
    uint64_t freed = 0;  // per lane of wave 0
    StChunk ch;          // wave 0's pool chunk
    SV s;                // wave 0
    for (uint64_t q = blockIdx.x; q < nb; q += gridDim.x) {
        const uint64_t sg = big[q];
        const uint32_t b = seg_start[sg];
        const uint32_t e = sg + 1 < nseg ? seg_start[sg + 1] : (uint32_t)m;
        __syncthreads();  // the previous source is done with the shared state
        if (wave == 0) {
            st_load(s, sk[b], hdr);
            if (lane == 0) { s_d = s.d; s_cap = s.cap; s_adj = s.adj; s_ok = 1u; }
        }
        __syncthreads();
        uint32_t stop = e;
        for (uint32_t p = b; p < e; ++p) {
            const uint32_t r = sv[p];
            const bool del = op[r] != OP_INSERT;
            const uint32_t v = dst[r];
            if (del) {
                const uint32_t d = s_d;
                const uint64_t* edges = reinterpret_cast<const uint64_t*>(pool + s_adj);
                const uint32_t* seqs = pool + s_adj + 2ull * s_cap;
                const uint32_t share = (d + NW - 1) / NW;
                const uint32_t lo = min(d, wave * share), hi = min(d, lo + share);
                uint32_t hits;
                const uint64_t bw = st_scan_oldest(edges, seqs, lo, hi, v, hits);
                if (lane == 0) { w_best[wave] = bw; w_hits[wave] = hits; }
                __syncthreads();  // every share scanned
            }
            if (wave == 0) {
                bool ok;
                if (del) {
                    uint64_t best = ~0ull;
                    uint32_t hits = 0;
                    for (int x = 0; x < NW; ++x) {
                        best = w_best[x] < best ? w_best[x] : best;
                        hits += w_hits[x];
                    }
                    ok = st_delete_at(s, v, best, hits, rule, pool, ctl, pool_words, ch, freed, acc, errw);
                } else {
                    ok = st_insert(s, v, w[r], rule, pool, ctl, pool_words, ch, freed, acc);
                }
                __threadfence_block();
                if (lane == 0) { s_d = s.d; s_cap = s.cap; s_adj = s.adj; s_ok = ok ? 1u : 0u; }
            }
            __syncthreads();  // the record is applied; the shared state is current
            if (!s_ok) {
                stop = p;
                break;
            }
        }
        if (wave == 0) st_store(s, stop == e, stop, e, sv, sg, rule, hdr, pool, errw, left, sdirty);
    }
    if (wave == 0) {
        if (lane == 0) freed += ch.end - ch.cur;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) freed += __shfl_xor(freed, o);
        if (lane == 0 && freed) atomicAdd(ctl + 1, (unsigned long long)freed);
    }
    __syncthreads();
    if (threadIdx.x < ST_CTRS && acc[threadIdx.x]) atomicAdd(out + threadIdx.x, acc[threadIdx.x]);
}

inline uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n + TB - 1) / TB, 1), 8192);
}

int bits_for_n(uint32_t n) {
    int b = 1;
    while (b < 32 && ((n - 1) >> b)) ++b;
    return b;
}

}  // namespace

namespace {
// The records flagged in left, in their order: out[pos[r]] = in[r] for each of the four arrays.
__global__ void k_st_gather(uint64_t m, const uint32_t* __restrict__ left, const uint64_t* __restrict__ pos,
                            const uint32_t* __restrict__ op, const uint32_t* __restrict__ src,
                            const uint32_t* __restrict__ dst, const uint32_t* __restrict__ w,
                            uint32_t* __restrict__ out, uint64_t k) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (uint64_t)gridDim.x * blockDim.x) {
        if (!left[r]) continue;
        const uint64_t p = pos[r];
        out[p] = op[r];
        out[k + p] = src[r];
        out[2 * k + p] = dst[r];
        out[3 * k + p] = w[r];
    }
}

void add_stats(bingo_update_stats* a, const bingo_update_stats& b) {
    a->inserted += b.inserted;
    a->deleted += b.deleted;
    a->not_found += b.not_found;
    a->match_scanned += b.match_scanned;
    a->match_candidates += b.match_candidates;
    for (int i = 0; i < 25; ++i) a->transitions[i] += b.transitions[i];
}

// A stream that runs out of pool is continued after a compaction (or a doubling of a
// library-sized pool) as long as each pass applies some of the records, at most this often.
constexpr uint32_t STREAM_RETRIES = 8;
int apply_stream(bingo_graph* g, uint64_t m, const uint32_t* op, const uint32_t* src, const uint32_t* dst,
                 const uint32_t* w, bingo_update_stats* h_stats, uint32_t retries, hipStream_t st);
}  // namespace

int update_stream(bingo_graph* g, uint64_t m, const uint32_t* op, const uint32_t* src, const uint32_t* dst,
                  const uint32_t* w, bingo_update_stats* h_stats, hipStream_t st) {
    bingo_update_stats sum{};
    // records applied here move edges without the edge locator: the next batch rebuilds it
    locator_invalidate(g);
    const int rc = apply_stream(g, m, op, src, dst, w, &sum, STREAM_RETRIES, st);
    if (h_stats) *h_stats = sum;
    // every record of a stream that returns OK was applied exactly once: inserted, deleted or
    // counted as an absent delete
    if (rc == BINGO_OK && sum.inserted + sum.deleted + sum.not_found != m) {
        fprintf(stderr, "libbingo: streaming update applied %llu of %llu records\n",
                (unsigned long long)(sum.inserted + sum.deleted + sum.not_found), (unsigned long long)m);
        return BINGO_E_INTERNAL;
    }
    return rc;
}

namespace {
int apply_stream(bingo_graph* g, uint64_t m, const uint32_t* op, const uint32_t* src, const uint32_t* dst,
                 const uint32_t* w, bingo_update_stats* h_stats, uint32_t retries, hipStream_t st) {
    if (m == 0) return BINGO_OK;
    if (m > (1ull << 31)) return BINGO_E_INVALID;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const size_t tmpb = std::max(sort_temp_bytes(m, false), scan_temp_bytes(m));
    const size_t bytes = al(m * 4) * 9 + al(m * 8) + al(SPARSE_WORK_WORDS(m) * 4) + al(ST_CTRS * 8) + 512 + tmpb;
    char* ws = (char*)ws_get(g, bytes);
    if (!ws) return BINGO_E_OOM;
    auto take = [&](uint64_t b) { char* r = ws; ws += al(b); return r; };
    uint32_t* ids = (uint32_t*)take(m * 4);
    uint32_t* sk = (uint32_t*)take(m * 4);
    uint32_t* sv = (uint32_t*)take(m * 4);
    uint32_t* head = (uint32_t*)take(m * 4);
    uint32_t* seg = (uint32_t*)take(m * 4);
    uint32_t* seg_src = (uint32_t*)take(m * 4);
    uint32_t* left = (uint32_t*)take(m * 4);
    uint32_t* sdirty = (uint32_t*)take(m * 4);  // per source segment: S(u) to rebuild
    uint32_t* srwork = (uint32_t*)take(SPARSE_WORK_WORDS(m) * 4);
    uint64_t* hx = (uint64_t*)take(m * 8);
    unsigned long long* out = (unsigned long long*)take(ST_CTRS * 8);
    unsigned long long* nseg = (unsigned long long*)take(256);
    uint32_t* big = (uint32_t*)take(m * 4);  // segments of the sources of at least ST_BIG_D edges
    unsigned long long* nbig = (unsigned long long*)take(256);
    void* tmp = ws;
    HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
    HIPCHK(hipMemsetAsync(out, 0, ST_CTRS * 8, st));
    HIPCHK(hipMemsetAsync(left, 0, m * 4, st));
    HIPCHK(hipMemsetAsync(sdirty, 0, m * 4, st));
    HIPCHK(hipMemsetAsync(nbig, 0, 8, st));
    phase_mark(g, st, true);
    hipLaunchKernelGGL(k_st_validate, dim3(grid_for(m)), dim3(TB), 0, st, m, g->n, op, src, dst, w, g->d_err);
    hipLaunchKernelGGL(k_st_iota, dim3(grid_for(m)), dim3(TB), 0, st, ids, m);
    sort_pairs_u32(src, ids, sk, sv, m, bits_for_n(g->n), tmp, st);
    hipLaunchKernelGGL(k_st_heads, dim3(grid_for(m)), dim3(TB), 0, st, sk, m, head);
    scan_u32_to_u64(head, hx, m, tmp, nseg, st);
    hipLaunchKernelGGL(k_st_starts, dim3(grid_for(m)), dim3(TB), 0, st, head, hx, m, sk, seg, seg_src);
    phase_mark(g, st, false);
    hipLaunchKernelGGL(k_st_apply, dim3(ST_GRID), dim3(TB), 0, st, (const uint32_t*)g->d_err,
                       (const unsigned long long*)nseg, m, sk, sv, seg, op, dst, w, g->hdr, g->pool, g->d_ctl,
                       g->pool_words, g->rule, g->d_err, out, left, sdirty, big, nbig);
    hipLaunchKernelGGL(k_st_apply_big, dim3(ST_BIG_GRID), dim3(STB), 0, st, (const uint32_t*)g->d_err,
                       (const unsigned long long*)nseg, m, sk, sv, seg, op, dst, w, g->hdr, g->pool, g->d_ctl,
                       g->pool_words, g->rule, g->d_err, out, left, sdirty, (const uint32_t*)big,
                       (const unsigned long long*)nbig);
    // S(u) and the sparse indexes of the sources whose records touched a vertex with sparse groups
    sparse_rebuild(g, seg_src, nseg, m, sdirty, srwork, st);
    // alias-table mode: the sources' inter-group tables (with bad records nothing changed: rewritten as they were)
    alias_rows(g, seg_src, nseg, m, st);
    phase_mark(g, st, false);
    unsigned long long o[ST_CTRS], ns = 0;
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(o, out, sizeof o, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&ns, nseg, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    if (err & (ERR_RANGE | ERR_WEIGHT)) return err_to_code(err);
    ++g->version;  // some records may have been applied before an out-of-pool stop
    if (h_stats) {
        bingo_update_stats part{};
        part.inserted = o[0];
        part.deleted = o[1];
        part.not_found = o[2];
        for (int i = 0; i < 25; ++i) part.transitions[i] = o[3 + i];
        part.match_scanned = o[28];
        part.match_candidates = o[29];
        add_stats(h_stats, part);
        if (!h_stats->touched_vertices) h_stats->touched_vertices = ns;  // the first pass saw every source
    }
    if (err != ERR_OOM || !retries) return err ? err_to_code(err) : BINGO_OK;
    // Out of pool: the records each stopped source did not apply are flagged.  Reclaim the
    // replaced blocks, or grow a pool the library sized, and apply those records, in their
    // order, once more (records of different sources are independent, so this equals the
    // stream applied in one pass).
    // left and its scan live in the workspace, which compaction and the second pass reuse: gather
    // the records into a buffer of their own first
    scan_u32_to_u64(left, hx, m, tmp, nseg, st);
    unsigned long long k = 0;
    HIPCHK(hipMemcpyAsync(&k, nseg, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (k == 0) return BINGO_E_OOM;
    uint32_t* rest = nullptr;
    if (hipMallocAsync((void**)&rest, k * 16, st) != hipSuccess) return BINGO_E_OOM;
    hipLaunchKernelGGL(k_st_gather, dim3(grid_for(m)), dim3(TB), 0, st, m, (const uint32_t*)left, (const uint64_t*)hx,
                       op, src, dst, w, rest, (uint64_t)k);
    unsigned long long ctl[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const uint64_t bigger = std::min<uint64_t>(g->pool_words * 2, 1ull << 35);
    const bool grow = g->pool_auto && bigger > g->pool_words;
    int rc = BINGO_E_OOM;
    if (ctl[1] > 0 || grow) rc = compact_pool(g, grow ? bigger : 0, st);
    if (rc == BINGO_OK) rc = apply_stream(g, k, rest, rest + k, rest + 2 * k, rest + 3 * k, h_stats, retries - 1, st);
    else rc = BINGO_E_OOM;
    HIPCHK(hipFreeAsync(rest, st));
    HIPCHK(hipStreamSynchronize(st));
    return rc;
}
}  // namespace

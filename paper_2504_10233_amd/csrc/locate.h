// locate.h -- the edge locator: an open-addressing hash multiset of the live
// edges, one slot per edge, key (u << 32 | dst) -> the edge's neighbour index
// in u's adjacency.  A batch delete names (src, dst), while the delete-and-swap
// of Sec. 4.2 and Sec. 5.2 starts from the neighbour index; the locator turns
// one into the other with a few probes instead of a scan of src's adjacency.
//
// Linear probing over a power-of-two table of 16-byte slots (the key, then the
// index in the low word of the second u64), so a probe reads one line.  A slot's
// key is EMPTY, a TOMB (a
// deleted edge; probes pass over it, a claim may take it) or a key.  Within one
// kernel slots only go from EMPTY or TOMB to a key (claims, by compare-and-swap)
// or from a key to TOMB (deletes); a slot's index field changes only when its
// own edge moves.  Duplicate edges (the same (u, dst) more than once) are
// separate slots of the same key, told apart by their index.
#pragma once
#include "dev.h"

constexpr uint64_t LOC_EMPTY = ~0ull;
constexpr uint64_t LOC_TOMB = ~0ull - 1;  // vertex ids stay below 2^31, so no key takes these values

struct LocView {
    uint64_t* tab;  // slot h: tab[2h] key, tab[2h + 1] neighbour index
    uint64_t mask;  // capacity - 1
};

struct LocSlot {
    uint64_t key, pos;
};
__device__ __forceinline__ LocSlot loc_slot(const LocView& L, uint64_t h) {
    const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(L.tab + 2 * h);
    return LocSlot{v.x, v.y};
}

__host__ __device__ __forceinline__ uint64_t loc_key(uint32_t u, uint32_t dst) { return ((uint64_t)u << 32) | dst; }

// splitmix64's output function (Steele, Lea and Flood, 2014) as the slot hash
__device__ __forceinline__ uint64_t loc_hash(uint64_t k) {
    k ^= k >> 30;
    k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27;
    k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return k;
}

// Visit the probe sequence of k in order, one 128-byte line (8 slots) per round of
// loads, so a sequence inside one line costs one memory round trip: f(h, key,
// index) is called for each slot until it returns true or an EMPTY slot ends the
// sequence.  Returns the slots visited.
template <class F>
__device__ __forceinline__ uint32_t loc_walk(const LocView& L, uint64_t k, F f) {
    const uint64_t h0 = loc_hash(k) & L.mask;
    uint64_t line = h0 & ~7ull;  // the capacity is a multiple of 8, so a line never wraps
    uint32_t first = (uint32_t)(h0 & 7), seen = 0;
    for (uint64_t s = 0; s <= L.mask; s += 8) {
        ulonglong2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<const ulonglong2*>(L.tab + 2 * (line + j));
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if ((uint32_t)j < first) continue;
            ++seen;
            if (v[j].x == LOC_EMPTY || f(line + j, v[j].x, (uint32_t)v[j].y)) return seen;
        }
        line = (line + 8) & L.mask;
        first = 0;
    }
    return seen;
}

// Slot holding the occurrence of k at neighbour index p; LOC_EMPTY when there is none.
__device__ __forceinline__ uint64_t loc_find(const LocView& L, uint64_t k, uint32_t p) {
    uint64_t found = LOC_EMPTY;
    loc_walk(L, k, [&](uint64_t h, uint64_t key, uint32_t pos) {
        if (key == k && pos == p) {
            found = h;
            return true;
        }
        return false;
    });
    return found;
}

// Put (k, p) in the first free slot of its probe sequence.  Returns 0 when the
// table has no free slot (never with the load the host keeps), 1 after taking
// a TOMB, 2 after taking an EMPTY slot.
__device__ __forceinline__ uint32_t loc_claim(const LocView& L, uint64_t k, uint32_t p) {
    const uint64_t h0 = loc_hash(k) & L.mask;
    uint64_t line = h0 & ~7ull;
    uint32_t first = (uint32_t)(h0 & 7);
    for (uint64_t s = 0; s <= L.mask; s += 8) {
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = L.tab[2 * (line + j)];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if ((uint32_t)j < first) continue;
            const uint64_t cur = v[j];
            if (cur != LOC_EMPTY && cur != LOC_TOMB) continue;
            unsigned long long* kp = (unsigned long long*)(L.tab + 2 * (line + j));
            if (atomicCAS(kp, (unsigned long long)cur, (unsigned long long)k) == cur) {
                L.tab[2 * (line + j) + 1] = p;
                return cur == LOC_EMPTY ? 2u : 1u;
            }
            // another claim took it first; a taken slot stays taken for the rest of the kernel
        }
        line = (line + 8) & L.mask;
        first = 0;
    }
    return 0u;
}

// ---------------------------------------------------------------------------
// Wave-cooperative probing.  Many copies of one edge make a run of slots of one
// key, which a lane walking alone would cross one line per memory round trip.
// So a lane first looks at its own first line only (loc_first_line,
// loc_claim_line); a lane whose sequence goes on past it is then served by the
// whole wave, 64 consecutive slots per load (lane i reads slot start + i) with
// the decision taken by ballots.  Every lane of the wave must call the wave
// functions (wave-uniform control flow).
// ---------------------------------------------------------------------------
// The slots of k's sequence in its first line, through f as in loc_walk.  Returns
// true when the sequence goes on past the line (*next: the following line).
template <class F>
__device__ __forceinline__ bool loc_first_line(const LocView& L, uint64_t k, uint64_t* next, uint32_t* seen, F f) {
    const uint64_t h0 = loc_hash(k) & L.mask;
    const uint64_t line = h0 & ~7ull;
    ulonglong2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<const ulonglong2*>(L.tab + 2 * (line + j));
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if ((uint64_t)j < (h0 & 7)) continue;
        ++*seen;
        if (v[j].x == LOC_EMPTY || f(line + j, v[j].x, (uint32_t)v[j].y)) return false;
    }
    *next = (line + 8) & L.mask;
    return true;
}

// Lanes below the first EMPTY of a window (all 64 when it has none).
__device__ __forceinline__ uint64_t loc_before_empty(uint64_t em) {
    return em ? ((1ull << (__ffsll((long long)em) - 1)) - 1) : ~0ull;
}

// Find, for every lane with want set, the slot of (k, p) from *next on (*found:
// the slot, or LOC_EMPTY when the sequence ends without it).
__device__ __forceinline__ void loc_wave_find(const LocView& L, bool want, uint64_t k, uint32_t p, uint64_t next,
                                              uint64_t* found) {
    const uint32_t lane = lane_id();
    uint64_t todo = __ballot(want);
    while (todo) {
        const int o = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const uint64_t kk = __shfl(k, o, 64);
        const uint32_t pp = __shfl(p, o, 64);
        uint64_t start = __shfl(next, o, 64), hit = LOC_EMPTY;
        for (uint64_t s = 0; s <= L.mask; s += 64) {
            const uint64_t h = (start + lane) & L.mask;
            const LocSlot c = loc_slot(L, h);
            const uint64_t em = __ballot(c.key == LOC_EMPTY);
            const uint64_t f = __ballot(c.key == kk && (uint32_t)c.pos == pp) & loc_before_empty(em);
            if (f) {
                hit = (start + (uint64_t)(__ffsll((long long)f) - 1)) & L.mask;
                break;
            }
            if (em) break;
            start = (start + 64) & L.mask;
        }
        if (lane == (uint32_t)o) *found = hit;
    }
}

// The first line of k's sequence for a claim of (k, p): 0 when the sequence goes on
// past the line without a free slot taken (*next: the following line), else 1 or 2
// as loc_claim returns.
__device__ __forceinline__ uint32_t loc_claim_line(const LocView& L, uint64_t k, uint32_t p, uint64_t* next) {
    const uint64_t h0 = loc_hash(k) & L.mask;
    const uint64_t line = h0 & ~7ull;
    uint64_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = L.tab[2 * (line + j)];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if ((uint64_t)j < (h0 & 7)) continue;
        const uint64_t cur = v[j];
        if (cur != LOC_EMPTY && cur != LOC_TOMB) continue;
        if (atomicCAS((unsigned long long*)(L.tab + 2 * (line + j)), (unsigned long long)cur, (unsigned long long)k) ==
            cur) {
            L.tab[2 * (line + j) + 1] = p;
            return cur == LOC_EMPTY ? 2u : 1u;
        }
    }
    *next = (line + 8) & L.mask;
    return 0u;
}

// Claims, for every lane with want set, the first free slot from *next on (*res: 0 when
// none, else as loc_claim).
__device__ __forceinline__ void loc_wave_claim(const LocView& L, bool want, uint64_t k, uint32_t p, uint64_t next,
                                               uint32_t* res) {
    const uint32_t lane = lane_id();
    uint64_t todo = __ballot(want);
    while (todo) {
        const int o = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const uint64_t kk = __shfl(k, o, 64);
        const uint32_t pp = __shfl(p, o, 64);
        uint64_t start = __shfl(next, o, 64);
        uint32_t got = 0;
        for (uint64_t s = 0; s <= L.mask && !got; s += 64) {
            const uint64_t h = (start + lane) & L.mask;
            const uint64_t cur = L.tab[2 * h];
            uint64_t fr = __ballot(cur == LOC_EMPTY || cur == LOC_TOMB);
            while (fr) {  // free slots in sequence order until one CAS succeeds
                const int j = __ffsll((long long)fr) - 1;
                fr &= fr - 1;
                uint32_t r = 0;
                if (lane == (uint32_t)j &&
                    atomicCAS((unsigned long long*)(L.tab + 2 * h), (unsigned long long)cur, (unsigned long long)kk) ==
                        cur) {
                    L.tab[2 * h + 1] = pp;
                    r = cur == LOC_EMPTY ? 2u : 1u;
                }
                got = __shfl(r, j, 64);
                if (got) break;
            }
            start = (start + 64) & L.mask;
        }
        if (lane == (uint32_t)o) *res = got;
    }
}

__device__ __forceinline__ uint32_t loc_wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Host side (locate.hip).
// Make the locator valid for a batch of at most n_ins inserts: built on first
// use or after locator_invalidate, rebuilt (grown when needed) when live edges,
// deleted slots and the batch's claims would pass the load limit.  Returns
// false when it cannot (no device memory): the batch then locates by scanning.
bool locator_prepare(bingo_graph* g, uint64_t n_ins, hipStream_t st);
// The locator view the batch pipeline uses (tab == nullptr: none).
LocView locator_view(const bingo_graph* g);
// Counters of an applied batch: slots turned TOMB, claims, claims of EMPTY slots, failed lookups.
void locator_after_batch(bingo_graph* g, uint64_t kills, uint64_t claims, uint64_t fresh, uint64_t bad);
void locator_invalidate(bingo_graph* g);
void locator_release(bingo_graph* g);

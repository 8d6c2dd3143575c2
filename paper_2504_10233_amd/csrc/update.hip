// update.hip -- batched edge insertions and deletions (Sec. 5.2, Fig. 10;
// Sec. 4.2 insertion / deletion on the radix groups).
//
// Pipeline (all on one stream):
//   1. validate; sort records by (src, op, dst) keeping batch order for inserts;
//      segment into touched vertices (the "group updates by vertex" step).
//   2. match deletes: every live edge and every insert of a touched vertex is
//      looked up among that vertex's delete targets; candidates are sorted by
//      (delete run, sequence number) so each run of k identical delete records
//      takes the k oldest live occurrences.
//   3. per touched vertex, the set X of deleted indices (sorted).
//   4. analysis (one wave per vertex): new counts c'_k, new degree, new types,
//      and the pool words needed; one scan and one bump allocate them.
//   5. mutation (one wave per vertex): two-phase delete-and-swap on the
//      adjacency (holes below the new degree filled by tail survivors in rank
//      order), appends, the same rule on every listed group that keeps its type,
//      renames of moved indices, fresh lists for groups that change type, and
//      the new header (the inter-group space, updated once per vertex).
#include "dev.h"
#include "locate.h"
#include <stdio.h>
#include <algorithm>
#include <string.h>
#include <vector>

namespace {

constexpr int TB = 256;
constexpr int WB = 256;
constexpr uint32_t NF = 0xFFFFFFFFu;
constexpr uint32_t MB = 1024;  // flat elements per matching block
constexpr uint32_t PART_BLOCKS = 2048;  // grid cap of the per-vertex kernels (blocks of 4 waves)


inline uint32_t grid_for(uint64_t n) {
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n + TB - 1) / TB, 1), 1u << 20);
}
int bits_for(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

#define GRID_LOOP(i, n) for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (uint64_t)gridDim.x * blockDim.x)

// Control block of one update pipeline run (u64 words, device memory):
//   [0] inserts  [1] deletes  [2] touched vertices T  [3] flat matching size F
//   [4] candidates C  [5] deleted-set entries  [6] pool words requested  [7] pool base
//   [8] overflow flags (bit 0: more candidates than the candidate buffer holds)  [9] records
//   [10] split work items  [11] split work chunks  [12] split pass-A survivor words
//   [13] large vertices (more than the split threshold of entries)
//   [16..47] statistics (inserted, deleted, not found, 25 type transitions)
//   [48..79] freed pool words (entry 48)
//   [80..84] edge locator: slots probed to match deletes, slots turned TOMB, claims,
//            claims of EMPTY slots, lookups that found no slot (a locator out of step)
// Every kernel reads its element counts from here, so the whole pipeline runs
// without host round trips and can be captured in a hipGraph; grids and
// buffers are sized by the batch-size bucket Rmax.
enum { UC_NI = 0, UC_ND = 1, UC_T = 2, UC_F = 3, UC_C = 4, UC_X = 5, UC_ALLOC = 6, UC_BASE = 7, UC_FLAGS = 8,
       UC_R = 9, UC_BIG_ITEMS = 10, UC_BIG_CHUNKS = 11, UC_BIG_SUR = 12, UC_NBIG = 13,
       UC_STATS = 16, UC_FREED = 48, UC_LPROBE = 80, UC_LKILL = 81, UC_LCLAIM = 82, UC_LFRESH = 83, UC_LBAD = 84,
       UC_WORDS = 96 };

__global__ void k_upd_begin(unsigned long long* __restrict__ uc, uint64_t ni, uint64_t nd, uint32_t* __restrict__ err) {
    const uint32_t i = threadIdx.x;
    if (i < UC_WORDS) uc[i] = i == UC_NI ? ni : (i == UC_ND ? nd : (i == UC_R ? ni + nd : 0ull));
    if (i == 0) *err = 0;
}

__global__ void k_fill_u32(uint32_t* __restrict__ a, uint64_t n, uint32_t v) {
    GRID_LOOP(i, n) a[i] = v;
}
__global__ void k_fill_u64(uint64_t* __restrict__ a, uint64_t n, uint64_t v) {
    GRID_LOOP(i, n) a[i] = v;
}

__global__ void k_upd_validate(uint32_t n, const unsigned long long* __restrict__ uc, const uint32_t* __restrict__ is,
                               const uint32_t* __restrict__ id, const uint32_t* __restrict__ iw,
                               const uint32_t* __restrict__ ds, const uint32_t* __restrict__ dd,
                               uint32_t* __restrict__ err) {
    const uint64_t ni = uc[UC_NI], nd = uc[UC_ND];
    uint32_t bad = 0;
    GRID_LOOP(i, ni) {
        if (is[i] >= n || id[i] >= n) bad |= ERR_RANGE;
        if (iw[i] == 0) bad |= ERR_WEIGHT;
    }
    GRID_LOOP(i, nd) {
        if (ds[i] >= n || dd[i] >= n) bad |= ERR_RANGE;
    }
    if (bad) atomicOr(err, bad);
}

// A rejected batch runs the rest of the pipeline as an empty one, so no kernel
// indexes a header with an out-of-range vertex.
__global__ void k_upd_gate(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err) {
    if (*err) uc[UC_NI] = uc[UC_ND] = uc[UC_R] = 0ull;
}

// insert j: key (src << (vb+1)); delete j: key (src << (vb+1)) | 1 << vb | dst;
// slots past the batch hold `pad`, which sorts after every record key
__global__ void k_upd_keys(const unsigned long long* __restrict__ uc, uint64_t rmax, const uint32_t* __restrict__ is,
                           const uint32_t* __restrict__ ds, const uint32_t* __restrict__ dd, int vb, uint64_t pad,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint64_t ni = uc[UC_NI], nd = uc[UC_ND];
    GRID_LOOP(r, rmax) {
        uint64_t k = pad;
        if (r < ni) {
            k = (uint64_t)is[r] << (vb + 1);
        } else if (r < ni + nd) {
            const uint64_t j = r - ni;
            k = ((uint64_t)ds[j] << (vb + 1)) | (1ull << vb) | dd[j];
        }
        keys[r] = k;
        vals[r] = (uint32_t)r;
    }
}

__device__ __forceinline__ uint32_t key_src(uint64_t k, int vb) { return (uint32_t)(k >> (vb + 1)); }
__device__ __forceinline__ uint32_t key_op(uint64_t k, int vb) { return (uint32_t)(k >> vb) & 1u; }
__device__ __forceinline__ uint32_t key_dst(uint64_t k, int vb) { return (uint32_t)(k & ((1ull << vb) - 1)); }

__global__ void k_seg_heads(const uint64_t* __restrict__ sk, const unsigned long long* __restrict__ uc, uint64_t rmax,
                            int vb, uint32_t* __restrict__ head) {
    const uint64_t R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(p, rmax) head[p] = (p < R && (p == 0 || key_src(sk[p], vb) != key_src(sk[p - 1], vb))) ? 1u : 0u;
}

// per touched vertex t: tv (vertex), ts (first record), tdl (first delete record)
__global__ void k_seg_fill(const uint64_t* __restrict__ sk, const unsigned long long* __restrict__ uc, int vb,
                           const uint32_t* __restrict__ head, const uint64_t* __restrict__ hx,
                           uint32_t* __restrict__ tv, uint32_t* __restrict__ ts, uint32_t* __restrict__ tdl,
                           uint32_t* __restrict__ rec_t) {
    const uint64_t R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(p, R) {
        const uint64_t t = hx[p] + head[p] - 1;
        rec_t[p] = (uint32_t)t;
        if (head[p]) { tv[t] = key_src(sk[p], vb); ts[t] = (uint32_t)p; }
        if (key_op(sk[p], vb) && (head[p] || !key_op(sk[p - 1], vb))) tdl[t] = (uint32_t)p;
    }
}

__global__ void k_seg_end(const unsigned long long* __restrict__ uc, const uint32_t* __restrict__ ts,
                          uint32_t* __restrict__ te, uint32_t* __restrict__ tdl) {
    const uint64_t T = uc[UC_T], R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(t, T) {
        const uint32_t end = (t + 1 < T) ? ts[t + 1] : (uint32_t)R;
        te[t] = end;
        if (tdl[t] == NF) tdl[t] = end;
    }
}

// flat size of the delete-matching space of t: its live edges and its inserts (0 past T;
// only the inserts when the edge locator finds the live edges);
// also the degree before the batch, dold[t], and the list of the vertices with more than
// `split` entries after the inserts (in no particular order)
__global__ void k_flat_size(unsigned long long* __restrict__ uc, uint64_t rmax, const uint32_t* __restrict__ tv,
                            const uint32_t* __restrict__ ts, const uint32_t* __restrict__ tdl,
                            const uint32_t* __restrict__ te, const uint32_t* __restrict__ hdr,
                            uint64_t* __restrict__ fsz, uint32_t* __restrict__ dold, uint32_t* __restrict__ vacap,
                            uint32_t* __restrict__ vnseq, uint64_t* __restrict__ vadj, uint32_t split,
                            uint32_t* __restrict__ blist, uint32_t ins_only) {
    const uint64_t T = uc[UC_T];
    GRID_LOOP(t, rmax) {
        uint64_t v = 0;
        if (t < T) {
            const uint32_t nd = te[t] - tdl[t];
            const uint32_t ni = tdl[t] - ts[t];
            const uint32_t* h = hdr + (size_t)tv[t] * HDR_WORDS;
            const uint32_t d = h[H_DEG];
            dold[t] = d;
            vacap[t] = h[H_ACAP];
            vnseq[t] = h[H_NSEQ];
            vadj[t] = hdr_adj(h);
            v = nd ? (uint64_t)(ins_only ? 0u : d) + ni : 0ull;
            if (split && d + ni > split) blist[atomicAdd(uc + UC_NBIG, 1ull)] = (uint32_t)t;
        }
        fsz[t] = v;
    }
}

// last t with foff[t] <= f, searching in [lo, hi]
__device__ __forceinline__ uint32_t find_t(const uint64_t* __restrict__ foff, uint32_t lo, uint32_t hi, uint64_t f) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Candidate search: every element of the flat space (live edges, then inserts,
// of each touched vertex with deletes) whose dst is among the vertex's delete
// targets becomes a candidate (run << 32 | seq, virtual index).  Each block
// takes a contiguous run of ranges of MB elements.  For DESC ranges at a time
// it first finds, one lane per range, the touched vertices owning the range's
// first and last element and where its delete targets start, so a range then
// needs only its staging loads before its elements: the offsets and header
// fields of the (at most MV) touched vertices it spans, from the per-vertex
// copies k_flat_size made, and the dst of their batch records (every 2^sh-th
// record when there are more than LDS_TARGETS).  The per-element vertex search
// and target search then run in LDS but for at most sh steps; a range that spans
// more vertices than MV searches them in global memory instead.  Consecutive
// ranges inside one vertex keep its staged state.  Hits collect in an LDS
// buffer that is written out (one atomic per flush) when it could not take
// another range, so the global atomics number about one per OUTCAP hits.
constexpr uint32_t LDS_TARGETS = 2048;
constexpr uint32_t MV = 128;      // staged vertices per range
constexpr uint32_t OUTCAP = 2048;  // buffered hits per block (>= MB + a range's worth)
constexpr uint32_t DESC = 64;     // ranges whose descriptors are found together (one lane each)
static_assert(OUTCAP >= 2 * MB, "the hit buffer takes a full range after any flush threshold");

// Wave-cooperative form of find_t over [0, tmax] (foff[0] = 0 <= f): each round
// probes 64 evenly spaced offsets at once and keeps the stride the answer lies
// in, so a search over 10^6 vertices takes 4 dependent loads instead of 20.
// Every lane of the wave calls it and gets the result.
__device__ __forceinline__ uint32_t wave_find_t(const uint64_t* __restrict__ foff, uint32_t tmax, uint64_t f) {
    const uint32_t lane = lane_id();
    uint32_t lo = 0, hi = tmax;  // invariant: foff[lo] <= f, answer in [lo, hi]
    while (hi - lo >= 64) {
        const uint32_t stride = (uint32_t)(((uint64_t)(hi - lo) + 64) / 64);  // 64 * stride > hi - lo
        const uint64_t t = (uint64_t)lo + (uint64_t)lane * stride;
        const bool le = t <= hi && foff[t] <= f;
        const uint64_t b = __ballot(le);  // lane 0 (t = lo) is always set
        const uint32_t k = 63 - __clzll(b);
        lo += k * stride;
        hi = (uint32_t)std::min<uint64_t>(hi, (uint64_t)lo + stride - 1);
    }
    const uint32_t t = lo + lane;
    const uint64_t b = __ballot(t <= hi && foff[t] <= f);
    return lo + (63 - __clzll(b));
}

__device__ __forceinline__ uint32_t find_t_lds(const uint64_t* __restrict__ fo, uint32_t nv, uint64_t f) {
    uint32_t lo = 0, hi = nv - 1;  // last k with fo[k] <= f
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (fo[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(TB) k_match(unsigned long long* __restrict__ uc, const uint64_t* __restrict__ foff,
                                              const uint32_t* __restrict__ ts, const uint32_t* __restrict__ tdl,
                                              const uint32_t* __restrict__ te, const uint32_t* __restrict__ vdeg,
                                              const uint32_t* __restrict__ vacap, const uint32_t* __restrict__ vnseq,
                                              const uint64_t* __restrict__ vadj, const uint64_t* __restrict__ sk,
                                              const uint32_t* __restrict__ sv, int vb, const uint32_t* __restrict__ id,
                                              const uint32_t* __restrict__ pool, uint64_t* __restrict__ ckey,
                                              uint32_t* __restrict__ cval, uint64_t cap, uint32_t ins_only) {
    __shared__ uint64_t s_fo[MV];
    __shared__ uint32_t s_v[8][MV];  // d, acap, nseq, adj lo, adj hi, ts, tdl, te
    __shared__ uint32_t tgt[LDS_TARGETS];
    __shared__ uint64_t okey[OUTCAP];
    __shared__ uint32_t oidx[OUTCAP];
    __shared__ uint32_t dlo[DESC], dhi[DESC], drb[DESC], dsh[DESC], dns[DESC];  // per-range descriptors
    __shared__ uint32_t cspan[2];    // first and last touched vertex of a chunk of ranges
    __shared__ uint32_t wtot[TB / 64];
    __shared__ uint32_t ocount;
    __shared__ unsigned long long obase;
    const uint64_t F = uc[UC_F], T = uc[UC_T];
    const uint64_t nblk = (F + MB - 1) / MB;
    constexpr int PER = MB / TB;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) ocount = 0;
    uint32_t held = ~0u;  // the one vertex whose staged fields and targets the LDS still holds (block-uniform)
    // each block takes a contiguous run of ranges, so consecutive ranges of
    // one large vertex reuse its staged header fields and targets
    const uint64_t per = (nblk + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = (uint64_t)blockIdx.x * per, b1 = std::min<uint64_t>(nblk, b0 + per);
    for (uint64_t c0 = b0; c0 < b1; c0 += DESC) {
        const uint32_t nc = (uint32_t)std::min<uint64_t>(DESC, b1 - c0);
        __syncthreads();  // the previous chunk's readers of the descriptors are done
        // the touched vertices owning the chunk's first and last element (waves 0 and 1, 64 probes per load)
        if (wave < 2) {
            const uint64_t f = wave == 0 ? c0 * MB : std::min<uint64_t>((c0 + nc) * MB, F) - 1;
            const uint32_t t = wave_find_t(foff, (uint32_t)T - 1, f);
            if (lane == 0) cspan[wave] = t;
        }
        __syncthreads();
        // each range's first (wave 0) and last (wave 1) owner, searched between the two
        if (wave < 2 && lane < nc) {
            const uint64_t f0 = (c0 + lane) * MB;
            const uint64_t f = wave == 0 ? f0 : std::min<uint64_t>(f0 + MB, F) - 1;
            const uint32_t t = find_t(foff, cspan[0], cspan[1], f);
            if (wave == 0) dlo[lane] = t; else dhi[lane] = t;
        }
        __syncthreads();
        if (wave == 0 && lane < nc) {
            const uint32_t rb = ts[dlo[lane]], re = te[dhi[lane]];
            uint32_t sh = 0;
            while (((re - rb) + (1u << sh) - 1) >> sh > LDS_TARGETS) ++sh;
            drb[lane] = rb;
            dsh[lane] = sh;
            dns[lane] = ((re - rb) + (1u << sh) - 1) >> sh;
        }
        for (uint32_t jr = 0; jr < nc; ++jr) {
            const uint64_t blk = c0 + jr;
            const uint64_t f0 = blk * MB;
            __syncthreads();  // descriptors written; the previous range's users of the shared state are done
            const uint32_t tlo = dlo[jr], thi = dhi[jr], rbase = drb[jr], tsh = dsh[jr];
            const bool vstaged = thi - tlo < MV;
            const bool reuse = tlo == thi && held == tlo;
            const uint32_t nv = thi - tlo + 1;
            if (!reuse) {
                if (vstaged) {
                    for (uint32_t k = threadIdx.x; k < nv; k += TB) {
                        const uint32_t t = tlo + k;
                        const uint64_t a = vadj[t];
                        s_fo[k] = foff[t];
                        s_v[0][k] = vdeg[t]; s_v[1][k] = vacap[t]; s_v[2][k] = vnseq[t];
                        s_v[3][k] = (uint32_t)a; s_v[4][k] = (uint32_t)(a >> 32);
                        s_v[5][k] = ts[t]; s_v[6][k] = tdl[t]; s_v[7][k] = te[t];
                    }
                }
                const uint32_t ns = dns[jr];
                for (uint32_t j = threadIdx.x; j < ns; j += TB) tgt[j] = key_dst(sk[rbase + (j << tsh)], vb);
            }
            held = tlo == thi ? tlo : ~0u;
            __syncthreads();
            // each thread looks at PER elements, in phases so that the loads of all
            // of them are in flight together: its vertex's fields, then every dst,
            // then the target searches, then the seq of every hit; hits stay in
            // registers until the block has placed them in the LDS buffer
            uint64_t hkey[PER];
            uint32_t hidx[PER];
            uint32_t nh = 0;
            uint32_t e_i[PER], e_d[PER], e_acap[PER], e_nseq[PER], e_ts[PER], e_tdl[PER], e_te[PER], e_dst[PER];
            uint64_t e_adj[PER];
            bool e_in[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const uint64_t f = f0 + (uint64_t)r * TB + threadIdx.x;
                hkey[r] = 0;
                hidx[r] = 0;
                e_in[r] = f < F;
                e_i[r] = e_d[r] = e_acap[r] = e_nseq[r] = e_ts[r] = e_tdl[r] = e_te[r] = 0;
                e_adj[r] = 0;
                if (e_in[r]) {
                    uint64_t fo;
                    if (vstaged) {
                        const uint32_t k = find_t_lds(s_fo, nv, f);
                        fo = s_fo[k];
                        e_d[r] = s_v[0][k]; e_acap[r] = s_v[1][k]; e_nseq[r] = s_v[2][k];
                        e_adj[r] = ((uint64_t)s_v[4][k] << 32) | s_v[3][k];
                        e_ts[r] = s_v[5][k]; e_tdl[r] = s_v[6][k]; e_te[r] = s_v[7][k];
                    } else {
                        const uint32_t t = find_t(foff, tlo, thi, f);
                        fo = foff[t];
                        e_d[r] = vdeg[t]; e_acap[r] = vacap[t]; e_nseq[r] = vnseq[t];
                        e_adj[r] = vadj[t];
                        e_ts[r] = ts[t]; e_tdl[r] = tdl[t]; e_te[r] = te[t];
                    }
                    // a vertex's flat range covers virtual indices from d when it holds only the inserts
                    e_i[r] = (uint32_t)(f - fo) + (ins_only ? e_d[r] : 0u);
                }
            }
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                e_dst[r] = 0;
                if (e_in[r] && e_i[r] < e_d[r]) e_dst[r] = pool[e_adj[r] + 2ull * e_i[r]];
            }
#pragma unroll
            for (int r = 0; r < PER; ++r)
                if (e_in[r] && e_i[r] >= e_d[r]) e_dst[r] = id[sv[e_ts[r] + (e_i[r] - e_d[r])]];
            uint32_t e_l[PER];
            bool e_hit[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                e_hit[r] = false;
                e_l[r] = 0;
                if (e_in[r]) {
                    const uint32_t dst = e_dst[r], tdlv = e_tdl[r], tev = e_te[r];
                    // lower bound of dst among the vertex's delete targets [tdlv, tev): first over
                    // the LDS samples at positions rbase + (j << tsh) inside [tdlv, tev), then
                    // over the records between two samples in global memory
                    const uint32_t jl = (tdlv - rbase + (1u << tsh) - 1) >> tsh;
                    const uint32_t jh = (tev - rbase + (1u << tsh) - 1) >> tsh;
                    uint32_t ja = jl, jb = jh;
                    while (ja < jb) {
                        const uint32_t mid = (ja + jb) >> 1;
                        if (tgt[mid] < dst) ja = mid + 1; else jb = mid;
                    }
                    uint32_t l = ja > jl ? rbase + ((ja - 1) << tsh) + 1 : tdlv;
                    uint32_t rr = ja < jh ? rbase + (ja << tsh) : tev;
                    while (l < rr) {
                        const uint32_t mid = (l + rr) >> 1;
                        if (key_dst(sk[mid], vb) < dst) l = mid + 1; else rr = mid;
                    }
                    e_hit[r] = l < tev && (tsh == 0 ? tgt[l - rbase] : key_dst(sk[l], vb)) == dst;
                    e_l[r] = l;
                }
            }
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                if (e_hit[r]) {
                    const uint32_t i = e_i[r];
                    const uint32_t seq = i < e_d[r] ? pool[e_adj[r] + 2ull * e_acap[r] + i] : e_nseq[r] + (i - e_d[r]);
                    hkey[nh] = ((uint64_t)e_l[r] << 32) | seq;
                    hidx[nh] = i;
                    ++nh;
                }
            }
            // place the hits at the end of the LDS buffer
            uint32_t x = nh;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= (uint32_t)o) x += y;
            }
            if (lane == 63) wtot[wave] = x;
            __syncthreads();
            uint32_t before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < TB / 64; ++w) {
                if (w < (int)wave) before += wtot[w];
                total += wtot[w];
            }
            const uint32_t o0 = ocount + before + x - nh;
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                if ((uint32_t)r < nh) {
                    okey[o0 + r] = hkey[r];
                    oidx[o0 + r] = hidx[r];
                }
            }
            __syncthreads();  // all threads have read ocount and written their hits
            if (threadIdx.x == 0) ocount += total;
            __syncthreads();
            // flush when the buffer could not take another full range
            if (ocount > OUTCAP - MB) {
                if (threadIdx.x == 0) obase = atomicAdd(uc + UC_C, (unsigned long long)ocount);
                __syncthreads();
                for (uint32_t k = threadIdx.x; k < ocount; k += TB) {
                    if (obase + k < cap) {
                        ckey[obase + k] = okey[k];
                        cval[obase + k] = oidx[k];
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) ocount = 0;
            }
        }
    }
    __syncthreads();
    if (ocount) {
        if (threadIdx.x == 0) obase = atomicAdd(uc + UC_C, (unsigned long long)ocount);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < ocount; k += TB) {
            if (obase + k < cap) {
                ckey[obase + k] = okey[k];
                cval[obase + k] = oidx[k];
            }
        }
    }
}

__global__ void k_check_overflow(unsigned long long* uc, uint64_t cap) {
    if (uc[UC_C] > cap) uc[UC_FLAGS] |= 1ull;
}

// first candidate position of every run (candidates sorted by run, then seq; padding last)
__global__ void k_cand_first(const uint64_t* __restrict__ ck, const unsigned long long* __restrict__ uc, uint64_t cap,
                             uint32_t* __restrict__ first) {
    const uint64_t C = std::min<uint64_t>(uc[UC_C], cap);
    GRID_LOOP(c, C) {
        const uint32_t run = (uint32_t)(ck[c] >> 32);
        if (c == 0 || (uint32_t)(ck[c - 1] >> 32) != run) first[run] = (uint32_t)c;
    }
}

// the rank-th oldest occurrence goes to the rank-th record of the run
__global__ void k_cand_assign(const uint64_t* __restrict__ ck, const uint32_t* __restrict__ cv,
                              const unsigned long long* __restrict__ uc, uint64_t cap,
                              const uint32_t* __restrict__ first, const uint64_t* __restrict__ sk,
                              const uint32_t* __restrict__ rec_t, uint32_t* __restrict__ matched,
                              uint32_t* __restrict__ ncnt) {
    const uint64_t C = std::min<uint64_t>(uc[UC_C], cap), R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(c, C) {
        const uint32_t run = (uint32_t)(ck[c] >> 32);
        const uint32_t rank = (uint32_t)c - first[run];
        // run length: records with exactly the same key
        uint64_t lo = run, hi = R;
        const uint64_t key = sk[run];
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (sk[mid] <= key) lo = mid + 1; else hi = mid;
        }
        if (rank < lo - run) {
            matched[run + rank] = cv[c];
            atomicAdd(&ncnt[rec_t[run]], 1u);
        }
    }
}

__global__ void k_xkeys(const unsigned long long* __restrict__ uc, uint64_t rmax, const uint32_t* __restrict__ matched,
                        const uint32_t* __restrict__ rec_t, uint64_t pad, uint64_t* __restrict__ xk) {
    const uint64_t R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(p, rmax) xk[p] = (p < R && matched[p] != NF) ? (((uint64_t)rec_t[p] << 32) | matched[p]) : pad;
}

__global__ void k_xextract(uint64_t R, const uint64_t* __restrict__ xk, uint32_t* __restrict__ xs) {
    GRID_LOOP(p, R) xs[p] = (uint32_t)xk[p];
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t n, uint32_t v);

// Per insert record (sorted position j in [ts[t], tdl[t]) of touched vertex t):
// its weight wv[j], contiguous per vertex, and its final adjacency index
// idest[j] (NF when the batch deletes it again), so the per-group passes of
// k_mutate neither gather weights nor search the deleted set for inserts.
__global__ void k_ins_prep(const unsigned long long* __restrict__ uc, uint64_t rmax, const uint32_t* __restrict__ sv,
                           const uint32_t* __restrict__ iw, const uint32_t* __restrict__ rec_t,
                           const uint32_t* __restrict__ ts, const uint32_t* __restrict__ tdl,
                           const uint32_t* __restrict__ dold, const uint32_t* __restrict__ ncnt,
                           const uint64_t* __restrict__ xoff, const uint32_t* __restrict__ xs,
                           uint32_t* __restrict__ wv, uint32_t* __restrict__ idest) {
    const uint64_t R = uc[UC_NI] + uc[UC_ND];
    GRID_LOOP(j, rmax) {
        if (j >= R) continue;
        const uint32_t t = rec_t[j];
        const uint32_t s0 = ts[t], s1 = tdl[t];
        if (j >= s1) continue;  // a delete record
        const uint32_t a = (uint32_t)j - s0, d = dold[t], N = ncnt[t];
        const uint32_t* X = xs + xoff[t];
        const uint32_t e = d + a, dn = d + (s1 - s0) - N;
        const uint32_t pe = lower_bound_u32(X, N, e);
        uint32_t dest;
        if (pe < N && X[pe] == e) dest = NF;
        else if (e < dn) dest = e;
        else dest = X[(e - dn) - (pe - lower_bound_u32(X, N, dn))];
        wv[j] = iw[sv[j]];
        idest[j] = dest;
    }
}

// ---------------------------------------------------------------------------
// Edge locator (locate.h) in the batch pipeline.  Matching probes it for the
// live edges (k_match then scans only the batch's inserts); after the mutation
// three kernels bring it in step: slots of deleted live edges turn TOMB, live
// edges that moved into holes take their new index, surviving inserts claim
// slots.  The kill pass comes first so that no two live slots of one key ever
// share an index; moves and claims touch disjoint index ranges (a moved edge is
// looked up by an index >= dn, every new index is below dn or an insert's own).
// ---------------------------------------------------------------------------
// Sum v over the block into *dst (one atomic per block).  Every thread calls it.
__device__ __forceinline__ void block_add(unsigned long long* dst, uint32_t v, uint32_t* sh) {
    v = loc_wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) s += sh[w];
        if (s) atomicAdd(dst, (unsigned long long)s);
    }
}

// Wave-uniform grid loop: every lane of a wave runs the same iterations (i may
// be past n), so the wave-cooperative probes of locate.h can run inside.
#define WAVE_LOOP(i, n)                                                                                    \
    for (uint64_t i##_b = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u), i = i##_b + lane_id(); \
         i##_b < (n); i##_b += (uint64_t)gridDim.x * blockDim.x, i = i##_b + lane_id())

// Candidates among the live edges: the first record of each run of equal delete
// records (its sorted position r is the run id k_match uses as well) probes the
// locator for its (src, dst) and emits every occurrence as (r << 32 | seq,
// neighbour index).  A block counts its hits, reserves their space with one
// atomic, then writes them: the first HOLD of a record from registers, the rest
// (a key with many copies) by its wave walking the sequence again.
__global__ void __launch_bounds__(TB) k_loc_match(unsigned long long* __restrict__ uc, const uint64_t* __restrict__ sk,
                                                  int vb, const uint32_t* __restrict__ rec_t,
                                                  const uint32_t* __restrict__ tv, const uint32_t* __restrict__ tdl,
                                                  const uint32_t* __restrict__ dold, const uint32_t* __restrict__ vacap,
                                                  const uint64_t* __restrict__ vadj, const uint32_t* __restrict__ pool,
                                                  LocView L, uint64_t* __restrict__ ckey, uint32_t* __restrict__ cval,
                                                  uint64_t cap) {
    constexpr uint32_t HOLD = 4;
    __shared__ uint32_t wt[TB / 64];
    __shared__ unsigned long long bb;
    const uint64_t R = uc[UC_NI] + uc[UC_ND];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t probes = 0, bad = 0;
    for (uint64_t base = (uint64_t)blockIdx.x * TB; base < R; base += (uint64_t)gridDim.x * TB) {
        const uint64_t r = base + threadIdx.x;
        bool head = false;
        uint64_t k = 0;
        uint32_t t = 0, d = 0;
        if (r < R) {
            t = rec_t[r];
            d = dold[t];
            const uint32_t dl = tdl[t];
            if (r >= dl) {
                const uint32_t dst = key_dst(sk[r], vb);
                head = r == dl || key_dst(sk[r - 1], vb) != dst;
                k = loc_key(tv[t], dst);
            }
        }
        // count the hits; keep the first HOLD indexes
        uint32_t nh = 0, hp[HOLD], hs[HOLD];
        uint64_t next = 0;
        bool lng = false;
        if (head)
            lng = loc_first_line(L, k, &next, &probes, [&](uint64_t, uint64_t key, uint32_t p) {
                // an index past the degree would mean a locator out of step: never used
                if (key == k) {
                    if (p < d) {
                        if (nh < HOLD) hp[nh] = p;
                        ++nh;
                    } else {
                        ++bad;
                    }
                }
                return false;
            });
        for (uint64_t todo = __ballot(lng); todo; todo &= todo - 1) {
            const int o = __ffsll((long long)todo) - 1;
            const uint64_t kk = __shfl(k, o, 64);
            const uint32_t dd = __shfl(d, o, 64);
            uint64_t start = __shfl(next, o, 64);
            uint32_t cnt = __shfl(nh, o, 64);
            for (uint64_t s = 0; s <= L.mask; s += 64) {
                const LocSlot c = loc_slot(L, (start + lane) & L.mask);
                const uint64_t em = __ballot(c.key == LOC_EMPTY), live = loc_before_empty(em);
                uint64_t m = __ballot(c.key == kk && (uint32_t)c.pos < dd) & live;
                const uint64_t bm = __ballot(c.key == kk && (uint32_t)c.pos >= dd) & live;
                const uint32_t nm = (uint32_t)__popcll(m);
#pragma unroll
                for (uint32_t q = 0; q < HOLD; ++q) {
                    if (q >= cnt && m) {
                        const uint32_t p = __shfl((uint32_t)c.pos, __ffsll((long long)m) - 1, 64);
                        if (lane == (uint32_t)o) hp[q] = p;
                        m &= m - 1;
                    }
                }
                if (lane == (uint32_t)o) {
                    nh += nm;
                    bad += (uint32_t)__popcll(bm);
                    probes += em ? (uint32_t)__ffsll((long long)em) : 64u;
                }
                cnt += nm;
                if (em) break;
                start = (start + 64) & L.mask;
            }
        }
        const uint64_t seqb = head ? vadj[t] + 2ull * vacap[t] : 0ull;
#pragma unroll
        for (uint32_t j = 0; j < HOLD; ++j)
            if (j < nh) hs[j] = pool[seqb + hp[j]];
        uint32_t x = nh;  // inclusive prefix over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= (uint32_t)o) x += y;
        }
        __syncthreads();  // the previous round's readers of wt and bb are done
        if (lane == 63) wt[wave] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < TB / 64; ++w) tot += wt[w];
            bb = tot ? atomicAdd(uc + UC_C, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        uint64_t ob = bb + x - nh;
        for (int w = 0; w < (int)wave; ++w) ob += wt[w];
#pragma unroll
        for (uint32_t j = 0; j < HOLD; ++j) {
            if (j < nh && ob + j < cap) {
                ckey[ob + j] = ((uint64_t)r << 32) | hs[j];
                cval[ob + j] = hp[j];
            }
        }
        // hits past the first HOLD: the wave walks the record's sequence from its start
        for (uint64_t todo = __ballot(nh > HOLD); todo; todo &= todo - 1) {
            const int o = __ffsll((long long)todo) - 1;
            const uint64_t kk = __shfl(k, o, 64), oo = __shfl(ob, o, 64), sb = __shfl(seqb, o, 64);
            const uint64_t rr = __shfl(r, o, 64);
            const uint32_t dd = __shfl(d, o, 64), nn = __shfl(nh, o, 64);
            uint64_t start = loc_hash(kk) & L.mask;
            uint32_t run = 0;
            for (uint64_t s = 0; s <= L.mask && run < nn; s += 64) {
                const LocSlot c = loc_slot(L, (start + lane) & L.mask);
                const uint64_t em = __ballot(c.key == LOC_EMPTY);
                const bool mine = c.key == kk && (uint32_t)c.pos < dd && ((loc_before_empty(em) >> lane) & 1ull);
                const uint64_t m = __ballot(mine);
                const uint32_t rank = run + (uint32_t)__popcll(m & lanemask_lt());
                if (mine && rank >= HOLD && rank < nn && oo + rank < cap) {
                    ckey[oo + rank] = (rr << 32) | pool[sb + (uint32_t)c.pos];
                    cval[oo + rank] = (uint32_t)c.pos;
                }
                run += (uint32_t)__popcll(m);
                if (em) break;
                start = (start + 64) & L.mask;
            }
        }
    }
    block_add(uc + UC_LPROBE, probes, wt);
    block_add(uc + UC_LBAD, bad, wt);
}

// The slots of the deleted live edges turn TOMB (a rejected batch changes nothing).
__global__ void __launch_bounds__(TB) k_loc_kill(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err,
                                                 const uint64_t* __restrict__ sk, int vb,
                                                 const uint32_t* __restrict__ rec_t, const uint32_t* __restrict__ tv,
                                                 const uint32_t* __restrict__ dold,
                                                 const uint32_t* __restrict__ matched, LocView L) {
    __shared__ uint32_t sh[TB / 64];
    const bool skip = *err != 0 || uc[UC_FLAGS] != 0;
    const uint64_t R = skip ? 0 : uc[UC_NI] + uc[UC_ND];
    uint32_t kills = 0, bad = 0, seen = 0;
    WAVE_LOOP(r, R) {
        bool act = false;
        uint32_t x = NF;
        uint64_t k = 0, found = LOC_EMPTY, next = 0;
        if (r < R) {
            // the record's own fields load beside its vertex's
            const uint32_t t = rec_t[r];
            x = matched[r];
            const uint64_t key = sk[r];
            act = x != NF && x < dold[t];  // not an insert record, not absent, not an insert of this batch
            if (act) k = loc_key(tv[t], key_dst(key, vb));
        }
        bool lng = false;
        if (act)
            lng = loc_first_line(L, k, &next, &seen, [&](uint64_t h, uint64_t key, uint32_t p) {
                if (key == k && p == x) {
                    found = h;
                    return true;
                }
                return false;
            });
        loc_wave_find(L, lng, k, x, next, &found);
        if (act) {
            if (found == LOC_EMPTY) {
                ++bad;
            } else {
                L.tab[2 * found] = LOC_TOMB;
                ++kills;
            }
        }
    }
    block_add(uc + UC_LKILL, kills, sh);
    block_add(uc + UC_LBAD, bad, sh);
}

// Live edges that move into a hole take their new index.  Entry e of the
// deleted sets belongs to touched vertex t = xks[e] >> 32 (xoff[t] <= e < xoff[t] + N); the
// virtual index v = dn + (e - xoff[t]) runs over [dn, d + ni), and a surviving
// old edge among them (v < d) goes to hole X[j] by the rank rule of the
// mutation (the rule k_ins_prep applies to inserts).  Runs before the mutation,
// so the edge's dst is read at v in the old adjacency.
__global__ void __launch_bounds__(TB) k_loc_move(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err,
                                                 const uint64_t* __restrict__ xks, const uint64_t* __restrict__ xoff,
                                                 const uint32_t* __restrict__ ncnt,
                                                 const uint32_t* __restrict__ xs, const uint32_t* __restrict__ tv,
                                                 const uint32_t* __restrict__ ts, const uint32_t* __restrict__ tdl,
                                                 const uint32_t* __restrict__ dold, const uint64_t* __restrict__ vadj,
                                                 const uint32_t* __restrict__ pool, LocView L) {
    __shared__ uint32_t sh[TB / 64];
    const bool skip = *err != 0 || uc[UC_FLAGS] != 0;
    const uint64_t NX = skip ? 0 : uc[UC_X];
    uint32_t bad = 0, seen = 0;
    WAVE_LOOP(e, NX) {
        bool act = false;
        uint32_t v = 0, hole = 0;
        uint64_t k = 0, found = LOC_EMPTY, next = 0;
        if (e < NX) {
            const uint32_t t = (uint32_t)(xks[e] >> 32), N = ncnt[t], d = dold[t], u = tv[t];
            const uint64_t xo = xoff[t], adj = vadj[t];
            const uint32_t* X = xs + xo;
            const uint32_t dn = d + (tdl[t] - ts[t]) - N;
            v = dn + (uint32_t)(e - xo);
            if (v < d) {  // an old edge (an insert is placed by k_loc_claim)
                const uint32_t dst = pool[adj + 2ull * v];  // issued before the searches of the deleted set
                const uint32_t pv = lower_bound_u32(X, N, v);
                if (!(pv < N && X[pv] == v)) {  // it survives
                    hole = X[(v - dn) - (pv - lower_bound_u32(X, N, dn))];
                    k = loc_key(u, dst);
                    act = true;
                }
            }
        }
        bool lng = false;
        if (act)
            lng = loc_first_line(L, k, &next, &seen, [&](uint64_t h, uint64_t key, uint32_t p) {
                if (key == k && p == v) {
                    found = h;
                    return true;
                }
                return false;
            });
        loc_wave_find(L, lng, k, v, next, &found);
        if (act) {
            if (found == LOC_EMPTY) ++bad; else L.tab[2 * found + 1] = hole;
        }
    }
    block_add(uc + UC_LBAD, bad, sh);
}

// Every insert that survives the batch claims a slot at its final index.
__global__ void __launch_bounds__(TB) k_loc_claim(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err,
                                                  const uint32_t* __restrict__ rec_t, const uint32_t* __restrict__ tv,
                                                  const uint32_t* __restrict__ tdl, const uint32_t* __restrict__ sv,
                                                  const uint32_t* __restrict__ id, const uint32_t* __restrict__ idest,
                                                  LocView L) {
    __shared__ uint32_t sh[TB / 64];
    const bool skip = *err != 0 || uc[UC_FLAGS] != 0;
    const uint64_t R = skip ? 0 : uc[UC_NI] + uc[UC_ND];
    uint32_t claims = 0, fresh = 0, bad = 0;
    WAVE_LOOP(r, R) {
        bool act = false;
        uint32_t dest = 0, res = 0;
        uint64_t k = 0, next = 0;
        if (r < R) {
            const uint32_t t = rec_t[r], o = sv[r];
            dest = idest[r];
            // an insert record (r < tdl[t]) that the batch does not delete again
            act = r < tdl[t] && dest != NF;
            if (act) k = loc_key(tv[t], id[o]);
        }
        bool lng = false;
        if (act) {
            res = loc_claim_line(L, k, dest, &next);
            lng = res == 0;
        }
        loc_wave_claim(L, lng, k, dest, next, &res);
        if (act) {
            if (res == 0) ++bad;
            else {
                ++claims;
                fresh += res == 2;
            }
        }
    }
    block_add(uc + UC_LCLAIM, claims, sh);
    block_add(uc + UC_LFRESH, fresh, sh);
    block_add(uc + UC_LBAD, bad, sh);
}

// ---------------------------------------------------------------------------
// per-vertex state shared by the analysis and mutation kernels
// ---------------------------------------------------------------------------
struct VState {
    uint32_t u, d, cap, nseq, mask;
    uint64_t adj;
    uint32_t ts, ni, nd, N, xoff;
    uint32_t d1, dn;
    uint64_t W;  // fixed-point biases: sum of the weights after the batch (unused for integer biases)
    // group indexes: adjacency capacity after the batch; S(u) block, capacity before and after
    // (the new capacity covers an upper bound on |S(u)| after the batch); sparse masks before
    // and after
    uint32_t ncap, sblk, scap, scapn, smo, smn;
    // lane k < 32
    uint32_t c, cn, app, del, told, tnew, lcap, info;
};

__device__ __forceinline__ uint32_t ins_rec(const uint32_t* __restrict__ sv, uint32_t ts, uint32_t a) {
    return sv[ts + a];
}

// weight of virtual index x: an old edge (x < d) or insert x - d
__device__ __forceinline__ uint32_t vweight(uint32_t x, const VState& s, const uint32_t* __restrict__ pool,
                                            const uint32_t* __restrict__ wv) {
    if (x < s.d) return pool[s.adj + 2ull * x + 1];
    return wv[s.ts + (x - s.d)];
}

__device__ void load_state(VState& s, uint32_t t, const uint32_t* __restrict__ tv, const uint32_t* __restrict__ ts,
                           const uint32_t* __restrict__ tdl, const uint32_t* __restrict__ te,
                           const uint32_t* __restrict__ ncnt, const uint64_t* __restrict__ xoff,
                           const uint32_t* __restrict__ xs, const uint32_t* __restrict__ hdr,
                           const uint32_t* __restrict__ pool, const uint32_t* __restrict__ wv, GroupRule rule) {
    const uint32_t lane = lane_id();
    s.u = tv[t];
    const uint32_t* h = hdr + (size_t)s.u * HDR_WORDS;
    s.d = h[H_DEG]; s.cap = h[H_ACAP]; s.nseq = h[H_NSEQ]; s.mask = h[H_MASK];
    s.adj = hdr_adj(h);
    s.ts = ts[t]; s.ni = tdl[t] - ts[t]; s.nd = te[t] - tdl[t];
    s.N = ncnt[t]; s.xoff = (uint32_t)xoff[t];
    s.d1 = s.d + s.ni; s.dn = s.d1 - s.N;
    s.c = lane < 32 ? slot_count(hdr_slot(h, lane, hdr_hi(h)), h[H_ONEMASK], lane) : 0u;
    s.info = lane < 32 ? h[H_INFO + lane] : 0u;
    s.lcap = lane < 32 ? (1u << ((h[H_LCAPLOG + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu)) : 0u;
    s.told = lane < 32 ? group_type(s.c, s.d, rule) : GT_EMPTY;
    // group-membership counts of the inserts and of the deleted entries; for
    // fixed-point biases also their weight sums (the decimal group's total is
    // not a count times a power of two)
    uint32_t app = 0, del = 0;
    uint64_t wadd = 0, wsub = 0;
    for (uint32_t a0 = 0; a0 < s.ni; a0 += 64) {
        const uint32_t a = a0 + lane;
        const uint32_t wr = a < s.ni ? wv[s.ts + a] : 0u;
        wadd += wr;
        const uint32_t w = member_word(wr, rule.fbits);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const uint64_t b = __ballot((w >> k) & 1u);
            if (lane == (uint32_t)k) app += __popcll(b);
        }
    }
    const uint32_t* X = xs + s.xoff;
    for (uint32_t j0 = 0; j0 < s.N; j0 += 64) {
        const uint32_t j = j0 + lane;
        const uint32_t wr = j < s.N ? vweight(X[j], s, pool, wv) : 0u;
        wsub += wr;
        const uint32_t w = member_word(wr, rule.fbits);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const uint64_t b = __ballot((w >> k) & 1u);
            if (lane == (uint32_t)k) del += __popcll(b);
        }
    }
    s.W = 0;
    if (rule.fbits) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            wadd += __shfl_xor(wadd, o);
            wsub += __shfl_xor(wsub, o);
        }
        s.W = ((((uint64_t)h[H_WHI]) << 32) | h[H_WLO]) + wadd - wsub;
    }
    s.app = app; s.del = del;
    s.cn = s.c + app - del;
    s.tnew = lane < 32 ? group_type(s.cn, s.dn, rule) : GT_EMPTY;
    s.ncap = s.dn > s.cap ? adj_cap_for(s.dn) : s.cap;
    s.sblk = h[H_SBLK];
    s.scap = h[H_SCAP];
    s.smo = (uint32_t)(__ballot(s.told == GT_SPARSE) & 0xFFFFFFFFull);
    s.smn = (uint32_t)(__ballot(s.tnew == GT_SPARSE) & 0xFFFFFFFFull);
    // |S(u)| after the batch is at most min(d', sum of the new sparse counts)
    uint64_t sub = s.tnew == GT_SPARSE ? s.cn : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sub += __shfl_xor(sub, o);
    sub = sub < s.dn ? sub : s.dn;
    s.scapn = s.smn ? (sub > s.scap ? s_cap_for((uint32_t)sub) : s.scap) : 0u;
}

__device__ __forceinline__ bool kept_listed(const VState& s) { return type_listed(s.told) && s.tnew == s.told; }

// list capacity of a listed group after the batch (capacities only grow while the type is kept)
__device__ __forceinline__ uint32_t new_lcap(const VState& s) {
    if (kept_listed(s)) return s.cn > s.lcap ? list_cap_for(s.cn) : s.lcap;
    return list_cap_for(s.cn);
}
// pool words of lane k's list block before the batch (lane < 32, listed groups)
__device__ __forceinline__ uint64_t old_block_words(const VState& s) {
    return list_block_words(s.lcap, index_cap_for(s.told, s.cap, s.scap));
}

// Pool words this vertex allocates, per lane: lane k < 32 a list block for group
// k (list and index) when the group becomes listed, changes between sparse and
// regular, outgrows its list, or its index outgrows its block (regular: the
// adjacency capacity grows; sparse: the S(u) capacity grows); lane 32 a new
// S(u) block.  The adjacency block is added by the callers.
__device__ __forceinline__ uint64_t lane_list_need(const VState& s) {
    if (lane_id() == 32) return (s.scapn && s.scapn != s.scap) ? (uint64_t)s.scapn : 0ull;
    if (!type_listed(s.tnew)) return 0;
    const uint32_t icn = index_cap_for(s.tnew, s.ncap, s.scapn);
    if (kept_listed(s)) {
        const bool moves = s.cn > s.lcap || icn != index_cap_for(s.told, s.cap, s.scap);
        return moves ? list_block_words(new_lcap(s), icn) : 0ull;
    }
    return list_block_words(list_cap_for(s.cn), icn);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Statistics are accumulated per lane in registers over a grid-stride loop and
// reduced per block into partials[block * 32 + i] (i: 0 inserted, 1 deleted,
// 2 not found, 3.. the 25 type transitions); k_stats_reduce sums the blocks.
// No global atomics: a per-vertex atomic on a handful of addresses would
// serialize in L2 across ~10^6 touched vertices.
// Eight waves per SIMD fit without spilling (the default allocation allowed seven).
__global__ void __launch_bounds__(WB) __attribute__((amdgpu_waves_per_eu(8, 8))) k_analyze(const unsigned long long* __restrict__ uc, const uint32_t* __restrict__ tv,
                                                const uint32_t* __restrict__ ts,
                                                const uint32_t* __restrict__ tdl, const uint32_t* __restrict__ te,
                                                const uint32_t* __restrict__ ncnt, const uint64_t* __restrict__ xoff,
                                                const uint32_t* __restrict__ xs, const uint32_t* __restrict__ hdr,
                                                const uint32_t* __restrict__ pool, const uint32_t* __restrict__ wv,
                                                GroupRule rule, uint64_t* __restrict__ need,
                                                unsigned long long* __restrict__ partials) {
    __shared__ unsigned long long red[WB / 64][32];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint64_t T = uc[UC_T];
    uint64_t acc = 0;  // lane i < 28 accumulates counter i
    for (uint64_t t = (uint64_t)blockIdx.x * (WB / 64) + wave; t < T; t += (uint64_t)gridDim.x * (WB / 64)) {
        VState s;
        load_state(s, (uint32_t)t, tv, ts, tdl, te, ncnt, xoff, xs, hdr, pool, wv, rule);
        uint64_t w = lane_list_need(s);
        if (lane == 0 && s.dn > s.cap) w += adj_block_words(adj_cap_for(s.dn));
        w = wave_sum(w);
        // type transitions over all 32 groups of the vertex
        const uint32_t code = lane < 32 ? s.told * 5 + s.tnew : 31u;
#pragma unroll
        for (int c = 0; c < 25; ++c) {
            const uint32_t k = __popcll(__ballot(code == (uint32_t)c));
            if (lane == (uint32_t)(3 + c)) acc += k;
        }
        if (lane == 0) { need[t] = w; acc += s.ni; }
        if (lane == 1) acc += s.N;
        if (lane == 2) acc += s.nd - s.N;
    }
    if (lane < 32) red[wave][lane] = acc;
    __syncthreads();
    if (threadIdx.x < 32) {
        unsigned long long v = 0;
#pragma unroll
        for (int w = 0; w < WB / 64; ++w) v += red[w][threadIdx.x];
        partials[(uint64_t)blockIdx.x * 32 + threadIdx.x] = v;
    }
}

// Sum per-block partials: out[i] = sum_b partials[b * 32 + i]; block i sums counter i.
__global__ void __launch_bounds__(256) k_stats_reduce(const unsigned long long* __restrict__ partials,
                                                      uint32_t nblocks, unsigned long long* __restrict__ out,
                                                      int accumulate) {
    __shared__ unsigned long long red[4];
    const uint32_t i = blockIdx.x;
    unsigned long long v = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += 256) v += partials[(uint64_t)b * 32 + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long sum = red[0] + red[1] + red[2] + red[3];
        if (accumulate) out[i] += sum; else out[i] = sum;
    }
}

// ---------------------------------------------------------------------------
// mutation
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ bool in_set(const uint32_t* __restrict__ X, uint32_t N, uint32_t v) {
    const uint32_t p = lower_bound_u32(X, N, v);
    return p < N && X[p] == v;
}
// new index of a surviving virtual index v (adjacency two-phase rule)
__device__ __forceinline__ uint32_t rho(uint32_t v, const uint32_t* __restrict__ X, uint32_t N, uint32_t dn,
                                        uint32_t nholes) {
    if (v < dn) return v;
    const uint32_t j = (v - dn) - (lower_bound_u32(X, N, v) - nholes);
    return X[j];
}

// The deleted set of the vertex k_mutate is working on: the sorted array in
// global memory and, for the large-vertex instance, every 2^sh-th entry of it
// in LDS (sh = 0: all of it), so a search takes its first steps in LDS and at
// most sh steps in global memory.
struct XView {
    const uint32_t* X;
    const uint32_t* L;  // nullptr: no LDS samples
    uint32_t N, nl, sh;
};
__device__ __forceinline__ uint32_t xv_lb(const XView& x, uint32_t v) {
    if (!x.L) return lower_bound_u32(x.X, x.N, v);
    uint32_t lo = 0, hi = x.nl;  // samples below v
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (x.L[mid] < v) lo = mid + 1; else hi = mid;
    }
    if (lo == 0) return 0;
    uint32_t a = ((lo - 1) << x.sh) + 1, b = min(lo << x.sh, x.N);
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (x.X[mid] < v) a = mid + 1; else b = mid;
    }
    return a;
}
__device__ __forceinline__ uint32_t xv_at(const XView& x, uint32_t j) {
    return (x.L && x.sh == 0) ? x.L[j] : x.X[j];
}
__device__ __forceinline__ bool xv_in(const XView& x, uint32_t v) {
    const uint32_t p = xv_lb(x, v);
    return p < x.N && xv_at(x, p) == v;
}
// in_set and rho with one search: NF for a deleted v, else its new index
__device__ __forceinline__ uint32_t xv_rho(const XView& x, uint32_t v, uint32_t dn, uint32_t nholes) {
    const uint32_t p = xv_lb(x, v);
    if (p < x.N && xv_at(x, p) == v) return NF;
    if (v < dn) return v;
    return xv_at(x, (v - dn) - (p - nholes));
}

// virtual list entry p of a kept group k: the old list, then new members (inserts with bit k)
// in insert order.  Positions p >= c are enumerated by the insert scans below.

// ---------------------------------------------------------------------------
// Split work.  A touched vertex is handled by one wave, but four of its passes
// are O(d) or O(c_k): copying the adjacency into a larger block, pass A of a
// kept listed group (renames and holes over the whole list), building a fresh
// list for a group that changed type, and finding the member of a group that
// became one-element.  On a hub these would keep one wave busy for
// milliseconds, so above `split` entries the wave records a work item instead
// and the k_big_* kernels process it in chunks over the whole GPU after
// k_mutate.  Items and chunks come from fixed-size tables; a wave that cannot
// reserve space does the pass itself.
//   k_big_pass  : one wave per chunk: adjacency copies, one-element members, and
//                 pass A of lists with at most BIG_HOLES holes (renames written
//                 in place, hole positions collected unordered)
//   k_big_count / k_big_apply : ordered output (fresh lists, pass A of lists
//                 with more holes): per-chunk counts, then ranks
//   k_big_holes : per pass-A item of the first kind, its holes sorted by
//                 position take the tail survivors in order
// ---------------------------------------------------------------------------
enum { BK_COPY = 1, BK_PASSA = 2, BK_FRESH = 3, BK_ONE = 4, BK_PASSH = 5, BK_HOLES = 6 };
constexpr uint32_t BIG_HOLES = 4096;
constexpr uint32_t BIG_NONE = 0xFFFFFFFFu;
constexpr uint32_t BIG_MIN_CHUNK = 2048;
constexpr uint32_t BIG_MAX_CHUNKS_PER_ITEM = 16;

struct BigItem {
    uint32_t kind, k, n, csize;    // pass, group, entries, entries per chunk
    uint32_t cbase, u, xoff, N;    // first chunk, vertex, its deleted set xs[xoff .. xoff + N)
    uint32_t dn, nholes, keep, reloc;
    uint32_t sur, hole, ocap, ncap;  // survivor words sur[..], hole slots sur[hole ..], adjacency capacities
    uint64_t a, b, aold;           // block offsets in pool words (meaning per kind, see k_big_apply)
    uint32_t nh;                   // BK_PASSH: holes of the list
    uint32_t iofs;                 // regular list: its inverted index starts iofs words into block b (0: none)
    unsigned long long hcnt;       // BK_PASSH: hole positions collected so far
};
static_assert(sizeof(BigItem) == 104, "BigItem layout");

struct BigCtx {
    BigItem* items;
    uint32_t* chunk_item;
    uint32_t* sur;  // tail survivors of deferred pass-A lists, smax words
    uint32_t imax, cmax, smax;
    uint32_t fbits;  // fraction bits of fixed-point biases (membership words)
};

// Reserve an item and its chunks (every lane calls; the result is uniform).
__device__ __forceinline__ bool big_reserve(const BigCtx& bc, unsigned long long* uc, uint32_t n, uint32_t& item,
                                            uint32_t& cbase, uint32_t& csize) {
    const uint32_t lane = lane_id();
    uint32_t cs = BIG_MIN_CHUNK;
    while ((uint64_t)cs * BIG_MAX_CHUNKS_PER_ITEM < n) cs <<= 1;
    const uint32_t nch = (n + cs - 1) / cs;
    unsigned long long it = 0, cb = 0;
    if (lane == 0) {
        it = atomicAdd(uc + UC_BIG_ITEMS, 1ull);
        cb = atomicAdd(uc + UC_BIG_CHUNKS, (unsigned long long)nch);
    }
    it = __shfl(it, 0, 64);
    cb = __shfl(cb, 0, 64);
    const bool ok = it < bc.imax && cb + nch <= bc.cmax;
    for (uint64_t g = cb + lane; g < cb + nch && g < bc.cmax; g += 64) bc.chunk_item[g] = ok ? (uint32_t)it : BIG_NONE;
    if (!ok && it < bc.imax && lane == 0) bc.items[it].kind = 0;  // a slot k_big_holes must skip
    item = (uint32_t)it;
    cbase = (uint32_t)cb;
    csize = cs;
    return ok;
}

// Arguments of the mutation shared by the per-vertex code.
struct MutArgs {
    const uint32_t *tv, *ts, *tdl, *te, *ncnt;
    const uint64_t *xoff;
    const uint32_t *xs;
    uint32_t *hdr, *pool;
    const uint32_t *sv, *id, *wv, *idest;
    const uint64_t* aoff;
    uint32_t* sur;
    uint32_t* sdirty;  // per touched vertex: 1 when S(u) must be rebuilt
    GroupRule rule;
};

template <bool SPLIT>
__device__ uint64_t mutate_one(uint64_t t, const MutArgs& A, uint64_t abase0, const XView& xv, const BigCtx& bc,
                               unsigned long long* uc, uint32_t split);

// The large-vertex instance (SPLIT) runs one wave per block with the deleted
// set's samples in dynamic LDS; the other runs WB-thread blocks, one vertex per
// wave at a time.
constexpr uint32_t XL_WORDS = 8192;  // LDS samples per large vertex (32 KiB)
constexpr int MUT_WAVES = 5;  // waves per SIMD the small-vertex instance is compiled for

template <bool SPLIT>
__device__ __forceinline__ void mutate_blocks(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err,
                                              const MutArgs& A, unsigned long long* __restrict__ partials,
                                              const uint32_t* __restrict__ dold, const uint32_t* __restrict__ blist,
                                              const BigCtx& bc, uint32_t split, unsigned long long* red,
                                              uint32_t* xl) {
    // a batch with bad input, a candidate overflow or no pool space changes nothing
    const bool skip = *err != 0 || uc[UC_FLAGS] != 0;
    const uint64_t T = skip ? 0 : uc[UC_T];
    const uint64_t abase0 = uc[UC_BASE];
    const uint32_t lane = lane_id();
    uint64_t freed_total = 0;  // lane 0 of each wave
    if constexpr (!SPLIT) {
        for (uint64_t t = (uint64_t)blockIdx.x * (WB / 64) + (threadIdx.x >> 6); t < T;
             t += (uint64_t)gridDim.x * (WB / 64)) {
            // vertices with more than `split` entries after the inserts belong to the other instance
            // (the degree from before the batch: headers are rewritten as vertices finish)
            if (split && dold[t] + (A.tdl[t] - A.ts[t]) > split) continue;
            const uint32_t N = A.ncnt[t];
            const XView xv{A.xs + A.xoff[t], nullptr, N, 0u, 0u};
            freed_total += mutate_one<false>(t, A, abase0, xv, bc, uc, split);
        }
    } else {
        // one block (one wave) per listed large vertex
        const uint64_t nb = skip ? 0 : uc[UC_NBIG];
        for (uint64_t i = blockIdx.x; i < nb; i += gridDim.x) {
            const uint64_t t = blist[i];
            const uint32_t N = A.ncnt[t];
            const uint32_t* X = A.xs + A.xoff[t];
            uint32_t sh = 0;
            while ((N >> sh) >= XL_WORDS) ++sh;
            const uint32_t nl = (N + (1u << sh) - 1) >> sh;
            __syncthreads();  // the previous vertex is done with xl
            for (uint32_t j = lane; j < nl; j += 64) xl[j] = X[(uint64_t)j << sh];
            __syncthreads();
            const XView xv{X, xl, N, nl, sh};
            freed_total += mutate_one<true>(t, A, abase0, xv, bc, uc, split);
        }
    }
    if (lane == 0) red[threadIdx.x >> 6] = freed_total;
    __syncthreads();
    if (threadIdx.x < 32) {
        unsigned long long v = 0;
        if (threadIdx.x == 0)
            for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) v += red[w];
        partials[(uint64_t)blockIdx.x * 32 + threadIdx.x] = v;  // counter 0: garbage words
    }
}

// The vertices up to `split` entries: a wave's work on one vertex is a chain of dependent loads, so
// the kernel is held to a register budget that keeps five waves per SIMD resident (4 without it;
// 6 and 8 spill enough registers to be slower).
__global__ void __launch_bounds__(WB) __attribute__((amdgpu_waves_per_eu(MUT_WAVES, MUT_WAVES)))
k_mutate(unsigned long long* __restrict__ uc, const uint32_t* __restrict__ err, MutArgs A,
         unsigned long long* __restrict__ partials, const uint32_t* __restrict__ dold,
         const uint32_t* __restrict__ blist, BigCtx bc, uint32_t split) {
    __shared__ unsigned long long red[WB / 64];
    mutate_blocks<false>(uc, err, A, partials, dold, blist, bc, split, red, nullptr);
}

// The vertices with more than `split` entries, one wave per block.
__global__ void __launch_bounds__(WB) k_mutate_split(unsigned long long* __restrict__ uc,
                                                     const uint32_t* __restrict__ err, MutArgs A,
                                                     unsigned long long* __restrict__ partials,
                                                     const uint32_t* __restrict__ dold,
                                                     const uint32_t* __restrict__ blist, BigCtx bc, uint32_t split) {
    __shared__ unsigned long long red[WB / 64];
    extern __shared__ uint32_t xl[];
    mutate_blocks<true>(uc, err, A, partials, dold, blist, bc, split, red, xl);
}

// Final adjacency word i (< dn) of a vertex whose kept entries may not have been
// copied to the new block yet: kept entries that were not deleted still sit in
// the old block.
__device__ __forceinline__ uint64_t final_word_xv(uint32_t i, const uint64_t* __restrict__ enew,
                                                  const uint64_t* __restrict__ eold, bool reloc, uint32_t keep,
                                                  const XView& xv) {
    if (reloc && i < keep && !xv_in(xv, i)) return eold[i];
    return enew[i];
}

// One touched vertex; returns (in every lane) the pool words it freed.  The
// SPLIT instance handles the vertices with more than `split` entries and may
// hand its long passes to k_big_apply; the other one handles the rest.
template <bool SPLIT>
__device__ uint64_t mutate_one(uint64_t t, const MutArgs& A, uint64_t abase0, const XView& xv, const BigCtx& bc,
                               unsigned long long* uc, uint32_t split) {
    const uint32_t* __restrict__ wv = A.wv;
    const uint32_t* __restrict__ idest = A.idest;
    uint32_t* __restrict__ pool = A.pool;
    const uint32_t fb = A.rule.fbits;
    VState s;
    load_state(s, (uint32_t)t, A.tv, A.ts, A.tdl, A.te, A.ncnt, A.xoff, A.xs, A.hdr, pool, wv, A.rule);
    const uint32_t lane = lane_id();
    const uint32_t N = s.N;
    const uint32_t nholes = xv_lb(xv, s.dn);  // deleted entries below the new degree
    const uint32_t* W = wv + s.ts;            // insert weights
    const uint32_t* D = idest + s.ts;         // insert final indices (NF: deleted)
    uint64_t abase = abase0 + A.aoff[t];
    uint64_t freed = 0;

    // ---- adjacency
    uint64_t nadj = s.adj;
    uint32_t ncap = s.cap;
    if (s.dn > s.cap) {
        ncap = adj_cap_for(s.dn);
        nadj = abase;
        abase += adj_block_words(ncap);
        if (lane == 0) freed += adj_block_words(s.cap) * (s.cap > 0);  // freed is summed over the wave
    }
    uint64_t* eold = reinterpret_cast<uint64_t*>(pool + s.adj);
    const uint32_t* qold = pool + s.adj + 2ull * s.cap;
    uint64_t* enew = reinterpret_cast<uint64_t*>(pool + nadj);
    uint32_t* qnew = pool + nadj + 2ull * ncap;
    const uint32_t keep = s.d < s.dn ? s.d : s.dn;
    const bool reloc = nadj != s.adj;
    if (reloc) {
        uint32_t it, cb, cs;
        if (SPLIT && keep > split && big_reserve(bc, uc, keep, it, cb, cs)) {
            // the kept entries that are not deleted are copied by k_big_apply
            if (lane == 0) {
                BigItem& bi = bc.items[it];
                bi.kind = BK_COPY; bi.k = 0; bi.n = keep; bi.csize = cs; bi.cbase = cb; bi.u = s.u;
                bi.xoff = s.xoff; bi.N = N; bi.dn = s.dn; bi.nholes = nholes; bi.keep = keep; bi.reloc = 1;
                bi.sur = 0; bi.hole = 0; bi.ocap = s.cap; bi.ncap = ncap; bi.a = s.adj; bi.b = nadj; bi.aold = s.adj;
                bi.nh = 0; bi.iofs = 0; bi.hcnt = 0;
            }
        } else {
            for (uint32_t i = lane; i < keep; i += 64) { enew[i] = eold[i]; qnew[i] = qold[i]; }
        }
    }
    __threadfence_block();
    // inserts that stay where they were appended
    for (uint32_t q = s.d + lane; q < s.dn; q += 64) {
        const uint32_t a = q - s.d;
        if (D[a] != NF) {
            enew[q] = (uint64_t)A.id[A.sv[s.ts + a]] | ((uint64_t)W[a] << 32);
            qnew[q] = s.nseq + a;
        }
    }
    // tail survivors fill the holes in rank order
    const uint32_t sany = s.smo | s.smn;
    bool smoved = false;  // a moved entry belongs to a sparse group (S(u) changes)
    for (uint32_t q = s.dn + lane; q < s.d1; q += 64) {
        if (q < s.d) {
            const uint32_t dest = xv_rho(xv, q, s.dn, nholes);
            if (dest != NF) {
                const uint64_t e = eold[q];
                enew[dest] = e; qnew[dest] = qold[q];
                smoved |= (member_word((uint32_t)(e >> 32), fb) & sany) != 0u;
            }
        } else {
            const uint32_t a = q - s.d, dest = D[a];
            if (dest != NF) {
                enew[dest] = (uint64_t)A.id[A.sv[s.ts + a]] | ((uint64_t)W[a] << 32);
                qnew[dest] = s.nseq + a;
            }
        }
    }
    __threadfence_block();

    // ---- listed groups that keep their type
    uint32_t newinfo = 0, newlcap = s.lcap;
    const bool kl = lane < 32 && kept_listed(s);
    uint32_t km = (uint32_t)(__ballot(kl) & 0xFFFFFFFFull);
    // per-lane (k) new block for kept lists that move (the list or its index outgrows the
    // block), or fresh lists; lane 32: a new S(u) block
    const uint64_t lneed = lane <= 32 ? lane_list_need(s) : 0ull;
    const uint32_t nlc = lane < 32 && type_listed(s.tnew) ? new_lcap(s) : 0u;
    uint64_t lx = lneed;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(lx, o, 64);
        if (lane >= (uint32_t)o) lx += y;
    }
    const uint64_t my_block = abase + (lx - lneed);
    abase += __shfl(lx, 63, 64);
    uint32_t* S = A.sur + s.xoff;
    while (km) {
        const int k = __ffs(km) - 1;
        km &= km - 1;
        const uint32_t ck = __shfl(s.c, k, 64), cnk = __shfl(s.cn, k, 64), appk = __shfl(s.app, k, 64);
        const uint32_t lcapk = __shfl(s.lcap, k, 64);
        const uint64_t oblk = (uint64_t)__shfl(s.info, k, 64) * LIST_UNIT_WORDS;
        const uint64_t nblk = __shfl(lneed, k, 64) ? __shfl(my_block, k, 64) : oblk;
        // a regular group's inverted index follows its list in the block: entry i = position of i
        const uint32_t iofs = ((s.smn >> k) & 1u) ? 0u : __shfl(nlc, k, 64);
        const uint32_t lenv = ck + appk;
        const uint32_t* Lold = pool + oblk;
        uint32_t* Lnew = pool + nblk;
        // pass B: survivors of the tail window [cnk, lenv) in order -> S[]
        uint32_t nsur = 0;
        // old-list part of the window
        for (uint32_t p0 = cnk; p0 < ck; p0 += 64) {
            const uint32_t p = p0 + lane;
            const uint32_t r = p < ck ? xv_rho(xv, Lold[p], s.dn, nholes) : NF;
            const uint64_t b = __ballot(r != NF);
            if (r != NF) S[nsur + __popcll(b & lanemask_lt())] = r;
            nsur += __popcll(b);
        }
        // new-member part: inserts with bit k, position ck + rank
        uint32_t rank = 0;
        for (uint32_t a0 = 0; a0 < s.ni; a0 += 64) {
            const uint32_t a = a0 + lane;
            const bool v = a < s.ni && ((member_word(W[a], fb) >> k) & 1u);
            const uint64_t b = __ballot(v);
            if (b) {
                const uint32_t p = ck + rank + __popcll(b & lanemask_lt());
                const uint32_t r = v && p >= cnk ? D[a] : NF;
                const uint64_t sb = __ballot(r != NF);
                if (r != NF) S[nsur + __popcll(sb & lanemask_lt())] = r;
                nsur += __popcll(sb);
                rank += __popcll(b);
            }
        }
        __threadfence_block();
        // pass A: final entries [0, cnk): kept entries renamed, holes take S[] in rank order
        uint32_t nh = 0;
        const uint32_t oldpart = ck < cnk ? ck : cnk;
        uint32_t it, cb, cs;
        bool defer = false;
        if (SPLIT && oldpart > split) {
            // holes among the first cnk virtual positions = deleted members of the group less the
            // deleted entries of the tail window; those among the new members are counted here
            const uint32_t delk = __shfl(s.del, k, 64);
            uint32_t hnew = 0;
            if (cnk > ck) {
                uint32_t r2 = 0;
                for (uint32_t a0 = 0; a0 < s.ni && ck + r2 < cnk; a0 += 64) {
                    const uint32_t a = a0 + lane;
                    const bool v = a < s.ni && ((member_word(W[a], fb) >> k) & 1u);
                    const uint64_t b = __ballot(v);
                    const uint32_t p = ck + r2 + __popcll(b & lanemask_lt());
                    hnew += __popcll(__ballot(v && p < cnk && D[a] == NF));
                    r2 += __popcll(b);
                }
            }
            const uint32_t nha = (delk - (lenv - cnk - nsur)) - hnew;  // holes in [0, oldpart)
            // the tail survivors (and the hole slots) move to the split survivor buffer: S is reused
            // by the next group
            const bool listed = nha <= BIG_HOLES;
            const uint32_t words = nsur + (listed ? nha : 0u);
            unsigned long long soff = 0;
            if (lane == 0) soff = atomicAdd(uc + UC_BIG_SUR, (unsigned long long)words);
            soff = __shfl(soff, 0, 64);
            // A regular group whose block stays finds its holes and renamed entries through its
            // inverted index (Sec. 4.2): O(deleted + moved entries) instead of a pass over the list.
            const bool by_index = iofs != 0 && nblk == oblk && listed;
            if (by_index) {
                unsigned long long it64 = 0;
                if (lane == 0) it64 = atomicAdd(uc + UC_BIG_ITEMS, 1ull);
                it64 = __shfl(it64, 0, 64);
                defer = soff + words <= bc.smax && it64 < bc.imax;
                if (!defer && it64 < bc.imax && lane == 0) bc.items[it64].kind = 0;  // a slot k_big_holes skips
                if (defer) {
                    for (uint32_t i = lane; i < nsur; i += 64) bc.sur[soff + i] = S[i];
                    uint32_t* H = bc.sur + soff + nsur;
                    const uint32_t* Iold = Lold + iofs;
                    // holes: the positions below cnk of deleted old members (a deleted member in the
                    // tail window leaves no hole)
                    uint32_t nhf = 0;
                    for (uint32_t j0 = 0; j0 < N; j0 += 64) {
                        const uint32_t j = j0 + lane;
                        // membership by the index's own check (a member's entry is its position, the list
                        // holds it there): the adjacency slot of a deleted edge may already hold a survivor
                        const uint32_t x = j < N ? xv_at(xv, j) : NF;
                        const uint32_t pos = x < s.d ? Iold[x] : NF;
                        const bool hole = pos < ck && Lold[pos] == x && pos < cnk;
                        const uint64_t hb = __ballot(hole);
                        if (hole) H[nhf + __popcll(hb & lanemask_lt())] = pos;
                        nhf += __popcll(hb);
                    }
                    __threadfence_block();
                    // renames: the survivors the adjacency moved from its tail [dn, d) into its holes
                    for (uint32_t q = s.dn + lane; q < s.d; q += 64) {
                        const uint32_t dest = xv_rho(xv, q, s.dn, nholes);
                        if (dest != NF) {
                            const uint32_t pos = Iold[q];
                            if (pos < cnk && Lold[pos] == q) {
                                Lnew[pos] = dest;
                                Lnew[iofs + dest] = pos;
                            }
                        }
                    }
                    if (lane == 0) {
                        BigItem& bi = bc.items[it64];
                        bi.kind = BK_HOLES; bi.k = (uint32_t)k; bi.n = 0; bi.csize = 0; bi.cbase = 0; bi.u = s.u;
                        bi.xoff = s.xoff; bi.N = N; bi.dn = s.dn; bi.nholes = nholes; bi.keep = keep; bi.reloc = 0;
                        bi.sur = (uint32_t)soff; bi.hole = (uint32_t)(soff + nsur); bi.ocap = 0; bi.ncap = 0;
                        bi.a = oblk; bi.b = nblk; bi.aold = 0; bi.nh = nha; bi.iofs = iofs; bi.hcnt = nhf;
                    }
                    nh = nha;
                }
            } else {
            defer = soff + words <= bc.smax && big_reserve(bc, uc, oldpart, it, cb, cs);
            if (defer) {
                for (uint32_t i = lane; i < nsur; i += 64) bc.sur[soff + i] = S[i];
                if (lane == 0) {
                    BigItem& bi = bc.items[it];
                    bi.kind = listed ? BK_PASSH : BK_PASSA; bi.k = (uint32_t)k; bi.n = oldpart; bi.csize = cs;
                    bi.cbase = cb; bi.u = s.u; bi.xoff = s.xoff; bi.N = N; bi.dn = s.dn; bi.nholes = nholes;
                    bi.keep = keep; bi.reloc = nblk != oblk ? 1u : 0u; bi.sur = (uint32_t)soff;
                    bi.hole = (uint32_t)(soff + nsur); bi.ocap = 0; bi.ncap = 0; bi.a = oblk; bi.b = nblk;
                    bi.aold = 0; bi.nh = nha; bi.iofs = iofs; bi.hcnt = 0;
                }
                nh = nha;
            }
            }
        }
        if (!defer) {
            for (uint32_t p0 = 0; p0 < oldpart; p0 += 64) {
                const uint32_t p = p0 + lane;
                const bool v = p < oldpart;
                const uint32_t e = v ? Lold[p] : 0u;
                const uint32_t r = v ? xv_rho(xv, e, s.dn, nholes) : 0u;
                const bool hole = v && r == NF;
                const uint64_t hb = __ballot(hole);
                if (v) {
                    const uint32_t val = hole ? S[nh + __popcll(hb & lanemask_lt())] : r;
                    if (val != e || nblk != oblk) {
                        Lnew[p] = val;
                        if (iofs) Lnew[iofs + val] = p;
                    }
                }
                nh += __popcll(hb);
            }
        }
        if (cnk > ck) {
            // new members at positions [ck, cnk)
            uint32_t r2 = 0;
            for (uint32_t a0 = 0; a0 < s.ni && ck + r2 < cnk; a0 += 64) {
                const uint32_t a = a0 + lane;
                const bool v = a < s.ni && ((member_word(W[a], fb) >> k) & 1u);
                const uint64_t b = __ballot(v);
                const uint32_t p = ck + r2 + __popcll(b & lanemask_lt());
                const bool inpre = v && p < cnk;
                const uint32_t r = inpre ? D[a] : 0u;
                const bool hole = inpre && r == NF;
                const uint64_t hb = __ballot(hole);
                if (inpre) {
                    const uint32_t val = hole ? S[nh + __popcll(hb & lanemask_lt())] : r;
                    Lnew[p] = val;
                    if (iofs) Lnew[iofs + val] = p;
                }
                nh += __popcll(hb);
                r2 += __popcll(b);
            }
        }
        __threadfence_block();
        if (lane == (uint32_t)k) {
            newinfo = (uint32_t)(nblk / LIST_UNIT_WORDS);
            if (nblk != oblk) { newlcap = nlc; freed += old_block_words(s); }
        }
    }

    // ---- groups that become listed or switch between sparse and regular: fresh lists
    const bool fresh = lane < 32 && type_listed(s.tnew) && !kept_listed(s);
    if (fresh) { newinfo = (uint32_t)(my_block / LIST_UNIT_WORDS); newlcap = nlc; }
    if (lane < 32 && type_listed(s.told) && !kept_listed(s)) freed += old_block_words(s);
    // S(u): a new block (its old one is freed), or none when no group is sparse any more
    const uint64_t nsblk = __shfl(lneed, 32, 64) ? __shfl(my_block, 32, 64) : (uint64_t)s.sblk * LIST_UNIT_WORDS;
    if (lane == 32 && s.scap && s.scapn != s.scap) freed += s.scap;
    const uint32_t fm = (uint32_t)(__ballot(fresh) & 0xFFFFFFFFull);
    // one-element groups: the surviving member
    const bool one = lane < 32 && s.tnew == GT_ONE;
    uint32_t member = NF;
    if (one && s.told == GT_ONE) member = xv_rho(xv, s.info, s.dn, nholes);
    // members found among the inserts
    if (__ballot(one && member == NF)) {
        for (uint32_t a0 = 0; a0 < s.ni; a0 += 64) {
            const uint32_t a = a0 + lane;
            const uint32_t dest = a < s.ni ? D[a] : NF;
            const uint32_t w = dest != NF ? member_word(W[a], fb) : 0u;
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const uint64_t b = __ballot((w >> k) & 1u);
                if (b) {
                    const int src = __ffsll((long long)b) - 1;
                    const uint32_t cand = __shfl(dest, src, 64);
                    if (lane == (uint32_t)k && one && member == NF) member = cand;
                }
            }
        }
    }
    const uint32_t need_scan = (uint32_t)(__ballot(one && member == NF) & 0xFFFFFFFFull);
    uint32_t fm_seq = fm, ns_seq = need_scan;
    if (SPLIT && s.dn > split && (fm | need_scan)) {
        // fresh lists and one-element members of a large vertex: split work
        uint32_t mm = fm | need_scan;
        while (mm) {
            const int k = __ffs(mm) - 1;
            mm &= mm - 1;
            uint32_t it, cb, cs;
            const uint64_t blk = (uint64_t)__shfl(newinfo, k, 64) * LIST_UNIT_WORDS;
            // a fresh regular list's inverted index follows the list (read in every lane)
            const uint32_t iofs = ((fm >> k) & 1u) && ((s.smn >> k) & 1u) == 0u ? __shfl(nlc, k, 64) : 0u;
            if (big_reserve(bc, uc, s.dn, it, cb, cs)) {
                if (lane == 0) {
                    BigItem& bi = bc.items[it];
                    bi.kind = ((fm >> k) & 1u) ? BK_FRESH : BK_ONE; bi.k = (uint32_t)k; bi.n = s.dn; bi.csize = cs;
                    bi.cbase = cb; bi.u = s.u; bi.xoff = s.xoff; bi.N = N; bi.dn = s.dn; bi.nholes = nholes;
                    bi.keep = keep; bi.reloc = reloc ? 1u : 0u; bi.sur = 0; bi.hole = 0; bi.ocap = 0; bi.ncap = 0;
                    bi.a = nadj; bi.b = blk; bi.aold = s.adj; bi.nh = 0; bi.hcnt = 0;
                    bi.iofs = iofs;
                }
                fm_seq &= ~(1u << k);
                ns_seq &= ~(1u << k);
            }
        }
    }
    if (fm_seq | ns_seq) {
        // one pass over the final adjacency
        uint32_t fill = 0;
        for (uint32_t i0 = 0; i0 < s.dn; i0 += 64) {
            const uint32_t i = i0 + lane;
            uint32_t w = 0;
            if (i < s.dn)
                w = member_word((uint32_t)((SPLIT ? final_word_xv(i, enew, eold, reloc, keep, xv) : enew[i]) >> 32), fb);
            uint32_t mm = fm_seq | ns_seq;
            while (mm) {
                const int k = __ffs(mm) - 1;
                mm &= mm - 1;
                const bool bit = (w >> k) & 1u;
                const uint64_t b = __ballot(bit);
                if ((fm_seq >> k) & 1u) {
                    const uint64_t blk = (uint64_t)__shfl(newinfo, k, 64) * LIST_UNIT_WORDS;
                    const uint32_t f = __shfl(fill, k, 64);
                    const uint32_t iofs = ((s.smn >> k) & 1u) ? 0u : __shfl(nlc, k, 64);
                    if (bit) {
                        const uint32_t pos = f + __popcll(b & lanemask_lt());
                        pool[blk + pos] = i;
                        if (iofs) pool[blk + iofs + i] = pos;  // a regular group's inverted index
                    }
                    if (lane == (uint32_t)k) fill += __popcll(b);
                } else if (b) {
                    const uint32_t first = i0 + (__ffsll((long long)b) - 1);
                    if (lane == (uint32_t)k && member == NF) member = first;
                }
            }
        }
    }

    // ---- header: the inter-group sampling space of the vertex
    uint32_t* h = A.hdr + (size_t)s.u * HDR_WORDS;
    const bool ne = lane < 32 && s.cn > 0;
    const uint64_t wsum = fb ? s.W : wave_sum(ne ? ((uint64_t)s.cn << lane) : 0ull);
    const uint32_t nmask = (uint32_t)(__ballot(ne) & 0xFFFFFFFFull);
    // one-element groups keep their member's destination in the count slot (a member
    // left to k_big_pass gets it from k_big_one_dst)
    const bool onek = lane < 32 && s.tnew == GT_ONE;
    uint32_t slot = s.cn;
    if (onek && member != NF)
        slot = (uint32_t)(SPLIT ? final_word_xv(member, enew, eold, reloc, keep, xv) : enew[member]);
    const uint32_t onemask = (uint32_t)(__ballot(onek) & 0xFFFFFFFFull);
    const uint32_t nhi = mask_hi(nmask);
    if (lane < 32) {
        if (lane <= nhi) h[H_CNT + (nhi - lane)] = slot;
        uint32_t inf = 0;
        if (type_listed(s.tnew)) inf = newinfo;
        else if (s.tnew == GT_ONE) inf = member;
        h[H_INFO + lane] = inf;
    }
    const uint32_t lg = (lane < 32 && type_listed(s.tnew)) ? (31 - __clz(newlcap)) : 0u;
    uint32_t packed = lg << (8 * (lane & 3));
    packed |= __shfl_xor(packed, 1);
    packed |= __shfl_xor(packed, 2);
    if (lane < 32 && (lane & 3) == 0) h[H_LCAPLOG + (lane >> 2)] = packed;
    freed = wave_sum(freed);
    if (lane == 0) {
        h[H_MASK] = nmask;
        h[H_ONEMASK] = onemask;
        h[H_DEG] = s.dn;
        h[H_WLO] = (uint32_t)wsum;
        h[H_WHI] = (uint32_t)(wsum >> 32);
        h[H_ADJLO] = (uint32_t)nadj;
        h[H_ADJHI] = adjhi_word(nadj, nhi);
        h[H_ACAP] = ncap;
        h[H_NSEQ] = s.nseq + s.ni;
        h[H_SCAP] = s.scapn;
        h[H_SBLK] = (uint32_t)(nsblk / LIST_UNIT_WORDS);
        if (!s.smn) h[H_SLEN] = 0;
    }
    // S(u) and the sparse groups' indexes over it are rebuilt after the mutation
    // (k_srebuild) when the vertex has a sparse group and S(u) or a sparse list may
    // have changed: the sparse mask or the S(u) block changed, a sparse list moved or
    // is fresh, or an inserted, deleted or moved entry belongs to a sparse group
    const bool touched_sparse = lane < 32 && ((sany >> lane) & 1u) && (s.app | s.del) != 0u;
    const bool sparse_block = lane < 32 && s.tnew == GT_SPARSE && lneed != 0;
    const bool dirty = s.smn != 0u && (s.smn != s.smo || s.scapn != s.scap ||
                                       __ballot(touched_sparse || sparse_block || smoved) != 0ull);
    if (lane == 0) A.sdirty[t] = dirty ? 1u : 0u;
    return freed;
}

// Split work: the deleted set of an item's vertex, with up to BIG_XL samples in LDS.
constexpr uint32_t BIG_XL = 1024;

__device__ __forceinline__ XView big_stage_x(const BigItem& bi, const uint32_t* __restrict__ xs, uint32_t* xl) {
    const uint32_t* X = xs + bi.xoff;
    uint32_t sh = 0;
    while ((bi.N >> sh) >= BIG_XL) ++sh;
    const uint32_t nl = (bi.N + (1u << sh) - 1) >> sh;
    for (uint32_t j = threadIdx.x; j < nl; j += blockDim.x) xl[j] = X[(uint64_t)j << sh];
    return XView{X, xl, bi.N, nl, sh};
}

// Entry p of an item in two steps, so a tile's loads are all in flight before
// the searches: big_load reads the raw words (pass A: the list entry in w0;
// fresh / one-element: the new adjacency word in w0 and, for a kept entry of a
// relocated adjacency, the old one in w1); big_eval gives the predicate: a hole
// of a pass-A list (other entries get their new index in *r), or bit k of the
// final adjacency word p.
__device__ __forceinline__ void big_load(const BigItem& bi, uint32_t p, const uint32_t* __restrict__ pool,
                                         uint64_t& w0, uint64_t& w1) {
    w1 = 0;
    if (bi.kind == BK_PASSA) { w0 = pool[bi.a + p]; return; }
    w0 = reinterpret_cast<const uint64_t*>(pool + bi.a)[p];
    if (bi.reloc && p < bi.keep) w1 = reinterpret_cast<const uint64_t*>(pool + bi.aold)[p];
}
__device__ __forceinline__ bool big_eval(const BigItem& bi, uint32_t p, uint64_t w0, uint64_t w1, const XView& xv,
                                         uint32_t* r, uint32_t fbits) {
    if (bi.kind == BK_PASSA) {
        *r = xv_rho(xv, (uint32_t)w0, bi.dn, bi.nholes);
        return *r == NF;
    }
    const uint64_t w = (bi.reloc && p < bi.keep && !xv_in(xv, p)) ? w1 : w0;
    return (member_word((uint32_t)(w >> 32), fbits) >> bi.k) & 1u;
}

constexpr uint32_t BIG_TPT = 8;  // entries per thread per tile (tiles of 2048 entries)

// Split work, pass 1: per chunk, the number of entries the chunk contributes
// (holes of a pass-A list, members of a fresh list; 0 for the other kinds).
// One block per chunk, grid-stride over the reserved chunks.
__global__ void __launch_bounds__(256) k_big_count(const unsigned long long* __restrict__ uc, BigCtx bc,
                                                   const uint32_t* __restrict__ xs, const uint32_t* __restrict__ pool,
                                                   uint32_t* __restrict__ ccnt) {
    __shared__ BigItem bi;
    __shared__ uint32_t red[4];
    __shared__ uint32_t xl[BIG_XL];
    const uint64_t used = std::min<uint64_t>(uc[UC_BIG_CHUNKS], bc.cmax);
    for (uint64_t g = blockIdx.x; g < used; g += gridDim.x) {
        const uint32_t it = bc.chunk_item[g];
        if (it == BIG_NONE) continue;
        __syncthreads();
        if (threadIdx.x == 0) bi = bc.items[it];
        __syncthreads();
        if (bi.kind != BK_PASSA && bi.kind != BK_FRESH) continue;
        const XView xv = big_stage_x(bi, xs, xl);
        __syncthreads();
        uint32_t c = 0;
        const uint32_t p0 = (uint32_t)(g - bi.cbase) * bi.csize;
        const uint32_t p1 = std::min(p0 + bi.csize, bi.n);
        for (uint32_t q0 = p0; q0 < p1; q0 += 256 * BIG_TPT) {
            uint64_t w0[BIG_TPT], w1[BIG_TPT];
#pragma unroll
            for (uint32_t j = 0; j < BIG_TPT; ++j) {
                const uint32_t p = q0 + j * 256 + threadIdx.x;
                w0[j] = w1[j] = 0;
                if (p < p1) big_load(bi, p, pool, w0[j], w1[j]);
            }
#pragma unroll
            for (uint32_t j = 0; j < BIG_TPT; ++j) {
                const uint32_t p = q0 + j * 256 + threadIdx.x;
                uint32_t r;
                if (p < p1 && big_eval(bi, p, w0[j], w1[j], xv, &r, bc.fbits)) ++c;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        if (lane_id() == 0) red[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) ccnt[g] = red[0] + red[1] + red[2] + red[3];
    }
}

// Split work, pass 2 of the ordered kinds.  An item's chunk g starts at rank
// ccnt[cbase] + ... + ccnt[g - 1] among the item's holes/members (an item has at
// most 16 chunks); the chunk is walked in tiles of 2048 consecutive entries
// (entry q0 + 256 j + thread), ranked by ballots.
//   BK_PASSA: a = old list, b = new list: hole -> next tail survivor
//             (bc.sur[sur + rank]), other entries renamed; written when changed
//             or when the list moved.
//   BK_FRESH: a = new adjacency, aold = old one, b = the list: ascending
//             indices of the final entries with bit k.
__global__ void __launch_bounds__(256) k_big_apply(const unsigned long long* __restrict__ uc, BigCtx bc,
                                                   const uint32_t* __restrict__ xs, uint32_t* __restrict__ pool,
                                                   const uint32_t* __restrict__ ccnt) {
    __shared__ BigItem bi;
    __shared__ uint32_t wsum[BIG_TPT][4], cbefore;
    __shared__ uint32_t xl[BIG_XL];
    const uint64_t used = std::min<uint64_t>(uc[UC_BIG_CHUNKS], bc.cmax);
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint64_t g = blockIdx.x; g < used; g += gridDim.x) {
        const uint32_t it = bc.chunk_item[g];
        if (it == BIG_NONE) continue;
        __syncthreads();
        if (threadIdx.x == 0) bi = bc.items[it];
        __syncthreads();
        if (bi.kind != BK_PASSA && bi.kind != BK_FRESH) continue;
        const XView xv = big_stage_x(bi, xs, xl);
        if (wave == 0) {
            uint32_t c = (uint64_t)bi.cbase + lane < g ? ccnt[bi.cbase + lane] : 0u;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
            if (lane == 0) cbefore = c;
        }
        __syncthreads();
        const uint32_t p0 = (uint32_t)(g - bi.cbase) * bi.csize;
        const uint32_t p1 = std::min(p0 + bi.csize, bi.n);
        // BK_PASSA / BK_FRESH: ordered output
        uint32_t base = cbefore;
        uint32_t* L = pool + bi.b;
        const uint32_t* S = bc.sur + bi.sur;
        for (uint32_t q0 = p0; q0 < p1; q0 += 256 * BIG_TPT) {
            uint64_t w0[BIG_TPT], w1[BIG_TPT];
#pragma unroll
            for (uint32_t j = 0; j < BIG_TPT; ++j) {
                const uint32_t p = q0 + j * 256 + threadIdx.x;
                w0[j] = w1[j] = 0;
                if (p < p1) big_load(bi, p, pool, w0[j], w1[j]);
            }
            uint32_t r[BIG_TPT];
            uint64_t b[BIG_TPT];
#pragma unroll
            for (uint32_t j = 0; j < BIG_TPT; ++j) {
                const uint32_t p = q0 + j * 256 + threadIdx.x;
                r[j] = 0;
                const bool pr = p < p1 && big_eval(bi, p, w0[j], w1[j], xv, &r[j], bc.fbits);
                b[j] = __ballot(pr);
                if (lane == 0) wsum[j][wave] = (uint32_t)__popcll(b[j]);
            }
            __syncthreads();
#pragma unroll
            for (uint32_t j = 0; j < BIG_TPT; ++j) {
                const uint32_t p = q0 + j * 256 + threadIdx.x;
                uint32_t rk = base + (uint32_t)__popcll(b[j] & lanemask_lt());
                for (uint32_t w = 0; w < wave; ++w) rk += wsum[j][w];
                base += wsum[j][0] + wsum[j][1] + wsum[j][2] + wsum[j][3];
                const bool pr = (b[j] >> lane) & 1ull;
                if (bi.kind == BK_FRESH) {
                    if (pr) {
                        L[rk] = p;
                        if (bi.iofs) L[bi.iofs + p] = rk;
                    }
                } else if (p < p1) {
                    const uint32_t e = (uint32_t)w0[j];
                    const uint32_t val = pr ? S[rk] : r[j];
                    if (val != e || bi.reloc) {
                        L[p] = val;
                        if (bi.iofs) L[bi.iofs + val] = p;
                    }
                }
            }
            __syncthreads();  // wsum is rewritten by the next tile
        }
    }
}

// Split work, the unordered kinds, one wave per chunk (the deleted set's samples
// in a per-wave LDS slice):
//   BK_COPY : a = old adjacency, b = new adjacency (capacities ocap, ncap):
//             kept entries [0, keep) not deleted are copied with their seq.
//   BK_ONE  : the first final entry with bit k becomes the group's member
//             (header info, set to NF by k_mutate, lowered by atomicMin).
//   BK_PASSH: a = old list, b = new list: other entries renamed (written when
//             changed or when the list moved); hole positions appended to
//             sur[hole ..] for k_big_holes.
constexpr uint32_t BIG_WXL = 1024;  // LDS samples per wave

__global__ void __launch_bounds__(256) k_big_pass(const unsigned long long* __restrict__ uc, BigCtx bc,
                                                  const uint32_t* __restrict__ xs, uint32_t* __restrict__ pool,
                                                  uint32_t* __restrict__ hdr) {
    __shared__ uint32_t xlw[4][BIG_WXL];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t* xl = xlw[wave];
    const uint64_t used = std::min<uint64_t>(uc[UC_BIG_CHUNKS], bc.cmax);
    for (uint64_t g = (uint64_t)blockIdx.x * 4 + wave; g < used; g += (uint64_t)gridDim.x * 4) {
        const uint32_t it = __builtin_amdgcn_readfirstlane(bc.chunk_item[g]);
        if (it == BIG_NONE) continue;
        const BigItem& bi = bc.items[it];
        const uint32_t kind = bi.kind;
        if (kind != BK_COPY && kind != BK_ONE && kind != BK_PASSH) continue;
        // the deleted set: every 2^sh-th entry in this wave's LDS slice
        const uint32_t* X = xs + bi.xoff;
        const uint32_t N = bi.N;
        uint32_t sh = 0;
        while ((N >> sh) >= BIG_WXL) ++sh;
        const uint32_t nl = (N + (1u << sh) - 1) >> sh;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t j = lane; j < nl; j += 64) xl[j] = X[(uint64_t)j << sh];
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        const XView xv{X, xl, N, nl, sh};
        const uint32_t p0 = (uint32_t)(g - bi.cbase) * bi.csize;
        const uint32_t p1 = std::min(p0 + bi.csize, bi.n);
        if (kind == BK_COPY) {
            const uint64_t* eo = reinterpret_cast<const uint64_t*>(pool + bi.a);
            const uint32_t* qo = pool + bi.a + 2ull * bi.ocap;
            uint64_t* en = reinterpret_cast<uint64_t*>(pool + bi.b);
            uint32_t* qn = pool + bi.b + 2ull * bi.ncap;
            for (uint32_t q0 = p0; q0 < p1; q0 += 64 * 4) {
                uint64_t e[4];
                uint32_t q[4];
#pragma unroll
                for (uint32_t j = 0; j < 4; ++j) {
                    const uint32_t p = q0 + j * 64 + lane;
                    if (p < p1) { e[j] = eo[p]; q[j] = qo[p]; }
                }
#pragma unroll
                for (uint32_t j = 0; j < 4; ++j) {
                    const uint32_t p = q0 + j * 64 + lane;
                    if (p < p1 && !xv_in(xv, p)) { en[p] = e[j]; qn[p] = q[j]; }
                }
            }
        } else if (kind == BK_ONE) {
            uint32_t first = NF;
            for (uint32_t q0 = p0; q0 < p1; q0 += 64) {
                const uint32_t p = q0 + lane;
                bool hit = false;
                if (p < p1) {
                    uint64_t w0, w1;
                    uint32_t r;
                    big_load(bi, p, pool, w0, w1);
                    hit = big_eval(bi, p, w0, w1, xv, &r, bc.fbits);
                }
                const uint64_t b = __ballot(hit);
                if (b) { first = q0 + (uint32_t)(__ffsll((long long)b) - 1); break; }
            }
            if (lane == 0 && first != NF) atomicMin(hdr + (size_t)bi.u * HDR_WORDS + H_INFO + bi.k, first);
        } else {
            const uint32_t* Lold = pool + bi.a;
            uint32_t* Lnew = pool + bi.b;
            uint32_t* H = bc.sur + bi.hole;
            unsigned long long* hc = &bc.items[it].hcnt;
            const uint32_t dn = bi.dn, nholes = bi.nholes, nh = bi.nh;
            const bool moved = bi.reloc != 0;
            for (uint32_t q0 = p0; q0 < p1; q0 += 64 * BIG_TPT) {
                uint32_t e[BIG_TPT];
#pragma unroll
                for (uint32_t j = 0; j < BIG_TPT; ++j) {
                    const uint32_t p = q0 + j * 64 + lane;
                    e[j] = p < p1 ? Lold[p] : 0u;
                }
#pragma unroll
                for (uint32_t j = 0; j < BIG_TPT; ++j) {
                    const uint32_t p = q0 + j * 64 + lane;
                    const uint32_t r = p < p1 ? xv_rho(xv, e[j], dn, nholes) : 0u;
                    const bool hole = p < p1 && r == NF;
                    const uint64_t hb = __ballot(hole);
                    if (hb) {
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(hc, (unsigned long long)__popcll(hb));
                        base = __shfl(base, 0, 64);
                        const uint64_t slot = base + __popcll(hb & lanemask_lt());
                        if (hole && slot < nh) H[slot] = p;
                    }
                    if (p < p1 && !hole && (r != e[j] || moved)) {
                        Lnew[p] = r;
                        if (bi.iofs) Lnew[bi.iofs + r] = p;
                    }
                }
            }
        }
    }
}

// Split work, the holes of BK_PASSH lists (collected by k_big_pass) and of BK_HOLES
// lists (found by k_mutate through the inverted index): one block per item sorts the hole
// positions (at most BIG_HOLES) in LDS; the i-th hole takes tail survivor i.
__global__ void __launch_bounds__(256) k_big_holes(const unsigned long long* __restrict__ uc, BigCtx bc,
                                                   uint32_t* __restrict__ pool) {
    __shared__ uint32_t hs[BIG_HOLES];
    const uint64_t nitems = std::min<uint64_t>(uc[UC_BIG_ITEMS], bc.imax);
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BigItem& bi = bc.items[it];
        if (bi.kind != BK_PASSH && bi.kind != BK_HOLES) continue;
        const uint32_t nh = (uint32_t)std::min<unsigned long long>(bi.nh, bi.hcnt);
        if (nh == 0) continue;
        uint32_t P = 1;
        while (P < nh) P <<= 1;
        const uint32_t* H = bc.sur + bi.hole;
        const uint32_t* S = bc.sur + bi.sur;
        uint32_t* L = pool + bi.b;
        __syncthreads();  // the previous item is done with hs
        for (uint32_t i = threadIdx.x; i < P; i += 256) hs[i] = i < nh ? H[i] : 0xFFFFFFFFu;
        __syncthreads();
        // bitonic sort, ascending
        for (uint32_t k2 = 2; k2 <= P; k2 <<= 1) {
            for (uint32_t j = k2 >> 1; j > 0; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += 256) {
                    const uint32_t ixj = i ^ j;
                    if (ixj > i) {
                        const uint32_t a = hs[i], b = hs[ixj];
                        if ((a > b) == ((i & k2) == 0)) { hs[i] = b; hs[ixj] = a; }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < nh; i += 256) {
            L[hs[i]] = S[i];
            if (bi.iofs) L[bi.iofs + S[i]] = hs[i];
        }
    }
}

// Split work, last step: a one-element member found by k_big_pass puts its
// destination in the group's count slot (the adjacency copies are complete).
__global__ void __launch_bounds__(256) k_big_one_dst(const unsigned long long* __restrict__ uc, BigCtx bc,
                                                     const uint32_t* __restrict__ pool, uint32_t* __restrict__ hdr) {
    const uint64_t nitems = std::min<uint64_t>(uc[UC_BIG_ITEMS], bc.imax);
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < nitems;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const BigItem& bi = bc.items[it];
        if (bi.kind != BK_ONE) continue;
        uint32_t* h = hdr + (size_t)bi.u * HDR_WORDS;
        const uint32_t member = h[H_INFO + bi.k];
        if (member < bi.n) h[H_CNT + (mask_hi(h[H_MASK]) - bi.k)] = pool[bi.a + 2ull * member];
    }
}

__global__ void k_add_u64(unsigned long long* dst, const unsigned long long* src) { *dst += *src; }

// Reserve the batch's pool words with one bump, unless the batch is already
// rejected (bad input or candidate overflow); no space sets ERR_OOM.
__global__ void k_alloc_check(unsigned long long* __restrict__ ctl, uint64_t pool_words,
                              unsigned long long* __restrict__ uc, uint32_t* __restrict__ err) {
    if (*err || uc[UC_FLAGS]) return;
    const unsigned long long used = ctl[0], total = uc[UC_ALLOC];
    if (used + total > pool_words) {
        atomicOr(err, ERR_OOM);
    } else {
        uc[UC_BASE] = used;
        ctl[0] = used + total;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Plans: one workspace (and captured graph) per power-of-two batch-size bucket.
// ---------------------------------------------------------------------------
struct UpdPlan {
    uint64_t rmax = 0, cmax = 0;
    char* ws = nullptr;
    size_t bytes = 0;
    uint32_t *is = nullptr, *id = nullptr, *iw = nullptr, *ds = nullptr, *dd = nullptr;  // staged inputs
    unsigned long long* uc = nullptr;
    uint64_t *keys, *sk, *hx, *fsz, *foff, *ckey, *cks, *xk, *xks, *needw, *aoff, *xoff;
    uint32_t *vals, *sv, *head, *rec_t, *tv, *tsa, *tdl, *te, *cval, *cvs, *first, *matched, *xs, *sur, *ncnt, *dold, *wv, *idest, *blist;
    uint32_t *vacap, *vnseq;  // header fields of the touched vertices before the batch (k_flat_size)
    uint32_t* sdirty;         // per touched vertex: S(u) to rebuild after the mutation
    uint32_t* srwork;         // scratch of the S(u) rebuild
    uint64_t* vadj;
    unsigned long long* parts;
    BigItem* big_items;
    uint32_t *chunk_item, *ccnt, *bsur;
    void* tmp;
    uint32_t split = 0;  // the split threshold the captured graph was made with
    LocView lv{nullptr, 0};  // the edge locator the captured graph was made with
    uint32_t grid_an = PART_BLOCKS, grid_mu = PART_BLOCKS;  // resident blocks of k_analyze, k_mutate
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
};

struct UpdPlans {
    std::vector<UpdPlan*> plans;
    hipStream_t cap_stream = nullptr;  // private stream for captures (never the legacy default stream)
};

static constexpr uint32_t MATCH_GRID = 2048;
static constexpr uint32_t BIG_IMAX = 65536;
static constexpr uint32_t BIG_CMAX = 1u << 19;
// survivor words for deferred pass-A lists: a hub's group windows hold about
// popcount(weight) entries per deleted edge, so the buffer scales with the bucket
static uint64_t big_smax(uint64_t R) { return std::min<uint64_t>(std::max<uint64_t>(1ull << 22, 4 * R), 1ull << 31); }
static constexpr uint32_t BIG_GRID = 2048;
static constexpr size_t PLAN_CACHE_BYTES = 16ull << 30;

static void plan_free(UpdPlan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    hipFree(p->ws);
    delete p;
}

// Blocks of `kernel` resident at once on the current device (occupancy times
// compute units), at most PART_BLOCKS.  The per-vertex kernels loop over their
// vertices with a grid stride, so every block gets the same share of
// latency-bound iterations; blocks beyond the resident count would only start
// when the first ones end and then run a whole second share.
static uint32_t resident_grid(const void* kernel, int block) {
    int dev = 0, cus = 0, per = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || per <= 0) per = 4;
    return (uint32_t)std::min<uint64_t>((uint64_t)cus * per, PART_BLOCKS);
}

static UpdPlan* plan_make(uint64_t rmax, uint64_t cmax) {
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t R = rmax, C = cmax;
    const size_t tmpb = std::max(std::max(sort_temp_bytes(R, true), sort_temp_bytes(C, true)),
                                 scan_temp_bytes(R + 1));
    const size_t bytes = al(R * 4) * 5 + al(UC_WORDS * 8) + al(R * 8) * 11 + al(C * 8) * 2 + al(R * 4) * 19 +
                         al(R * 8) + al(C * 4) * 2 + al(PART_BLOCKS * 32 * 8) + al(BIG_IMAX * sizeof(BigItem)) +
                         2 * al(BIG_CMAX * 4) + al(big_smax(R) * 4) + al(SPARSE_WORK_WORDS(R) * 4) + tmpb + 4096;
    UpdPlan* p = new UpdPlan();
    p->rmax = R;
    p->cmax = C;
    p->grid_an = resident_grid((const void*)k_analyze, WB);
    p->grid_mu = resident_grid((const void*)k_mutate, WB);
    if (hipMalloc(&p->ws, bytes) != hipSuccess) { delete p; return nullptr; }
    p->bytes = bytes;
    char* w = p->ws;
    auto take = [&](uint64_t b) { char* r = w; w += al(b); return r; };
    p->is = (uint32_t*)take(R * 4); p->id = (uint32_t*)take(R * 4); p->iw = (uint32_t*)take(R * 4);
    p->ds = (uint32_t*)take(R * 4); p->dd = (uint32_t*)take(R * 4);
    p->uc = (unsigned long long*)take(UC_WORDS * 8);
    p->keys = (uint64_t*)take(R * 8); p->sk = (uint64_t*)take(R * 8); p->hx = (uint64_t*)take(R * 8);
    p->fsz = (uint64_t*)take(R * 8); p->foff = (uint64_t*)take(R * 8); p->xk = (uint64_t*)take(R * 8);
    p->xks = (uint64_t*)take(R * 8); p->needw = (uint64_t*)take(R * 8); p->aoff = (uint64_t*)take(R * 8);
    p->xoff = (uint64_t*)take(R * 8);
    p->ckey = (uint64_t*)take(C * 8); p->cks = (uint64_t*)take(C * 8);
    p->vals = (uint32_t*)take(R * 4); p->sv = (uint32_t*)take(R * 4); p->head = (uint32_t*)take(R * 4);
    p->rec_t = (uint32_t*)take(R * 4); p->tv = (uint32_t*)take(R * 4); p->tsa = (uint32_t*)take(R * 4);
    p->tdl = (uint32_t*)take(R * 4); p->te = (uint32_t*)take(R * 4); p->first = (uint32_t*)take(R * 4);
    p->matched = (uint32_t*)take(R * 4); p->xs = (uint32_t*)take(R * 4); p->ncnt = (uint32_t*)take(R * 4);
    p->dold = (uint32_t*)take(R * 4);
    p->wv = (uint32_t*)take(R * 4);
    p->idest = (uint32_t*)take(R * 4);
    p->blist = (uint32_t*)take(R * 4);
    p->vacap = (uint32_t*)take(R * 4);
    p->vnseq = (uint32_t*)take(R * 4);
    p->sdirty = (uint32_t*)take(R * 4);
    p->srwork = (uint32_t*)take(SPARSE_WORK_WORDS(R) * 4);
    p->vadj = (uint64_t*)take(R * 8);
    p->sur = (uint32_t*)take(R * 8);
    p->cval = (uint32_t*)take(C * 4); p->cvs = (uint32_t*)take(C * 4);
    p->parts = (unsigned long long*)take(PART_BLOCKS * 32 * 8);
    p->big_items = (BigItem*)take(BIG_IMAX * sizeof(BigItem));
    p->chunk_item = (uint32_t*)take(BIG_CMAX * 4);
    p->ccnt = (uint32_t*)take(BIG_CMAX * 4);
    p->bsur = (uint32_t*)take(big_smax(R) * 4);
    p->tmp = w;
    return p;
}

static uint64_t pow2_at_least(uint64_t x, uint64_t lo) {
    uint64_t c = lo;
    while (c < x) c <<= 1;
    return c;
}

// The whole pipeline for one batch, sizes from the control block; no host round trips.
// With p->lv.tab set, deletes are located through the edge locator, which the
// pipeline then keeps in step.
static void enqueue_update(bingo_graph* g, UpdPlan* p, hipStream_t st) {
    const uint64_t R = p->rmax, C = p->cmax;
    const LocView lv = p->lv;
    const uint32_t ins_only = lv.tab ? 1u : 0u;
    const int vb = std::max(1, bits_for((uint64_t)g->n - 1));
    const int cbits = bits_for(R) + 32;  // candidate key: run (< R) << 32 | seq
    const uint64_t xpad = cbits >= 64 ? ~0ull : (1ull << cbits) - 1;
    const uint32_t vgrid_a = (uint32_t)std::min<uint64_t>((R + 3) / 4, p->grid_an);
    const uint32_t vgrid_m = (uint32_t)std::min<uint64_t>((R + 3) / 4, p->grid_mu);
    unsigned long long* uc = p->uc;
    uint32_t* err = g->d_err;
    hipLaunchKernelGGL(k_upd_validate, dim3(grid_for(R)), dim3(TB), 0, st, g->n, (const unsigned long long*)uc, p->is,
                       p->id, p->iw, p->ds, p->dd, err);
    hipLaunchKernelGGL(k_upd_gate, dim3(1), dim3(1), 0, st, uc, (const uint32_t*)err);
    // 1. records sorted by (src, op, dst); segments per touched vertex
    hipLaunchKernelGGL(k_upd_keys, dim3(grid_for(R)), dim3(TB), 0, st, (const unsigned long long*)uc, R, p->is, p->ds,
                       p->dd, vb, ~0ull, p->keys, p->vals);
    sort_pairs_u64_dn(p->keys, p->vals, p->sk, p->sv, R, uc + UC_R, 2 * vb + 1, p->tmp, st);
    hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(R)), dim3(TB), 0, st, p->sk, (const unsigned long long*)uc, R, vb,
                       p->head);
    scan_u32_to_u64(p->head, p->hx, R, p->tmp, uc + UC_T, st);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(R)), dim3(TB), 0, st, p->tdl, R, NF);
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(R)), dim3(TB), 0, st, p->sk, (const unsigned long long*)uc, vb,
                       p->head, p->hx, p->tv, p->tsa, p->tdl, p->rec_t);
    hipLaunchKernelGGL(k_seg_end, dim3(grid_for(R)), dim3(TB), 0, st, (const unsigned long long*)uc, p->tsa, p->te,
                       p->tdl);
    hipLaunchKernelGGL(k_flat_size, dim3(grid_for(R)), dim3(TB), 0, st, uc, R, p->tv,
                       p->tsa, p->tdl, p->te, g->hdr, p->fsz, p->dold, p->vacap, p->vnseq, p->vadj, g->update_split,
                       p->blist, ins_only);
    scan_u64(p->fsz, p->foff, R, p->tmp, uc + UC_F, st);
    // 2. delete matching: candidates, sorted by (run, seq); the k oldest per run
    hipLaunchKernelGGL(k_match, dim3(MATCH_GRID), dim3(TB), 0, st, uc, p->foff, p->tsa, p->tdl, p->te, p->dold,
                       p->vacap, p->vnseq, p->vadj, p->sk, p->sv, vb, p->id, g->pool, p->ckey, p->cval, C, ins_only);
    if (lv.tab)
        hipLaunchKernelGGL(k_loc_match, dim3(grid_for(R)), dim3(TB), 0, st, uc, (const uint64_t*)p->sk, vb,
                           (const uint32_t*)p->rec_t, (const uint32_t*)p->tv, (const uint32_t*)p->tdl,
                           (const uint32_t*)p->dold, (const uint32_t*)p->vacap, (const uint64_t*)p->vadj,
                           (const uint32_t*)g->pool, lv, p->ckey, p->cval, C);
    hipLaunchKernelGGL(k_check_overflow, dim3(1), dim3(1), 0, st, uc, C);
    sort_pairs_u64_dn(p->ckey, p->cval, p->cks, p->cvs, C, uc + UC_C, cbits, p->tmp, st);
    hipLaunchKernelGGL(k_cand_first, dim3(grid_for(C)), dim3(TB), 0, st, p->cks, (const unsigned long long*)uc, C,
                       p->first);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(R)), dim3(TB), 0, st, p->matched, R, NF);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(R)), dim3(TB), 0, st, p->ncnt, R, 0u);
    hipLaunchKernelGGL(k_cand_assign, dim3(grid_for(C)), dim3(TB), 0, st, p->cks, p->cvs,
                       (const unsigned long long*)uc, C, p->first, p->sk, p->rec_t, p->matched, p->ncnt);
    // 3. the deleted indices of every touched vertex, sorted
    hipLaunchKernelGGL(k_xkeys, dim3(grid_for(R)), dim3(TB), 0, st, (const unsigned long long*)uc, R, p->matched,
                       p->rec_t, xpad, p->xk);
    sort_keys_u64(p->xk, p->xks, R, cbits, p->tmp, st);
    hipLaunchKernelGGL(k_xextract, dim3(grid_for(R)), dim3(TB), 0, st, R, p->xks, p->xs);
    scan_u32_to_u64(p->ncnt, p->xoff, R, p->tmp, uc + UC_X, st);
    hipLaunchKernelGGL(k_ins_prep, dim3(grid_for(R)), dim3(TB), 0, st, (const unsigned long long*)uc, R, p->sv, p->iw,
                       p->rec_t, p->tsa, p->tdl, p->dold, p->ncnt, p->xoff, p->xs, p->wv, p->idest);
    // 4. analysis and one bump allocation
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(R)), dim3(TB), 0, st, p->needw, R, 0ull);
    hipLaunchKernelGGL(k_analyze, dim3(vgrid_a), dim3(WB), 0, st, (const unsigned long long*)uc, p->tv, p->tsa, p->tdl,
                       p->te, p->ncnt, p->xoff, p->xs, g->hdr, g->pool, p->wv, g->rule, p->needw, p->parts);
    hipLaunchKernelGGL(k_stats_reduce, dim3(32), dim3(256), 0, st, (const unsigned long long*)p->parts, vgrid_a,
                       uc + UC_STATS, 0);
    scan_u64(p->needw, p->aoff, R, p->tmp, uc + UC_ALLOC, st);
    hipLaunchKernelGGL(k_alloc_check, dim3(1), dim3(1), 0, st, g->d_ctl, g->pool_words, uc, err);
    // the edge locator in step with what the mutation will do (before it: the moved edges' dst
    // are read in the old adjacency; a rejected batch skips these as it skips the mutation)
    if (lv.tab) {
        hipLaunchKernelGGL(k_loc_kill, dim3(grid_for(R)), dim3(TB), 0, st, uc, (const uint32_t*)err,
                           (const uint64_t*)p->sk, vb, (const uint32_t*)p->rec_t, (const uint32_t*)p->tv,
                           (const uint32_t*)p->dold, (const uint32_t*)p->matched, lv);
        hipLaunchKernelGGL(k_loc_move, dim3(grid_for(R)), dim3(TB), 0, st, uc, (const uint32_t*)err,
                           (const uint64_t*)p->xks, (const uint64_t*)p->xoff, (const uint32_t*)p->ncnt,
                           (const uint32_t*)p->xs,
                           (const uint32_t*)p->tv, (const uint32_t*)p->tsa, (const uint32_t*)p->tdl,
                           (const uint32_t*)p->dold, (const uint64_t*)p->vadj, (const uint32_t*)g->pool, lv);
        hipLaunchKernelGGL(k_loc_claim, dim3(grid_for(R)), dim3(TB), 0, st, uc, (const uint32_t*)err,
                           (const uint32_t*)p->rec_t, (const uint32_t*)p->tv, (const uint32_t*)p->tdl,
                           (const uint32_t*)p->sv, (const uint32_t*)p->id, (const uint32_t*)p->idest, lv);
    }

    // 5. mutation (a no-op for a rejected batch)
    BigCtx bc{p->big_items, p->chunk_item, p->bsur, BIG_IMAX, BIG_CMAX, (uint32_t)big_smax(R), g->rule.fbits};
    const uint32_t split = g->update_split;
    const MutArgs ma{p->tv, p->tsa, p->tdl, p->te, p->ncnt, p->xoff, p->xs, g->hdr, g->pool, p->sv, p->id, p->wv,
                     p->idest, p->aoff, p->sur, p->sdirty, g->rule};
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(R)), dim3(TB), 0, st, p->sdirty, R, 0u);
    hipLaunchKernelGGL(k_mutate, dim3(vgrid_m), dim3(WB), 0, st, uc, (const uint32_t*)err, ma, p->parts,
                       (const uint32_t*)p->dold, (const uint32_t*)p->blist, bc, split);
    hipLaunchKernelGGL(k_stats_reduce, dim3(32), dim3(256), 0, st, (const unsigned long long*)p->parts, vgrid_m,
                       uc + UC_FREED, 0);
    if (split) {
        // vertices with more than `split` entries, then the passes they handed over
        const uint32_t sgrid = (uint32_t)std::min<uint64_t>(R, PART_BLOCKS);
        hipLaunchKernelGGL(k_mutate_split, dim3(sgrid), dim3(64), XL_WORDS * 4, st, uc, (const uint32_t*)err, ma,
                           p->parts, (const uint32_t*)p->dold, (const uint32_t*)p->blist, bc, split);
        hipLaunchKernelGGL(k_stats_reduce, dim3(32), dim3(256), 0, st, (const unsigned long long*)p->parts, sgrid,
                           uc + UC_FREED, 1);
        hipLaunchKernelGGL(k_big_pass, dim3(BIG_GRID), dim3(256), 0, st, (const unsigned long long*)uc, bc,
                           (const uint32_t*)p->xs, g->pool, g->hdr);
        hipLaunchKernelGGL(k_big_count, dim3(BIG_GRID), dim3(256), 0, st, (const unsigned long long*)uc, bc,
                           (const uint32_t*)p->xs, (const uint32_t*)g->pool, p->ccnt);
        hipLaunchKernelGGL(k_big_apply, dim3(BIG_GRID), dim3(256), 0, st, (const unsigned long long*)uc, bc,
                           (const uint32_t*)p->xs, g->pool, (const uint32_t*)p->ccnt);
        hipLaunchKernelGGL(k_big_holes, dim3(BIG_GRID), dim3(256), 0, st, (const unsigned long long*)uc, bc, g->pool);
        hipLaunchKernelGGL(k_big_one_dst, dim3(64), dim3(256), 0, st, (const unsigned long long*)uc, bc,
                           (const uint32_t*)g->pool, g->hdr);
    }
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(1), 0, st, g->d_ctl + 1, (const unsigned long long*)(uc + UC_FREED));
    // S(u) and the sparse groups' indexes of the vertices whose reduced list may have changed
    sparse_rebuild(g, p->tv, uc + UC_T, R, p->sdirty, p->srwork, st);
    // alias-table mode: the touched vertices' inter-group tables (a rejected batch rewrites them unchanged)
    alias_rows(g, p->tv, uc + UC_T, R, st);
}

static UpdPlan* get_plan(bingo_graph* g, uint64_t rmax, uint64_t cmax_min) {
    if (!g->upd) g->upd = new UpdPlans();
    UpdPlans* ps = g->upd;
    for (size_t i = 0; i < ps->plans.size(); ++i) {
        UpdPlan* p = ps->plans[i];
        if (p->rmax == rmax) {
            if (p->cmax >= cmax_min) return p;
            hipDeviceSynchronize();
            plan_free(p);
            ps->plans.erase(ps->plans.begin() + i);
            break;
        }
    }
    // small batches get a candidate buffer the one-block sort takes (a batch with more candidates than
    // that retries once with a larger plan)
    const uint64_t cmax =
        std::max<uint64_t>(cmax_min, rmax <= 1024 ? 4096ull : std::max<uint64_t>(4 * rmax, 1ull << 16));
    // keep the cached workspaces bounded: drop the largest others first
    size_t total = 0;
    for (auto* p : ps->plans) total += p->bytes;
    while (!ps->plans.empty() && total > PLAN_CACHE_BYTES) {
        size_t big = 0;
        for (size_t i = 1; i < ps->plans.size(); ++i)
            if (ps->plans[i]->bytes > ps->plans[big]->bytes) big = i;
        total -= ps->plans[big]->bytes;
        hipDeviceSynchronize();
        plan_free(ps->plans[big]);
        ps->plans.erase(ps->plans.begin() + big);
    }
    UpdPlan* p = plan_make(rmax, cmax);
    if (p) ps->plans.push_back(p);
    return p;
}

void update_drop_graphs(bingo_graph* g) {
    if (!g->upd) return;
    for (auto* p : g->upd->plans) {
        if (p->exec) hipGraphExecDestroy(p->exec);
        if (p->graph) hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
}

void update_release(bingo_graph* g) {
    if (!g->upd) return;
    for (auto* p : g->upd->plans) plan_free(p);
    if (g->upd->cap_stream) hipStreamDestroy(g->upd->cap_stream);
    delete g->upd;
    g->upd = nullptr;
}

int update_batch(bingo_graph* g, uint64_t n_ins, const uint32_t* is, const uint32_t* id, const uint32_t* iw,
                 uint64_t n_del, const uint32_t* ds, const uint32_t* dd, bingo_update_stats* h_stats, hipStream_t st) {
    const uint64_t R = n_ins + n_del;
    if (h_stats) memset(h_stats, 0, sizeof(*h_stats));
    if (R == 0) return BINGO_OK;
    if (R > (1ull << 31)) return BINGO_E_INVALID;
    const uint64_t rmax = pow2_at_least(R, 1024);
    uint64_t cmin = 0;
    bool compacted = false, grown = false;
    // the edge locator, made ready for this batch's claims (when it cannot be, deletes are
    // located by scanning)
    locator_prepare(g, n_ins, st);
    for (int attempt = 0; attempt < 6; ++attempt) {
        UpdPlan* p = get_plan(g, rmax, cmin);
        if (!p) return BINGO_E_OOM;
        const LocView lv = locator_view(g);
        if (n_ins) {
            HIPCHK(hipMemcpyAsync(p->is, is, n_ins * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(p->id, id, n_ins * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(p->iw, iw, n_ins * 4, hipMemcpyDeviceToDevice, st));
        }
        if (n_del) {
            HIPCHK(hipMemcpyAsync(p->ds, ds, n_del * 4, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(p->dd, dd, n_del * 4, hipMemcpyDeviceToDevice, st));
        }
        hipLaunchKernelGGL(k_upd_begin, dim3(1), dim3(128), 0, st, p->uc, n_ins, n_del, g->d_err);
        phase_mark(g, st, true);
        bool launched = false;
        if (p->exec && (p->split != g->update_split || p->lv.tab != lv.tab || p->lv.mask != lv.mask)) {
            hipGraphExecDestroy(p->exec);
            hipGraphDestroy(p->graph);
            p->exec = nullptr;
            p->graph = nullptr;
        }
        if (g->update_graphs && !p->graph_failed) {
            if (!p->exec) {
                p->split = g->update_split;
                p->lv = lv;
                if (!g->upd->cap_stream &&
                    hipStreamCreateWithFlags(&g->upd->cap_stream, hipStreamNonBlocking) != hipSuccess)
                    g->upd->cap_stream = nullptr;
                hipStream_t cs = g->upd->cap_stream;
                bool ok = cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    enqueue_update(g, p, cs);
                    ok = hipStreamEndCapture(cs, &p->graph) == hipSuccess && p->graph;
                }
                if (ok) ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
                if (!ok) {
                    p->graph_failed = true;
                    (void)hipGetLastError();
                }
            }
            if (p->exec && hipGraphLaunch(p->exec, st) == hipSuccess) launched = true;
        }
        if (!launched) {
            p->lv = lv;
            enqueue_update(g, p, st);
        }
        phase_mark(g, st, false);
        unsigned long long uc[UC_WORDS];
        uint32_t err = 0;
        HIPCHK(hipMemcpyAsync(uc, p->uc, sizeof uc, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&err, g->d_err, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (err == ERR_OOM && !grown) {
            // the pool is full (nothing was applied): reclaim the blocks earlier batches replaced,
            // once; then, for a pool the library sized, move to an arena twice the size
            unsigned long long ctl[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (!compacted && ctl[1] > 0) {
                compacted = true;
                if (compact_pool(g, 0, st) == BINGO_OK) continue;
            }
            grown = true;
            const uint64_t bigger = std::min<uint64_t>(g->pool_words * 2, 1ull << 35);
            if (g->pool_auto && bigger > g->pool_words && compact_pool(g, bigger, st) == BINGO_OK) continue;
        }
        if (err) return err_to_code(err);
        if (uc[UC_FLAGS] & 1ull) {  // more candidates than the buffer held: nothing changed, retry larger
            cmin = pow2_at_least(uc[UC_C], 1ull << 16) * 2;
            continue;
        }
        if (h_stats) {
            h_stats->inserted = uc[UC_STATS + 0];
            h_stats->deleted = uc[UC_STATS + 1];
            h_stats->not_found = uc[UC_STATS + 2];
            h_stats->touched_vertices = uc[UC_T];
            h_stats->match_scanned = uc[UC_F] + uc[UC_LPROBE];
            h_stats->match_candidates = uc[UC_C];
            for (int i = 0; i < 25; ++i) h_stats->transitions[i] = uc[UC_STATS + 3 + i];
        }
        if (lv.tab) locator_after_batch(g, uc[UC_LKILL], uc[UC_LCLAIM], uc[UC_LFRESH], uc[UC_LBAD]);
        else locator_invalidate(g);  // the batch did not keep it in step
        ++g->version;
        return BINGO_OK;
    }
    return BINGO_E_CAPACITY;
}

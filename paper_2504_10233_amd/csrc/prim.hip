// prim.hip -- device-wide exclusive scan and stable LSD radix sort (8-bit
// digits) for gfx950.  Digit ranks inside a wave come from eight ballots that
// isolate the lanes sharing a digit (wave64 match), then a popcount of the
// lower lanes; per-wave digit counts are combined through LDS.  Sorts of at
// most 4096 entries run as one bitonic block in LDS instead.
#include "dev.h"
#include <stdio.h>

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr uint64_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
constexpr uint64_t RAW_PART_MAX = 2048;  // tiles whose sums each tile adds up itself

// a tile of 4096 keys per block of 1024 threads (16 waves, so a compute unit keeps
// enough loads in flight when the grid has about one block per CU)
constexpr int SORT_BLOCK = 1024;
constexpr int SORT_WAVES = SORT_BLOCK / 64;
constexpr int SORT_SUBTILES = 4;
constexpr uint64_t SORT_TILE = (uint64_t)SORT_BLOCK * SORT_SUBTILES;
constexpr int RADIX = 256;

inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Block-wide exclusive scan of one u64 per thread; returns the block total in *total.
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const T* __restrict__ in, uint64_t n,
                                                            uint64_t* __restrict__ part) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += (uint64_t)in[base + i];
    uint64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// part: the tiles' bases (scanned), or with raw_part their sums, of which each block
// adds up those before it itself (one launch fewer than scanning them first).
template <typename T>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_tile(const T* __restrict__ in, uint64_t* __restrict__ out,
                                                          uint64_t n, const uint64_t* __restrict__ part,
                                                          unsigned long long* __restrict__ total, int raw_part) {
    uint64_t tbase = 0;
    if (part && raw_part) {
        uint64_t acc = 0;
        for (uint64_t j = threadIdx.x; j < blockIdx.x; j += SCAN_BLOCK) acc += part[j];
        block_exclusive_scan(acc, &tbase);
    } else if (part) {
        tbase = part[blockIdx.x];
    }
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : (T)0;
        s += (uint64_t)v[i];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_scan(s, &tot) + tbase;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += (uint64_t)v[i];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = tbase + tot;
}

template <typename T>
void scan_impl(const T* in, uint64_t* out, uint64_t n, void* temp, unsigned long long* d_total, hipStream_t st) {
    if (n == 0) {
        if (d_total) hipMemsetAsync(d_total, 0, 8, st);
        return;
    }
    const uint64_t nb = cdiv(n, SCAN_TILE);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile<T>, dim3(1), dim3(SCAN_BLOCK), 0, st, in, out, n, (const uint64_t*)nullptr,
                           d_total, 0);
        return;
    }
    uint64_t* part = (uint64_t*)temp;
    void* rest = (char*)temp + align256(nb * 8);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)nb), dim3(SCAN_BLOCK), 0, st, in, n, part);
    if (nb <= RAW_PART_MAX) {  // each tile adds up the sums before it
        hipLaunchKernelGGL(k_scan_tile<T>, dim3((uint32_t)nb), dim3(SCAN_BLOCK), 0, st, in, out, n,
                           (const uint64_t*)part, d_total, 1);
        return;
    }
    scan_impl<uint64_t>(part, part, nb, rest, nullptr, st);  // in place: each tile reads then writes its own range
    hipLaunchKernelGGL(k_scan_tile<T>, dim3((uint32_t)nb), dim3(SCAN_BLOCK), 0, st, in, out, n,
                       (const uint64_t*)part, d_total, 0);
}

// ------------------------------------------------------------------ radix sort
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int sh) {
    return (uint32_t)(k >> sh) & 0xFFu;
}

template <typename K>
__global__ void __launch_bounds__(SORT_BLOCK) k_digit_hist(const K* __restrict__ keys, uint64_t n,
                                                           const unsigned long long* __restrict__ dn, int sh,
                                                           uint32_t* __restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[RADIX];
    if (dn) n = std::min<uint64_t>(n, *dn);
    if (threadIdx.x < RADIX) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    K k[SORT_SUBTILES];
#pragma unroll
    for (int i = 0; i < SORT_SUBTILES; ++i) {
        const uint64_t idx = base + (uint64_t)i * SORT_BLOCK + threadIdx.x;
        k[i] = idx < n ? keys[idx] : (K)0;
    }
#pragma unroll
    for (int i = 0; i < SORT_SUBTILES; ++i)
        if (base + (uint64_t)i * SORT_BLOCK + threadIdx.x < n) atomicAdd(&h[digit_of(k[i], sh)], 1u);
    __syncthreads();
    if (threadIdx.x < RADIX) hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

template <typename K, bool HAS_V>
__global__ void __launch_bounds__(SORT_BLOCK) k_digit_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                              K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              uint64_t n, const unsigned long long* __restrict__ dn,
                                                              int sh, const uint64_t* __restrict__ offs,
                                                              uint32_t nblocks) {
    __shared__ uint64_t run[RADIX];
    __shared__ uint32_t tot[RADIX];
    if (dn) n = std::min<uint64_t>(n, *dn);
    __shared__ uint32_t wc[SORT_WAVES][RADIX];
    const int tid = threadIdx.x, wave = tid >> 6;
    if (tid < RADIX) {
        run[tid] = offs[(uint64_t)tid * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < SORT_WAVES; ++w) wc[w][tid] = 0;
    }
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    const uint64_t below = lanemask_lt();
    // the tile's keys and values, all loads issued before the first subtile is ranked
    K keys[SORT_SUBTILES];
    uint32_t vals[SORT_SUBTILES];
#pragma unroll
    for (int i = 0; i < SORT_SUBTILES; ++i) {
        const uint64_t idx = base + (uint64_t)i * SORT_BLOCK + tid;
        keys[i] = idx < n ? kin[idx] : (K)0;
        vals[i] = (HAS_V && idx < n) ? vin[idx] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SORT_SUBTILES; ++i) {
        const uint64_t idx = base + (uint64_t)i * SORT_BLOCK + tid;
        const bool valid = idx < n;
        const K key = keys[i];
        const uint32_t val = vals[i];
        const uint32_t dg = digit_of(key, sh);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t lrank = __popcll(peers & below);
        if (valid && lrank == 0) wc[wave][dg] = __popcll(peers);
        __syncthreads();
        // per digit, the keys of the lower waves (an exclusive scan down each column)
        if (tid < RADIX) {
            uint32_t acc = 0;
#pragma unroll
            for (int w = 0; w < SORT_WAVES; ++w) {
                const uint32_t c = wc[w][tid];
                wc[w][tid] = acc;
                acc += c;
            }
            tot[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint64_t pos = run[dg] + wc[wave][dg] + lrank;
            kout[pos] = key;
            if (HAS_V) vout[pos] = val;
        }
        __syncthreads();
        if (tid < RADIX) {
            run[tid] += tot[tid];
#pragma unroll
            for (int w = 0; w < SORT_WAVES; ++w) wc[w][tid] = 0;
        }
        __syncthreads();
    }
}

// Small sorts (capacity up to BSORT_MAX) in one block: a bitonic network in LDS
// over (the key's digits the LSD passes would look at, input position), which
// orders exactly as the stable LSD sort does, replacing its 3 to 5 launches per
// 8-bit pass.
constexpr uint32_t BSORT_MAX = 4096;
constexpr int BSORT_BLOCK = 1024;

template <typename K, bool HAS_V>
__global__ void __launch_bounds__(BSORT_BLOCK) k_block_sort(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                            K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                            uint32_t n, const unsigned long long* __restrict__ dn,
                                                            K mask) {
    __shared__ K sk[BSORT_MAX];
    __shared__ uint32_t si[BSORT_MAX];
    const uint32_t m = dn ? (uint32_t)std::min<uint64_t>(n, *dn) : n;
    if (m == 0) return;
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += BSORT_BLOCK) {
        // padding sorts after every entry: the largest masked key, then the largest position
        sk[i] = i < m ? (K)(kin[i] & mask) : mask;
        si[i] = i < m ? i : ~0u;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = threadIdx.x; q < (P >> 1); q += BSORT_BLOCK) {
                const uint32_t a = 2 * j * (q / j) + (q % j), b = a + j;
                const bool up = (a & k) == 0;
                const K ka = sk[a], kb = sk[b];
                const uint32_t ia = si[a], ib = si[b];
                const bool gt = ka > kb || (ka == kb && ia > ib);
                if (gt == up) {
                    sk[a] = kb; sk[b] = ka;
                    si[a] = ib; si[b] = ia;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < m; i += BSORT_BLOCK) {
        const uint32_t src = si[i];
        kout[i] = kin[src];
        if (HAS_V) vout[i] = vin[src];
    }
}

// Stable LSD sort of the first min(n, *dn) entries (all n when dn is null);
// grids are sized by n, so a device-side count keeps the launch sequence fixed.
template <typename K, bool HAS_V>
void sort_impl(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, uint64_t n, int bits, void* temp,
               hipStream_t st, const unsigned long long* dn = nullptr) {
    if (n == 0) return;
    const int passes = bits <= 0 ? 0 : (bits + 7) / 8;
    const uint64_t nb = cdiv(n, SORT_TILE);
    char* t = (char*)temp;
    uint32_t* hist = (uint32_t*)t;           t += align256(nb * RADIX * 4);
    uint64_t* offs = (uint64_t*)t;           t += align256(nb * RADIX * 8);
    K* ktmp = (K*)t;                         t += align256(n * sizeof(K));
    uint32_t* vtmp = (uint32_t*)t;           t += align256(HAS_V ? n * 4 : 0);
    void* scratch = t;
    if (passes == 0) {
        hipMemcpyAsync(kout, kin, n * sizeof(K), hipMemcpyDeviceToDevice, st);
        if (HAS_V) hipMemcpyAsync(vout, vin, n * 4, hipMemcpyDeviceToDevice, st);
        return;
    }
    if (n <= BSORT_MAX) {
        const int pb = 8 * passes;  // the LSD passes look at whole digits
        const K mask = pb >= (int)(8 * sizeof(K)) ? (K)~(K)0 : (K)(((K)1 << pb) - 1);
        hipLaunchKernelGGL((k_block_sort<K, HAS_V>), dim3(1), dim3(BSORT_BLOCK), 0, st, kin, vin, kout, vout,
                           (uint32_t)n, dn, mask);
        return;
    }
    const K* ck = kin;
    const uint32_t* cv = vin;
    for (int p = 0; p < passes; ++p) {
        // the last pass lands in kout
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        K* nk = to_out ? kout : ktmp;
        uint32_t* nv = to_out ? vout : vtmp;
        const int sh = 8 * p;
        hipLaunchKernelGGL((k_digit_hist<K>), dim3((uint32_t)nb), dim3(SORT_BLOCK), 0, st, ck, n, dn, sh, hist,
                           (uint32_t)nb);
        scan_impl<uint32_t>(hist, offs, nb * RADIX, scratch, nullptr, st);
        hipLaunchKernelGGL((k_digit_scatter<K, HAS_V>), dim3((uint32_t)nb), dim3(SORT_BLOCK), 0, st, ck, cv, nk,
                           nv, n, dn, sh, (const uint64_t*)offs, (uint32_t)nb);
        ck = nk;
        cv = nv;
    }
}

}  // namespace

size_t scan_temp_bytes(uint64_t n) {
    size_t b = 0;
    while (n > SCAN_TILE) {
        n = cdiv(n, SCAN_TILE);
        b += align256(n * 8);
    }
    return b + 256;
}

size_t sort_temp_bytes(uint64_t n, bool wide_keys) {
    const uint64_t nb = cdiv(n ? n : 1, SORT_TILE);
    return align256(nb * RADIX * 4) + align256(nb * RADIX * 8) + align256(n * (wide_keys ? 8 : 4)) +
           align256(n * 4) + scan_temp_bytes(nb * RADIX) + 256;
}

void scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, void* temp, unsigned long long* d_total,
                     hipStream_t st) {
    scan_impl<uint32_t>(in, out, n, temp, d_total, st);
}
void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, void* temp, unsigned long long* d_total,
              hipStream_t st) {
    scan_impl<uint64_t>(in, out, n, temp, d_total, st);
}
void sort_pairs_u32(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, uint64_t n, int bits,
                    void* temp, hipStream_t st) {
    sort_impl<uint32_t, true>(ki, vi, ko, vo, n, bits, temp, st);
}
void sort_pairs_u64(const uint64_t* ki, const uint32_t* vi, uint64_t* ko, uint32_t* vo, uint64_t n, int bits,
                    void* temp, hipStream_t st) {
    sort_impl<uint64_t, true>(ki, vi, ko, vo, n, bits, temp, st);
}
void sort_keys_u64(const uint64_t* ki, uint64_t* ko, uint64_t n, int bits, void* temp, hipStream_t st) {
    sort_impl<uint64_t, false>(ki, nullptr, ko, nullptr, n, bits, temp, st);
}
void sort_pairs_u64_dn(const uint64_t* ki, const uint32_t* vi, uint64_t* ko, uint32_t* vo, uint64_t nmax,
                       const unsigned long long* dn, int bits, void* temp, hipStream_t st) {
    sort_impl<uint64_t, true>(ki, vi, ko, vo, nmax, bits, temp, st, dn);
}

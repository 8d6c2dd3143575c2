// probe.hip -- measurement aid: the rate of random line reads this device
// sustains over a large buffer.  It gives the walk kernels' roofline an
// achievable ceiling next to the published HBM peak: a walk transition is a
// short chain of dependent random line reads (header, list entry, adjacency
// word), so the relevant ceiling is random-line throughput, not streaming
// bandwidth.  A second probe replays a walk query's recorded visits over the
// graph's own headers and adjacency, the walk's access pattern without its
// arithmetic.  Nothing of the method runs here.
#include "dev.h"

namespace {

constexpr int PB = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014)
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

// Independent form: the address of read r of lane l is a hash of (seed, l, r),
// so a lane keeps UNROLL reads in flight.  Dependent form: the next address
// also hashes the previous line's first word, so each lane is one pointer
// chase, like one walk.  Each read loads LINE bytes as 16-byte vectors.
template <int LINE, bool DEP>
__global__ void __launch_bounds__(PB) k_probe(const uint4* __restrict__ table, uint64_t nlines, uint32_t reads,
                                              uint64_t seed, uint32_t* __restrict__ sink) {
    constexpr int V = LINE / 16;
    constexpr int UNROLL = DEP ? 1 : 4;
    const uint64_t lane = (uint64_t)blockIdx.x * PB + threadIdx.x;
    uint32_t acc = 0;
    uint64_t chain = mix64(seed ^ (lane * 0x9E3779B97F4A7C15ull));
    for (uint32_t r = 0; r < reads; r += UNROLL) {
        uint4 x[UNROLL][V];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const uint64_t h = DEP ? mix64(chain + r) : mix64(chain + r + k);
            const uint64_t line = (uint64_t)(((unsigned __int128)h * nlines) >> 64);
#pragma unroll
            for (int q = 0; q < V; ++q) x[k][q] = table[line * V + q];
        }
#pragma unroll
        for (int k = 0; k < UNROLL; ++k)
#pragma unroll
            for (int q = 0; q < V; ++q) acc ^= x[k][q].x ^ x[k][q].y ^ x[k][q].z ^ x[k][q].w;
        if (DEP) chain ^= (uint64_t)x[0][0].x << 17 | acc;
    }
    sink[lane] = acc;
}

template <int LINE, bool DEP>
void launch_probe(const void* table, uint64_t nlines, uint32_t lanes, uint32_t reads, uint64_t seed, uint32_t* sink,
                  hipStream_t st) {
    hipLaunchKernelGGL((k_probe<LINE, DEP>), dim3(lanes / PB), dim3(PB), 0, st, (const uint4*)table, nlines, reads,
                       seed, sink);
}

// Replay of a walk query's visit stream: lane l takes chains l, l + lanes, ...
// of `chain` consecutive visits.  Per visit it reads the 64-byte header line of
// the visited vertex, then `extra` random adjacency entries of that vertex
// (extra_x256 / 256 on average, a seeded coin deciding the fraction), whose
// address needs the header's adjacency offset.  DEP: the next visit's address
// also waits on what was read, as a walk's next header waits on the neighbour
// it read; otherwise visits are independent and only the header-to-adjacency
// dependency remains.  Counts the lines it read.
template <bool DEP>
__global__ void __launch_bounds__(PB) k_probe_replay(const uint32_t* __restrict__ visits, uint64_t nv, uint32_t chain,
                                                     const uint32_t* __restrict__ hdr, uint32_t n,
                                                     const uint32_t* __restrict__ pool, uint32_t extra_x256,
                                                     uint64_t seed, uint32_t zero,
                                                     unsigned long long* __restrict__ ctr) {
    const uint64_t lane = (uint64_t)blockIdx.x * PB + threadIdx.x, lanes = (uint64_t)gridDim.x * PB;
    const uint64_t nchains = (nv + chain - 1) / chain;
    uint32_t acc = 0;
    unsigned long long lines = 0;
    for (uint64_t c = lane; c < nchains; c += lanes) {
        const uint64_t e = std::min<uint64_t>(nv, (c + 1) * chain);
        for (uint64_t i = c * chain; i < e; ++i) {
            const uint32_t v = DEP ? visits[i] ^ (acc & zero) : visits[i];
            if (v >= n) continue;
            const uint32_t* h = hdr + (size_t)v * HDR_WORDS;
            const uint4* hl = (const uint4*)h;
            const uint4 x0 = hl[0], x1 = hl[1], x2 = hl[2], x3 = hl[3];
            acc ^= x0.x ^ x1.y ^ x2.z ^ x3.w;
            ++lines;
            const uint32_t d = x0.y;  // H_DEG
            if (d) {
                const uint64_t adj = ((uint64_t)(x1.y & H_ADJHI_MASK) << 32) | x1.x;  // H_ADJHI, H_ADJLO
                const uint64_t r = mix64(seed ^ (i * 0x9E3779B97F4A7C15ull));
                const uint32_t k = (extra_x256 >> 8) + ((uint32_t)(r & 255u) < (extra_x256 & 255u) ? 1u : 0u);
                for (uint32_t j = 0; j < k; ++j) {
                    const uint32_t pos = (uint32_t)(((mix64(r + j + 1) >> 32) * d) >> 32);
                    acc ^= pool[adj + 2ull * pos];
                    ++lines;
                }
            }
        }
    }
    // one atomic per wave
    for (int o = 32; o > 0; o >>= 1) lines += __shfl_xor(lines, o, 64);
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(ctr, lines);
        atomicXor(ctr + 1, (unsigned long long)acc);
    }
}
static_assert(H_DEG == 1 && H_ADJLO == 4 && H_ADJHI == 5, "k_probe_replay reads these words from the header line");

}  // namespace

extern "C" int bingo_probe_replay(bingo_graph* g, const uint32_t* d_visits, uint64_t n_visits, uint32_t chain,
                                  uint32_t lanes, uint32_t extra_x256, uint32_t dependent, uint64_t seed,
                                  unsigned long long* d_counters, float* h_ms, void* stream) {
    if (!g || !d_counters || !h_ms || (n_visits && !d_visits)) return BINGO_E_INVALID;
    if (g->radix_base == 4) return BINGO_E_INVALID;
    if (chain == 0 || lanes == 0 || lanes % PB || extra_x256 > 64 * 256) return BINGO_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(d_counters, 0, 16, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    if (n_visits && dependent)
        hipLaunchKernelGGL(k_probe_replay<true>, dim3(lanes / PB), dim3(PB), 0, st, d_visits, n_visits, chain, g->hdr,
                           g->n, g->pool, extra_x256, seed, 0u, d_counters);
    else if (n_visits)
        hipLaunchKernelGGL(k_probe_replay<false>, dim3(lanes / PB), dim3(PB), 0, st, d_visits, n_visits, chain,
                           g->hdr, g->n, g->pool, extra_x256, seed, 0u, d_counters);
    HIPCHK(hipEventRecord(e1, st));
    const hipError_t le = hipGetLastError();
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(h_ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return le == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

extern "C" int bingo_probe_random_reads(const void* d_table, uint64_t table_bytes, uint32_t lanes, uint32_t reads,
                                        uint32_t dependent, uint32_t line_bytes, uint64_t seed, uint32_t* d_sink,
                                        float* h_ms, void* stream) {
    if (!d_table || !d_sink || !h_ms) return BINGO_E_INVALID;
    if (line_bytes != 64 && line_bytes != 128) return BINGO_E_INVALID;
    if (table_bytes < (1ull << 16) || table_bytes % line_bytes) return BINGO_E_INVALID;
    if (lanes == 0 || lanes % PB || reads == 0 || reads % 4) return BINGO_E_INVALID;
    const uint64_t nlines = table_bytes / line_bytes;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
    if (line_bytes == 64) {
        if (dependent) launch_probe<64, true>(d_table, nlines, lanes, reads, seed, d_sink, st);
        else launch_probe<64, false>(d_table, nlines, lanes, reads, seed, d_sink, st);
    } else {
        if (dependent) launch_probe<128, true>(d_table, nlines, lanes, reads, seed, d_sink, st);
        else launch_probe<128, false>(d_table, nlines, lanes, reads, seed, d_sink, st);
    }
    HIPCHK(hipEventRecord(e1, st));
    const hipError_t le = hipGetLastError();
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(h_ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return le == hipSuccess ? BINGO_OK : BINGO_E_HIP;
}

// probe.hip -- measurement aid: the rate of random line reads this device
// sustains over a large buffer.  It gives the walk kernels' roofline an
// achievable ceiling next to the published HBM peak: a walk transition is a
// short chain of dependent random line reads (header, list entry, adjacency
// word), so the relevant ceiling is random-line throughput, not streaming
// bandwidth.  Nothing of the method runs here.
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

}  // namespace

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

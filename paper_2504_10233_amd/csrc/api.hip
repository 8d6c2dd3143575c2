// api.hip -- the extern "C" entry points of libbingo (declared in bingo.h).
#include "dev.h"
#include "locate.h"
#include <stdio.h>
#include <string.h>
#include <new>
#include <stdlib.h>
#include <cmath>

void* ws_get(bingo_graph* g, size_t bytes) {
    // a pending asynchronous PPR histogram still reads its visit bins here
    if (ppr_drain(g) != BINGO_OK) return nullptr;
    if (bytes <= g->ws_bytes && g->ws) return g->ws;
    hipDeviceSynchronize();
    if (g->ws) hipFree(g->ws);
    g->ws = nullptr;
    g->ws_bytes = 0;
    const size_t want = bytes + bytes / 4 + 4096;
    if (hipMalloc(&g->ws, want) != hipSuccess) {
        g->ws = nullptr;
        return nullptr;
    }
    g->ws_bytes = want;
    return g->ws;
}

// Record the next phase boundary of the current call on its stream.
void phase_mark(bingo_graph* g, hipStream_t st, bool first) {
    if (first) g->nev = 0;
    if (g->nev >= PHASE_EVENTS) return;
    if (!g->ev[g->nev] && hipEventCreate(&g->ev[g->nev]) != hipSuccess) return;
    if (hipEventRecord(g->ev[g->nev], st) == hipSuccess) g->nev++;
}

int err_to_code(uint32_t bits) {
    if (bits & ERR_RANGE) return BINGO_E_RANGE;
    if (bits & ERR_WEIGHT) return BINGO_E_WEIGHT;
    if (bits & ERR_OOM) return BINGO_E_OOM;
    if (bits & ERR_INTERNAL) return BINGO_E_INTERNAL;
    return BINGO_OK;
}

static void release(bingo_graph* g) {
    if (!g) return;
    update_release(g);
    locator_release(g);
    for (int i = 0; i < PHASE_EVENTS; ++i)
        if (g->ev[i]) hipEventDestroy(g->ev[i]);
    for (int i = 0; i < WALK_SLOTS; ++i)
        if (g->slot_ev[i]) hipEventDestroy(g->slot_ev[i]);
    for (hipEvent_t e : {g->ppr_done, g->ppr_h0, g->ppr_h1})
        if (e) hipEventDestroy(e);
    hipFree(g->hdr);
    hipFree(g->alias);
    hipFree(g->pool);
    hipFree(g->d_ctl);
    hipFree(g->d_err);
    hipFree(g->ppr_off);
    hipFree(g->ppr_vtx);
    hipFree(g->ppr_cnt);
    hipFree(g->ws);
    hipFree(g->aux);
    hipFree(g->n2v_idx);
    hipFree(g->n2v_off);
    delete g;
}

extern "C" {

int bingo_build(const bingo_config* cfg, uint32_t n, uint64_t m, const uint32_t* d_src, const uint32_t* d_dst,
                const uint32_t* d_w, void* stream, bingo_graph** out) {
    if (!out) return BINGO_E_INVALID;
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(bingo_config)) return BINGO_E_INVALID;
    if (n == 0 || n >= (1u << 31) || m >= (1ull << 32)) return BINGO_E_INVALID;
    if (m && (!d_src || !d_dst || !d_w)) return BINGO_E_INVALID;
    if (cfg->adaptive > 1 || cfg->alpha_pct > 100 || cfg->beta_pct > 100) return BINGO_E_INVALID;
    if (cfg->frac_bits > 16 || cfg->alias_table > 1 || (cfg->alias_table && cfg->frac_bits)) return BINGO_E_INVALID;
    const uint32_t radix = cfg->radix_base ? cfg->radix_base : 2u;
    if ((radix != 2 && radix != 4) || cfg->reserved) return BINGO_E_INVALID;
    if (radix == 4 && (cfg->frac_bits || cfg->alias_table)) return BINGO_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    bingo_graph* g = new (std::nothrow) bingo_graph();
    if (!g) return BINGO_E_OOM;
    g->n = n;
    g->rule.adaptive = cfg->adaptive;
    g->rule.alpha = cfg->alpha_pct;
    g->rule.beta = cfg->beta_pct;
    g->rule.fbits = cfg->frac_bits;
    g->rule.alias = nullptr;
    g->alias_mode = cfg->alias_table;
    g->pool_words = cfg->pool_bytes / 4;
    g->pool_auto = cfg->pool_bytes == 0;
    g->radix_base = radix;
    const size_t hdr_words = radix == 4 ? (size_t)H4_WORDS : (size_t)HDR_WORDS;
    g->hdr = nullptr; g->pool = nullptr; g->d_ctl = nullptr; g->d_err = nullptr; g->alias = nullptr;
    if (hipMalloc(&g->hdr, (size_t)n * hdr_words * 4) != hipSuccess ||
        hipMalloc(&g->d_ctl, CTL_WORDS * 8) != hipSuccess || hipMalloc(&g->d_err, 4) != hipSuccess) {
        release(g);
        return BINGO_E_OOM;
    }
    if (hipMemsetAsync(g->hdr, 0, (size_t)n * hdr_words * 4, st) != hipSuccess ||
        hipMemsetAsync(g->d_ctl, 0, CTL_WORDS * 8, st) != hipSuccess) {
        release(g);
        return BINGO_E_HIP;
    }
    const int rc = build_graph(g, m, d_src, d_dst, d_w, st);
    if (rc != BINGO_OK) {
        hipStreamSynchronize(st);
        release(g);
        return rc;
    }
    *out = g;
    return BINGO_OK;
}

int bingo_quantize_biases(uint64_t m, const float* d_bias, double lambda, uint32_t frac_bits, uint32_t* d_w,
                          void* stream) {
    if (m && (!d_bias || !d_w)) return BINGO_E_INVALID;
    if (frac_bits < 1 || frac_bits > 16 || !(lambda > 0.0) || std::isinf(lambda)) return BINGO_E_INVALID;
    return quantize_biases(m, d_bias, lambda, frac_bits, d_w, (hipStream_t)stream);
}

int bingo_update_batch(bingo_graph* g, uint64_t n_ins, const uint32_t* d_ins_src, const uint32_t* d_ins_dst,
                       const uint32_t* d_ins_w, uint64_t n_del, const uint32_t* d_del_src, const uint32_t* d_del_dst,
                       void* stream, bingo_update_stats* h_stats) {
    if (!g || g->radix_base != 2) return BINGO_E_INVALID;
    if (n_ins && (!d_ins_src || !d_ins_dst || !d_ins_w)) return BINGO_E_INVALID;
    if (n_del && (!d_del_src || !d_del_dst)) return BINGO_E_INVALID;
    return update_batch(g, n_ins, d_ins_src, d_ins_dst, d_ins_w, n_del, d_del_src, d_del_dst, h_stats,
                        (hipStream_t)stream);
}

int bingo_update_stream(bingo_graph* g, uint64_t n, const uint32_t* d_op, const uint32_t* d_src,
                        const uint32_t* d_dst, const uint32_t* d_w, void* stream, bingo_update_stats* h_stats) {
    if (!g || g->radix_base != 2 || (n && (!d_op || !d_src || !d_dst || !d_w))) return BINGO_E_INVALID;
    return update_stream(g, n, d_op, d_src, d_dst, d_w, h_stats, (hipStream_t)stream);
}

int bingo_walk(const bingo_graph* g, uint64_t n_walks, const uint32_t* d_starts, uint64_t walk_id_base,
               uint32_t length, uint64_t seed, uint32_t* d_paths, uint64_t* d_steps_taken, uint32_t mode,
               void* stream) {
    if (!g || (n_walks && (!d_starts || !d_paths))) return BINGO_E_INVALID;
    if (mode > BINGO_WALK_PER_STEP || length == 0xFFFFFFFFu) return BINGO_E_INVALID;
    if (g->radix_base == 4) {
        if (mode != BINGO_WALK_PERSISTENT) return BINGO_E_INVALID;
        return launch_walk4(const_cast<bingo_graph*>(g), n_walks, d_starts, walk_id_base, length, seed, d_paths,
                            d_steps_taken, (hipStream_t)stream);
    }
    return launch_walk(const_cast<bingo_graph*>(g), n_walks, d_starts, walk_id_base, length, seed, d_paths,
                       d_steps_taken, mode, (hipStream_t)stream);
}

int bingo_walk_batch(const bingo_graph* g, uint32_t n_queries, const bingo_walk_query* h_queries, void* stream) {
    if (!g || g->radix_base != 2 || n_queries > BINGO_WALK_BATCH_MAX || (n_queries && !h_queries)) return BINGO_E_INVALID;
    for (uint32_t i = 0; i < n_queries; ++i) {
        const bingo_walk_query& q = h_queries[i];
        if ((q.n_walks && (!q.d_starts || !q.d_paths)) || q.length == 0xFFFFFFFFu) return BINGO_E_INVALID;
    }
    return launch_walk_batch(const_cast<bingo_graph*>(g), n_queries, h_queries, (hipStream_t)stream);
}

int bingo_node2vec(bingo_graph* g, uint64_t n_walks, const uint32_t* d_starts, uint64_t walk_id_base,
                   uint32_t length, double p, double q, uint64_t seed, uint32_t* d_paths, uint64_t* d_counts,
                   void* stream) {
    if (!g || g->radix_base != 2 || (n_walks && (!d_starts || !d_paths)) || length == 0xFFFFFFFFu)
        return BINGO_E_INVALID;
    return run_node2vec(g, n_walks, d_starts, walk_id_base, length, p, q, seed, d_paths, d_counts,
                        (hipStream_t)stream);
}

int bingo_ppr(bingo_graph* g, uint32_t n_sources, const uint32_t* d_sources, uint32_t walks_per_source,
              uint32_t term_threshold, uint32_t max_len, uint64_t seed, uint64_t walk_id_base, uint32_t mode,
              uint64_t* h_total_entries, uint64_t* h_total_steps, void* stream) {
    if (!g || g->radix_base != 2 || !h_total_entries || n_sources == 0 || walks_per_source == 0 || !d_sources)
        return BINGO_E_INVALID;
    if (mode > BINGO_WALK_PER_STEP) return BINGO_E_INVALID;
    if ((uint64_t)n_sources * walks_per_source >= (1ull << 40)) return BINGO_E_INVALID;
    return run_ppr(g, n_sources, d_sources, walks_per_source, term_threshold, max_len, seed, walk_id_base, mode,
                   h_total_entries, h_total_steps, (hipStream_t)stream);
}

int bingo_ppr_async(bingo_graph* g, uint32_t n_sources, const uint32_t* d_sources, uint32_t walks_per_source,
                    uint32_t term_threshold, uint32_t max_len, uint64_t seed, uint64_t walk_id_base,
                    uint64_t* h_total_steps, void* stream, void* hist_stream) {
    if (!g || g->radix_base != 2 || n_sources == 0 || walks_per_source == 0 || !d_sources) return BINGO_E_INVALID;
    if ((uint64_t)n_sources * walks_per_source >= (1ull << 40)) return BINGO_E_INVALID;
    uint64_t entries = 0;
    return run_ppr(g, n_sources, d_sources, walks_per_source, term_threshold, max_len, seed, walk_id_base,
                   BINGO_WALK_PERSISTENT, &entries, h_total_steps, (hipStream_t)stream, (hipStream_t)hist_stream);
}

int bingo_ppr_wait(bingo_graph* g, uint64_t* h_total_entries, float* h_hist_ms) {
    if (!g) return BINGO_E_INVALID;
    return ppr_wait(g, h_total_entries, h_hist_ms);
}

int bingo_ppr_fetch(bingo_graph* g, uint64_t* d_offsets, uint32_t* d_vertex, uint32_t* d_count, uint64_t capacity,
                    void* stream) {
    if (!g || !d_offsets || !d_vertex || !d_count || !g->ppr_off) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    if (capacity < g->ppr_entries) return BINGO_E_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(d_offsets, g->ppr_off, ((uint64_t)g->ppr_nsrc + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (g->ppr_entries) {
        HIPCHK(hipMemcpyAsync(d_vertex, g->ppr_vtx, g->ppr_entries * 4, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(d_count, g->ppr_cnt, g->ppr_entries * 4, hipMemcpyDeviceToDevice, st));
    }
    return BINGO_OK;
}

int bingo_export(bingo_graph* g, uint32_t* h_buf, uint64_t cap_words, uint64_t* h_len, void* stream) {
    if (!g || !h_len) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    if (g->radix_base == 4) return export_graph4(g, 0, g->n, h_buf, cap_words, h_len, (hipStream_t)stream);
    return export_graph(g, 0, g->n, h_buf, cap_words, h_len, (hipStream_t)stream);
}

int bingo_export_range(bingo_graph* g, uint32_t u_begin, uint32_t u_end, uint32_t* h_buf, uint64_t cap_words,
                       uint64_t* h_len, void* stream) {
    if (!g || !h_len) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    if (g->radix_base == 4) return export_graph4(g, u_begin, u_end, h_buf, cap_words, h_len, (hipStream_t)stream);
    return export_graph(g, u_begin, u_end, h_buf, cap_words, h_len, (hipStream_t)stream);
}

int bingo_export_index_range(bingo_graph* g, uint32_t u_begin, uint32_t u_end, uint32_t* h_buf, uint64_t cap_words,
                             uint64_t* h_len, void* stream) {
    if (!g || !h_len || g->radix_base != 2) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    return export_index(g, u_begin, u_end, h_buf, cap_words, h_len, (hipStream_t)stream);
}

int bingo_compact(bingo_graph* g, uint64_t pool_bytes, void* stream) {
    if (!g || g->radix_base != 2) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    if (pool_bytes > (1ull << 37)) return BINGO_E_INVALID;
    return compact_pool(g, pool_bytes / 4, (hipStream_t)stream);
}

int bingo_memory(bingo_graph* g, bingo_mem_stats* out, void* stream) {
    if (!g || !out) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    memset(out, 0, sizeof(*out));
    if (g->radix_base == 4) return memory_stats4(g, out, (hipStream_t)stream);
    return memory_stats(g, out, (hipStream_t)stream);
}

int bingo_status(bingo_graph* g, void* stream) {
    if (!g) return BINGO_E_INVALID;
    if (int rc = ppr_drain(g)) return rc;
    hipStream_t st = (hipStream_t)stream;
    uint32_t bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, g->d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemsetAsync(g->d_err, 0, 4, st));
    return err_to_code(bits);
}

uint32_t bingo_num_vertices(const bingo_graph* g) { return g ? g->n : 0u; }

int bingo_set_tuning(bingo_graph* g, const bingo_tuning* t) {
    if (!g || !t || t->struct_size != sizeof(bingo_tuning)) return BINGO_E_INVALID;
    if (t->walk_variant > 1 || t->blocks_per_cu > 64 || t->update_graphs > 1 || t->ppr_bins > 1 ||
        t->update_locate > 1)
        return BINGO_E_INVALID;
    if (t->update_split != 0 && t->update_split < 64) return BINGO_E_INVALID;
    const uint32_t qc = t->queue_chunk ? t->queue_chunk : 256u;
    if (qc < 16 || qc > 4096 || (qc & (qc - 1))) return BINGO_E_INVALID;
    const uint32_t ds = t->dense_spec ? t->dense_spec : 2u;
    if (ds != 1 && ds != 2 && ds != 4) return BINGO_E_INVALID;
    g->dense_spec = ds;
    g->ppr_bins = t->ppr_bins;
    g->update_split = t->update_split;
    g->walk_variant = t->walk_variant;
    g->blocks_per_cu = t->blocks_per_cu;
    g->queue_chunk = qc;
    g->update_graphs = t->update_graphs;
    g->wave_degree = t->wave_degree;
    g->update_locate = t->update_locate;
    return BINGO_OK;
}

int bingo_get_tuning(const bingo_graph* g, bingo_tuning* t) {
    if (!g || !t) return BINGO_E_INVALID;
    t->struct_size = sizeof(bingo_tuning);
    t->walk_variant = g->walk_variant;
    t->blocks_per_cu = g->blocks_per_cu;
    t->queue_chunk = g->queue_chunk;
    t->update_graphs = g->update_graphs;
    t->dense_spec = g->dense_spec;
    t->ppr_bins = g->ppr_bins;
    t->update_split = g->update_split;
    t->wave_degree = g->wave_degree;
    t->update_locate = g->update_locate;
    return BINGO_OK;
}

int bingo_last_phase_ms(bingo_graph* g, float* h_ms, uint32_t cap, uint32_t* h_n) {
    if (!g || !h_n) return BINGO_E_INVALID;  // a pending histogram records no phase: no wait
    const uint32_t n = g->nev > 1 ? g->nev - 1 : 0;
    *h_n = n;
    if (!h_ms) return BINGO_OK;
    if (cap < n) return BINGO_E_CAPACITY;
    if (n) HIPCHK(hipEventSynchronize(g->ev[n]));
    for (uint32_t i = 0; i < n; ++i) HIPCHK(hipEventElapsedTime(&h_ms[i], g->ev[i], g->ev[i + 1]));
    return BINGO_OK;
}

void bingo_destroy(bingo_graph* g) {
    if (!g) return;
    hipDeviceSynchronize();
    release(g);
}

const char* bingo_strerror(int code) {
    switch (code) {
        case BINGO_OK: return "ok";
        case BINGO_E_INVALID: return "invalid argument";
        case BINGO_E_RANGE: return "vertex id out of range";
        case BINGO_E_WEIGHT: return "zero edge weight";
        case BINGO_E_OOM: return "device memory pool exhausted";
        case BINGO_E_CAPACITY: return "output buffer too small";
        case BINGO_E_HIP: return "HIP runtime error";
        case BINGO_E_INTERNAL: return "internal consistency check failed";
        default: return "unknown error";
    }
}

}  // extern "C"

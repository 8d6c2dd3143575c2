/*
 * bingo.h -- C ABI of the MI355X implementation of radix-based bias
 * factorization for random walks on dynamic graphs (Bingo, arXiv 2504.10233).
 *
 * Plain C: no HIP or torch types appear here.  Streams are passed as void*
 * (a hipStream_t, or NULL for the default stream).  Pointers named d_* are
 * device pointers; h_* are host pointers.  Every call is asynchronous on the
 * given stream unless its comment says it synchronizes.
 *
 * Errors.  Calls return 0 (BINGO_OK) or a negative code.  Argument errors
 * (null pointers, sizes out of range) and device-pool exhaustion are reported
 * synchronously and leave the graph unchanged.  Data errors found on the
 * device (a vertex id >= n, a zero weight) make the whole call a no-op; they
 * are returned by the calls that synchronize and by bingo_status().
 *
 * Ownership.  Input and output buffers belong to the caller and must stay
 * valid until the stream work that uses them has finished.  A bingo_graph owns
 * all of its device memory and releases it in bingo_destroy().
 *
 * Concurrency.  A handle is not thread-safe.  bingo_walk and bingo_walk_batch
 * calls may overlap each other on different streams, any number of them: each
 * call takes one of 64 per-handle counter slots in turn, and when the call that
 * held its slot last ran on another stream and has not finished, the new call's
 * stream first waits for it (so more than 64 calls in flight on distinct
 * streams serialize in part, but never share counters).  bingo_update_batch,
 * bingo_update_stream, bingo_ppr and bingo_node2vec must not overlap any other
 * call on the same handle.
 *
 * Determinism.  Results are a pure function of (graph version, inputs, seed,
 * walk id base); they do not depend on stream, launch shape or timing.
 */
#ifndef BINGO_H
#define BINGO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BINGO_OK = 0,
    BINGO_E_INVALID = -1,   /* null pointer, zero or oversized count, bad config */
    BINGO_E_RANGE = -2,     /* a vertex id >= n (device-detected) */
    BINGO_E_WEIGHT = -3,    /* a zero weight (device-detected) */
    BINGO_E_OOM = -4,       /* the device pool cannot hold the result */
    BINGO_E_CAPACITY = -5,  /* a caller-supplied output buffer is too small */
    BINGO_E_HIP = -6,       /* a HIP runtime call failed */
    BINGO_E_INTERNAL = -7   /* a consistency check of the library's own bookkeeping failed */
};

/* Group types of the adaptive representation (Sec. 5.1, Eq. eq:group). */
enum { BINGO_T_EMPTY = 0, BINGO_T_ONE = 1, BINGO_T_DENSE = 2, BINGO_T_SPARSE = 3, BINGO_T_REGULAR = 4 };

/* Walk execution forms: one persistent launch that keeps each walk in a
 * thread until it ends (default), or one launch per step over all walks (the
 * step-by-step form of the paper's Sec. 6, item iii). */
enum { BINGO_WALK_PERSISTENT = 0, BINGO_WALK_PER_STEP = 1 };

typedef struct bingo_graph bingo_graph;

typedef struct {
    uint32_t struct_size;   /* sizeof(bingo_config) */
    uint32_t adaptive;      /* 1: group adaption (Sec. 5.1); 0: every non-empty group regular */
    uint32_t alpha_pct;     /* dense threshold alpha in percent (paper: 40) */
    uint32_t beta_pct;      /* sparse threshold beta in percent (paper: 10) */
    uint64_t pool_bytes;    /* device arena for adjacency and group lists; 0 = sized by the library
                               (twice the input plus 16 MB, doubled by bingo_update_batch when a
                               batch does not fit even after compaction); otherwise a fixed size */
    uint32_t frac_bits;     /* 0: integer biases.  F in 1..16: every weight is a fixed-point bias with
                               F fraction bits (Sec. 4.3, see bingo_quantize_biases): bits F..31 are
                               its integer part, decomposed into radix groups F..31; a nonzero
                               fraction (weight mod 2^F) puts the edge in the decimal group, kept in
                               slot 0 with total sum(fraction); slots 1..F-1 stay empty.  A walk step
                               draws r in [0, sum of weights), takes the integer groups in ascending
                               k and the decimal group last; inside the decimal group a candidate
                               (from its list, or the whole adjacency when it is dense) is accepted
                               when the top F bits of the next random word are below its fraction. */
    uint32_t alias_table;   /* 0: inter-group choice by inverse transform over the groups in ascending k
                               (default).  1: by an alias table over the 32 groups, as the paper
                               prints it (Sec. 4.1): slot j = top 5 bits of the next random word,
                               x = below64(W), group j if x < cut_j else alias_j, with an exact
                               integer Walker/Vose table (512 B per vertex beside the header,
                               rebuilt for every vertex an update touches).  Integer biases only
                               (frac_bits must be 0). */
    uint32_t radix_base;    /* 0 or 2: the method's power-of-two groups.  4: radix base 4
                               (Supplement S.2): a weight is read as base-4 digits d_k (k = 0..15) and
                               group k splits into subgroups s = 3k + v - 1 of the edges whose digit k
                               is v = 1..3, each member carrying v 4^k; a step takes the first
                               subgroup in ascending s with r < sum of c_s v 4^k (r = below64(W)),
                               then a member by the subgroup's type from (c_s, d) under the rule of
                               Sec. 5.1 (dense: i = below32(d) until digit k of w_i is v).  A static
                               structure: bingo_walk (persistent form), bingo_export /
                               bingo_export_range (base-4 dump layout, see bingo_export),
                               bingo_memory, bingo_status, tuning and bingo_destroy; every other call
                               returns BINGO_E_INVALID.  Integer biases only, no alias table. */
    uint32_t reserved;      /* 0 */
} bingo_config;

typedef struct {
    uint64_t inserted;          /* insert records applied */
    uint64_t deleted;           /* delete records that removed an edge */
    uint64_t not_found;         /* delete records with no live matching edge */
    uint64_t touched_vertices;  /* vertices with at least one record */
    uint64_t transitions[25];   /* [old*5 + new] group-type changes over all groups of touched vertices */
    uint64_t match_scanned;     /* entries read to locate the deletes: locator slots probed and the
                                   inserts of vertices with deletes (with update_locate = 0: their live
                                   edges and inserts, scanned) */
    uint64_t match_candidates;  /* entries whose dst is among their vertex's delete targets */
} bingo_update_stats;

typedef struct {
    uint64_t vertices, edges;
    uint64_t pool_bytes, pool_used_bytes, pool_garbage_bytes;
    uint64_t header_bytes;          /* per-vertex inter-group sampling space */
    uint64_t adjacency_bytes;       /* live edges: dst, weight, seq (12 B each) */
    uint64_t adjacency_reserved_bytes;
    uint64_t list_bytes;            /* live entries of listed (sparse + regular) groups */
    uint64_t list_reserved_bytes;
    uint64_t groups_by_type[5];     /* number of groups per type */
    uint64_t model_ga_bytes;        /* paper's memory model with adaption (Sec. 5.1) */
    uint64_t model_bs_bytes;        /* ... and without (all regular, Sec. 6.2) */
    uint64_t alias_bytes;           /* inter-group alias rows (alias_table = 1): 512 B per vertex, else 0 */
    uint64_t index_bytes;           /* live group indexes (Sec. 4.2, 5.1): 4 d per regular group, 4 |S(u)|
                                       per sparse group and for S(u) itself */
    uint64_t index_reserved_bytes;  /* their capacities in the pool (list_reserved_bytes counts the lists) */
    uint64_t locator_bytes;         /* edge locator of bingo_update_batch (16 B per slot; 0 when none) */
} bingo_mem_stats;

/*
 * bingo_build -- build the dynamic graph and its sampling space from COO edges
 * (Sec. 4.1 sampling-space construction: Eq. eq:dwi decomposition, Eq. eq:wpk
 * group totals; Sec. 5.1 group adaption).
 *   n           number of vertices, 1 <= n < 2^31.
 *   m           number of edges, m < 2^32.
 *   d_src, d_dst, d_w   m device uint32 each; weights must be >= 1.
 * The edges of vertex u keep their input order; an edge's sequence number is
 * its rank among u's edges.  Synchronizes the stream.  Returns BINGO_E_RANGE or
 * BINGO_E_WEIGHT (and no graph) for bad input.  *out receives the handle.
 */
int bingo_build(const bingo_config* cfg, uint32_t n, uint64_t m,
                const uint32_t* d_src, const uint32_t* d_dst, const uint32_t* d_w,
                void* stream, bingo_graph** out);

/*
 * bingo_quantize_biases -- floating-point biases as stored weights (Sec. 4.3:
 * amortization factor lambda, integer and decimal parts).
 *   d_bias      m device float32 biases.
 *   lambda      the amortization factor (> 0, finite).
 *   frac_bits   F, 1..16: fraction bits kept (resolution 2^-F of lambda * b).
 *   d_w         m device uint32 outputs: floor(lambda * b * 2^F), with lambda * b
 *               one IEEE double product rounded to nearest; 0 where that is not
 *               a number in [1, 2^32) (negative, not finite, too small or too
 *               large), which bingo_build / bingo_update_batch then reject as a
 *               zero weight.
 * Build the graph with bingo_config.frac_bits = F.  Asynchronous.
 */
int bingo_quantize_biases(uint64_t m, const float* d_bias, double lambda, uint32_t frac_bits, uint32_t* d_w,
                          void* stream);

/*
 * bingo_update_batch -- apply one batch of edge insertions and deletions
 * (Sec. 5.2 parallel batched updates; Sec. 4.2 insertion and deletion).
 * All insertions are applied first, then all deletions, then one rebuild per
 * touched vertex.  Inserts of a vertex are appended in batch order.  A delete
 * record (s, t) removes the live edge s->t with the smallest sequence number
 * (the earliest version); records with no live match are counted in
 * not_found.  Deleted entries are removed from the adjacency and from every
 * listed group by the two-phase delete-and-swap (Fig. 10b), holes and tail
 * survivors paired in ascending order.  Types are recomputed from the new
 * counts; groups that change to a listed type get a fresh ascending list.
 *   d_ins_*     n_ins device uint32 each (weights >= 1).
 *   d_del_*     n_del device uint32 each.
 *   h_stats     optional; filled after the call (the call synchronizes).
 * The records are staged into a workspace of the batch's power-of-two size
 * bucket (at least 1024 records); the pipeline reads every count from device
 * memory, so one captured hipGraph per bucket serves every batch of that
 * bucket (bingo_tuning.update_graphs).  The library allocates a bucket's
 * workspace at its first use and keeps it with the handle.
 * When the pool cannot hold the batch's new blocks and holds blocks that
 * earlier batches replaced (pool_garbage_bytes > 0), the call compacts the pool
 * once (bingo_compact at the current size) and runs the batch again; if it
 * still does not fit and the library sized the pool (bingo_config.pool_bytes =
 * 0), it compacts into an arena twice the size (at most 2^37 bytes) and runs the
 * batch again.
 * Returns BINGO_E_RANGE / BINGO_E_WEIGHT (batch not applied), BINGO_E_OOM
 * (pool or workspace too small even after compaction; batch not applied),
 * BINGO_E_INVALID (more than 2^31 records) or BINGO_E_CAPACITY (delete
 * matching kept overflowing its candidate buffer; batch not applied).
 */
int bingo_update_batch(bingo_graph* g, uint64_t n_ins, const uint32_t* d_ins_src,
                       const uint32_t* d_ins_dst, const uint32_t* d_ins_w,
                       uint64_t n_del, const uint32_t* d_del_src, const uint32_t* d_del_dst,
                       void* stream, bingo_update_stats* h_stats);

/*
 * bingo_update_stream -- streaming updates (Sec. 4.2 insertion and deletion):
 * n records applied one at a time in the given order; record i has exactly the
 * meaning of a bingo_update_batch call that holds that record alone, so inserts
 * and deletes may interleave and a delete sees every earlier record.
 *   d_op        n device uint32: 0 insert (d_src[i], d_dst[i], d_w[i]), 1 delete
 *               of the live edge d_src[i] -> d_dst[i] with the smallest sequence
 *               number (d_w[i] ignored; not found is counted, not an error).
 *   d_src, d_dst, d_w   n device uint32 each (weights of inserts >= 1).
 *   h_stats     optional: inserted / deleted / not_found / transitions summed over
 *               the records (as the batches of one would report them);
 *               touched_vertices = distinct sources; match_scanned / match_candidates
 *               = adjacency entries scanned by deletes and those with the target dst.
 * The records of one source are applied by one wave in order, different
 * sources in parallel; a delete scans the vertex's adjacency and the lists of
 * the groups it touches.  Synchronizes the stream.  Returns BINGO_E_RANGE (an
 * id >= n or an op other than 0/1) or BINGO_E_WEIGHT (a zero insert weight)
 * with nothing applied.  When the pool cannot hold a record's new blocks, that
 * source stops before the record and the other sources continue; then, if the
 * pool holds blocks that earlier updates replaced or the library sized it
 * (bingo_config.pool_bytes = 0), the call compacts it (into an arena twice the
 * size for a library-sized pool) and applies the records not yet applied, in
 * their order; this repeats, at most 8 times, while a pass runs out.  Records
 * of different sources are independent, so the result is that of the whole
 * stream.  BINGO_E_OOM if a source still runs out: it keeps the records before
 * the failing one (the structure is consistent).  On BINGO_OK every record was applied exactly once
 * (inserted + deleted + not_found = n, checked on the host; BINGO_E_INTERNAL
 * otherwise).
 */
int bingo_update_stream(bingo_graph* g, uint64_t n, const uint32_t* d_op, const uint32_t* d_src,
                        const uint32_t* d_dst, const uint32_t* d_w, void* stream, bingo_update_stats* h_stats);

/*
 * bingo_walk -- biased first-order walks of fixed length (DeepWalk, Sec. 2.2).
 * Walk j has id walk_id_base + j and starts at d_starts[j]; step s of that walk
 * draws from the Philox-4x32-10 stream keyed by (seed, id, s).  Each step picks
 * a group with probability c_k 2^k / W (Eq. eq:group_prob) and then a member
 * uniformly (Eq. eq:pvp), by rejection on the adjacency for dense groups.
 *   d_paths        n_walks * (length + 1) uint32, row-major; entry 0 is the
 *                  start; after a vertex without out-edges the rest is
 *                  0xFFFFFFFF.
 *   d_steps_taken  optional, one uint64 that receives the transitions taken
 *                  (overwritten, not accumulated).
 *   mode           BINGO_WALK_PERSISTENT or BINGO_WALK_PER_STEP.
 * Start ids >= n give BINGO_E_RANGE at the next synchronizing call and the
 * paths are left unspecified.
 */
int bingo_walk(const bingo_graph* g, uint64_t n_walks, const uint32_t* d_starts,
               uint64_t walk_id_base, uint32_t length, uint64_t seed,
               uint32_t* d_paths, uint64_t* d_steps_taken, uint32_t mode, void* stream);

/*
 * bingo_walk_noalloc -- bingo_walk in the persistent form, for callers that
 * cannot allocate: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid allocation.  It makes no allocation of any kind (no
 * device or host memory, no events, no library routine that allocates), and
 * launches only kernels (no memset or copy nodes).
 *   Arguments and results are those of bingo_walk(g, n_walks, d_starts,
 *   walk_id_base, length, seed, d_paths, d_steps_taken, BINGO_WALK_PERSISTENT,
 *   stream): the same paths and transition count, bit for bit.
 *   Scratch: the kernels' work-queue head and transition counter live in a
 *   fixed 256-byte device array of the library, one per GPU, held until the
 *   process ends; its size does not depend on n_walks or length, so no input
 *   size is refused for it.  Its device address is looked up once per GPU, at
 *   the first call made with that GPU current.  Each call clears it on the
 *   stream before use.
 *   Concurrency: every call on one GPU shares that array, so calls that
 *   overlap on one GPU (on different streams or threads) race and give wrong
 *   paths and counts; serialize them (one stream, or events).
 * BINGO_E_INVALID for a null handle, a null d_starts or d_paths with
 * n_walks > 0, or a length of 0xFFFFFFFF; BINGO_E_HIP if the device address
 * lookup or a launch fails.  Start ids >= n as in bingo_walk.
 */
int bingo_walk_noalloc(const bingo_graph* g, uint64_t n_walks, const uint32_t* d_starts,
                       uint64_t walk_id_base, uint32_t length, uint64_t seed,
                       uint32_t* d_paths, uint64_t* d_steps_taken, void* stream);

/* One DeepWalk query of a batch: the arguments of one bingo_walk call. */
typedef struct {
    uint64_t n_walks;
    const uint32_t* d_starts;    /* n_walks device uint32 */
    uint64_t walk_id_base;
    uint32_t length;             /* transitions per walk */
    uint32_t reserved;           /* 0 */
    uint64_t seed;
    uint32_t* d_paths;           /* n_walks * (length + 1) device uint32 */
    uint64_t* d_steps_taken;     /* optional, one device uint64 */
} bingo_walk_query;

#define BINGO_WALK_BATCH_MAX 32

/*
 * bingo_walk_batch -- several DeepWalk queries (Sec. 2.2) in one persistent
 * launch: one device work queue over all their walks, so small queries do not
 * each pay a launch and a partly idle GPU (the serving loop merges the queries
 * waiting for a slot this way).  Query i's paths and step count are exactly
 * those of bingo_walk(g, q.n_walks, q.d_starts, q.walk_id_base, q.length,
 * q.seed, q.d_paths, q.d_steps_taken, BINGO_WALK_PERSISTENT): every walk is
 * keyed by its own query's (seed, id).
 *   n_queries   0..BINGO_WALK_BATCH_MAX.
 *   h_queries   host array of n_queries descriptors (read during the call).
 * Asynchronous on the stream.  BINGO_E_INVALID for a bad count, a descriptor
 * with n_walks > 0 and a null pointer, or a length of 0xFFFFFFFF; start ids >= n
 * as in bingo_walk.
 */
int bingo_walk_batch(const bingo_graph* g, uint32_t n_queries, const bingo_walk_query* h_queries, void* stream);

/*
 * bingo_node2vec -- second-order walks (Sec. 2.2, Eq. node2vec): from u, having
 * come from w, the walk moves to v with probability proportional to
 * w_uv * f(w, v), f = 1/p if v = w, 1 if the structure holds an edge w -> v,
 * 1/q otherwise.  Sampled by rejection on the first-order step (the approach
 * the paper adopts from KnightKing, Sec. 8): propose v as bingo_walk would,
 * accept with probability f / max(1/p, 1, 1/q).  The first transition of a
 * walk has no previous vertex and is first-order.
 *   Random words: proposal t of step s of walk id draws its first-order step
 *   from the Philox stream (seed, id, s) starting at block t * 2^16 (proposal
 *   0 is the bingo_walk step) and its acceptance word is word 0 of block
 *   t * 2^16 + 0xFFFF; it is accepted iff that word < floor(f / f_max * 2^32)
 *   (computed in IEEE double), without a draw when f = f_max.  So p = q = 1
 *   reproduces bingo_walk exactly.  A step stops the walk after 2^15
 *   rejected proposals (only reachable when a threshold is 0).
 *   d_starts, d_paths  as bingo_walk (paths n_walks * (length + 1)).
 *   d_counts           optional device uint64[2]: transitions, proposals.
 * The first call after the structure changed rebuilds the neighbour index
 * (a sorted copy of every vertex's destinations, 4 bytes per edge, kept with
 * the handle).  Asynchronous on the stream apart from that rebuild.
 * BINGO_E_INVALID for p or q not positive and finite.
 */
int bingo_node2vec(bingo_graph* g, uint64_t n_walks, const uint32_t* d_starts, uint64_t walk_id_base,
                   uint32_t length, double p, double q, uint64_t seed, uint32_t* d_paths, uint64_t* d_counts,
                   void* stream);

/*
 * bingo_ppr -- personalized PageRank by Monte-Carlo visit counts (Sec. 1 and
 * Sec. 6.1).  Source index q runs walks_per_source walks with ids
 * walk_id_base + q * walks_per_source + r.  The start counts as a visit;
 * before every transition the walk ends if the next word of its stream is
 * below term_threshold (= floor(p * 2^32) for termination probability p), at
 * a vertex without out-edges, or after max_len transitions.  The result is,
 * per source, the visited vertices in ascending order with their counts; it
 * stays in the handle until bingo_ppr_fetch or the next bingo_ppr.
 * Synchronizes; *h_total_entries receives the number of (vertex, count)
 * pairs and *h_total_steps (optional) the transitions taken.
 */
int bingo_ppr(bingo_graph* g, uint32_t n_sources, const uint32_t* d_sources,
              uint32_t walks_per_source, uint32_t term_threshold, uint32_t max_len,
              uint64_t seed, uint64_t walk_id_base, uint32_t mode,
              uint64_t* h_total_entries, uint64_t* h_total_steps, void* stream);

/*
 * bingo_ppr_async -- bingo_ppr in the persistent form whose visit histogram is
 * left running, so that it can overlap the next update batch (the histogram
 * reads only the visit bins, never the graph).  The walk phase runs on stream
 * and the call waits for it as bingo_ppr does; the histogram is then enqueued
 * on hist_stream (after the walk) and the call returns.  *h_total_steps
 * (optional) receives the transitions.  The result is complete once
 * bingo_ppr_wait returns; bingo_ppr_fetch waits for it by itself.  Until then
 * the handle accepts bingo_update_batch, which runs beside the histogram, and
 * bingo_ppr / bingo_ppr_async, whose walk waits for it on the device (its
 * result then gives way to the new query's); every other call on the handle
 * first waits for it on the host, except bingo_last_phase_ms, which reports
 * [walk-length bound pass, walk kernel] for it without waiting (the
 * histogram's time comes from bingo_ppr_wait).  When a bin overflows, the query reruns with exact
 * per-walk segments and finishes before returning.  Same results as bingo_ppr.
 * BINGO_E_INVALID as bingo_ppr.
 */
int bingo_ppr_async(bingo_graph* g, uint32_t n_sources, const uint32_t* d_sources,
                    uint32_t walks_per_source, uint32_t term_threshold, uint32_t max_len,
                    uint64_t seed, uint64_t walk_id_base, uint64_t* h_total_steps,
                    void* stream, void* hist_stream);

/*
 * bingo_ppr_wait -- wait for the histogram of the last bingo_ppr_async (no-op
 * after a synchronous bingo_ppr): *h_total_entries (optional) receives the
 * (vertex, count) pairs of the last result and *h_hist_ms (optional) the
 * histogram's device time (0 when there was none pending).
 */
int bingo_ppr_wait(bingo_graph* g, uint64_t* h_total_entries, float* h_hist_ms);

/*
 * bingo_ppr_fetch -- copy the last PPR result: d_offsets (n_sources + 1
 * uint64, CSR offsets per source), d_vertex and d_count (capacity uint32
 * each).  Returns BINGO_E_CAPACITY if capacity is below the entry count.
 */
int bingo_ppr_fetch(bingo_graph* g, uint64_t* d_offsets, uint32_t* d_vertex, uint32_t* d_count,
                    uint64_t capacity, void* stream);

/*
 * bingo_export -- canonical dump of the whole structure into host memory, as
 * little-endian uint32 words: for each vertex u ascending: d, next sequence
 * number, non-empty group mask, then (dst, weight, seq) for each neighbor
 * index, then for each non-empty group k ascending: k, type, count, followed
 * by the member index (one-element group) or the list in order (sparse and
 * regular groups).  With h_buf == NULL only *h_len (words) is set.
 * Synchronizes.  Returns BINGO_E_CAPACITY if cap_words is too small.
 * A radix-base-4 graph dumps, per vertex: d, the mask of non-empty subgroups
 * (subgroups 0..31, then 32..47: two words), (dst, weight) per neighbor index,
 * then for each non-empty subgroup s ascending: s, type, count, followed by the
 * member index or the list.
 */
int bingo_export(bingo_graph* g, uint32_t* h_buf, uint64_t cap_words, uint64_t* h_len, void* stream);

/*
 * bingo_export_range -- the same dump restricted to vertices [u_begin, u_end),
 * for sampled checks of large graphs.
 */
int bingo_export_range(bingo_graph* g, uint32_t u_begin, uint32_t u_end, uint32_t* h_buf, uint64_t cap_words,
                       uint64_t* h_len, void* stream);

/*
 * bingo_export_index_range -- the group indexes of vertices [u_begin, u_end)
 * (Sec. 4.2: the inverted index that maps a neighbor index to its position in
 * a group's list; Sec. 5.1: the reduced neighbor list S(u) of a vertex, the
 * ascending neighbor indices of its edges that belong to at least one sparse
 * group, over whose positions a sparse group keeps its smaller index).  Host
 * memory, little-endian uint32 words, for each vertex u ascending: |S(u)|,
 * then S(u); then for each sparse or regular group k ascending: k, followed
 * by, for a regular group, its index read at the list's members in list order
 * (index[L[p]] for p = 0..c-1, which is p for a consistent index), for a
 * sparse group, for each s < |S(u)|, the position of S[s] in the group's list
 * or 0xFFFFFFFF when S[s] is not a member.  The structures live in the pool
 * with the lists (bingo_mem_stats counts them); walks never read them.  With
 * h_buf == NULL only *h_len (words) is set.  Synchronizes.  BINGO_E_INVALID
 * for a bad range, BINGO_E_CAPACITY if cap_words is too small.
 */
int bingo_export_index_range(bingo_graph* g, uint32_t u_begin, uint32_t u_end, uint32_t* h_buf,
                             uint64_t cap_words, uint64_t* h_len, void* stream);

/*
 * bingo_compact -- pool compaction (the dynamic arrays of Sec. 5.2 grow by
 * moving to a block of twice the capacity; the old block is left behind as
 * garbage).  Every live block -- each vertex's adjacency block and the list
 * block of each listed group, at their capacities -- is copied into a fresh
 * arena in vertex order and the headers take the new offsets.  Capacities and
 * contents do not change, so neither does bingo_export nor any walk.
 *   pool_bytes  size of the new arena; 0 keeps the current size.  At most 2^37
 *               bytes (BINGO_E_INVALID above).
 * The new arena is allocated before the old one is freed, so both are held
 * during the copy.  Returns BINGO_E_OOM, with nothing changed, when the live
 * blocks do not fit pool_bytes or the allocation fails.  Synchronizes the
 * stream.  Must not overlap any other call on the handle.  bingo_update_batch
 * and bingo_update_stream call it by themselves when the pool is full.
 */
int bingo_compact(bingo_graph* g, uint64_t pool_bytes, void* stream);

/*
 * bingo_check_locator -- consistency of the edge locator of bingo_update_batch
 * (the update_locate tuning): *h_bad receives the number of live edges whose
 * (src, dst, neighbour index) has no slot, plus the difference between the
 * live slots and the live edges, plus one when the library's own count of live
 * slots is off; 0 means every live edge has exactly its slot.  *h_live
 * (optional) receives the live slots.  Synchronizes.  BINGO_E_INVALID for a
 * null handle or h_bad, a radix-base-4 graph, or no locator in step (none
 * built yet, or made stale by bingo_update_stream or a batch run without it).
 */
int bingo_check_locator(bingo_graph* g, uint64_t* h_bad, uint64_t* h_live, void* stream);

/* bingo_memory -- device memory by structure (synchronizes). */
int bingo_memory(bingo_graph* g, bingo_mem_stats* out, void* stream);

/* bingo_status -- sticky device-detected error of the last call (synchronizes), then cleared. */
int bingo_status(bingo_graph* g, void* stream);

/*
 * bingo_last_phase_ms -- device time of each phase of the last bingo_walk,
 * bingo_ppr, bingo_node2vec or bingo_update_batch call on this handle,
 * measured with HIP events recorded on that call's stream.  bingo_walk:
 * [walk kernel]; bingo_node2vec: [neighbour index rebuild, walk kernel];
 * bingo_ppr: [walk-length bound pass and scan, walk kernel, visit histogram];
 * bingo_update_batch: [the device pipeline of the batch, from the sort of its
 * records to the last mutation kernel; the graph launch when one is used].  *h_n
 * receives the number of phases; h_ms (capacity cap) may be NULL.
 * Synchronizes on the last event.
 */
int bingo_last_phase_ms(bingo_graph* g, float* h_ms, uint32_t cap, uint32_t* h_n);

/*
 * Launch tuning of the persistent walk kernels.  Results never depend on it
 * (walks are keyed by seed and walk id); only speed does.
 *   walk_variant     0: the lanes of a wave take each step together;
 *                    1: attempt-interleaved lanes (a lane still rejecting in a
 *                       dense group does not hold back lanes that are done).
 *   blocks_per_cu    resident 256-thread blocks per compute unit for the
 *                    persistent grid; 0 = as many as occupancy allows.
 *   queue_chunk      walk ids a wave takes per queue atomic (power of two,
 *                    16..4096); 0 = default (256).
 *   update_graphs    1: bingo_update_batch replays one captured hipGraph per
 *                    power-of-two batch-size bucket (default); 0: it launches
 *                    the same kernels one by one.
 *   dense_spec       dense-rejection attempts issued together per round (1, 2
 *                    or 4; 0 = default 2).  The attempt indices come from the
 *                    step's random stream alone, so a round's loads are
 *                    independent; the first accepting attempt in stream order
 *                    wins, and results do not depend on this value.
 *   ppr_bins         persistent bingo_ppr: 1 (default) appends each source's
 *                    visits to a bin of fixed capacity (one atomic per source
 *                    per wave iteration) and reruns the query with exact
 *                    per-walk segments if a bin overflows; 0 always uses the
 *                    segments (a length pass first).  Same results either way.
 *   update_split     bingo_update_batch: a touched vertex's passes over more
 *                    than this many entries (copying a grown adjacency, the
 *                    rename-and-fill pass over a kept list, building a fresh
 *                    list, finding a new one-element member) are split into
 *                    chunks spread over the GPU instead of running in the
 *                    vertex's wave.  0 = never split; otherwise at least 64;
 *                    default 4096.  Same results either way.
 *   wave_degree      attempt-interleaved walk kernels (walk_variant 1, used by
 *                    bingo_walk, bingo_ppr and the serving loop): a step whose
 *                    group is dense at a vertex of degree >= wave_degree is
 *                    served by the whole wave (wave per vertex: the rejection
 *                    attempts of one round drawn and loaded by 8 lanes at once,
 *                    the first accepting one in stream order taken by ballot)
 *                    instead of by its own lane (thread per walk).  0 (default)
 *                    = never.  Same results either way.
 *   update_locate    bingo_update_batch: 1 (default) finds the live edges a
 *                    delete names through the edge locator, a hash multiset of
 *                    the live edges keyed by (src, dst) that gives an edge's
 *                    neighbour index in a few probes (16 bytes per slot, at
 *                    least 1.6 slots per edge; built by the first batch that
 *                    needs it, kept in step by every batch, rebuilt after
 *                    bingo_update_stream or a batch run with 0); 0 scans the
 *                    adjacency of every source with deletes instead.  Same
 *                    results either way.
 */
typedef struct {
    uint32_t struct_size;
    uint32_t walk_variant;
    uint32_t blocks_per_cu;
    uint32_t queue_chunk;
    uint32_t update_graphs;
    uint32_t dense_spec;
    uint32_t ppr_bins;
    uint32_t update_split;
    uint32_t wave_degree;
    uint32_t update_locate;
} bingo_tuning;

int bingo_set_tuning(bingo_graph* g, const bingo_tuning* t);
int bingo_get_tuning(const bingo_graph* g, bingo_tuning* t);

/*
 * Serving loop.  A scheduler thread owned by the server keeps the graph
 * resident and runs requests in submission order, with these rules (the
 * paper's consistency rule, Sec. 6 item ii: a query sees exactly the update
 * batches submitted before it):
 *   - a walk query runs once every update batch submitted before it has been
 *     applied and a slot (one of max_inflight streams) and its device memory
 *     (counted against hbm_budget_bytes; 0 = unlimited) are free;
 *     admitted queries run concurrently;
 *   - an update batch runs once every query submitted before it has finished.
 * Requests are admitted first-in first-out.  Results equal those of the same
 * requests issued one by one through bingo_walk / bingo_update_batch.  The
 * graph handle must not be used directly while a server is attached to it.
 */
typedef struct bingo_server bingo_server;

typedef struct {
    uint32_t struct_size;       /* sizeof(bingo_server_config) */
    uint32_t max_inflight;      /* concurrent walk launches, 1..64 */
    uint64_t hbm_budget_bytes;  /* device bytes of admitted queries; 0 = no limit */
    uint32_t max_batch;         /* walk queries merged into one launch (bingo_walk_batch),
                                   0 or 1 = none, at most BINGO_WALK_BATCH_MAX */
    uint32_t reserved;          /* 0 */
} bingo_server_config;

typedef struct {
    uint32_t kind;              /* 0 walk query, 1 update batch */
    int32_t status;             /* BINGO_OK or an error code */
    uint64_t epoch;             /* update batches submitted before the request */
    double queue_us;            /* submission to start on the device */
    double latency_us;          /* submission to result ready */
    uint64_t steps;             /* transitions taken (walk query) */
    uint64_t path_words;        /* n_walks * (length + 1) (walk query) */
    uint64_t updates_applied;   /* inserted + deleted (update batch) */
    uint64_t updates_not_found; /* delete records without a live edge (update batch) */
} bingo_request_info;

/* bingo_server_create -- start the scheduler thread on a built graph. */
int bingo_server_create(bingo_graph* g, const bingo_server_config* cfg, bingo_server** out);

/*
 * bingo_server_submit_walk -- enqueue a DeepWalk query (same semantics as
 * bingo_walk); h_starts is copied before the call returns.  *ticket names the
 * request in bingo_server_wait.
 */
int bingo_server_submit_walk(bingo_server* s, uint64_t n_walks, const uint32_t* h_starts, uint32_t length,
                             uint64_t seed, uint64_t walk_id_base, uint64_t* ticket);

/* bingo_server_submit_update -- enqueue an update batch (same semantics as
 * bingo_update_batch); host arrays are copied before the call returns. */
int bingo_server_submit_update(bingo_server* s, uint64_t n_ins, const uint32_t* h_ins_src,
                               const uint32_t* h_ins_dst, const uint32_t* h_ins_w, uint64_t n_del,
                               const uint32_t* h_del_src, const uint32_t* h_del_dst, uint64_t* ticket);

/*
 * bingo_server_wait -- block until the request is done; a walk query's paths
 * (path_words uint32, row-major as in bingo_walk) are copied to h_paths when
 * it is non-NULL and cap_words suffices (else BINGO_E_CAPACITY and the request
 * stays available).  The ticket is released on return.  Returns the request's
 * status.
 */
int bingo_server_wait(bingo_server* s, uint64_t ticket, uint32_t* h_paths, uint64_t cap_words,
                      bingo_request_info* info);

/* bingo_server_destroy -- finish all submitted requests, stop the thread, free the server. */
int bingo_server_destroy(bingo_server* s);

/*
 * bingo_probe_random_reads -- measurement aid, not part of the method.  Times
 * one kernel of `lanes` threads that each read `reads` random lines of
 * `line_bytes` (64 or 128) from d_table, giving the random-line read rate this
 * device sustains (the ceiling that bounds the walk kernels, whose transitions
 * are short chains of dependent random line reads).
 *   d_table      device buffer of table_bytes bytes (at least 64 KiB, a
 *                multiple of line_bytes; contents arbitrary, only read).
 *   lanes        multiple of 256; reads a multiple of 4.
 *   dependent    0: a lane's addresses hash (seed, lane, read index), so each
 *                lane keeps 4 reads in flight; 1: each address also hashes the
 *                previous line's content (one pointer chase per lane).
 *   d_sink       lanes uint32 written (keeps the reads live).
 *   h_ms         receives the kernel time from HIP events on the stream.
 * Synchronizes.  BINGO_E_INVALID for a bad size or line width.
 */
int bingo_probe_random_reads(const void* d_table, uint64_t table_bytes, uint32_t lanes, uint32_t reads,
                             uint32_t dependent, uint32_t line_bytes, uint64_t seed, uint32_t* d_sink,
                             float* h_ms, void* stream);

/*
 * bingo_probe_replay -- measurement aid, not part of the method.  Replays a walk
 * query's visit stream over the graph's own header array and adjacency pool:
 * the access pattern of the walk kernels without their arithmetic, giving an
 * achievable rate for that pattern next to the uniform random-read probe.
 *   d_visits     n_visits device uint32 vertex ids in replay order (ids >= n
 *                are skipped); a chain of `chain` consecutive visits plays one
 *                walk, and lane l of `lanes` (a multiple of 256) takes chains
 *                l, l + lanes, ...
 *   per visit    the 64-byte header line of the vertex, then extra_x256 / 256
 *                (at most 64 on average) random adjacency entries of it, whose
 *                address depends on the header's adjacency offset.
 *   dependent    1: the next visit's address also depends on what was read
 *                (one chain of dependent reads per walk, as in the walk kernels);
 *                0: visits are independent (the pattern's ceiling).
 *   d_counters   two device uint64: [0] the lines read, [1] a checksum that
 *                keeps the reads live (both cleared first).
 *   h_ms         receives the kernel time from HIP events on the stream.
 * Synchronizes.  BINGO_E_INVALID for a null or radix-4 handle, a zero chain, a
 * bad lane count or extra_x256 above 64 * 256.
 */
int bingo_probe_replay(bingo_graph* g, const uint32_t* d_visits, uint64_t n_visits, uint32_t chain, uint32_t lanes,
                       uint32_t extra_x256, uint32_t dependent, uint64_t seed, unsigned long long* d_counters,
                       float* h_ms, void* stream);

/* bingo_num_vertices -- n of the handle. */
uint32_t bingo_num_vertices(const bingo_graph* g);

/* bingo_destroy -- release the handle and all its device memory. */
void bingo_destroy(bingo_graph* g);

/* bingo_strerror -- static description of a return code. */
const char* bingo_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* BINGO_H */

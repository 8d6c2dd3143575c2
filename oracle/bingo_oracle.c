/*
 * bingo_oracle.c -- plain, slow CPU oracle for radix-based bias factorization
 * (Bingo, arXiv 2504.10233).  TEST INFRASTRUCTURE ONLY: nothing on the GPU
 * product path links, loads or calls this file.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark use it.
 *
 * It computes, with every free choice of the paper fixed, exactly what the GPU
 * path must reproduce bit for bit:
 *   - Philox-4x32-10 counter-based stream keyed by (seed, walk id, step),
 *     written from its published description (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11);
 *   - exact bounded integer draws by Lemire's multiply-and-reject method
 *     ("Fast random integer generation in an interval", ACM TOMACS 2019);
 *   - radix decomposition of each weight into power-of-two groups (paper
 *     Sec. 4.1, Eq. eq:dwi) and the group totals W(p_k) = c_k * 2^k
 *     (Eq. eq:wpk);
 *   - group adaption into empty / one-element / dense / sparse / regular
 *     groups (Sec. 5.1, Eq. eq:group, alpha = 40, beta = 10);
 *   - the two-stage sampling step (Sec. 4.1, Eq. eq:group_prob and eq:pvp)
 *     with rejection on the adjacency for dense groups (Sec. 5.1); the
 *     inter-group choice by inverse transform or, as the paper prints it, by
 *     an alias table over the groups (Sec. 4.1);
 *   - floating-point biases (Sec. 4.3, Fig. SAMPLING2): scaling by the
 *     amortization factor lambda, an integer part decomposed into radix
 *     groups and a decimal part collected in one group sampled by rejection;
 *   - DeepWalk and personalized-PageRank walks (Sec. 2.2 and Sec. 6.1);
 *   - node2vec second-order walks by rejection on the first-order sampler
 *     (Sec. 2.2, Eq. node2vec; the KnightKing approach the paper adopts);
 *   - the batched update workflow: per vertex insert, then delete, then
 *     rebuild, oldest duplicate deleted first, two-phase parallel
 *     delete-and-swap (Sec. 5.2, Fig. 10);
 *   - a canonical little-endian dump of the whole structure and the memory
 *     model of Sec. 4.4 and Sec. 6.2.
 *
 * Readings where the paper is silent are listed at each function.  Loops are
 * plain; OpenMP is used only over independent walks (results do not depend on
 * the thread count because every walk writes only its own output).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

enum { T_EMPTY = 0, T_ONE = 1, T_DENSE = 2, T_SPARSE = 3, T_REGULAR = 4 };
enum { O_OK = 0, O_EINVAL = -1, O_ERANGE = -2, O_EWEIGHT = -3, O_ENOMEM = -4 };
#define STOPV 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (SC'11): two 32x32->64 multiplies per round, key bumped   */
/* by the Weyl constants between rounds, ten rounds.                         */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void o_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The random stream of one walk step.  key = (seed low, seed high); counter =
 * (walk low, walk high, step, block).  Words are taken in output order from
 * block 0, then block 1, ...  next64 = first word in the high half. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[3];
    uint32_t blk;
    uint32_t buf[4];
    int idx;
    uint64_t words;      /* words consumed (statistics only) */
} ostream;

static void st_init(ostream *s, uint64_t seed, uint64_t walk, uint32_t step) {
    s->key[0] = (uint32_t)seed; s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = (uint32_t)walk; s->ctr[1] = (uint32_t)(walk >> 32); s->ctr[2] = step;
    s->blk = 0; s->idx = 4; s->words = 0;
}

static uint32_t st_next32(ostream *s) {
    if (s->idx == 4) {
        uint32_t c[4] = {s->ctr[0], s->ctr[1], s->ctr[2], s->blk};
        o_philox(c, s->key, s->buf);
        s->blk++;
        s->idx = 0;
    }
    s->words++;
    return s->buf[s->idx++];
}

static uint64_t st_next64(ostream *s) {
    uint64_t hi = st_next32(s);
    uint64_t lo = st_next32(s);
    return (hi << 32) | lo;
}

void o_stream_words(uint64_t seed, uint64_t walk, uint32_t step, uint32_t nwords, uint32_t *out) {
    ostream s; st_init(&s, seed, walk, step);
    for (uint32_t i = 0; i < nwords; i++) out[i] = st_next32(&s);
}

/* ------------------------------------------------------------------------ */
/* Lemire's exact bounded draw, for a generic word width W (1..64 bits).    */
/* x is a W-bit word; m = x * n; l = m mod 2^W.  If l < n, the threshold    */
/* t = (2^W - n) mod n is computed and x is redrawn while l < t.  The result */
/* is m >> W, uniform on [0, n).  The 32- and 64-bit draws of the walk are   */
/* this same function with W = 32 and W = 64.                                */
/* ------------------------------------------------------------------------ */
typedef uint64_t (*word_fn)(void *ctx);

static uint64_t below_bits(uint64_t n, int W, word_fn next, void *ctx) {
    u128 two_w = (u128)1 << W;
    u128 mask = two_w - 1;
    u128 x = next(ctx);
    u128 m = x * n;
    u128 l = m & mask;
    if (l < n) {
        u128 t = (two_w - n) % n;
        while (l < t) {
            x = next(ctx);
            m = x * n;
            l = m & mask;
        }
    }
    return (uint64_t)(m >> W);
}

static uint64_t wf32(void *ctx) { return st_next32((ostream *)ctx); }
static uint64_t wf64(void *ctx) { return st_next64((ostream *)ctx); }

static uint32_t st_below32(ostream *s, uint32_t n) { return (uint32_t)below_bits(n, 32, wf32, s); }
static uint64_t st_below64(ostream *s, uint64_t n) { return below_bits(n, 64, wf64, s); }

/* Test hook: a draw from a caller-supplied list of W-bit words.  Past the end of
 * the list the all-ones word is returned: (2^W - 1) n mod 2^W = 2^W - n is never
 * below the threshold (2^W - n) mod n, so the draw always ends. */
typedef struct { const uint64_t *w; uint64_t n, i; int overrun; int W; } wordlist;
static uint64_t wf_list(void *ctx) {
    wordlist *l = (wordlist *)ctx;
    if (l->i >= l->n) { l->overrun = 1; return l->W >= 64 ? UINT64_MAX : (1ull << l->W) - 1; }
    return l->w[l->i++];
}
/* Returns the draw; *consumed = words used, or UINT64_MAX if the list ran out. */
uint64_t o_below_bits_words(uint64_t n, int W, const uint64_t *words, uint64_t nwords, uint64_t *consumed) {
    wordlist l = {words, nwords, 0, 0, W};
    uint64_t r = below_bits(n, W, wf_list, &l);
    *consumed = l.overrun ? UINT64_MAX : l.i;
    return r;
}

/* Test hook: draw once from every single W-bit word x in [0, 2^W) (W <= 24); counts[v] gets the
 * number of words accepted with result v, and the number of rejected words is returned. */
uint64_t o_below_bits_all_words(uint64_t n, int W, uint64_t *counts) {
    uint64_t rejected = 0;
    for (uint64_t x = 0; x < (1ull << W); x++) {
        uint64_t used;
        uint64_t v = o_below_bits_words(n, W, &x, 1, &used);
        if (used == UINT64_MAX) rejected++;
        else counts[v]++;
    }
    return rejected;
}

uint32_t o_below32(uint64_t seed, uint64_t walk, uint32_t step, uint32_t n) {
    ostream s; st_init(&s, seed, walk, step); return st_below32(&s, n);
}
uint64_t o_below64(uint64_t seed, uint64_t walk, uint32_t step, uint64_t n) {
    ostream s; st_init(&s, seed, walk, step); return st_below64(&s, n);
}

/* ------------------------------------------------------------------------ */
/* Group adaption (Sec. 5.1, Eq. eq:group).  The printed cases overlap; the  */
/* reading fixed here is a precedence, first match wins, with strict integer */
/* comparisons: c = 0 empty; c = 1 one-element; 100c > alpha*d dense;         */
/* 100c < beta*d sparse; otherwise regular.  Without adaption (the paper's   */
/* "BS" baseline, Sec. 6.2) every non-empty group is regular.                 */
/* ------------------------------------------------------------------------ */
int o_type(uint64_t c, uint64_t d, int adaptive, uint32_t alpha, uint32_t beta) {
    if (c == 0) return T_EMPTY;
    if (!adaptive) return T_REGULAR;
    if (c == 1) return T_ONE;
    if (100 * c > (uint64_t)alpha * d) return T_DENSE;
    if (100 * c < (uint64_t)beta * d) return T_SPARSE;
    return T_REGULAR;
}
static int listed(int t) { return t == T_SPARSE || t == T_REGULAR; }

/* Inter-group selection by inverse transform over the groups in ascending
 * bit order (Eq. eq:group_prob): the smallest k with r < sum_{j<=k} c_j 2^j.
 * r must lie in [0, W). */
int o_pick_group(const uint32_t c[32], uint64_t r) {
    uint64_t acc = 0;
    for (int k = 0; k < 32; k++) {
        acc += (uint64_t)c[k] << k;
        if (r < acc) return k;
    }
    return -1;
}

/* Inter-group alias table (Sec. 4.1, Walker / Vose), exact in integers.  The
 * 32 slots are the 32 groups; every slot holds W units, group k owns 32 T_k
 * units in total (T_k its group total, W = sum T_k).  Readings fixed here:
 * the small groups (32 T_k < W) and the large ones (32 T_k >= W) are taken in
 * ascending k, each as a first-in first-out queue; the front small slot s
 * keeps 32 T_s of its own units and takes the rest, W - 32 T_s, from the
 * front large group l, which joins the back of the small queue once what it
 * has left drops below W; slots left over keep all W units.  A draw takes
 * slot j from the top 5 bits of the next word, then x = below64(W), and
 * selects j when x < cut[j], else alias[j].  Group k is then selected by
 * exactly 32 T_k of the 32 W (j, x) pairs. */
void o_alias_table(const uint64_t T[32], uint64_t cut[32], uint32_t alias[32]) {
    u128 W = 0, U[32];
    for (int k = 0; k < 32; k++) W += T[k];
    for (int k = 0; k < 32; k++) U[k] = (u128)T[k] * 32;
    int small[32], large[32], ns = 0, nl = 0, hs = 0, hl = 0;
    for (int k = 0; k < 32; k++) {
        if (U[k] < W) small[ns++] = k; else large[nl++] = k;
    }
    for (int k = 0; k < 32; k++) { cut[k] = (uint64_t)W; alias[k] = (uint32_t)k; }
    while (hs < ns && hl < nl) {
        const int sm = small[hs++], l = large[hl];
        cut[sm] = (uint64_t)U[sm];
        alias[sm] = (uint32_t)l;
        U[l] -= W - U[sm];
        if (U[l] < W) { hl++; small[ns++] = l; }
    }
}

/* Test hook: the group selected by slot j and value x. */
int o_alias_pick(const uint64_t T[32], uint32_t j, uint64_t x) {
    uint64_t cut[32]; uint32_t alias[32];
    o_alias_table(T, cut, alias);
    return x < cut[j] ? (int)j : (int)alias[j];
}

/* ------------------------------------------------------------------------ */
/* Graph state.                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t c;        /* members of the group */
    uint8_t type;
    uint32_t one;      /* member index of a one-element group */
    uint32_t *list;    /* member indices of a listed group */
    uint32_t len, cap;
} ogroup;

typedef struct {
    uint32_t d, cap, next_seq;
    uint32_t *dst, *w, *seq;
    ogroup g[32];
} ovtx;

typedef struct {
    uint32_t n;
    int adaptive;
    uint32_t alpha, beta;
    uint32_t fbits;    /* 0: integer biases; F > 0: fixed-point biases with F fraction bits */
    int alias;         /* 1: inter-group choice by the alias table instead of inverse transform */
    ovtx *v;
} ograph;

/* ------------------------------------------------------------------------ */
/* Floating-point biases (Sec. 4.3, Fig. SAMPLING2).  Readings fixed here:   */
/*  - a bias b becomes the stored weight floor(lambda * b * 2^F): lambda * b */
/*    is one IEEE double product rounded to nearest, the scaling by 2^F is   */
/*    exact; a result that is not finite, negative, zero or not below 2^32  */
/*    is stored as 0, which the build and the update reject as a bad weight; */
/*  - the integer part (bits F..31) is radix-decomposed like an integer     */
/*    bias: group k >= F holds the edges with bit k set, total c_k 2^k;     */
/*  - the decimal part q = weight mod 2^F puts the edge in the decimal group */
/*    (slot 0) when q > 0; the group's total is the sum of its q;           */
/*    slots 1..F-1 stay empty;                                               */
/*  - inter-group selection draws r in [0, W) (W = sum of the weights) and   */
/*    takes the integer groups in ascending k, the decimal group last;       */
/*  - inside the decimal group, by its type: the one member; or a candidate  */
/*    drawn uniformly from the list (listed types) or the whole adjacency   */
/*    (dense), accepted when the top F bits of the next word are below its  */
/*    q, else a new candidate (rejection with bound 2^F).                    */
/* With F = 0 everything reduces to the integer case.                        */
/* ------------------------------------------------------------------------ */
uint32_t o_quantize_one(float b, double lambda, uint32_t F) {
    double s = (double)b * lambda;
    if (!(s >= 0.0) || isinf(s)) return 0;
    double t = ldexp(s, (int)F);
    if (!(t < 4294967296.0)) return 0;
    return (uint32_t)t;
}

void o_quantize(uint64_t m, const float *b, double lambda, uint32_t F, uint32_t *out) {
    for (uint64_t i = 0; i < m; i++) out[i] = o_quantize_one(b[i], lambda, F);
}

/* Group membership word of a stored weight: bit k says "member of group k". */
static uint32_t mword(const ograph *G, uint32_t w) {
    if (!G->fbits) return w;
    uint32_t fm = (1u << G->fbits) - 1u;
    return (w & ~fm) | ((w & fm) ? 1u : 0u);
}

static void *xrealloc(void *p, size_t sz) {
    void *q = realloc(p, sz ? sz : 1);
    if (!q) { fprintf(stderr, "oracle: out of host memory\n"); abort(); }
    return q;
}

static void adj_reserve(ovtx *x, uint32_t need) {
    if (need <= x->cap) return;
    uint32_t c = x->cap ? x->cap : 1;
    while (c < need) c *= 2;
    x->dst = xrealloc(x->dst, (size_t)c * 4);
    x->w = xrealloc(x->w, (size_t)c * 4);
    x->seq = xrealloc(x->seq, (size_t)c * 4);
    x->cap = c;
}

static void list_push(ogroup *g, uint32_t v) {
    if (g->len == g->cap) {
        g->cap = g->cap ? 2 * g->cap : 4;
        g->list = xrealloc(g->list, (size_t)g->cap * 4);
    }
    g->list[g->len++] = v;
}

static void list_clear(ogroup *g) { free(g->list); g->list = NULL; g->len = g->cap = 0; }

/* Fresh structure of group k of vertex x from its adjacency: listed groups
 * hold the member indices in ascending order; a one-element group keeps its
 * single member; dense and empty groups keep nothing. */
static void group_fresh(const ograph *G, ovtx *x, int k) {
    ogroup *g = &x->g[k];
    list_clear(g);
    g->one = 0;
    if (g->type == T_ONE) {
        for (uint32_t i = 0; i < x->d; i++) if (mword(G, x->w[i]) >> k & 1u) { g->one = i; break; }
    } else if (listed(g->type)) {
        for (uint32_t i = 0; i < x->d; i++) if (mword(G, x->w[i]) >> k & 1u) list_push(g, i);
    }
}

static void vertex_recount(ograph *G, ovtx *x, uint32_t c[32]) {
    for (int k = 0; k < 32; k++) c[k] = 0;
    for (uint32_t i = 0; i < x->d; i++)
        for (int k = 0; k < 32; k++) c[k] += mword(G, x->w[i]) >> k & 1u;
}

static void vertex_fresh(ograph *G, ovtx *x) {
    uint32_t c[32];
    vertex_recount(G, x, c);
    for (int k = 0; k < 32; k++) {
        x->g[k].c = c[k];
        x->g[k].type = (uint8_t)o_type(c[k], x->d, G->adaptive, G->alpha, G->beta);
        group_fresh(G, x, k);
    }
}

void o_free(ograph *G) {
    if (!G) return;
    for (uint32_t u = 0; u < G->n; u++) {
        ovtx *x = &G->v[u];
        free(x->dst); free(x->w); free(x->seq);
        for (int k = 0; k < 32; k++) free(x->g[k].list);
    }
    free(G->v);
    free(G);
}

/* Build (a snapshot of the dynamic graph, Sec. 2.1).  Edges of vertex u keep
 * their input order; seq of an edge is its rank among u's edges, and the
 * per-vertex sequence counter starts at d. */
int o_build(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
            int adaptive, uint32_t alpha, uint32_t beta, uint32_t fbits, int alias, ograph **out) {
    *out = NULL;
    if (n == 0 || fbits > 16 || (alias && fbits)) return O_EINVAL;
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] >= n || dst[e] >= n) return O_ERANGE;
        if (w[e] == 0) return O_EWEIGHT;
    }
    ograph *G = calloc(1, sizeof(ograph));
    G->n = n; G->adaptive = adaptive; G->alpha = alpha; G->beta = beta; G->fbits = fbits; G->alias = alias;
    G->v = calloc(n, sizeof(ovtx));
    if (!G->v) { free(G); return O_ENOMEM; }
    uint32_t *deg = calloc(n, 4);
    for (uint64_t e = 0; e < m; e++) deg[src[e]]++;
    for (uint32_t u = 0; u < n; u++) adj_reserve(&G->v[u], deg[u]);
    free(deg);
    for (uint64_t e = 0; e < m; e++) {
        ovtx *x = &G->v[src[e]];
        x->dst[x->d] = dst[e]; x->w[x->d] = w[e]; x->seq[x->d] = x->d;
        x->d++;
    }
    for (uint32_t u = 0; u < n; u++) {
        G->v[u].next_seq = G->v[u].d;
        vertex_fresh(G, &G->v[u]);
    }
    *out = G;
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* One sampling step from vertex u (Sec. 4.1 two-stage sampling, Sec. 5.1    */
/* dense rejection).  Order of random words: the PPR termination word, then  */
/* the 64-bit group draw, then member draws.                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t steps, sel[5], dense_attempts, words;
} ostats;

static uint32_t step_from(const ograph *G, uint32_t u, ostream *s, int ppr, uint32_t thr, ostats *st) {
    const ovtx *x = &G->v[u];
    if (x->d == 0) return STOPV;
    if (ppr && st_next32(s) < thr) return STOPV;
    uint64_t W = 0;
    uint32_t c[32];
    int k;
    if (G->alias) {
        uint64_t T[32];
        for (int j = 0; j < 32; j++) { T[j] = (uint64_t)x->g[j].c << j; W += T[j]; }
        const uint32_t slot = st_next32(s) >> 27;
        const uint64_t r = st_below64(s, W);
        k = o_alias_pick(T, slot, r);
    } else if (!G->fbits) {
        for (int j = 0; j < 32; j++) { c[j] = x->g[j].c; W += (uint64_t)c[j] << j; }
        uint64_t r = st_below64(s, W);
        k = o_pick_group(c, r);
    } else {
        /* integer groups F..31 ascending, then the decimal group (slot 0) */
        const uint32_t F = G->fbits, fm = (1u << F) - 1u;
        for (uint32_t i = 0; i < x->d; i++) W += x->w[i];
        uint64_t r = st_below64(s, W), acc = 0;
        k = 0;
        for (int j = (int)F; j < 32; j++) {
            acc += (uint64_t)x->g[j].c << j;
            if (r < acc) { k = j; break; }
        }
        if (k == 0) {
            const ogroup *g = &x->g[0];
            uint32_t i;
            if (g->type == T_ONE) {
                i = g->one;
            } else {
                for (;;) {
                    i = listed(g->type) ? g->list[st_below32(s, g->c)] : st_below32(s, x->d);
                    if (st) st->dense_attempts++;
                    if ((st_next32(s) >> (32 - F)) < (x->w[i] & fm)) break;
                }
            }
            if (st) { st->steps++; st->sel[g->type]++; }
            return x->dst[i];
        }
    }
    const ogroup *g = &x->g[k];
    uint32_t i;
    if (g->type == T_ONE) {
        i = g->one;
    } else if (listed(g->type)) {
        i = g->list[st_below32(s, g->c)];
    } else { /* dense: rejection over the whole neighbor list */
        for (;;) {
            i = st_below32(s, x->d);
            if (st) st->dense_attempts++;
            if (x->w[i] >> k & 1u) break;
        }
    }
    if (st) { st->steps++; st->sel[g->type]++; }
    return x->dst[i];
}

/* Exported single step, for tests. */
uint32_t o_step(const ograph *G, uint32_t u, uint64_t seed, uint64_t walk, uint32_t step,
                int ppr, uint32_t thr) {
    ostream s; st_init(&s, seed, walk, step);
    return step_from(G, u, &s, ppr, thr, NULL);
}

/* Biased DeepWalk: walk j has id base + j, starts at starts[j], and takes up
 * to len transitions; step s of walk id uses the stream (seed, id, s).  The
 * path holds len + 1 entries; after a stop (a vertex without out-edges) the
 * rest is 0xFFFFFFFF.  Returns the number of transitions taken. */
uint64_t o_deepwalk(const ograph *G, uint64_t nwalks, const uint32_t *starts, uint64_t base,
                    uint32_t len, uint64_t seed, uint32_t *paths, int nthreads, uint64_t *stats_out) {
    uint64_t total = 0;
    uint64_t agg[8] = {0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        ostats st; memset(&st, 0, sizeof st);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
        for (int64_t j = 0; j < (int64_t)nwalks; j++) {
            uint32_t *p = paths + (uint64_t)j * (len + 1);
            uint32_t u = starts[j];
            p[0] = u;
            uint32_t s = 0;
            for (; s < len; s++) {
                ostream rs; st_init(&rs, seed, base + (uint64_t)j, s);
                uint32_t v = step_from(G, u, &rs, 0, 0, &st);
                if (v == STOPV) break;
                p[s + 1] = v;
                u = v;
            }
            for (; s < len; s++) p[s + 1] = STOPV;
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            total += st.steps;
            for (int t = 0; t < 5; t++) agg[t] += st.sel[t];
            agg[5] += st.dense_attempts;
        }
    }
    if (stats_out) for (int t = 0; t < 6; t++) stats_out[t] = agg[t];
    return total;
}

/* ------------------------------------------------------------------------ */
/* node2vec (Sec. 2.2, Eq. node2vec): the walker at u that came from w moves */
/* to neighbour v with probability proportional to w_uv * f(w, v), where     */
/* f = 1/p if v = w, 1 if w has an edge to v, 1/q otherwise.  The paper       */
/* samples it as KnightKing does (Sec. 8): propose v from the first-order     */
/* sampler at u and accept it with probability f(w, v) / max(1/p, 1, 1/q).   */
/* Readings fixed here:                                                       */
/*  - "distance 1" means an edge w -> v in the current (directed) structure;  */
/*  - the first transition of a walk has no previous vertex and is a plain    */
/*    first-order step;                                                       */
/*  - acceptance is an integer test: thr_c = 2^32 when f_c is the maximum     */
/*    (accept without a draw), else floor(f_c / f_max * 2^32) computed in     */
/*    IEEE double, and the proposal is accepted iff its acceptance word is    */
/*    below thr_c;                                                            */
/*  - proposal t of step s of walk id draws its first-order step from the     */
/*    stream (seed, id, s) starting at block t * 2^16, and its acceptance     */
/*    word is word 0 of block t * 2^16 + 0xFFFF; so proposal 0 uses exactly   */
/*    the DeepWalk stream of the step, and p = q = 1 gives the DeepWalk path; */
/*  - a step gives up after 2^15 proposals and the walk stops (unreachable    */
/*    unless some thr_c is 0).                                                */
/* ------------------------------------------------------------------------ */
#define N2V_MAX_PROPOSALS (1u << 15)

static void st_init_blk(ostream *s, uint64_t seed, uint64_t walk, uint32_t step, uint32_t blk0) {
    st_init(s, seed, walk, step);
    s->blk = blk0;
}

/* Edge w -> v present?  Plain scan of w's adjacency. */
static int has_edge(const ograph *G, uint32_t w, uint32_t v) {
    const ovtx *x = &G->v[w];
    for (uint32_t i = 0; i < x->d; i++)
        if (x->dst[i] == v) return 1;
    return 0;
}

/* Acceptance thresholds for classes distance 0, 1, 2; 2^32 means always. */
int o_node2vec_thresholds(double p, double q, uint64_t thr[3]) {
    if (!(p > 0.0) || !(q > 0.0)) return -1;
    const double f[3] = {1.0 / p, 1.0, 1.0 / q};
    double fmax = f[0];
    if (f[1] > fmax) fmax = f[1];
    if (f[2] > fmax) fmax = f[2];
    for (int c = 0; c < 3; c++) {
        if (f[c] == fmax) thr[c] = 1ull << 32;
        else {
            double t = (f[c] / fmax) * 4294967296.0;
            thr[c] = (uint64_t)t;  /* floor: t is positive and below 2^32 */
        }
    }
    return 0;
}

uint32_t o_node2vec_step(const ograph *G, uint32_t prev, uint32_t u, uint64_t seed, uint64_t id, uint32_t s,
                         const uint64_t thr[3], uint64_t *proposals) {
    for (uint32_t t = 0; t < N2V_MAX_PROPOSALS; t++) {
        ostream rs; st_init_blk(&rs, seed, id, s, t << 16);
        uint32_t v = step_from(G, u, &rs, 0, 0, NULL);
        if (proposals) (*proposals)++;
        if (v == STOPV) return STOPV;
        if (prev == STOPV) return v;
        int c = v == prev ? 0 : (has_edge(G, prev, v) ? 1 : 2);
        if (thr[c] >> 32) return v;
        ostream as; st_init_blk(&as, seed, id, s, (t << 16) | 0xFFFFu);
        if (st_next32(&as) < thr[c]) return v;
    }
    return STOPV;
}

/* Walk j has id base + j, starts at starts[j] and takes up to len transitions;
 * paths as in o_deepwalk.  Returns the transitions taken; *proposals_out
 * receives the number of proposals (first-order steps) drawn. */
uint64_t o_node2vec(const ograph *G, uint64_t nwalks, const uint32_t *starts, uint64_t base, uint32_t len,
                    uint64_t seed, double p, double q, uint32_t *paths, int nthreads, uint64_t *proposals_out) {
    uint64_t thr[3];
    if (o_node2vec_thresholds(p, q, thr)) return 0;
    uint64_t total = 0, props = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total, props)
#endif
    for (int64_t j = 0; j < (int64_t)nwalks; j++) {
        uint32_t *path = paths + (uint64_t)j * (len + 1);
        uint32_t u = starts[j], prev = STOPV;
        path[0] = u;
        uint32_t s = 0;
        for (; s < len; s++) {
            uint32_t v = o_node2vec_step(G, prev, u, seed, base + (uint64_t)j, s, thr, &props);
            if (v == STOPV) break;
            path[s + 1] = v;
            prev = u;
            u = v;
            total++;
        }
        for (; s < len; s++) path[s + 1] = STOPV;
    }
    if (proposals_out) *proposals_out = props;
    return total;
}

/* ------------------------------------------------------------------------ */
/* Personalized PageRank by Monte-Carlo visit counts.  For source index q   */
/* and walk r < R the walk id is base + q*R + r.  The start vertex counts as */
/* a visit; before every transition the walk stops if the next word of its  */
/* stream is below thr (thr = floor(p * 2^32) for termination probability p),*/
/* at a vertex without out-edges, or after cap transitions.  Every vertex    */
/* reached counts one visit.  The result per source is (vertex, count) pairs */
/* sorted by vertex.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t nsrc;
    uint64_t *off;
    uint32_t *vtx, *cnt;
    uint64_t total_steps;
    uint64_t sel[6];
} oppr;

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

oppr *o_ppr(const ograph *G, uint32_t nsrc, const uint32_t *sources, uint32_t R, uint32_t thr,
            uint32_t cap, uint64_t seed, uint64_t base, int nthreads) {
    oppr *P = calloc(1, sizeof(oppr));
    P->nsrc = nsrc;
    P->off = calloc((size_t)nsrc + 1, 8);
    uint32_t **hv = calloc(nsrc ? nsrc : 1, sizeof(uint32_t *));
    uint32_t **hc = calloc(nsrc ? nsrc : 1, sizeof(uint32_t *));
    uint64_t *hn = calloc(nsrc ? nsrc : 1, 8);
    uint64_t total = 0, agg[6] = {0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        ostats st; memset(&st, 0, sizeof st);
        uint32_t *vis = NULL; uint64_t vcap = 0;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t q = 0; q < (int64_t)nsrc; q++) {
            uint64_t nv = 0;
            for (uint32_t r = 0; r < R; r++) {
                uint64_t id = base + (uint64_t)q * R + r;
                uint32_t u = sources[q];
                if (nv + cap + 1 > vcap) { vcap = 2 * (nv + cap + 1); vis = xrealloc(vis, vcap * 4); }
                vis[nv++] = u;
                for (uint32_t s = 0; s < cap; s++) {
                    ostream rs; st_init(&rs, seed, id, s);
                    uint32_t v = step_from(G, u, &rs, 1, thr, &st);
                    if (v == STOPV) break;
                    vis[nv++] = v;
                    u = v;
                }
            }
            qsort(vis, nv, 4, cmp_u32);
            uint64_t distinct = 0;
            for (uint64_t i = 0; i < nv; i++) if (i == 0 || vis[i] != vis[i - 1]) distinct++;
            hv[q] = malloc(distinct * 4 + 4); hc[q] = malloc(distinct * 4 + 4);
            uint64_t o = 0;
            for (uint64_t i = 0; i < nv; i++) {
                if (i == 0 || vis[i] != vis[i - 1]) { hv[q][o] = vis[i]; hc[q][o] = 0; o++; }
                hc[q][o - 1]++;
            }
            hn[q] = distinct;
        }
        free(vis);
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            total += st.steps;
            for (int t = 0; t < 5; t++) agg[t] += st.sel[t];
            agg[5] += st.dense_attempts;
        }
    }
    for (uint32_t q = 0; q < nsrc; q++) P->off[q + 1] = P->off[q] + hn[q];
    uint64_t ne = P->off[nsrc];
    P->vtx = malloc(ne * 4 + 4); P->cnt = malloc(ne * 4 + 4);
    for (uint32_t q = 0; q < nsrc; q++) {
        memcpy(P->vtx + P->off[q], hv[q], hn[q] * 4);
        memcpy(P->cnt + P->off[q], hc[q], hn[q] * 4);
        free(hv[q]); free(hc[q]);
    }
    free(hv); free(hc); free(hn);
    P->total_steps = total;
    memcpy(P->sel, agg, sizeof agg);
    return P;
}

uint64_t o_ppr_entries(const oppr *P) { return P->off[P->nsrc]; }
uint64_t o_ppr_steps(const oppr *P) { return P->total_steps; }
void o_ppr_stats(const oppr *P, uint64_t out[6]) { memcpy(out, P->sel, sizeof P->sel); }
void o_ppr_fetch(const oppr *P, uint64_t *off, uint32_t *vtx, uint32_t *cnt) {
    uint64_t ne = P->off[P->nsrc];
    memcpy(off, P->off, ((size_t)P->nsrc + 1) * 8);
    memcpy(vtx, P->vtx, ne * 4);
    memcpy(cnt, P->cnt, ne * 4);
}
void o_ppr_free(oppr *P) { if (!P) return; free(P->off); free(P->vtx); free(P->cnt); free(P); }

/* ------------------------------------------------------------------------ */
/* Two-phase parallel delete-and-swap (Sec. 5.2, Fig. 10b).  Deleting N      */
/* entries from an array of length len: the tail window [len-N, len) is      */
/* handled first -- its deleted entries simply disappear -- and its          */
/* surviving entries fill the deleted positions in front of the window.     */
/* Reading fixed here: holes and tail survivors are paired by rank in        */
/* ascending position order.  del[] flags the entries to delete; on return   */
/* moved_from[j] / moved_to[j] (j < *nmoved) list the moves.                 */
/* ------------------------------------------------------------------------ */
static uint32_t two_phase(uint32_t *a, uint32_t len, const uint8_t *del,
                          uint32_t *moved_from, uint32_t *moved_to, uint32_t *nmoved) {
    uint32_t N = 0;
    for (uint32_t i = 0; i < len; i++) N += del[i];
    uint32_t newlen = len - N;
    uint32_t h = 0, s = newlen, nm = 0;
    for (;;) {
        while (h < newlen && !del[h]) h++;
        while (s < len && del[s]) s++;
        if (h >= newlen) break;
        /* a hole in front pairs with the next tail survivor */
        a[h] = a[s];
        if (moved_from) { moved_from[nm] = s; moved_to[nm] = h; }
        nm++;
        h++; s++;
    }
    if (nmoved) *nmoved = nm;
    return newlen;
}

/* Test hook: two-phase compaction of a u32 array in place. */
uint32_t o_two_phase(uint32_t *a, uint32_t len, const uint8_t *del) {
    return two_phase(a, len, del, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Batched update (Sec. 5.2).  All insertions of the batch, then all         */
/* deletions, then one rebuild per vertex.  Readings fixed here:             */
/*  - inserts of a vertex are appended in batch order, seq = next_seq++;     */
/*  - deleting edge (u, t) k times removes the k live occurrences of (u, t)  */
/*    with the smallest seq (the earliest version first), same-batch inserts */
/*    included; requests beyond the live occurrences are counted not_found; */
/*  - the adjacency is compacted with the two-phase rule, and moved indices  */
/*    are renamed in the lists;                                              */
/*  - a group that is listed and keeps the same type gets its new member     */
/*    indices appended in ascending order, then its deleted entries removed  */
/*    with the two-phase rule, then renames;                                 */
/*  - group types are a pure function of (c, d) after the batch; a group    */
/*    that becomes listed or switches between sparse and regular gets a      */
/*    fresh ascending list; a one-element group's member is recomputed.      */
/* stats: [0] inserted, [1] deleted, [2] not found, [3..27] 5x5 type         */
/* transitions old*5+new over every group of every touched vertex.           */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t dst, seq, idx; } occ;

static int cmp_occ(const void *a, const void *b) {
    const occ *x = a, *y = b;
    if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    return 0;
}

int o_update(ograph *G, uint64_t nI, const uint32_t *Isrc, const uint32_t *Idst, const uint32_t *Iw,
             uint64_t nD, const uint32_t *Dsrc, const uint32_t *Ddst, uint64_t *stats) {
    uint32_t n = G->n;
    for (uint64_t j = 0; j < nI; j++) {
        if (Isrc[j] >= n || Idst[j] >= n) return O_ERANGE;
        if (Iw[j] == 0) return O_EWEIGHT;
    }
    for (uint64_t j = 0; j < nD; j++)
        if (Dsrc[j] >= n || Ddst[j] >= n) return O_ERANGE;
    uint64_t st[28]; memset(st, 0, sizeof st);

    /* group the batch by vertex: a bucket of insert and delete positions */
    uint64_t *ic = calloc((size_t)n + 1, 8), *dc = calloc((size_t)n + 1, 8);
    for (uint64_t j = 0; j < nI; j++) ic[Isrc[j] + 1]++;
    for (uint64_t j = 0; j < nD; j++) dc[Dsrc[j] + 1]++;
    for (uint32_t u = 0; u < n; u++) { ic[u + 1] += ic[u]; dc[u + 1] += dc[u]; }
    uint64_t *ib = malloc(nI * 8 + 8), *db = malloc(nD * 8 + 8);
    uint64_t *ifill = calloc(n, 8), *dfill = calloc(n, 8);
    for (uint64_t j = 0; j < nI; j++) { uint32_t u = Isrc[j]; ib[ic[u] + ifill[u]++] = j; }
    for (uint64_t j = 0; j < nD; j++) { uint32_t u = Dsrc[j]; db[dc[u] + dfill[u]++] = j; }
    free(ifill); free(dfill);

    for (uint32_t u = 0; u < n; u++) {
        uint64_t ni = ic[u + 1] - ic[u], nd = dc[u + 1] - dc[u];
        if (ni == 0 && nd == 0) continue;
        ovtx *x = &G->v[u];
        uint8_t oldt[32];
        for (int k = 0; k < 32; k++) oldt[k] = x->g[k].type;
        uint32_t d0 = x->d;

        /* 1. inserts, appended in batch order */
        adj_reserve(x, (uint32_t)(x->d + ni));
        for (uint64_t a = 0; a < ni; a++) {
            uint64_t j = ib[ic[u] + a];
            x->dst[x->d] = Idst[j]; x->w[x->d] = Iw[j]; x->seq[x->d] = x->next_seq++;
            x->d++;
            st[0]++;
        }
        uint32_t d1 = x->d;

        /* 2. deletes: mark the oldest live occurrences */
        uint8_t *del = calloc(d1 ? d1 : 1, 1);
        if (nd) {
            uint32_t *tg = malloc(nd * 4);
            for (uint64_t a = 0; a < nd; a++) tg[a] = Ddst[db[dc[u] + a]];
            qsort(tg, nd, 4, cmp_u32);
            occ *oc = malloc((size_t)d1 * sizeof(occ) + sizeof(occ));
            uint32_t no = 0;
            for (uint32_t i = 0; i < d1; i++) {
                /* is dst_i among the delete targets?  binary search */
                uint64_t lo = 0, hi = nd;
                while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (tg[mid] < x->dst[i]) lo = mid + 1; else hi = mid; }
                if (lo < nd && tg[lo] == x->dst[i]) { oc[no].dst = x->dst[i]; oc[no].seq = x->seq[i]; oc[no].idx = i; no++; }
            }
            qsort(oc, no, sizeof(occ), cmp_occ);
            uint64_t a = 0; uint32_t o = 0;
            while (a < nd) {
                uint32_t t = tg[a];
                uint64_t kt = 0;
                while (a < nd && tg[a] == t) { kt++; a++; }
                while (o < no && oc[o].dst < t) o++;
                uint64_t taken = 0;
                while (o < no && oc[o].dst == t && taken < kt) { del[oc[o].idx] = 1; taken++; o++; }
                while (o < no && oc[o].dst == t) o++;
                st[1] += taken;
                st[2] += kt - taken;
            }
            free(tg); free(oc);
        }

        /* new counts and types after the batch */
        uint32_t nc[32]; uint8_t newt[32];
        uint32_t N = 0;
        for (uint32_t i = 0; i < d1; i++) N += del[i];
        uint32_t d2 = d1 - N;
        for (int k = 0; k < 32; k++) nc[k] = 0;
        for (uint32_t i = 0; i < d1; i++) if (!del[i]) for (int k = 0; k < 32; k++) nc[k] += mword(G, x->w[i]) >> k & 1u;
        for (int k = 0; k < 32; k++) newt[k] = (uint8_t)o_type(nc[k], d2, G->adaptive, G->alpha, G->beta);

        /* 3. kept listed groups: append the new member indices, ascending */
        for (int k = 0; k < 32; k++) {
            if (!(listed(oldt[k]) && newt[k] == oldt[k])) continue;
            for (uint32_t i = d0; i < d1; i++) if (mword(G, x->w[i]) >> k & 1u) list_push(&x->g[k], i);
        }

        /* 4. two-phase delete-and-swap on the adjacency; rho maps moved indices */
        uint32_t *perm = malloc((size_t)d1 * 4 + 4);
        for (uint32_t i = 0; i < d1; i++) perm[i] = i;
        uint32_t *mf = malloc((size_t)d1 * 4 + 4), *mt = malloc((size_t)d1 * 4 + 4), nm = 0;
        two_phase(perm, d1, del, mf, mt, &nm);
        uint32_t *rho = malloc((size_t)d1 * 4 + 4);
        for (uint32_t i = 0; i < d1; i++) rho[i] = i;
        for (uint32_t j = 0; j < nm; j++) {
            rho[mf[j]] = mt[j];
            x->dst[mt[j]] = x->dst[mf[j]]; x->w[mt[j]] = x->w[mf[j]]; x->seq[mt[j]] = x->seq[mf[j]];
        }
        x->d = d2;

        /* 5. kept listed groups: two-phase on the list, then rename */
        for (int k = 0; k < 32; k++) {
            if (!(listed(oldt[k]) && newt[k] == oldt[k])) continue;
            ogroup *g = &x->g[k];
            uint8_t *ld = calloc(g->len ? g->len : 1, 1);
            for (uint32_t p = 0; p < g->len; p++) ld[p] = del[g->list[p]];
            g->len = two_phase(g->list, g->len, ld, NULL, NULL, NULL);
            for (uint32_t p = 0; p < g->len; p++) g->list[p] = rho[g->list[p]];
            free(ld);
        }

        /* 6. recount, reclassify, rebuild converted groups */
        for (int k = 0; k < 32; k++) {
            ogroup *g = &x->g[k];
            int keep = listed(oldt[k]) && newt[k] == oldt[k];
            g->c = nc[k];
            g->type = newt[k];
            if (!keep) group_fresh(G, x, k);
            st[3 + oldt[k] * 5 + newt[k]]++;
        }
        free(del); free(perm); free(mf); free(mt); free(rho);
    }
    free(ic); free(dc); free(ib); free(db);
    if (stats) memcpy(stats, st, sizeof st);
    return O_OK;
}

/* ------------------------------------------------------------------------ */
/* Canonical dump: for each vertex u ascending: d, next_seq, nonempty mask,  */
/* then (dst, w, seq) for each index, then for each non-empty group k        */
/* ascending: k, type, c, followed by the member (one-element) or the list   */
/* in order (listed groups); dense groups add nothing.  Little-endian u32.   */
/* ------------------------------------------------------------------------ */
static uint64_t dump_vertex(const ovtx *x, uint32_t *out) {
    uint64_t o = 0;
    uint32_t mask = 0;
    for (int k = 0; k < 32; k++) if (x->g[k].c) mask |= 1u << k;
#define PUT(v) do { if (out) out[o] = (v); o++; } while (0)
    PUT(x->d); PUT(x->next_seq); PUT(mask);
    for (uint32_t i = 0; i < x->d; i++) { PUT(x->dst[i]); PUT(x->w[i]); PUT(x->seq[i]); }
    for (int k = 0; k < 32; k++) {
        const ogroup *g = &x->g[k];
        if (!g->c) continue;
        PUT((uint32_t)k); PUT(g->type); PUT(g->c);
        if (g->type == T_ONE) PUT(g->one);
        else if (listed(g->type)) for (uint32_t p = 0; p < g->len; p++) PUT(g->list[p]);
    }
#undef PUT
    return o;
}

/* Returns the number of u32 words; writes them if out != NULL. */
uint64_t o_dump(const ograph *G, uint32_t *out) {
    uint64_t o = 0;
    for (uint32_t u = 0; u < G->n; u++) o += dump_vertex(&G->v[u], out ? out + o : NULL);
    return o;
}

/* The same for vertices [u0, u1) only. */
uint64_t o_dump_range(const ograph *G, uint32_t u0, uint32_t u1, uint32_t *out) {
    uint64_t o = 0;
    for (uint32_t u = u0; u < u1 && u < G->n; u++) o += dump_vertex(&G->v[u], out ? out + o : NULL);
    return o;
}

/* ------------------------------------------------------------------------ */
/* Group indexes (Sec. 4.2 inverted index, Sec. 5.1 sparse and regular      */
/* groups).  The inverted index of a listed group maps a neighbour index to  */
/* its position in the group's list.  A regular group keeps it over all d    */
/* neighbour indices.  A sparse group keeps it over the positions of the     */
/* reduced neighbour list S(u): the neighbour indices, ascending, of the     */
/* edges in at least one sparse group of u (reading of the garbled example), */
/* so that index has |S| entries.  Dump per vertex u ascending: |S|, then S; */
/* then for each listed group k ascending: k, followed by, for a regular     */
/* group, its inverted index read at the list's members in list order        */
/* (inv[L[p]] for p = 0..c-1), for a sparse group its index over S (entry s: */
/* the position of S[s] in the list, or 0xFFFFFFFF when S[s] is not in it).  */
/* ------------------------------------------------------------------------ */
static uint64_t index_vertex(const ograph *G, const ovtx *x, uint32_t *out) {
    uint64_t o = 0;
#define PUT(v) do { if (out) out[o] = (v); o++; } while (0)
    uint32_t smask = 0;
    for (int k = 0; k < 32; k++) if (x->g[k].type == T_SPARSE) smask |= 1u << k;
    uint32_t *S = malloc(((size_t)x->d + 1) * 4);
    uint32_t ns = 0;
    for (uint32_t i = 0; i < x->d; i++) if (mword(G, x->w[i]) & smask) S[ns++] = i;
    PUT(ns);
    for (uint32_t s = 0; s < ns; s++) PUT(S[s]);
    uint32_t *inv = malloc(((size_t)x->d + 1) * 4);
    for (int k = 0; k < 32; k++) {
        const ogroup *g = &x->g[k];
        if (!listed(g->type)) continue;
        PUT((uint32_t)k);
        if (g->type == T_REGULAR) {
            for (uint32_t i = 0; i < x->d; i++) inv[i] = 0xFFFFFFFFu;
            for (uint32_t p = 0; p < g->len; p++) inv[g->list[p]] = p;
            for (uint32_t p = 0; p < g->len; p++) PUT(inv[g->list[p]]);
        } else {
            for (uint32_t s = 0; s < ns; s++) {
                uint32_t pos = 0xFFFFFFFFu;
                for (uint32_t p = 0; p < g->len; p++) if (g->list[p] == S[s]) { pos = p; break; }
                PUT(pos);
            }
        }
    }
    free(inv);
    free(S);
#undef PUT
    return o;
}

/* Index dump of vertices [u0, u1); returns the number of u32 words, writes them if out != NULL. */
uint64_t o_index_dump_range(const ograph *G, uint32_t u0, uint32_t u1, uint32_t *out) {
    uint64_t o = 0;
    for (uint32_t u = u0; u < u1 && u < G->n; u++) o += index_vertex(G, &G->v[u], out ? out + o : NULL);
    return o;
}

/* ------------------------------------------------------------------------ */
/* Memory model.  out[0] adjacency bytes (12 per edge); out[t] for t = 1..4  */
/* group bytes by type (one-element, dense, sparse, regular) under adaption: */
/* one-element 4, dense 0, regular                                           */
/* 4(c + d) (list + full inverted index), sparse 4c for the list plus 4|S|   */
/* for its inverted index, where S(u) is the reduced neighbor list of edges  */
/* in at least one sparse group (4|S| once more per vertex for S itself,     */
/* out[6]); out[7] the all-regular baseline 4 sum(c + d) over non-empty      */
/* groups; out[8] the naive bound of Sec. 4.4, 4 (d K + sum popc w_i).       */
/* ------------------------------------------------------------------------ */
void o_memory(const ograph *G, uint64_t out[9]) {
    memset(out, 0, 9 * 8);
    for (uint32_t u = 0; u < G->n; u++) {
        const ovtx *x = &G->v[u];
        out[0] += 12ull * x->d;
        uint32_t smask = 0;
        for (int k = 0; k < 32; k++) if (x->g[k].type == T_SPARSE) smask |= 1u << k;
        uint64_t S = 0, popc = 0;
        for (uint32_t i = 0; i < x->d; i++) {
            const uint32_t mw = mword(G, x->w[i]);
            if (mw & smask) S++;
            popc += (uint64_t)__builtin_popcount(mw);
        }
        for (int k = 0; k < 32; k++) {
            const ogroup *g = &x->g[k];
            switch (g->type) {
            case T_ONE: out[1] += 4; break;
            case T_DENSE: break;
            case T_SPARSE: out[3] += 4ull * g->c + 4ull * S; break;
            case T_REGULAR: out[4] += 4ull * ((uint64_t)g->c + x->d); break;
            default: break;
            }
            if (g->c) out[7] += 4ull * ((uint64_t)g->c + x->d);
        }
        out[6] += 4ull * S;
        out[8] += 4ull * ((uint64_t)x->d * 32 + popc);
    }
}

uint32_t o_n(const ograph *G) { return G->n; }

/* ======================================================================== */
/* Radix base 4 (Supplement S.2, Fig. 17).                                   */
/*                                                                           */
/* Every weight is written in base 4, w = sum_k d_k 4^k with digits d_k in   */
/* {0,1,2,3} (k = 0..15).  Group k holds the edges with d_k != 0; its        */
/* members do not all carry the same bias, so it is split into subgroups     */
/* (k, v), v = 1..3, of the edges whose digit is v: every member of (k, v)   */
/* carries v 4^k, and the subgroup's total is c_{k,v} v 4^k.  A step picks   */
/* the group by its total, then the subgroup inside it by c_{k,v} v, then a  */
/* member uniformly.  Readings fixed here: both choices are inverse          */
/* transform in ascending order on one draw r = below64(W) (the group's      */
/* residual r - sum of the lower groups picks the subgroup), which is the    */
/* same as one ascending scan over the 48 subgroups s = 3k + v - 1 with      */
/* totals T_s = c_s v 4^k; the member of a subgroup is drawn as for a power- */
/* of-two group, by the subgroup's type from (c_s, d) under the rule of      */
/* Sec. 5.1 (one-element: its member; listed: L_s[below32(c_s)]; dense:      */
/* i = below32(d) until digit k of w_i is v).  Build and walks only: the     */
/* paper leaves updates of nested subgroups open.                            */
/* ======================================================================== */
#define R4_SUB 48

typedef struct {
    uint32_t d;
    uint32_t *dst, *w;
    ogroup s[R4_SUB];
} o4vtx;

typedef struct {
    uint32_t n;
    int adaptive;
    uint32_t alpha, beta;
    o4vtx *v;
} o4graph;

static uint32_t r4_digit(uint32_t w, int k) { return (w >> (2 * k)) & 3u; }

int o4_build(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, int adaptive,
             uint32_t alpha, uint32_t beta, o4graph **out) {
    *out = NULL;
    if (n == 0) return O_EINVAL;
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] >= n || dst[e] >= n) return O_ERANGE;
        if (w[e] == 0) return O_EWEIGHT;
    }
    o4graph *G = calloc(1, sizeof(o4graph));
    G->n = n; G->adaptive = adaptive; G->alpha = alpha; G->beta = beta;
    G->v = calloc(n, sizeof(o4vtx));
    uint32_t *deg = calloc(n, 4);
    for (uint64_t e = 0; e < m; e++) deg[src[e]]++;
    for (uint32_t u = 0; u < n; u++) {
        G->v[u].dst = malloc((size_t)(deg[u] ? deg[u] : 1) * 4);
        G->v[u].w = malloc((size_t)(deg[u] ? deg[u] : 1) * 4);
    }
    free(deg);
    /* edges of u in input order */
    for (uint64_t e = 0; e < m; e++) {
        o4vtx *x = &G->v[src[e]];
        x->dst[x->d] = dst[e]; x->w[x->d] = w[e]; x->d++;
    }
    for (uint32_t u = 0; u < n; u++) {
        o4vtx *x = &G->v[u];
        for (int s = 0; s < R4_SUB; s++) {
            const int k = s / 3;
            const uint32_t v = (uint32_t)(s % 3) + 1u;
            ogroup *g = &x->s[s];
            g->c = 0;
            for (uint32_t i = 0; i < x->d; i++) g->c += r4_digit(x->w[i], k) == v;
            g->type = (uint8_t)o_type(g->c, x->d, adaptive, alpha, beta);
            g->one = 0;
            if (g->type == T_ONE) {
                for (uint32_t i = 0; i < x->d; i++) if (r4_digit(x->w[i], k) == v) { g->one = i; break; }
            } else if (listed(g->type)) {
                for (uint32_t i = 0; i < x->d; i++) if (r4_digit(x->w[i], k) == v) list_push(g, i);
            }
        }
    }
    *out = G;
    return O_OK;
}

void o4_free(o4graph *G) {
    if (!G) return;
    for (uint32_t u = 0; u < G->n; u++) {
        free(G->v[u].dst); free(G->v[u].w);
        for (int s = 0; s < R4_SUB; s++) free(G->v[u].s[s].list);
    }
    free(G->v);
    free(G);
}

/* Subgroup selection for tests: the first s (ascending) with r < sum_{j<=s} T_j. */
int o4_pick_subgroup(const uint32_t c[R4_SUB], uint64_t r) {
    uint64_t acc = 0;
    for (int s = 0; s < R4_SUB; s++) {
        acc += (uint64_t)c[s] * (uint64_t)(s % 3 + 1) << (2 * (s / 3));
        if (r < acc) return s;
    }
    return -1;
}

static uint32_t o4_step_from(const o4graph *G, uint32_t u, ostream *s) {
    const o4vtx *x = &G->v[u];
    if (x->d == 0) return STOPV;
    uint32_t c[R4_SUB];
    uint64_t W = 0;
    for (int j = 0; j < R4_SUB; j++) {
        c[j] = x->s[j].c;
        W += (uint64_t)c[j] * (uint64_t)(j % 3 + 1) << (2 * (j / 3));
    }
    const int sg = o4_pick_subgroup(c, st_below64(s, W));
    const ogroup *g = &x->s[sg];
    const int k = sg / 3;
    const uint32_t v = (uint32_t)(sg % 3) + 1u;
    uint32_t i;
    if (g->type == T_ONE) {
        i = g->one;
    } else if (listed(g->type)) {
        i = g->list[st_below32(s, g->c)];
    } else {
        for (;;) {
            i = st_below32(s, x->d);
            if (r4_digit(x->w[i], k) == v) break;
        }
    }
    return x->dst[i];
}

uint32_t o4_step(const o4graph *G, uint32_t u, uint64_t seed, uint64_t walk, uint32_t step) {
    ostream s; st_init(&s, seed, walk, step);
    return o4_step_from(G, u, &s);
}

/* DeepWalk on the base-4 structure, with the walk ids, streams and path layout of o_deepwalk. */
uint64_t o4_deepwalk(const o4graph *G, uint64_t nwalks, const uint32_t *starts, uint64_t base, uint32_t len,
                     uint64_t seed, uint32_t *paths, int nthreads) {
    uint64_t total = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
#endif
    for (int64_t j = 0; j < (int64_t)nwalks; j++) {
        uint32_t *p = paths + (uint64_t)j * (len + 1);
        uint32_t u = starts[j];
        p[0] = u;
        uint32_t t = 0;
        for (; t < len; t++) {
            ostream rs; st_init(&rs, seed, base + (uint64_t)j, t);
            const uint32_t nx = o4_step_from(G, u, &rs);
            if (nx == STOPV) break;
            p[t + 1] = nx;
            u = nx;
        }
        total += t;
        for (; t < len; t++) p[t + 1] = STOPV;
    }
    return total;
}

/* Canonical dump of the base-4 structure: for each vertex ascending: d, the */
/* mask of non-empty subgroups (two words: subgroups 0..31, 32..47), then    */
/* (dst, w) per index, then for each non-empty subgroup s ascending: s,      */
/* type, c, and the member (one-element) or the list (listed).               */
uint64_t o4_dump(const o4graph *G, uint32_t *out) {
    uint64_t o = 0;
#define PUT(v) do { if (out) out[o] = (v); o++; } while (0)
    for (uint32_t u = 0; u < G->n; u++) {
        const o4vtx *x = &G->v[u];
        uint64_t mask = 0;
        for (int s = 0; s < R4_SUB; s++) if (x->s[s].c) mask |= 1ull << s;
        PUT(x->d); PUT((uint32_t)mask); PUT((uint32_t)(mask >> 32));
        for (uint32_t i = 0; i < x->d; i++) { PUT(x->dst[i]); PUT(x->w[i]); }
        for (int s = 0; s < R4_SUB; s++) {
            const ogroup *g = &x->s[s];
            if (!g->c) continue;
            PUT((uint32_t)s); PUT(g->type); PUT(g->c);
            if (g->type == T_ONE) PUT(g->one);
            else if (listed(g->type)) for (uint32_t p = 0; p < g->len; p++) PUT(g->list[p]);
        }
    }
#undef PUT
    return o;
}

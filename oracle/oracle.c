/*
 * CPU oracle for MESSI's data-parallel hot path (iSAX build + exact k-NN).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library: the breakpoint
 * table, the summation orders, the partition and the search are all written
 * out again here, plainly, from the paper (Peng, Fatourou, Palpanas, "MESSI:
 * In-Memory Data Series Indexing", ICDE 2020) and the textbook definitions it
 * cites.  Plain loops, fp64 wherever the method leaves the precision open.
 * Built with gcc -O2 -ffp-contract=off so that every + and * is one IEEE
 * operation in the order written.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes):
 *   - z-normalisation: population sigma, two passes, sums in "fold-halving"
 *     order (defined at fh64 below); sigma = 0 gives an all-zero series.
 *   - PAA: fp32, fold-halving sum of the segment then one division by m.
 *   - breakpoints: beta_j = fl32(Phi^-1(j / 2^b)), j = 1 .. 2^b - 1 (standard
 *     normal quantiles); a PAA value equal to a breakpoint takes the upper
 *     region, i.e. the symbol is #{j : beta_j <= p}.
 *   - word and root key: segment 0 first; the root child of a series takes
 *     the top bit of every symbol, segment 0 as the most significant bit.
 *   - leaf partition: the order-free top-down rule of oracle_build_leaves.
 *   - lower bound: query PAA (not the query's iSAX word) against the node's
 *     region, per segment; MINDIST^2 = m * sum_i d_i^2.
 *   - k-NN answer: the k smallest (D64, index) pairs, D64 the canonical
 *     sequential fp64 squared distance of oracle_d64.
 *   - BF16 filter of the batched search (beyond the paper): the filtered
 *     value and its rounding bound E, derived term by term at
 *     oracle_bf16_error_bound; a member may be discarded only if f - E > U.
 *   - DTW search (the paper's closing experiment): a Sakoe-Chiba band of
 *     half-width r around the diagonal (the caller picks r; the paper's
 *     window of 10% of the length is r = floor(L / 10)), the squared DTW of
 *     the textbook recurrence in fp64, the query's LB_Keogh envelope over
 *     that band, and per segment its maximum / minimum against the node's
 *     region as the index bound (oracle_mindist_dtw_sq).
 *
 * Parity pins live in tests/ (they compare against the paper's worked word,
 * textbook quantiles, closed forms, invariants and brute force).  Functions
 * with no external pin say "parity unpinned" in their comment; there are none
 * at present.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Fold-halving sums.  Pad the values with +0.0 to a power of two P, then    */
/* repeatedly replace v[i] by v[i] + v[i + P/2] for i < P/2 and halve P,     */
/* until one value is left.  Every + is one IEEE operation in the stated     */
/* precision.  buf must hold the next power of two >= len.                   */
/* ------------------------------------------------------------------------ */

static int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

static double fh64(double* buf, int len) {
    int p = next_pow2(len);
    for (int i = len; i < p; ++i) buf[i] = 0.0;
    for (int h = p / 2; h >= 1; h /= 2)
        for (int i = 0; i < h; ++i) buf[i] = buf[i] + buf[i + h];
    return buf[0];
}

static float fh32(float* buf, int len) {
    int p = next_pow2(len);
    for (int i = len; i < p; ++i) buf[i] = 0.0f;
    for (int h = p / 2; h >= 1; h /= 2)
        for (int i = 0; i < h; ++i) buf[i] = buf[i] + buf[i + h];
    return buf[0];
}

/* ------------------------------------------------------------------------ */
/* Breakpoints: standard normal quantiles (iSAX, Preliminaries section).     */
/* Phi(x) = erfc(-x / sqrt 2) / 2 in long double; each quantile by plain     */
/* bisection (the smallest x with Phi(x) >= p), then rounded to fp32.        */
/* ------------------------------------------------------------------------ */

static long double phi_ld(long double x) {
    return 0.5L * erfcl(-x / sqrtl(2.0L));
}

/* For p < 1/2 the root is negative, where erfc(-x / sqrt 2) is small and
 * accurate to its own relative precision; p > 1/2 uses Phi^-1(p) = -Phi^-1(1 - p)
 * and p = 1/2 gives 0 (dyadic p, so 1 - p is exact). */
static long double quantile_ld(long double p) {
    if (p == 0.5L) return 0.0L;
    if (p > 0.5L) return -quantile_ld(1.0L - p);
    long double lo = -40.0L, hi = 0.0L;
    for (int it = 0; it < 400; ++it) {
        long double mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (phi_ld(mid) < p) lo = mid; else hi = mid;
    }
    return hi;
}

/* out[j-1] = beta_j for j = 1 .. 2^b - 1.  Returns the count or -1. */
int oracle_breakpoints(int card_bits, float* out) {
    if (card_bits < 1 || card_bits > 8 || !out) return -1;
    int a = 1 << card_bits;
    for (int j = 1; j < a; ++j) out[j - 1] = (float)quantile_ld((long double)j / (long double)a);
    return a - 1;
}

/* ------------------------------------------------------------------------ */
/* z-normalisation (Preliminaries: mean 0, standard deviation 1).            */
/* ------------------------------------------------------------------------ */

void oracle_znorm(const float* x, int64_t n, int32_t len, float* z) {
    int p = next_pow2(len);
    double* buf = (double*)malloc(sizeof(double) * (size_t)p);
    double* c = (double*)malloc(sizeof(double) * (size_t)len);
    for (int64_t r = 0; r < n; ++r) {
        const float* row = x + (size_t)r * (size_t)len;
        float* out = z + (size_t)r * (size_t)len;
        for (int j = 0; j < len; ++j) buf[j] = (double)row[j];
        double mu = fh64(buf, len) / (double)len;
        for (int j = 0; j < len; ++j) c[j] = (double)row[j] - mu;
        for (int j = 0; j < len; ++j) buf[j] = c[j] * c[j];
        double var = fh64(buf, len) / (double)len;
        if (var == 0.0) {
            for (int j = 0; j < len; ++j) out[j] = 0.0f;
            continue;
        }
        double sigma = sqrt(var);
        for (int j = 0; j < len; ++j) out[j] = (float)(c[j] / sigma);
    }
    free(buf);
    free(c);
}

/* ------------------------------------------------------------------------ */
/* PAA (Keogh et al. 2001, as used by iSAX): the mean of each of w equal     */
/* segments of length m = len / w.  fp32, fold-halving order.                */
/* ------------------------------------------------------------------------ */

void oracle_paa(const float* z, int64_t n, int32_t len, int32_t w, float* paa) {
    int m = len / w;
    float* buf = (float*)malloc(sizeof(float) * (size_t)next_pow2(m));
    for (int64_t r = 0; r < n; ++r) {
        const float* row = z + (size_t)r * (size_t)len;
        for (int i = 0; i < w; ++i) {
            for (int j = 0; j < m; ++j) buf[j] = row[i * m + j];
            float s = fh32(buf, m);
            paa[(size_t)r * (size_t)w + (size_t)i] = s / (float)m;
        }
    }
    free(buf);
}

/* PAA of a query in fp64 (used by the oracle's own pruned search). */
static void paa64(const float* q, int32_t len, int32_t w, double* out) {
    int m = len / w;
    double* buf = (double*)malloc(sizeof(double) * (size_t)next_pow2(m));
    for (int i = 0; i < w; ++i) {
        for (int j = 0; j < m; ++j) buf[j] = (double)q[i * m + j];
        out[i] = fh64(buf, m) / (double)m;
    }
    free(buf);
}

/* ------------------------------------------------------------------------ */
/* SAX symbols: the index of the region the PAA value falls in, i.e. the     */
/* number of breakpoints <= p (a value on a breakpoint goes up).             */
/* bp holds beta_1 .. beta_{2^b - 1} from oracle_breakpoints(b).            */
/* ------------------------------------------------------------------------ */

void oracle_symbols(const float* paa, int64_t n, int32_t w, int32_t card_bits, const float* bp, uint8_t* words) {
    int a = 1 << card_bits;
    for (int64_t r = 0; r < n; ++r)
        for (int i = 0; i < w; ++i) {
            float p = paa[(size_t)r * (size_t)w + (size_t)i];
            int s = 0;
            for (int j = 1; j < a; ++j)
                if (bp[j - 1] <= p) s++;
            words[(size_t)r * (size_t)w + (size_t)i] = (uint8_t)s;
        }
}

/* Root child of each series: top bit of every symbol, segment 0 = MSB. */
void oracle_root_keys(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits, uint32_t* keys) {
    for (int64_t r = 0; r < n; ++r) {
        uint32_t k = 0;
        for (int i = 0; i < w; ++i) {
            uint32_t top = ((uint32_t)words[(size_t)r * (size_t)w + (size_t)i] >> (card_bits - 1)) & 1u;
            k |= top << (w - 1 - i);
        }
        keys[r] = k;
    }
}

/* ------------------------------------------------------------------------ */
/* Leaf partition (index tree of the Preliminaries and Algorithm             */
/* TreeConstruction / SplitNode), written as an order-free top-down rule so   */
/* that leaf membership has one answer whatever the insertion order:         */
/*   - root children: one per non-empty root key, card 1 in every segment;   */
/*   - a node with <= cap series is a leaf;                                  */
/*   - else, among segments whose cardinality can still grow, split on the   */
/*     one whose next bit divides the node most evenly (min |n0 - n1|, ties  */
/*     to the lowest segment); children take bit 0 then bit 1, keep the      */
/*     parent's series order, and empty children are dropped;                */
/*   - a node over capacity whose segments are all at full cardinality is an */
/*     (overflow) leaf.                                                      */
/* Leaves come out in depth-first order (root key ascending, 0 before 1);    */
/* members are in ascending series index.                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint8_t card[16];
    uint8_t prefix[16];
    uint32_t start;
    uint32_t count;
} oracle_leaf;

/* An internal node of the partition and the segment it split on. */
typedef struct {
    uint8_t card[16];
    uint8_t prefix[16];
    int32_t seg;
} oracle_split;

typedef struct {
    const uint8_t* words;
    int32_t w, b;
    int64_t cap;
    oracle_leaf* leaves;
    int64_t n_leaves;
    uint32_t* pos;
    int64_t n_pos;
    /* per-depth scratch for the members of the two children */
    uint32_t* scratch;
    /* appends: nodes that must split on a given segment (may be NULL) */
    const oracle_split* forced;
    int64_t n_forced;
    /* every internal node with its segment, in the order met (may be NULL) */
    oracle_split* inner;
    int64_t n_inner;
} build_ctx;

static int forced_segment(const build_ctx* ctx, const uint8_t* card, const uint8_t* prefix) {
    for (int64_t f = 0; f < ctx->n_forced; ++f)
        if (memcmp(ctx->forced[f].card, card, (size_t)ctx->w) == 0 &&
            memcmp(ctx->forced[f].prefix, prefix, (size_t)ctx->w) == 0)
            return ctx->forced[f].seg;
    return -1;
}

static void emit_leaf(build_ctx* ctx, const uint8_t* card, const uint8_t* prefix, const uint32_t* members,
                      int64_t cnt) {
    oracle_leaf* lf = &ctx->leaves[ctx->n_leaves++];
    memset(lf, 0, sizeof *lf);
    memcpy(lf->card, card, (size_t)ctx->w);
    memcpy(lf->prefix, prefix, (size_t)ctx->w);
    lf->start = (uint32_t)ctx->n_pos;
    lf->count = (uint32_t)cnt;
    for (int64_t j = 0; j < cnt; ++j) ctx->pos[ctx->n_pos++] = members[j];
}

static void split_node(build_ctx* ctx, const uint8_t* card, const uint8_t* prefix, uint32_t* members, int64_t cnt) {
    int w = ctx->w, b = ctx->b;
    if (cnt <= ctx->cap) {
        emit_leaf(ctx, card, prefix, members, cnt);
        return;
    }
    /* a node that split before an append splits on the same segment again */
    int best = forced_segment(ctx, card, prefix);
    if (best < 0) {
        int64_t best_gap = 0;
        for (int i = 0; i < w; ++i) {
            if (card[i] >= b) continue;
            int shift = b - 1 - card[i];
            int64_t n1 = 0;
            for (int64_t j = 0; j < cnt; ++j)
                n1 += (ctx->words[(size_t)members[j] * (size_t)w + (size_t)i] >> shift) & 1;
            int64_t n0 = cnt - n1;
            int64_t gap = n0 > n1 ? n0 - n1 : n1 - n0;
            if (best < 0 || gap < best_gap) {
                best = i;
                best_gap = gap;
            }
        }
    }
    if (best < 0) { /* every segment at full cardinality */
        emit_leaf(ctx, card, prefix, members, cnt);
        return;
    }
    if (ctx->inner) {
        oracle_split* sp = &ctx->inner[ctx->n_inner++];
        memset(sp, 0, sizeof *sp);
        memcpy(sp->card, card, (size_t)w);
        memcpy(sp->prefix, prefix, (size_t)w);
        sp->seg = best;
    }
    int shift = b - 1 - card[best];
    uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)cnt);
    int64_t n0 = 0;
    for (int64_t j = 0; j < cnt; ++j)
        if (((ctx->words[(size_t)members[j] * (size_t)w + (size_t)best] >> shift) & 1) == 0) tmp[n0++] = members[j];
    int64_t n1 = 0;
    for (int64_t j = 0; j < cnt; ++j)
        if (((ctx->words[(size_t)members[j] * (size_t)w + (size_t)best] >> shift) & 1) == 1) tmp[n0 + n1++] = members[j];
    uint8_t ccard[16], cpre[16];
    memcpy(ccard, card, 16);
    memcpy(cpre, prefix, 16);
    ccard[best] = (uint8_t)(card[best] + 1);
    if (n0 > 0) {
        cpre[best] = (uint8_t)(prefix[best] * 2 + 0);
        split_node(ctx, ccard, cpre, tmp, n0);
    }
    if (n1 > 0) {
        cpre[best] = (uint8_t)(prefix[best] * 2 + 1);
        split_node(ctx, ccard, cpre, tmp + n0, n1);
    }
    free(tmp);
}

/* Returns the number of leaves (<= n), or -1 on bad arguments.  leaves must
 * hold n entries and pos n entries. */
int64_t oracle_build_leaves_ex(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits, int64_t cap,
                               const oracle_split* forced, int64_t n_forced, oracle_leaf* leaves, uint32_t* pos,
                               oracle_split* inner, int64_t* n_inner);

int64_t oracle_build_leaves(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits, int64_t cap,
                            oracle_leaf* leaves, uint32_t* pos) {
    return oracle_build_leaves_ex(words, n, w, card_bits, cap, NULL, 0, leaves, pos, NULL, NULL);
}

/* The same, and (inner may be NULL) every internal node with the segment it
 * split on.  forced (n_forced entries, may be NULL) lists nodes that must
 * split on a given segment: appending series to an index is this partition of
 * all the series with the previous index's internal nodes as `forced`
 * (Algorithm TreeConstruction inserts each new series into the leaf its word
 * reaches and splits a leaf that gets too full; the existing splits stay, a
 * leaf that gets no new series stays as it is, and an over-full one is split
 * by the same balance rule).  inner must hold (w (card_bits - 1) + 2)
 * (n / (cap + 1) + 1) entries: internal nodes hold more than cap series, the
 * nodes of one depth are disjoint, and a path refines at most w (card_bits - 1)
 * times below the root children. */
int64_t oracle_build_leaves_ex(const uint8_t* words, int64_t n, int32_t w, int32_t card_bits, int64_t cap,
                               const oracle_split* forced, int64_t n_forced, oracle_leaf* leaves, uint32_t* pos,
                               oracle_split* inner, int64_t* n_inner) {
    if (n < 1 || w < 1 || w > 16 || card_bits < 1 || card_bits > 8 || cap < 1) return -1;
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    oracle_root_keys(words, n, w, card_bits, keys);
    int64_t nkeys = (int64_t)1 << w;
    /* stable counting sort of series by root key */
    int64_t* start = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
    for (int64_t r = 0; r < n; ++r) start[keys[r] + 1]++;
    for (int64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nkeys);
    memcpy(fill, start, sizeof(int64_t) * (size_t)nkeys);
    for (int64_t r = 0; r < n; ++r) order[fill[keys[r]]++] = (uint32_t)r;
    build_ctx ctx;
    memset(&ctx, 0, sizeof ctx);
    ctx.words = words; ctx.w = w; ctx.b = card_bits; ctx.cap = cap; ctx.leaves = leaves; ctx.pos = pos;
    ctx.forced = forced; ctx.n_forced = forced ? n_forced : 0; ctx.inner = inner;
    for (int64_t k = 0; k < nkeys; ++k) {
        int64_t cnt = start[k + 1] - start[k];
        if (cnt == 0) continue;
        uint8_t card[16] = {0}, prefix[16] = {0};
        for (int i = 0; i < w; ++i) {
            card[i] = 1;
            prefix[i] = (uint8_t)((k >> (w - 1 - i)) & 1);
        }
        split_node(&ctx, card, prefix, order + start[k], cnt);
    }
    free(keys); free(start); free(order); free(fill);
    if (n_inner) *n_inner = ctx.n_inner;
    return ctx.n_leaves;
}

/* ------------------------------------------------------------------------ */
/* Distances.                                                               */
/* ------------------------------------------------------------------------ */

/* Canonical squared Euclidean distance: sum over j = 0 .. len-1, in that
 * order, of (q_j - x_j)^2 with q_j, x_j widened to fp64; every - , * and +
 * rounded on its own (no fused multiply-add). */
double oracle_d64(const float* q, const float* x, int32_t len) {
    double s = 0.0;
    for (int j = 0; j < len; ++j) {
        double d = (double)q[j] - (double)x[j];
        s = s + d * d;
    }
    return s;
}

/* Region [lo, hi] of symbol prefix `prefix` at cardinality `card` (of b bits
 * maximum): lo = beta_{prefix * 2^(b - card)}, hi = beta_{(prefix + 1) * 2^(b - card)},
 * with beta_0 = -inf and beta_{2^b} = +inf. */
static void region(const float* bp, int card_bits, int card, int prefix, double* lo, double* hi) {
    int a = 1 << card_bits;
    int ilo = prefix << (card_bits - card);
    int ihi = (prefix + 1) << (card_bits - card);
    *lo = (ilo == 0) ? -INFINITY : (double)bp[ilo - 1];
    *hi = (ihi == a) ? INFINITY : (double)bp[ihi - 1];
}

/* iSAX lower bound (Shieh & Keogh 2008) of a query PAA against a node
 * (card[w], prefix[w]): m * sum_i d_i^2, d_i the distance from the query's
 * segment mean to the segment's region; regions widened by `slack` on both
 * sides (0 for the textbook value).  fp64. */
double oracle_mindist_sq(const double* qpaa, int32_t w, int32_t m, const uint8_t* card, const uint8_t* prefix,
                         int32_t card_bits, const float* bp, double slack) {
    double s = 0.0;
    for (int i = 0; i < w; ++i) {
        double lo, hi;
        region(bp, card_bits, card[i], prefix[i], &lo, &hi);
        lo -= slack;
        hi += slack;
        double d = 0.0;
        if (qpaa[i] < lo) d = lo - qpaa[i];
        else if (qpaa[i] > hi) d = qpaa[i] - hi;
        s += d * d;
    }
    return (double)m * s;
}

/* Same, from a float query PAA (for tests). */
double oracle_mindist_sq_f(const float* qpaa, int32_t w, int32_t m, const uint8_t* card, const uint8_t* prefix,
                           int32_t card_bits, const float* bp) {
    double qp[16];
    for (int i = 0; i < w; ++i) qp[i] = (double)qpaa[i];
    return oracle_mindist_sq(qp, w, m, card, prefix, card_bits, bp, 0.0);
}

/* ------------------------------------------------------------------------ */
/* k smallest by (distance, index): a sorted array with insertion.          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t k, size;
    double* d;
    int64_t* idx;
} topk_t;

static int pair_less(double da, int64_t ia, double db, int64_t ib) {
    return da < db || (da == db && ia < ib);
}

static void topk_insert(topk_t* t, double d, int64_t idx) {
    if (t->size == t->k && !pair_less(d, idx, t->d[t->k - 1], t->idx[t->k - 1])) return;
    int pos = (t->size < t->k) ? t->size++ : t->k - 1;
    while (pos > 0 && pair_less(d, idx, t->d[pos - 1], t->idx[pos - 1])) {
        t->d[pos] = t->d[pos - 1];
        t->idx[pos] = t->idx[pos - 1];
        pos--;
    }
    t->d[pos] = d;
    t->idx[pos] = idx;
}

/* ------------------------------------------------------------------------ */
/* Brute-force exact k-NN (the definition of the answer).                   */
/* ------------------------------------------------------------------------ */

double oracle_dtw64(const float* q, const float* x, int32_t len, int32_t r);

typedef struct {
    const float* data;
    int64_t r0, r1;
    int32_t len;
    const float* queries;
    int32_t nq, k;
    int32_t band;   /* < 0: Euclidean (D64); else DTW with this half-width */
    double* d;      /* [nq][k] */
    int64_t* idx;   /* [nq][k] */
    int32_t* size;  /* [nq] */
} brute_job;

static void* brute_worker(void* arg) {
    brute_job* j = (brute_job*)arg;
    for (int32_t q = 0; q < j->nq; ++q) {
        topk_t t = {j->k, 0, j->d + (size_t)q * (size_t)j->k, j->idx + (size_t)q * (size_t)j->k};
        const float* qs = j->queries + (size_t)q * (size_t)j->len;
        for (int64_t r = j->r0; r < j->r1; ++r) {
            const float* x = j->data + (size_t)r * (size_t)j->len;
            topk_insert(&t, j->band < 0 ? oracle_d64(qs, x, j->len) : oracle_dtw64(qs, x, j->len, j->band), r);
        }
        j->size[q] = t.size;
    }
    return NULL;
}

static int knn_brute_any(const float* data, int64_t n, int32_t len, const float* queries, int32_t nq, int32_t k,
                         int32_t band, int nthreads, int64_t row_offset, int64_t* out_idx, double* out_d64);

/* out_d64 / out_idx: [nq][k], ascending (D64, index).  Rows are data[n][len].
 * Uses nthreads threads over contiguous row ranges, merged at the end.
 * row_offset is added to every returned index (for scans of a slice). */
int oracle_knn_brute(const float* data, int64_t n, int32_t len, const float* queries, int32_t nq, int32_t k,
                     int nthreads, int64_t row_offset, int64_t* out_idx, double* out_d64) {
    return knn_brute_any(data, n, len, queries, nq, k, -1, nthreads, row_offset, out_idx, out_d64);
}

/* The same under DTW with a band of half-width r (ascending (DTW64, index)). */
int oracle_knn_brute_dtw(const float* data, int64_t n, int32_t len, const float* queries, int32_t nq, int32_t k,
                         int32_t r, int nthreads, int64_t* out_idx, double* out_d) {
    if (r < 0) return -1;
    return knn_brute_any(data, n, len, queries, nq, k, r, nthreads, 0, out_idx, out_d);
}

static int knn_brute_any(const float* data, int64_t n, int32_t len, const float* queries, int32_t nq, int32_t k,
                         int32_t band, int nthreads, int64_t row_offset, int64_t* out_idx, double* out_d64) {
    if (n < 1 || len < 1 || nq < 0 || k < 1 || k > n) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > n) nthreads = (int)n;
    brute_job* jobs = (brute_job*)calloc((size_t)nthreads, sizeof(brute_job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        brute_job* j = &jobs[t];
        j->data = data; j->len = len; j->queries = queries; j->nq = nq; j->k = k; j->band = band;
        j->r0 = n * t / nthreads; j->r1 = n * (t + 1) / nthreads;
        j->d = (double*)malloc(sizeof(double) * (size_t)nq * (size_t)k + 8);
        j->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)nq * (size_t)k + 8);
        j->size = (int32_t*)calloc((size_t)nq + 1, sizeof(int32_t));
        if (pthread_create(&th[t], NULL, brute_worker, j) != 0) {
            brute_worker(j);
            th[t] = 0;
        }
    }
    for (int t = 0; t < nthreads; ++t)
        if (th[t]) pthread_join(th[t], NULL);
    for (int32_t q = 0; q < nq; ++q) {
        topk_t t = {k, 0, out_d64 + (size_t)q * (size_t)k, out_idx + (size_t)q * (size_t)k};
        for (int w = 0; w < nthreads; ++w)
            for (int32_t i = 0; i < jobs[w].size[q]; ++i)
                topk_insert(&t, jobs[w].d[(size_t)q * (size_t)k + (size_t)i], jobs[w].idx[(size_t)q * (size_t)k + (size_t)i]);
        for (int32_t i = 0; i < k; ++i) out_idx[(size_t)q * (size_t)k + (size_t)i] += row_offset;
    }
    for (int t = 0; t < nthreads; ++t) {
        free(jobs[t].d); free(jobs[t].idx); free(jobs[t].size);
    }
    free(jobs);
    free(th);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Plain iSAX exact search (Algorithms ExactSearch .. CalculateRealDistance, */
/* with the leaves visited in ascending lower bound, as the priority queues  */
/* deliver them): a leaf whose bound exceeds the current k-th distance ends  */
/* the search; inside a leaf, a series whose own word's bound exceeds it is   */
/* skipped; otherwise its real distance is computed and the k best kept.     */
/*                                                                          */
/* Exactness: the data's words come from fp32 PAA values, which may differ   */
/* from the exact segment means by at most e = (ceil(log2 m) + 2) 2^-23 A,   */
/* A = max |value| in the collection; every region is widened by e so the     */
/* bound stays below the true distance, and a bound is compared with the     */
/* k-th D64 after scaling it down by (1 - 2^-40).  Ties on the bound are      */
/* visited (an equal distance with a lower index may displace).              */
/* Must return exactly oracle_knn_brute's answer.                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lb;
    int64_t id;
} lb_item;

static int lb_cmp(const void* a, const void* b) {
    const lb_item* x = (const lb_item*)a;
    const lb_item* y = (const lb_item*)b;
    if (x->lb < y->lb) return -1;
    if (x->lb > y->lb) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

/* stats (may be NULL): [nq][4] = leaves visited, series bounded, real distances, leaves total */
int oracle_knn_isax(const float* data, int64_t n, int32_t len, const uint8_t* words, int32_t w, int32_t card_bits,
                    const oracle_leaf* leaves, int64_t n_leaves, const uint32_t* pos, const float* queries,
                    int32_t nq, int32_t k, int64_t* out_idx, double* out_d64, int64_t* stats) {
    if (n < 1 || len < 1 || w < 1 || len % w || k < 1 || k > n) return -1;
    int m = len / w;
    float bp[255];
    oracle_breakpoints(card_bits, bp);
    double amax = 0.0;
    for (int64_t i = 0; i < n * (int64_t)len; ++i) {
        double a = fabs((double)data[i]);
        if (a > amax) amax = a;
    }
    int lg = 0;
    while ((1 << lg) < m) lg++;
    double slack = (double)(lg + 2) * ldexp(1.0, -23) * amax;
    lb_item* order = (lb_item*)malloc(sizeof(lb_item) * (size_t)n_leaves);
    uint8_t full[16];
    for (int i = 0; i < 16; ++i) full[i] = (uint8_t)card_bits;
    for (int32_t q = 0; q < nq; ++q) {
        const float* qs = queries + (size_t)q * (size_t)len;
        double qp[16];
        paa64(qs, len, w, qp);
        for (int64_t l = 0; l < n_leaves; ++l) {
            order[l].lb = oracle_mindist_sq(qp, w, m, leaves[l].card, leaves[l].prefix, card_bits, bp, slack);
            order[l].id = l;
        }
        qsort(order, (size_t)n_leaves, sizeof(lb_item), lb_cmp);
        topk_t t = {k, 0, out_d64 + (size_t)q * (size_t)k, out_idx + (size_t)q * (size_t)k};
        int64_t visited = 0, bounded = 0, real = 0;
        for (int64_t o = 0; o < n_leaves; ++o) {
            double bsf = (t.size == k) ? t.d[k - 1] : INFINITY;
            if (order[o].lb * (1.0 - ldexp(1.0, -40)) > bsf) break;
            const oracle_leaf* lf = &leaves[order[o].id];
            visited++;
            for (uint32_t j = 0; j < lf->count; ++j) {
                uint32_t r = pos[lf->start + j];
                bsf = (t.size == k) ? t.d[k - 1] : INFINITY;
                double lbx = oracle_mindist_sq(qp, w, m, full, words + (size_t)r * (size_t)w, card_bits, bp, slack);
                bounded++;
                if (lbx * (1.0 - ldexp(1.0, -40)) > bsf) continue;
                real++;
                topk_insert(&t, oracle_d64(qs, data + (size_t)r * (size_t)len, len), (int64_t)r);
            }
        }
        if (stats) {
            stats[(size_t)q * 4 + 0] = visited;
            stats[(size_t)q * 4 + 1] = bounded;
            stats[(size_t)q * 4 + 2] = real;
            stats[(size_t)q * 4 + 3] = n_leaves;
        }
    }
    free(order);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* BF16 filter of the batched search (an extension beyond the paper, whose   */
/* search computes real distances only).  The filtered squared distance of a */
/* pair is                                                                   */
/*   f = fl32(fl32(nq + nx) - 2 s),                                          */
/*   s = fp32 sum over j = 0 .. len-1, in that order, of the exact products  */
/*       bf16(q_j) * bf16(x_j)  (8-bit significands: the product is exact    */
/*       in fp32),                                                           */
/*   nq = fl32(|q|^2), nx = fl32(|x|^2), each from a sequential fp64 sum,    */
/* with bf16() rounding to nearest, ties to even.                            */
/* ------------------------------------------------------------------------ */

float oracle_bf16_round(float v) {
    uint32_t u;
    memcpy(&u, &v, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

void oracle_bf16_round_array(const float* in, int64_t n, float* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_bf16_round(in[i]);
}

void oracle_bf16_filter_values(const float* q, const float* x, int64_t npairs, int32_t len, float* out) {
    for (int64_t p = 0; p < npairs; ++p) {
        const float* qp = q + (size_t)p * (size_t)len;
        const float* xp = x + (size_t)p * (size_t)len;
        double a2 = 0.0, b2 = 0.0;
        float s = 0.0f;
        for (int j = 0; j < len; ++j) {
            a2 = a2 + (double)qp[j] * (double)qp[j];
            b2 = b2 + (double)xp[j] * (double)xp[j];
            float prod = oracle_bf16_round(qp[j]) * oracle_bf16_round(xp[j]);
            s = s + prod;
        }
        float nsum = (float)a2 + (float)b2;
        out[p] = nsum - 2.0f * s;
    }
}

/* Bound E on |f - D|, D = |q - x|^2 exact, for ANY order and ANY rounding    */
/* (nearest or directed) of the fp32 accumulation of s.  With a = |q|,        */
/* b = |x|, u_b = 2^-8 (BF16 unit roundoff), u32 = 2^-24, and               */
/* gamma_n = n u / (1 - n u) for u = 2^-23 (a directed fp32 rounding has      */
/* relative error below 2^-23):                                              */
/*   [0] operands:   2 (2 u_b + u_b^2) a b.  bf16(q_j) bf16(x_j) differs     */
/*       from q_j x_j by at most (2 u_b + u_b^2) |q_j x_j|; summed, and by   */
/*       Cauchy-Schwarz sum |q_j x_j| <= a b; doubled by the factor 2 of s.  */
/*   [1] accumulation: 2 gamma_{len-1} (1 + u_b)^2 a b.  Summing len terms in */
/*       any order errs by at most gamma_{len-1} sum |p_j| (the standard     */
/*       recursive-summation bound), and sum |p_j| <= |bf16(q)| |bf16(x)|     */
/*       <= (1 + u_b)^2 a b; doubled likewise.                              */
/*   [2] norms:      2 u32 (a^2 + b^2): one rounding of each fp64 norm to    */
/*       fp32, plus as much again covering the fp64 sums' own error.         */
/*   [3] first add:  u32 (a^2 + b^2) (1 + 2 u32).                            */
/*   [4] final subtraction: 2 u32 (a + b)^2, since |nq + nx - 2 s| is at most */
/*       (a + b)^2 times a factor below 2.                                   */
/* E = [0] + [1] + [2] + [3] + [4] in fp64, i.e.                              */
/*   (4 u_b + 2 u_b^2 + 2 gamma (1 + u_b)^2) a b + 3 u32 (a^2 + b^2)          */
/*   + 2 u32 (a + b)^2  (to first order).                                    */
double oracle_bf16_error_bound(double a2, double b2, int32_t len, double* terms) {
    const double ub = ldexp(1.0, -8), u32 = ldexp(1.0, -24), u = ldexp(1.0, -23);
    const double nu = (double)(len > 1 ? len - 1 : 0) * u;
    const double gamma = nu / (1.0 - nu);
    const double a = sqrt(a2), b = sqrt(b2);
    double t[5];
    t[0] = 2.0 * (2.0 * ub + ub * ub) * a * b;
    t[1] = 2.0 * gamma * (1.0 + ub) * (1.0 + ub) * a * b;
    t[2] = 2.0 * u32 * (a2 + b2);
    t[3] = u32 * (a2 + b2) * (1.0 + 2.0 * u32);
    t[4] = 2.0 * u32 * (a + b) * (a + b);
    double e = 0.0;
    for (int i = 0; i < 5; ++i) {
        if (terms) terms[i] = t[i];
        e = e + t[i];
    }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Approximate search (Section 4, approxSearch): the leaf whose summary is   */
/* closest to the query -- the smallest MINDIST of the query's PAA (fp64) to */
/* the leaf's regions, ties to the lowest leaf id -- and the k best of its   */
/* members by (D64, index).  A leaf with fewer than k members is extended to */
/* the following members in depth-first leaf order (the member range moves   */
/* back from the end of the collection), and at most 4096 members are taken. */
/* Each query's chosen leaf goes to out_leaf; with leaf_override >= 0 that   */
/* leaf is used instead of the argmin (to check a near-tie).                 */
/* ------------------------------------------------------------------------ */

void oracle_leaf_bounds(const float* query, int32_t len, int32_t w, int32_t card_bits, const oracle_leaf* leaves,
                        int64_t n_leaves, double* out) {
    int m = len / w;
    float bp[255];
    oracle_breakpoints(card_bits, bp);
    double qp[16];
    paa64(query, len, w, qp);
    for (int64_t l = 0; l < n_leaves; ++l)
        out[l] = oracle_mindist_sq(qp, w, m, leaves[l].card, leaves[l].prefix, card_bits, bp, 0.0);
}

int oracle_knn_approx(const float* data, int64_t n, int32_t len, int32_t w, int32_t card_bits,
                      const oracle_leaf* leaves, int64_t n_leaves, const uint32_t* pos, const float* queries,
                      int32_t nq, int32_t k, int64_t leaf_override, int64_t* out_leaf, int64_t* out_idx,
                      double* out_d64) {
    if (n < 1 || len < 1 || w < 1 || len % w || k < 1 || k > n || k > 4096) return -1;
    double* lb = (double*)malloc(sizeof(double) * (size_t)n_leaves);
    for (int32_t q = 0; q < nq; ++q) {
        const float* qs = queries + (size_t)q * (size_t)len;
        int64_t best = leaf_override;
        if (best < 0) {
            oracle_leaf_bounds(qs, len, w, card_bits, leaves, n_leaves, lb);
            best = 0;
            for (int64_t l = 1; l < n_leaves; ++l)
                if (lb[l] < lb[best]) best = l;
        }
        out_leaf[q] = best;
        int64_t cnt = leaves[best].count;
        if (cnt < k) cnt = k;
        if (cnt > 4096) cnt = 4096;
        if (cnt > n) cnt = n;
        int64_t r0 = leaves[best].start;
        if (r0 > n - cnt) r0 = n - cnt;
        topk_t t = {k, 0, out_d64 + (size_t)q * (size_t)k, out_idx + (size_t)q * (size_t)k};
        for (int64_t r = r0; r < r0 + cnt; ++r) {
            const uint32_t row = pos[r];
            topk_insert(&t, oracle_d64(qs, data + (size_t)row * (size_t)len, len), (int64_t)row);
        }
    }
    free(lb);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dynamic time warping (the paper's closing experiment: the index is left   */
/* as it is, and searched with the LB_Keogh envelope of the query).          */
/*                                                                          */
/* DTW^2(q, x) under a Sakoe-Chiba band of half-width r is the smallest sum  */
/* of (q_i - x_j)^2 over the monotone warping paths from (0, 0) to           */
/* (L-1, L-1) whose cells all satisfy |i - j| <= r.  It is computed by the   */
/* textbook recurrence                                                       */
/*   D(i, j) = c(i, j) + min(D(i-1, j), D(i, j-1), D(i-1, j-1)),  D(0,0) = c  */
/* in fp64, c = fl64(d * d) with d = fl64(q_i - x_j), each sum rounded once.  */
/* A cell's value is a fixed function of its three neighbours, so every      */
/* order of evaluating the cells gives these same values.  r >= L - 1 is the */
/* unconstrained DTW; r = 0 leaves only the diagonal, the squared Euclidean  */
/* distance summed in index order (oracle_d64).                              */
/* ------------------------------------------------------------------------ */
double oracle_dtw64(const float* q, const float* x, int32_t len, int32_t r) {
    if (r > len - 1) r = len - 1;
    if (r < 0) r = 0;
    double* prev = (double*)malloc(sizeof(double) * (size_t)len);
    double* cur = (double*)malloc(sizeof(double) * (size_t)len);
    for (int32_t i = 0; i < len; ++i) {
        const int32_t lo = i - r > 0 ? i - r : 0, hi = i + r < len - 1 ? i + r : len - 1;
        const int32_t plo = i - 1 - r > 0 ? i - 1 - r : 0, phi = i - 1 + r < len - 1 ? i - 1 + r : len - 1;
        for (int32_t j = lo; j <= hi; ++j) {
            const double d = (double)q[i] - (double)x[j];
            const double c = d * d;
            double best = INFINITY;
            if (i == 0 && j == 0) best = 0.0;
            if (i > 0 && j >= plo && j <= phi && prev[j] < best) best = prev[j];
            if (i > 0 && j - 1 >= plo && j - 1 <= phi && prev[j - 1] < best) best = prev[j - 1];
            if (j - 1 >= lo && cur[j - 1] < best) best = cur[j - 1];
            cur[j] = c + best;
        }
        double* t = prev;
        prev = cur;
        cur = t;
    }
    const double out = prev[len - 1];
    free(prev);
    free(cur);
    return out;
}

/* The query's envelope over the band (LB_Keogh): up[j] / lo[j] = the largest /
 * smallest q_t with |t - j| <= r. */
void oracle_envelope(const float* q, int32_t len, int32_t r, float* up, float* lo) {
    for (int32_t j = 0; j < len; ++j) {
        const int32_t a = j - r > 0 ? j - r : 0, b = j + r < len - 1 ? j + r : len - 1;
        float u = q[a], l = q[a];
        for (int32_t t = a + 1; t <= b; ++t) {
            if (q[t] > u) u = q[t];
            if (q[t] < l) l = q[t];
        }
        up[j] = u;
        lo[j] = l;
    }
}

/* LB_Keogh^2: the squared distance from x to the envelope (0 inside it),
 * fp64, summed in index order.  Every warping path in the band matches each
 * x_j with some q_t, |t - j| <= r, which lies inside [lo_j, up_j]. */
double oracle_lb_keogh(const float* up, const float* lo, const float* x, int32_t len) {
    double s = 0.0;
    for (int32_t j = 0; j < len; ++j) {
        double d = 0.0;
        if (x[j] > up[j]) d = (double)x[j] - (double)up[j];
        else if (x[j] < lo[j]) d = (double)lo[j] - (double)x[j];
        s += d * d;
    }
    return s;
}

/* The index bound under DTW: per segment i, U_i = max of up and L_i = min of
 * lo over the segment's m values; against the node's region [a, b] (widened
 * by slack), d_i = a - U_i if U_i < a, L_i - b if L_i > b, else 0; bound =
 * m sum_i d_i^2.  A series whose segment mean lies in [a, b] has at least m of
 * (mean - U_i)^2 in its LB_Keogh terms over the segment (mean of the positive
 * parts, Cauchy-Schwarz), so the bound is below LB_Keogh, hence below DTW. */
double oracle_mindist_dtw_sq(const float* up, const float* lo, int32_t len, int32_t w, const uint8_t* card,
                             const uint8_t* prefix, int32_t card_bits, const float* bp, double slack) {
    const int32_t m = len / w;
    double s = 0.0;
    for (int32_t i = 0; i < w; ++i) {
        double U = -INFINITY, L = INFINITY;
        for (int32_t t = i * m; t < (i + 1) * m; ++t) {
            if ((double)up[t] > U) U = (double)up[t];
            if ((double)lo[t] < L) L = (double)lo[t];
        }
        double a, b;
        region(bp, card_bits, card[i], prefix[i], &a, &b);
        a -= slack;
        b += slack;
        double d = 0.0;
        if (U < a) d = a - U;
        else if (L > b) d = L - b;
        s += d * d;
    }
    return (double)m * s;
}

/* Exact DTW k-NN through the index: leaves in ascending DTW bound, stop at
 * the first whose bound exceeds the k-th distance; inside a leaf, skip a
 * series whose word's bound or whose LB_Keogh exceeds it; else its DTW.  The
 * slack and the (1 - 2^-40) scaling are those of oracle_knn_isax.  Must return
 * exactly oracle_knn_brute_dtw's answer.  stats (may be NULL): [nq][4] =
 * leaves visited, series bounded, LB_Keogh computed, DTW computed. */
int oracle_knn_isax_dtw(const float* data, int64_t n, int32_t len, const uint8_t* words, int32_t w,
                        int32_t card_bits, const oracle_leaf* leaves, int64_t n_leaves, const uint32_t* pos,
                        const float* queries, int32_t nq, int32_t k, int32_t r, int64_t* out_idx, double* out_d,
                        int64_t* stats) {
    if (n < 1 || len < 1 || w < 1 || len % w || k < 1 || k > n || r < 0) return -1;
    const int32_t m = len / w;
    float bp[255];
    oracle_breakpoints(card_bits, bp);
    double amax = 0.0;
    for (int64_t i = 0; i < n * (int64_t)len; ++i) {
        double a = fabs((double)data[i]);
        if (a > amax) amax = a;
    }
    int lg = 0;
    while ((1 << lg) < m) lg++;
    const double slack = (double)(lg + 2) * ldexp(1.0, -23) * amax;
    const double shrink = 1.0 - ldexp(1.0, -40);
    lb_item* order = (lb_item*)malloc(sizeof(lb_item) * (size_t)n_leaves);
    float* up = (float*)malloc(sizeof(float) * (size_t)len);
    float* lo = (float*)malloc(sizeof(float) * (size_t)len);
    uint8_t full[16];
    for (int i = 0; i < 16; ++i) full[i] = (uint8_t)card_bits;
    for (int32_t q = 0; q < nq; ++q) {
        const float* qs = queries + (size_t)q * (size_t)len;
        oracle_envelope(qs, len, r, up, lo);
        for (int64_t l = 0; l < n_leaves; ++l) {
            order[l].lb = oracle_mindist_dtw_sq(up, lo, len, w, leaves[l].card, leaves[l].prefix, card_bits, bp, slack);
            order[l].id = l;
        }
        qsort(order, (size_t)n_leaves, sizeof(lb_item), lb_cmp);
        topk_t t = {k, 0, out_d + (size_t)q * (size_t)k, out_idx + (size_t)q * (size_t)k};
        int64_t visited = 0, bounded = 0, keogh = 0, real = 0;
        for (int64_t o = 0; o < n_leaves; ++o) {
            double bsf = (t.size == k) ? t.d[k - 1] : INFINITY;
            if (order[o].lb * shrink > bsf) break;
            const oracle_leaf* lf = &leaves[order[o].id];
            visited++;
            for (uint32_t j = 0; j < lf->count; ++j) {
                const uint32_t row = pos[lf->start + j];
                const float* x = data + (size_t)row * (size_t)len;
                bsf = (t.size == k) ? t.d[k - 1] : INFINITY;
                bounded++;
                if (oracle_mindist_dtw_sq(up, lo, len, w, full, words + (size_t)row * (size_t)w, card_bits, bp,
                                          slack) * shrink > bsf)
                    continue;
                keogh++;
                if (oracle_lb_keogh(up, lo, x, len) * shrink > bsf) continue;
                real++;
                topk_insert(&t, oracle_dtw64(qs, x, len, r), (int64_t)row);
            }
        }
        if (stats) {
            stats[(size_t)q * 4 + 0] = visited;
            stats[(size_t)q * 4 + 1] = bounded;
            stats[(size_t)q * 4 + 2] = keogh;
            stats[(size_t)q * 4 + 3] = real;
        }
    }
    free(order);
    free(up);
    free(lo);
    return 0;
}

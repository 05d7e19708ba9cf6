/*
 * messi.h -- C ABI of an MI355X (gfx950) implementation of MESSI's data-parallel
 * hot path: iSAX index construction and exact k-NN search under Euclidean
 * distance (Peng, Fatourou, Palpanas, "MESSI: In-Memory Data Series Indexing",
 * ICDE 2020).
 *
 * Problem (paper, Preliminaries, "Similarity Search"): given a collection of N
 * series of one length L and a query of that length, find the series with the
 * smallest Euclidean distance to the query.  This library returns the k
 * smallest, ordered by (distance, series index): ties go to the lower index.
 *
 * Conventions
 *  - Pointers named series / queries / out_* are DEVICE pointers (memory the
 *    caller allocated on the GPU, e.g. with hipMalloc or a torch CUDA tensor)
 *    unless the name says host_.  A host pointer where a device pointer is
 *    required is rejected with MESSI_EINVAL.
 *  - Series are fp32, row-major [n][len]; series i is the i-th row.
 *  - Every call runs on the calling thread's current HIP device.  The
 *    synchronous calls (messi_build, messi_knn, messi_znorm) return after the
 *    device work has finished.
 *  - Errors: functions returning int return MESSI_OK (0) or a negative
 *    MESSI_E* code; functions returning a pointer return NULL on error.  In
 *    both cases messi_last_error() gives the code and a message (per thread).
 *    A MESSI_EDEVICE error leaves the index unusable: free it and rebuild.
 */
#ifndef MESSI_H
#define MESSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MESSI_OK 0
#define MESSI_EINVAL -1    /* bad argument: null/host pointer, sizes out of range, non-finite input */
#define MESSI_ENOMEM -2    /* device allocation failed or the memory budget is exceeded */
#define MESSI_EDEVICE -3   /* a HIP runtime call or kernel launch failed */
#define MESSI_ENODEV -4    /* no usable GPU */
#define MESSI_EBUSY -5     /* server has no free slot (non-blocking submit) */
#define MESSI_EOVERFLOW -6 /* more candidates tie within rounding of a query's k-th distance than its buffer holds */

#define MESSI_MAX_SEGMENTS 16
#define MESSI_MAX_LEN 1024
#define MESSI_MAX_DTW_BAND 27  /* largest Sakoe-Chiba half-width of messi_knn_dtw */
#define MESSI_MAX_K 1024

/* Search modes of messi_knn_ex. */
#define MESSI_MODE_FP32 0        /* ordered leaf scan, fp32 early-abandoning squared ED */
#define MESSI_MODE_BF16 1        /* BF16 filter with a rounding bound, then exact fp32 distances: a
                                    batch runs the matrix-core filter; a call of one query runs the
                                    FP32 mode's ordered scan, where each member whose word bound
                                    survives is first tested on its BF16 row (half the bytes) */
#define MESSI_MODE_APPROX 2      /* the paper's approximate search (Section 4, approxSearch): the k best
                                    of the members of the leaf with the smallest bound (extended to
                                    the following leaves in depth-first order when it holds fewer
                                    than k, at most 4096 members), ordered by the canonical fp64
                                    distance.  Not exact: no other leaf is visited. */

typedef struct messi_index messi_index;

/* A leaf of the index: per segment i, the node's symbol prefix prefix[i] of
 * card[i] bits (segments >= `segments` are 0), and the range
 * [start, start + count) of the leaf's members in the position array. */
typedef struct {
    uint8_t card[16];
    uint8_t prefix[16];
    uint32_t start;
    uint32_t count;
} messi_leaf;

/* Options of an index (messi_build_ex); a zeroed struct gives the defaults.
 * The build reads znorm, bf16_shadow and stream; the others are kept with the
 * index and govern its searches and servers. */
typedef struct {
    int32_t znorm;       /* 1: z-normalise `series` in place before summarising (see messi_znorm) */
    int32_t bf16_shadow; /* 1: also keep a BF16 copy of every row, in leaf order, and fp32 squared
                            norms; required by MESSI_MODE_BF16 (costs 2 * len bytes per series) */
    void* stream;        /* hipStream_t for the build; NULL = the null stream */
    int32_t mode;        /* search mode of messi_knn (MESSI_MODE_*; MESSI_MODE_BF16 needs bf16_shadow) */
    int32_t max_slots;   /* slot cap of a server created on this index with max_slots = 0 (0: 256) */
    uint64_t budget_bytes; /* device bytes one search workspace (one per stream) may take; a call that
                              needs more fails with MESSI_ENOMEM (0: no cap).  Also the budget of a
                              server created with budget_bytes = 0 (0 there: 8 GiB) */
    int32_t scan_chunk;  /* members per work unit of the ordered scan: 256, 512 or 1024 (0: 512) */
    uint32_t cand_cap;   /* candidate slots per query (0: 2^20 for a call of one query, else 64 k per
                            query, at least 2^14, 2^16 in BF16 mode); at least 2 k is used.  A small
                            value exercises the overflow recovery described at messi_knn_ex */
    int32_t row_filter_max_q; /* MESSI_MODE_BF16 calls of at most this many queries take the ordered
                                 scan with the BF16 row filter instead of the matrix-core filter
                                 (0: 1; negative: never) */
} messi_opts;

typedef struct {
    int64_t n;
    int32_t len, segments, card_bits, leaf_cap;
    int64_t n_leaves;
    int64_t max_leaf;        /* largest leaf (> leaf_cap only for leaves of identical words) */
    int32_t levels;          /* split levels the build ran */
    int32_t has_bf16;
    uint64_t device_bytes;   /* device memory the index owns */
    float data_absmax;       /* max |x| over the collection (used for the bound's slack) */
    double ms_znorm, ms_summarize, ms_bucket, ms_split, ms_finalize, ms_shadow, ms_total;
    int32_t fine_segments;   /* segments of the fine summary the search reads before a row (0: none) */
    int32_t fine_length;     /* values per fine segment */
} messi_info;

/* Per-call counters and timings of messi_knn_ex (totals over the call's queries).
 * Filled only when a non-NULL pointer is passed (counting adds device atomics). */
typedef struct {
    int64_t leaves_total;     /* n_leaves * nq */
    int64_t leaves_kept;      /* (query, leaf) pairs whose bound did not exceed the first upper bound */
    int64_t leaves_scanned;   /* pairs whose members were examined */
    int64_t series_bounded;   /* per-series lower bounds computed (coarse words in the ordered scan) */
    int64_t series_distance;  /* fp32 distances (FP32 mode) or BF16 filter evaluations (BF16 mode) */
    int64_t series_abandoned; /* fp32 distances stopped early */
    int64_t series_recheck;   /* BF16 mode: compensated fp32 rechecks */
    int64_t candidates;       /* canonical fp64 distances computed for the final order */
    int64_t bytes_scan;       /* algorithmic HBM bytes of the scan kernels (words + rows read) */
    double ms_total, ms_prep, ms_leaf_lb, ms_approx, ms_order, ms_scan, ms_final;
    int32_t scan_launches;
    /* scan kernel, per block (device wall clock): mean time in leaf control,
       member filtering and distances, mean and max block lifetime */
    double scan_ms_control, scan_ms_filter, scan_ms_distance, scan_ms_block_mean, scan_ms_block_max;
    /* BF16 mode, and FP32 calls of several queries (the FP32 matrix-core
       filter on the fp32 rows, for rows of a length divisible by 4 and at
       most 256): device time of the filter and of the recheck kernels; BF16
       mode only: the filter's multiply-add work (2 * padded len per pair) */
    double ms_bf16_filter, ms_bf16_recheck;
    int64_t bf16_flops;
    int32_t bf16_rounds;
    /* FP32 mode: queries whose candidate buffer overflowed and whose scan was
       run a second time from the k-th buffered distance */
    int32_t reruns;
    /* BF16 mode and the FP32 filter: queries answered again by the one-query
       FP32 path because their candidate or filter-pair buffer overflowed */
    int32_t fallbacks;
    /* FP32 mode: device time after the first scan pass (candidate fix-up,
       the second pass when needed); ms_scan is then the first pass alone */
    double ms_fixup;
    /* BF16 mode: queries of a leaf staged in LDS at a time by the filter, and
       the most queries any leaf had in one round (above the former, the
       filter stages a leaf's queries in several turns) */
    int32_t bf16_stage_queries;
    int32_t bf16_max_leaf_queries;
    /* ordered scan: members whose full word was bounded (those that passed
       their coarse word's bound; series_bounded counts the coarse bounds),
       and members bounded by their fine summary (those that passed the word
       bound, when the index has a fine summary) */
    int64_t series_word_bounded;
    int64_t series_fine_bounded;
    /* FP32 mode, calls of one query: device time of the scan's first kernel
       (coarse-word and word bounds), within ms_scan */
    double ms_scan_coarse;
} messi_knn_stats;

/* ---- index ------------------------------------------------------------- */

/* Build the iSAX index of series[n][len] (paper: Index Construction, Algorithms
 * CreateIndex, CalculateiSAXSummaries, TreeConstruction).  Per series: PAA over
 * `segments` equal segments, an iSAX word of card_bits-bit symbols against
 * N(0,1) breakpoints, the root child from the top bit of every symbol; then
 * leaves of at most leaf_cap series by balanced binary splits (a leaf holds
 * more only if all its series have the same full word).  `series` is used as
 * given (call messi_znorm first for z-normalised data) and is BORROWED: it must
 * stay valid and unchanged until messi_free.  Limits: 1 <= n < 2^32,
 * 1 <= segments <= 16, len % segments == 0, len <= 1024, 1 <= card_bits <= 8,
 * leaf_cap >= 1.  Non-finite values -> MESSI_EINVAL. */
messi_index* messi_build(const float* series, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                         int32_t leaf_cap);
/* The same with options (opts may be NULL: all defaults).  Beyond messi_build's
 * checks: MESSI_EINVAL for a mode other than MESSI_MODE_*, MESSI_MODE_BF16
 * without bf16_shadow, scan_chunk not in {0, 256, 512, 1024}, max_slots < 0. */
messi_index* messi_build_ex(const float* series, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                            int32_t leaf_cap, const messi_opts* opts);

/* Exact k-NN (paper: Query Answering, Algorithms ExactSearch .. CalculateRealDistance,
 * generalised from 1 to k).  queries[nq][len] (device, fp32); out_idx[nq][k]
 * (device, int64) and out_dist[nq][k] (device, fp32) receive, per query, the k
 * series with the smallest (distance, index), ascending; distances are
 * fl32(sqrt(D)), D the squared distance summed in fp64 in index order.
 * 1 <= k <= min(n, 1024); nq == 0 is a no-op.  Runs in the index's search
 * mode (messi_opts.mode; MESSI_MODE_FP32 by default) on the null stream.
 * Synchronous. */
int messi_knn(const messi_index* index, const float* queries, int32_t nq, int32_t k, int64_t* out_idx,
              float* out_dist);

/* Same, with a k per query, a search mode (MESSI_MODE_*), a stream
 * (hipStream_t, NULL = null stream) and optional counters (stats may be NULL,
 * host memory).
 *   k_per_query  device int32[nq]: query q's k, 1 <= k_per_query[q] <= k_max;
 *                NULL: every query takes k_max
 *   k_max        1 <= k_max <= min(n, 1024): the row length of the outputs
 *   out_idx, out_dist  device [nq][k_max]; row q holds query q's k_per_query[q]
 *                answers, ascending (distance, index), and its remaining
 *                entries are set to index -1 and distance +inf
 * The call synchronises `stream` before returning, so that per-query errors (a
 * non-finite query, a candidate-buffer overflow) are reported by its return
 * code.  Concurrent calls on one index from different streams are allowed;
 * each stream gets its own search workspace (capped by messi_opts.budget_bytes).
 * Every query keeps a buffer of candidate distances (messi_opts.cand_cap).  If
 * a query's buffer overflows, its scan reruns from the k-th buffered distance;
 * if that overflows too, the call (FP32 mode) retries with a buffer 16 times
 * larger, twice at most.  In BF16 mode a query whose candidates or filter pairs
 * overflow their buffers is answered again, alone, in FP32 mode.
 * MESSI_EOVERFLOW remains only for inputs with more exact ties at the k-th
 * distance than the buffer can hold.  MESSI_EINVAL also for k_per_query
 * values outside [1, k_max] (checked before any search work). */
int messi_knn_ex(const messi_index* index, const float* queries, int32_t nq, const int32_t* k_per_query,
                 int32_t k_max, int32_t mode, void* stream, int64_t* out_idx, float* out_dist,
                 messi_knn_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the exact
 * FP32 search of messi_knn_ex (MESSI_MODE_FP32, one k for every query) with
 * no allocation of any kind.  Its search buffers live in one array of static
 * device memory of MESSI_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * library's load until the process ends; the caller passes only the inputs
 * and outputs (device pointers, as messi_knn_ex; out_* are [nq][k]).  The
 * buffers need about 24 bytes per leaf and query plus the candidate buffer
 * (at least 8 MiB for one query, 128 KiB per query of a batch below
 * k = 256, 512 bytes per unit of k above that); a call that needs more than
 * the array holds fails with MESSI_ENOMEM before any device work.  The
 * candidate buffer takes whatever the array has left, and an overflow of it
 * returns MESSI_EOVERFLOW (no retry with a larger buffer).  Every call on a
 * GPU shares that GPU's array: the library serialises the calls of a process
 * (each returns after its stream has finished the work), and calls that
 * overlap on one GPU from outside that lock (another copy of the library)
 * would race.  The array keeps the last call's contents; the kernels clear
 * what must start at zero.  Synchronises `stream` (hipStream_t, NULL = null
 * stream).  Errors as messi_knn_ex. */
#define MESSI_NOALLOC_SCRATCH_BYTES (64ull << 20)
int messi_knn_noalloc(const messi_index* index, const float* queries, int32_t nq, int32_t k, void* stream,
                      int64_t* out_idx, float* out_dist);

void messi_free(messi_index* index); /* NULL-safe; synchronises the device */

int messi_index_info(const messi_index* index, messi_info* out);

/* Words in input order: host_words[n][segments], segment 0 first. */
int messi_export_words(const messi_index* index, uint8_t* host_words);

/* Append series to a built index (paper: Algorithm TreeConstruction inserts
 * each series into the leaf its word reaches and splits a leaf that becomes
 * too full, SplitNode).  `series` is the collection with the new rows after
 * the old ones: rows [0, n) must be the rows the index was built on (it may
 * be a new allocation holding them), rows [n, new_n) are appended.  The new
 * index is the top-down partition of all new_n series in which every node
 * that split before splits on the same segment: the existing splits stay, a
 * leaf that gets no new series keeps its members, a region that held no
 * series gets a leaf, and a leaf over leaf_cap is split by the same balance
 * rule as the build.  The index then borrows `series` (as messi_build does);
 * its BF16 shadow, if any, is rebuilt.  Limits as messi_build (new_n < 2^32,
 * new_n >= n).  Not to be called while searches or a server use the index.
 * On error the index is unchanged.  Synchronous. */
int messi_append(messi_index* index, const float* series, int64_t new_n, void* stream);

/* Leaves in depth-first order (root key ascending, bit 0 before bit 1) and the
 * position array: host_leaves[n_leaves], host_pos[n]; leaf l's members are
 * host_pos[start .. start + count), ascending series index. */
int messi_export_leaves(const messi_index* index, messi_leaf* host_leaves, uint32_t* host_pos);

/* Exact k-NN under dynamic time warping on the same index (paper, closing
 * experiment: the index is unchanged; the query's LB_Keogh envelope is built
 * and the index searched with it; warping window 10% of the length, i.e.
 * band = len / 10).  DTW^2(q, x) is the smallest sum of (q_i - x_j)^2 over the
 * monotone warping paths from (0, 0) to (len-1, len-1) whose cells satisfy
 * |i - j| <= band (a Sakoe-Chiba band); band = 0 is the Euclidean distance.
 * Leaves are visited in ascending envelope bound (per segment, the envelope's
 * extreme values against the node's region), members are bounded by their
 * words, then by LB_Keogh against the envelope, then by the query's distance
 * to the member's own envelope (its min and max over each band window), then
 * get their DTW; the final
 * order is the canonical fp64 DTW (every step rounded once, no fused
 * multiply-add).  Outputs as messi_knn_ex: out_idx[nq][k], out_dist[nq][k] =
 * fl32(sqrt(DTW^2)), ascending (distance, index).  Limits: 0 <= band <= 27,
 * 1 <= k <= min(n, 1024).  Synchronous (stream-ordered work, then a wait).
 * Errors as messi_knn_ex; stats (optional, host) as there, with
 * series_distance = LB_Keogh computed and series_recheck = DTW computed. */
int messi_knn_dtw(const messi_index* index, const float* queries, int32_t nq, int32_t k, int32_t band,
                  void* stream, int64_t* out_idx, float* out_dist, messi_knn_stats* stats);

/* ---- building blocks ---------------------------------------------------- */

/* z-normalise series[n][len] in place (paper, Preliminaries: mean 0, standard
 * deviation 1).  Mean and population variance in fp64, summed in fold-halving
 * order (pad to a power of two with zeros, add the upper half onto the lower
 * half until one value is left); z = fl32((x - mean) / sigma); sigma = 0 gives
 * zeros.  Synchronous when stream == NULL, else stream-ordered. */
int messi_znorm(float* series, int64_t n, int32_t len, void* stream);

/* The windows of a long series as a collection (paper, Preliminaries: a
 * streaming series is cut into subsequences of the query length by a sliding
 * window, and those are indexed).  Writes window r = long_series[r * step ..
 * r * step + len) to out_rows[r][len] for r = 0 .. count - 1, where
 * count = (m - len) / step + 1 (a tail shorter than a step is left out).  With
 * znorm = 1 each window is z-normalised by its own statistics exactly as
 * messi_znorm does (the same fp64 sums, bit for bit); with znorm = 0 it is
 * copied.  long_series[m] and out_rows[count][len] are device memory and must
 * not overlap.  The result is an ordinary collection for messi_build; a k-NN
 * answer's index r is the window starting at r * step.  Limits: 1 <= len <=
 * 1024, m >= len, step >= 1, count < 2^32, znorm in {0, 1}.  Non-finite values
 * with znorm = 1 -> MESSI_EINVAL.  Synchronous. */
int messi_windows(const float* long_series, int64_t m, int32_t len, int64_t step, int32_t znorm, float* out_rows,
                  void* stream);

/* The iSAX breakpoints of card_bits bits: host_out[j - 1] = fl32(Phi^-1(j / 2^b)),
 * j = 1 .. 2^b - 1.  Host-only; needs no GPU. */
int messi_breakpoints(int32_t card_bits, float* host_out);

/* Code and message of the calling thread's last error; returns the code. */
int messi_last_error(char* buf, size_t len);

/* ---- serving (continuous batching) -------------------------------------- */

typedef struct messi_server messi_server;

typedef struct {
    uint64_t tag;        /* as submitted */
    int32_t k;
    int32_t status;      /* MESSI_OK or an error code */
    double t_submit_ms;  /* server clock when submitted */
    double t_done_ms;    /* server clock when the result was ready */
    int64_t idx[MESSI_MAX_K];
    float dist[MESSI_MAX_K];
} messi_result;

/* Server mode flags, OR-ed into `mode` of messi_server_create. */
#define MESSI_SERVER_BATCH_ONLY 0x100 /* BF16: launches of one query also take the matrix-core filter */
#define MESSI_SERVER_NO_GRAPHS 0x200  /* enqueue every launch eagerly instead of replaying HIP graphs */
#define MESSI_SERVER_SLOTS 0x400      /* BF16: the slot engine (one graph replay advances every query by a
                                         window of its leaf order) instead of lanes of batches */

/* A request loop that keeps `index` on the device and answers exact k-NN
 * queries with continuous batching (an extension beyond the paper, which
 * answers queries one after another, Section 5).  Queries submitted while
 * others run are admitted into free slots as soon as a slot frees up and
 * share batched launches; the slots are spread over up to four lanes, each a
 * HIP stream with its own workspace, that run concurrently.  A lane's launch
 * is recorded once per batch shape into a HIP graph and replayed afterwards.
 * In BF16 mode, a query that is alone in the queue when a lane frees up is a
 * launch of one (unless MESSI_SERVER_BATCH_ONLY), since a batch of one gains
 * nothing from the matrix-core filter: the FP32 search when the index has a
 * fine summary (messi_info.fine_segments > 0), else the ordered scan with the
 * BF16 row filter (see messi_knn_ex).  A result never
 * depends on which queries shared its batch: each query carries its own
 * status, and a query whose BF16 buffers overflow is answered again, alone,
 * in FP32 mode before its result is posted.  When most queries of BF16
 * batches overflow (a moving average above one half), batches take the FP32
 * matrix-core filter instead (rows of a length divisible by 4, at most 256),
 * with a BF16 batch every 256 batches.
 *   budget_bytes  device memory the server may use for per-query state; the
 *                 slot count is min(max_slots, budget_bytes / per-query need);
 *                 0 takes the index's messi_opts.budget_bytes (8 GiB if that is 0).
 *                 Launches of one query in FP32 take the split scan, whose
 *                 buffers (4 bytes per series, per lane of up to 4) come out
 *                 of the budget first when it holds them beside one query per
 *                 lane; otherwise those launches use the one-kernel scan.
 *                 A lone query may use its lane's whole candidate buffer; a
 *                 retry after a candidate-buffer overflow takes 16 times that
 *                 (256 times on a second retry), beyond the budget until it
 *                 completes
 *   max_slots     0 takes the index's messi_opts.max_slots (256 if that is 0)
 *   mode          MESSI_MODE_FP32 or MESSI_MODE_BF16 (needs the BF16 shadow),
 *                 optionally OR-ed with MESSI_SERVER_* flags.  With
 *                 MESSI_SERVER_SLOTS (BF16) the slots are those of the slot
 *                 engine: each step (one graph replay) admits queries into
 *                 free slots, advances every active slot by one filter round
 *                 over the next window of its leaf order and retires the
 *                 slots it finishes; one FP32 lane answers lone queries
 *                 (unless MESSI_SERVER_BATCH_ONLY) and retries
 * Returns NULL on error: MESSI_EINVAL (null index, max_slots < 0, bad mode or
 * flags, BF16 without a shadow), MESSI_ENOMEM (budget below one query's need,
 * or an allocation failed), MESSI_EDEVICE.  The index must outlive the
 * server. */
messi_server* messi_server_create(const messi_index* index, size_t budget_bytes, int32_t max_slots, int32_t mode);

/* Copy host_query[len] (host memory, the index's length) and enqueue it.
 * Non-blocking: returns MESSI_OK, MESSI_EINVAL (null pointer, k outside
 * [1, min(n, MESSI_MAX_K)]) or MESSI_EBUSY (2^20 queries already waiting). */
int messi_server_submit(messi_server* server, const float* host_query, int32_t k, uint64_t tag);

/* Move up to max_out finished results into out (host array, caller-owned);
 * returns how many (>= 0) or MESSI_EINVAL.  Results come in completion order. */
int messi_server_poll(messi_server* server, messi_result* out, int32_t max_out);

typedef struct {
    int64_t batches;          /* launches (a batch, or one query alone) */
    int64_t bf16_batches;     /* of which in BF16 mode */
    int64_t row_filter;       /* BF16 launches of one query, answered alone (see above) */
    int64_t requeued;         /* queries re-queued after a buffer overflow */
    int64_t eager_launches;   /* launches enqueued operation by operation */
    int64_t graphs_recorded;  /* launches recorded into a new HIP graph (then replayed) */
    int64_t graph_replays;    /* launches that replayed a recorded graph */
    int32_t lanes, batch;     /* lanes and queries per lane */
    int64_t device_bytes;     /* device memory of the lanes' and the engine's workspaces and staging at
                                 the last launch (within budget_bytes); the HIP runtime's own queue and
                                 scratch memory is not counted */
    int64_t slot_steps;       /* BF16 mode: steps of the slot engine */
    int64_t slot_admitted;    /* BF16 mode: queries admitted into slots */
    int64_t slots;            /* BF16 mode: the engine's slots */
} messi_server_counters;

/* Counters of the server so far (host struct, caller-owned).  MESSI_OK or
 * MESSI_EINVAL (null argument). */
int messi_server_stats(messi_server* server, messi_server_counters* out);

/* Milliseconds on the server clock (the one t_submit_ms / t_done_ms use). */
double messi_server_clock_ms(const messi_server* server);

/* Drop the queries still waiting for a slot (they get no result), finish the
 * admitted ones, stop the worker and free everything.  NULL-safe. */
void messi_server_destroy(messi_server* server);

#ifdef __cplusplus
}
#endif

#endif /* MESSI_H */

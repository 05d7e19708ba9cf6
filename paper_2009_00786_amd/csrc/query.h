// Query-side state shared by the FP32 and BF16 search paths and the server.
#pragma once

#include "common.h"

namespace messi {

constexpr int kNB = 1024;            // lower-bound bins used to order the surviving leaves
constexpr int kApproxMax = 4096;     // members of the first leaf evaluated for the first bound
constexpr int kApproxBlocks = 128;   // blocks per query for that leaf
constexpr int kMaxFinal = 4096;      // candidates ordered by fp64 distance per query
constexpr int kChunk = 1024;         // members filtered per step of the scan

// Relative error margins (see the exactness notes in query.hip).
constexpr float kRhoEd = 1.52587890625e-05f;  // 2^-16, fp32 squared-distance error margin
constexpr float kRhoLb = 2.44140625e-04f;     // 2^-12, lower-bound error margin

struct Cand {
    float d;       // fp32 squared distance
    uint32_t idx;  // series index
};

// Per-query search state (device).
struct QState {
    float paa[16];
    float norm2;
    float delta;             // widening of every region (covers fp32 PAA error of data and query)
    uint32_t U;              // current upper bound on the k-th squared distance (float bits)
    uint32_t ncand;          // candidates appended
    uint32_t ticket;         // next position in the ordered leaf list
    uint32_t nsurv;          // leaves in the ordered list
    uint32_t done;           // no more leaves can improve the answer
    uint32_t lbmax;          // max leaf bound (float bits)
    unsigned long long argmin;  // (bound bits << 32) | leaf of the smallest bound
    uint32_t approx_leaf;
    uint32_t approx_full;    // the first leaf was evaluated completely
    float range;             // bound range mapped onto the bins
    int32_t k;
    uint32_t err;            // 0 ok, 1 non-finite query, 2 candidate overflow, 3 final overflow, 4 too few
    uint32_t active;         // slot in use (server); 1 for plain calls
    uint32_t kstride;        // output row stride
    uint32_t pad0;
};

// Counters accumulated over a call (device).
struct QCounters {
    unsigned long long kept, scanned, bounded, distance, abandoned, recheck, final_cands, bytes;
};

struct QArgs {
    const float* series;
    int64_t n;
    int32_t L, w, m, b;
    const uint4* words;
    const uint32_t* pos;
    const Leaf* leaves;
    int32_t nL;
    const float* bp;
    const float* norms;          // bf16 path: squared norms in leaf order
    const uint16_t* shadow;      // bf16 path: bf16 rows in leaf order
    const float* queries;        // [nq][L]
    int32_t nq;
    QState* qs;
    float* lb;                   // [nq][nL]
    uint32_t* order;             // [nq][nL]
    uint32_t* bins;              // [nq][kNB]
    uint32_t* cursor;            // [nq][kNB]
    float* approx_d;             // [nq][kApproxMax]
    Cand* cand;                  // [nq][cap]
    uint32_t cap;
    float absmax_data;
    int32_t lg_m;                // ceil(log2 m)
    QCounters* counters;         // nullptr = no counting
    uint32_t* err_any;
    unsigned long long* prof;    // nullptr = no phase timing; else [blocks][4]
    int64_t* out_idx;
    float* out_dist;
};

// Per-(index, stream) search workspace, grown on demand.
struct Workspace {
    int32_t nq = 0, nL = 0;
    uint32_t cap = 0;
    DevBuf qs, lb, order, bins, cursor, approx_d, cand, counters, err, prof;
    // BF16 path
    int32_t bf_nq = 0;
    size_t bf_pairs_cap = 0, bf_leafq_cap = 0;
    DevBuf qb, qnorm, leaf_cnt, leaf_off, leaf_cur, leaf_q, pairs, npairs, scan_scr;
    // timing of the BF16 kernels of the last call (filled when timing is on)
    double bf_ms_filter = 0, bf_ms_recheck = 0;
    int bf_rounds = 0;
};

// The batched BF16 filter + compensated fp32 recheck (bf16.hip); runs after the
// shared prefix (prep, leaf bounds, first bound, leaf order) and before the
// shared fp64 final ordering.
int bf16_scan(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s, bool timing);

// For k > 1, lower every query's bound to its current k-th candidate distance.
int refresh_bounds(QArgs& a, hipStream_t s);

// Enqueue a whole search on `s` without waiting (used by the server): kq is an
// optional device array of per-query k (<= kmax; outputs have row stride kmax);
// the call's error flags are copied to *host_err (pinned) when the stream
// reaches that point.  knn_error_code turns those flags into a MESSI_E* code.
int knn_enqueue(const Index* ix, const float* queries, int32_t nq, int32_t kmax, const int32_t* kq, int32_t mode,
                hipStream_t s, int64_t* out_idx, float* out_dist, uint32_t* host_err);
int knn_error_code(uint32_t err);

}  // namespace messi

// Query-side state shared by the FP32 and BF16 search paths and the server.
#pragma once

#include <algorithm>

#include "common.h"

namespace messi {

constexpr int kNB = 1024;            // lower-bound bins used to order the surviving leaves
constexpr int kApproxMax = 4096;     // members of the first leaf evaluated for the first bound
// blocks per query for that leaf: for one or two queries a wave per member
// of a full leaf, so no wave waits on a second row
inline int approx_blocks(int nq) { return nq <= 2 ? 512 : nq <= 8 ? 256 : 128; }
constexpr int kMaxFinal = 4096;      // candidates ordered by fp64 distance per query
constexpr int kChunk = 1024;         // most members per scan work unit (the index's scan_chunk: 256, 512 or 1024)
constexpr int kHistBins = 4096;      // candidate-distance histogram (k > 1 bound)
constexpr int kSplitMaxQ = 1;        // calls of at most this many queries run the split Euclidean scan

// Relative error margins (see the exactness notes in query.hip).
constexpr float kRhoEd = 1.52587890625e-05f;  // 2^-16, fp32 squared-distance error margin
constexpr float kRhoLb = 2.44140625e-04f;     // 2^-12, lower-bound error margin
constexpr float kRhoDtw = 2.44140625e-04f;    // 2^-12, fp32 banded-DTW error margin (L <= 1024)

struct Cand {
    float d;       // fp32 squared distance
    uint32_t idx;  // series index
};

// One surviving leaf at its place in the bound order.
struct OrdRec {
    uint32_t start;  // first member (leaf order)
    uint32_t count;  // members
    float lb;        // lower bound of the leaf
    uint32_t moff;   // members of all earlier leaves in the order
};

// One leaf-bound block's share of the smallest leaf bound and the largest one.
struct LbPart {
    unsigned long long key;  // (bound bits << 32) | leaf, smallest in the block
    uint32_t mx;             // largest bound bits in the block
    uint32_t pad;
};

// Scan statistics per block: scanned leaves, members bounded by their coarse
// word, members that reached the distance stage, abandoned, bytes read, fp32
// distances after a BF16 row test, BF16 rows tested, members bounded by their
// full word, members bounded by their fine summary.
constexpr int kBlkCnt = 9;

// Per-query search state (device).
struct QState {
    float paa[16];           // ED: the query PAA; DTW: per segment the envelope's minimum
    float paa_hi[16];        // ED: the query PAA; DTW: per segment the envelope's maximum
    float norm2;
    float delta;             // widening of every region (covers fp32 PAA error of data and query)
    uint32_t U;              // current upper bound on the k-th squared distance (float bits)
    uint32_t ncand;          // candidates appended
    uint32_t nmemb;          // members of the ordered leaves
    uint32_t nsurv;          // leaves in the ordered list
    uint32_t ovf;            // the candidate buffer overflowed in this pass
    uint32_t lbmax;          // max leaf bound (float bits)
    unsigned long long argmin;  // (bound bits << 32) | leaf of the smallest bound
    float range;             // bound range mapped onto the bins
    int32_t k;
    uint32_t err;            // 0 ok, 1 non-finite query, 2 candidate overflow, 3 final overflow, 4 too few
    uint32_t active;         // slot in use (server); 1 for plain calls
    uint32_t kstride;        // output row stride
    int32_t hbase;           // histogram bin of a distance = (float bits >> 16) - hbase, clamped
    uint32_t rerun;          // the scan runs a second pass from a tightened bound
    float qamax;             // largest |value| of the query
    uint32_t skip_start;     // first member of the leaf whose distances the first bound appended
                             //   as candidates (the scan's first pass skips it); ~0: none
};

// Counters accumulated over a call (device).
struct QCounters {
    unsigned long long kept, scanned, bounded, distance, abandoned, recheck, final_cands, bytes, reruns;
};

struct QArgs {
    const float* series;
    int64_t n;
    int32_t L, w, m, b;
    const uint4* words;
    const uint2* cwords;         // [n] coarse words, leaf order
    const uint8_t* fwords;       // [n][kFineStride] fine summaries, input order (nullptr: none)
    int32_t wf, mf, lg_mf;       // fine segments, their length, ceil(log2 mf)
    int32_t csh;                 // coarse symbol = symbol >> csh
    int32_t skip_approx;         // 1: the first bound's leaf is appended as candidates, not scanned (split scan)
    uint32_t approx_min;         // exact search: the first bound's members reach at least this many (the
                                 //   approximate search takes the leaf alone: 0)
    const uint32_t* pos;
    const Leaf* leaves;
    int32_t nL;
    const float* bp;
    const uint16_t* shadow;      // bf16 path: bf16 rows in leaf order [n][Lp]
    // BF16 row filter of the ordered scan (bf16_row_prep fills these)
    const uint2* sx;             // [n] member terms of the filter's extra k-step
    const uint16_t* qb;          // [nq][Lp] 2 q rounded to BF16
    const float2* qnorm;         // [nq] (|q|^2, |q|) from fp64 sums
    const uint4* qx;             // [nq] query terms of the extra k-step
    int32_t Lp;                  // BF16 row length (L rounded up to 32)
    float one_minus_h;           // 1 - h of the drop test, rounded down
    float rf_tau;                // the row filter runs while U > rf_tau |q|^2
    // DTW search
    int32_t band;                // Sakoe-Chiba half-width; < 0: Euclidean search
    float rho_d;                 // relative error margin of the distances kept (ED or DTW)
    uint32_t chunk;              // members per scan chunk (<= kChunk)
    uint32_t chunk_lo, chunk_hi; // the scan takes chunks [chunk_lo, chunk_hi) of each query's order
    Cand* todo;                  // [nq][todo_nseg][todo_seg] DTW: (LB_Keogh, series) waiting for their DTW,
    uint32_t todo_cap;           //   a segment per scan block of the query; todo_cap = todo_nseg * todo_seg
    uint32_t todo_seg, todo_nseg;
    uint32_t* todo_cnt;          // [nq][todo_nseg] entries in each segment
    float* env;                  // [nq][2][L] DTW: the query's envelope, upper then lower
    Cand* ec;                    // [nq][ec_nseg][ec_seg] DTW: waiting series within the candidate-side bound,
    uint32_t ec_cap;             //   a segment per block of the bound kernel; ec_cap = ec_nseg * ec_seg
    uint32_t ec_seg, ec_nseg;
    uint32_t* ec_cnt;            // [nq][ec_nseg] entries in each segment
    const float* queries;        // [nq][L]
    int32_t nq;
    QState* qs;
    float* lb;                   // [nq][nL]
    uint32_t* order;             // [nq][nL] leaf ids in bound order
    OrdRec* rec;                 // [nq][nL] the same leaves with start, count, bound, member offset
    uint32_t* chunk_first;       // [nq][max_chunks] order position holding the first member of each chunk
    uint32_t max_chunks;
    uint32_t* bins;              // [nq][kNB] leaves per bound bin
    uint32_t* mbins;             // [nq][kNB] members per bound bin
    unsigned long long* cursor;  // [nq][kNB] per bin: (leaves placed << 32 | their members), zeroed per call
    uint32_t* hist;              // [nq][kHistBins] candidate-distance histogram
    float* approx_d;             // [nq][kApproxMax]
    LbPart* lbpart;              // [nq][leaf-bound blocks]
    Cand* cand;                  // [nq][cap]
    uint32_t* seg;               // split scan: [nq][max_chunks][chunk] word survivors of each chunk (nullptr: no split)
    uint32_t* segcnt;            // split scan: [nq][max_chunks] their counts
    uint32_t cap;
    float absmax_data;
    int32_t lg_m;                // ceil(log2 m)
    QCounters* counters;         // nullptr = no counting
    uint32_t* err_any;
    uint32_t* host_err;          // one-query calls: mapped pinned host word the final kernel stores its error
                                 //   bit in as well (the host zeroes it first), so no read-back copy is needed
    unsigned long long* prof;    // nullptr = no phase timing; else [blocks][4]
    unsigned long long* blk_cnt; // scan counters per block [blocks][5] (with counters)
    int64_t* out_idx;
    float* out_dist;
    // the serving engine's slots (nullptr for a plain call): a kernel of the
    // query head runs for slots in kSlotAdmit only, a filter round for slots in
    // kSlotActive (over their window of the leaf order), the final kernel for
    // slots in kSlotFinal
    uint32_t* phase;             // [nq]
    uint32_t* win;               // [nq][3]: window of order positions [r0, r1) this step, and the round
};

// Wait for the stream before a workspace buffer is reallocated.  Refused
// (MESSI_EDEVICE, nothing waited for) while the stream is being captured
// into a graph, so that a capture never records an allocation: the caller
// then runs the launch eagerly, which sizes the workspace.
inline int growth_sync(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        set_error(MESSI_EDEVICE, "a search workspace would grow while its stream is being captured");
        return MESSI_EDEVICE;
    }
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    return MESSI_OK;
}

// Phases of a slot of the serving engine.
constexpr uint32_t kSlotFree = 0, kSlotAdmit = 1, kSlotActive = 2, kSlotFinal = 3, kSlotDone = 4;

// Whether the slot of query q sits out a kernel meant for slots in `want`.
__device__ __forceinline__ bool slot_off(const QArgs& a, int q, uint32_t want) {
    return a.phase != nullptr && a.phase[q] != want;
}

// Per-(index, stream) search workspace, grown on demand.
struct Workspace {
    uint64_t gen = 0;  // bumped whenever a buffer is reallocated (recorded graphs hold the old addresses)
    int32_t nq = 0, nL = 0;
    size_t cand_slots = 0;  // candidate slots over all queries (a call uses nq * cap of them)
    uint32_t max_chunks = 0;
    DevBuf qs, lb, order, rec, chunk_first, bins, mbins, cursor, hist, approx_d, cand, counters, err, prof, blk_cnt,
        status, lbpart;
    DevBuf seg, segcnt;  // split scan (calls of at most kSplitMaxQ queries)
    int32_t seg_nq = 0;
    DevBuf slot_phase, slot_win, slot_q, slot_k;  // the serving engine's slots
    int32_t slot_n = 0;
    DevBuf todo, env, todo_cnt, ec, ec_cnt;  // DTW search
    size_t todo_slots = 0, env_floats = 0, todo_cnt_n = 0, ec_slots = 0, ec_cnt_n = 0;
    uint32_t* h_err = nullptr;  // pinned copy of the call's error flags
    uint32_t* h_flag = nullptr;  // mapped, coherent pinned word for one-query calls (host address)
    uint32_t* d_flag = nullptr;  //   and its device address
    // BF16 path
    int32_t bf_nq = 0;
    size_t bf_pairs_cap = 0, bf_leafq_cap = 0;
    DevBuf qb, qnorm, qx, leaf_cnt, leaf_off, leaf_cur, leaf_q, leaf_act, pairs, npairs;
    // timing of the BF16 kernels of the last call (filled when timing is on)
    double bf_ms_filter = 0, bf_ms_recheck = 0;
    int bf_rounds = 0, bf_stage_queries = 0, bf_max_leaf_q = 0;
    // statistics read-back: phase events and pinned staging, made on first use
    hipEvent_t ev[9] = {};
    QCounters* h_counters = nullptr;
    unsigned long long* h_prof = nullptr;    // [4096][4]
    unsigned long long* h_blk_cnt = nullptr; // [4096][5]
    int ensure_stats();
    // device bytes held by the workspace's buffers
    size_t device_bytes() const;
    // (Re)allocate b with `bytes` bytes unless that takes the workspace past the
    // index's budget_bytes option (MESSI_ENOMEM).  b is empty after a failure.
    int grow(const Index* ix, DevBuf& b, size_t bytes);
    ~Workspace();
};

// The batched BF16 filter + compensated fp32 recheck (bf16.hip); runs after the
// shared prefix (prep, leaf bounds, first bound, leaf order) and before the
// shared fp64 final ordering.
// f32: the FP32 filter on the fp32 rows instead (f32_filter_ok(ix) must
// hold); probe: the call may wait on the stream to see how wide its batch is
// (else it takes the FP32 filter's growing rounds).
int bf16_scan(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s, bool timing, bool f32 = false,
              bool probe = false);
// Whether the FP32 filter takes the index's rows (length a multiple of 4, at
// most 256, rows 16-byte aligned).
bool f32_filter_ok(const Index* ix);

// One BF16 filter round of the serving engine's active slots (a.phase, a.win).
int bf16_slot_round(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s);

// The BF16 row filter of the ordered scan: per query 2 q in BF16, its norms
// and the extra k-step terms (into the workspace), and the filter's fields of a.
int bf16_row_prep(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s);

// Whether a BF16-mode call of nq queries runs the ordered scan with the BF16
// row filter (few queries) instead of the batched matrix-core filter.
bool row_filter_path(const Index* ix, int32_t mode, int32_t nq, bool matrix_only);

// For k > 1, lower every query's bound to its current k-th candidate distance.
int refresh_bounds(QArgs& a, hipStream_t s);

// Enqueue a whole search on `s` without waiting (used by the server): kq is an
// optional device array of per-query k (<= kmax; outputs have row stride kmax);
// the call's error flags are copied to *host_err (pinned) and, if host_status
// is given, every query's own status to host_status[nq] (pinned) when the
// stream reaches that point.  knn_error_code turns the flags into a MESSI_E*
// code, query_error_code a query's status.
// cap_min raises the per-query candidate buffer above its default.
// matrix_only keeps a BF16 call of few queries on the matrix-core filter.
// split = false keeps a one-query FP32 call off the split scan (and its
// workspace free of the split_scan_bytes it would take).  cap_limit (nonzero)
// caps the default candidate buffer per query (never below 2 kmax; cap_min
// still raises it).
int knn_enqueue(const Index* ix, const float* queries, int32_t nq, int32_t kmax, const int32_t* kq, int32_t mode,
                hipStream_t s, int64_t* out_idx, float* out_dist, uint32_t* host_err, uint32_t* host_status,
                uint32_t cap_min = 0, bool matrix_only = false, bool split = true, uint32_t cap_limit = 0);
// Host-mapped arrays (their device addresses) through which the server and
// the serving engine's step exchange slots: S slots, rows of the index's length.
struct SlotIO {
    const uint32_t* ctl;   // [S] nonzero: the slot takes the query staged for it in this step
    const float* q;        // [S][L] staged queries
    const int32_t* k;      // [S] their k
    uint32_t* phase;       // [S] every slot's phase after the step (kSlot*)
    uint32_t* status;      // [S] a slot finished in the step: its QState::err (0: answered)
    int64_t* idx;          // [S][MESSI_MAX_K] a finished slot's answer (row stride MESSI_MAX_K)
    float* dist;           // [S][MESSI_MAX_K]
};

// Enqueue one step of the serving engine on s (BF16 mode, an index with the
// BF16 shadow): slots marked in io.ctl are admitted (the query head: bounds,
// first bound, leaf order); every active slot takes one filter round over the
// next window of its leaf order (16 positions, then four times the previous
// window, at most 65536); a slot whose order is exhausted, or whose next leaf
// lies in a bin wholly above its U, gets its final answer; io.phase and
// io.status report every slot.  Capturable in a HIP graph once a first call
// has sized the workspace (it allocates only when the slot count grows).
int slot_step_enqueue(const Index* ix, hipStream_t s, int32_t S, const SlotIO& io);

// Device bytes a workspace holds whatever its query count (statistics
// staging, the BF16 filter's per-leaf counters).
size_t workspace_fixed_bytes(const Index* ix);
// Device bytes of the split scan's survivor segments and counts, held by the
// workspace of a stream once a one-query FP32 call has run on it.
size_t split_scan_bytes(const Index* ix);
// Exact FP32 k-NN of nq queries at one k (as knn_enqueue in MESSI_MODE_FP32)
// with every search buffer carved from the device region [base, base + bytes)
// (256-byte aligned) instead of a workspace: allocates nothing.  The
// candidate buffers take the room left after the fixed buffers.  MESSI_ENOMEM
// when even the default candidate buffer does not fit.  Waits for the stream;
// the region's earlier contents do not matter (the kernels clear what must
// start at zero).
int knn_view(const Index* ix, const float* queries, int32_t nq, int32_t k, hipStream_t s, int64_t* out_idx,
             float* out_dist, void* base, size_t bytes);
// Default candidate slots per query for a call of nq queries with k <= kmax.
uint32_t default_cap(const Index* ix, int32_t nq, int32_t kmax, int32_t mode);
int knn_error_code(uint32_t err);
int query_error_code(uint32_t status);

// Slots of the BF16 filter's (query, member) survivor list for a batch of nq.
inline size_t bf16_pairs_cap(int32_t nq) { return std::min<size_t>((size_t)nq * 65536, (size_t)1 << 28); }

// Device bytes of search workspace one query needs (for a memory budget).
size_t workspace_bytes_per_query(const Index* ix, int32_t mode, uint32_t cap);

// Generation of the (index, stream) workspace, 0 if there is none yet.
uint64_t workspace_generation(const Index* ix, hipStream_t s);

}  // namespace messi

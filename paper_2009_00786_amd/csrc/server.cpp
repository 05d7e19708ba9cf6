// Request loop with continuous batching over a resident index.
//
// The server owns a worker thread and a few "lanes"; a lane is a HIP stream
// with its own pinned staging buffers and search workspace.  Submitted queries
// wait in a FIFO; whenever a lane is free, the worker moves up to the lane's
// batch size of waiting queries into it and enqueues one batched search
// (mixed k allowed) on the lane's stream without waiting.  Lanes run
// concurrently, so queries that arrive while other batches are on the GPU are
// admitted as soon as a lane frees up and their work overlaps on the device.
// The lane count and batch size follow from the device-memory budget: every
// admitted query holds its share of a lane's workspace until it completes.
//
// In BF16 mode a lone waiting query (the queue holds at most one when a lane
// frees up) becomes a launch of one: a batch of one gains nothing from the
// matrix-core filter, whose cost is a pass over the BF16 rows of every leaf
// the query visits.  On an index with a fine summary it runs the FP32
// search, whose one-query scan bounds each member by its coarse word, word
// and fine summary before any row; otherwise the ordered scan with the BF16
// row filter (half a row per member that passes its word).  As soon as
// queries queue up they go in batches on the matrix-core filter.
//
// With MESSI_SERVER_SLOTS (BF16) the batches give way to a slot engine: S
// slots on one stream, and a step (one replay of a recorded HIP graph) that
// admits the queries placed in free slots (their head: bounds, first bound,
// leaf order), runs one BF16 filter round in which every active slot takes
// the next window of its own leaf order (16 positions, then four times the
// last), and finishes every slot whose order is exhausted or whose next leaf
// lies in a bin wholly above its bound.  A query retires at the end of the
// step that finishes it; its slot takes a waiting query in the next step.
// Slots and host exchange queries, phases and answers through mapped pinned
// memory.  Lone queries and retries go to one FP32 lane.
//
// A BF16 batch whose queries mostly overflow the filter's buffers (its
// margin is too wide for the data: short rows, many near-equal distances)
// costs a filter pass and then every query again alone; when that share
// exceeds one half (a moving average over BF16 batches), batches go to the
// FP32 matrix-core filter instead, with a BF16 batch every 256 to notice
// when BF16 pays again.
//
// A lane's whole launch (copies in, the search, copies out) is recorded once
// per batch shape (query count, largest k, mode, buffer size) into a HIP graph
// and replayed afterwards: the first batch of a shape runs eagerly, which
// also sizes the workspace, the second records the graph.  A graph is dropped
// when the workspace it points into is reallocated.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <thread>
#include <vector>

#include "query.h"

namespace messi {

void release_workspace(const Index* ix, hipStream_t s);
size_t workspace_device_bytes(const Index* ix, hipStream_t s);
int trim_candidates(const Index* ix, hipStream_t s, size_t slots);

namespace {

struct Pending {
    std::vector<float> q;
    int32_t k;
    uint64_t tag;
    double t_submit;
    bool fp32 = false;  // answered alone in FP32 mode (after a buffer overflow)
    int grow = 0;       // its candidate buffer is 16^grow times the default
};

// A recorded launch: the shape it was recorded for decides everything the
// launch does (grids, buffer sizes); the lane's buffers are fixed.
typedef std::tuple<int32_t, int32_t, int32_t, uint32_t> Shape;  // nq, kmax, mode, cap_min

struct Recorded {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;  // workspace generation it was recorded against
};

constexpr size_t kMaxGraphsPerLane = 256;

struct Lane {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    int32_t kmax = 0;
    int32_t mode = MESSI_MODE_BF16;  // of the batch in flight
    std::set<Shape> seen;            // shapes run eagerly once
    std::map<Shape, Recorded> graphs;
    DevBuf d_q, d_k, d_idx, d_dist;
    float* h_q = nullptr;
    int32_t* h_k = nullptr;
    int64_t* h_idx = nullptr;
    float* h_dist = nullptr;
    uint32_t* h_err = nullptr;
    uint32_t* h_status = nullptr;  // per query of the batch in flight
    uint32_t cap_min = 0;          // of the launch in flight
    std::vector<Pending> batch;
    size_t staging_bytes() const { return d_q.bytes + d_k.bytes + d_idx.bytes + d_dist.bytes; }
};

// The BF16 serving engine: S slots on one stream, advanced together one step
// (one replay of a recorded graph) at a time.  Host and device exchange
// slots through mapped pinned memory (io holds the device addresses).
struct Engine {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    int32_t S = 0;
    bool busy = false;
    uint32_t* h_ctl = nullptr;
    float* h_q = nullptr;
    int32_t* h_k = nullptr;
    uint32_t* h_phase = nullptr;
    uint32_t* h_status = nullptr;
    int64_t* h_idx = nullptr;
    float* h_dist = nullptr;
    SlotIO io{};
    std::vector<Pending> held;  // the query each slot holds
    std::vector<char> used;
    int32_t n_used = 0;
    Recorded step;              // the recorded step
};

constexpr size_t kMaxPending = 1u << 20;
// candidate slots the budget charges per admitted query: enough for any k
constexpr uint32_t kSlotCap = std::max<uint32_t>(1u << 14, 64u * MESSI_MAX_K);

}  // namespace

struct Server {
    const Index* ix = nullptr;
    int32_t mode = MESSI_MODE_BF16;
    bool row_filter = true;  // BF16 mode: a launch of one query is answered alone, off the matrix-core filter
    bool split = true;       // FP32 launches of one query take the split scan (its buffers are in the budget)
    uint32_t lane_cap = kSlotCap;  // candidate slots of a lane (batch x kSlotCap): a lone query may use them all
    // BF16 mode: the share of a BF16 batch's queries that overflowed (moving
    // average); above one half, batches go to the FP32 matrix-core filter
    // (every 256th batch still tries BF16, to notice when it pays again)
    double bf16_overflow = 0.0;
    int64_t fp32_batches_since = 0;
    bool f32_filter = false;  // the index's rows suit the FP32 filter
    bool use_graphs = true;
    int32_t batch = 1;  // queries per lane
    messi_server_counters stats{};  // guarded by mu
    std::vector<Lane> lanes;
    Engine eng;         // BF16 mode: the slot engine (the lanes answer lone queries and retries in FP32)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> pending;
    std::deque<messi_result*> ready;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int device = 0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }

    // The lane's launch as stream operations: copies in, the search, copies out.
    int enqueue(Lane& ln, int32_t nq, uint32_t cap_min) {
        const int L = ix->len;
        MESSI_HIP_TRY(hipMemcpyAsync(ln.d_q.p, ln.h_q, sizeof(float) * (size_t)nq * L, hipMemcpyHostToDevice, ln.s));
        MESSI_HIP_TRY(hipMemcpyAsync(ln.d_k.p, ln.h_k, sizeof(int32_t) * (size_t)nq, hipMemcpyHostToDevice, ln.s));
        MESSI_TRY(knn_enqueue(ix, ln.d_q.as<float>(), nq, ln.kmax, ln.d_k.as<int32_t>(), ln.mode, ln.s,
                              ln.d_idx.as<int64_t>(), ln.d_dist.as<float>(), ln.h_err, ln.h_status, cap_min,
                              !row_filter, split, lane_cap));
        MESSI_HIP_TRY(hipMemcpyAsync(ln.h_idx, ln.d_idx.p, sizeof(int64_t) * (size_t)nq * ln.kmax,
                                     hipMemcpyDeviceToHost, ln.s));
        MESSI_HIP_TRY(hipMemcpyAsync(ln.h_dist, ln.d_dist.p, sizeof(float) * (size_t)nq * ln.kmax,
                                     hipMemcpyDeviceToHost, ln.s));
        return MESSI_OK;
    }

    static void drop_graph(Recorded& r) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        r.exec = nullptr;
    }

    // Record the lane's launch for this shape; false (and the stream left as it
    // was) if recording is not possible, then the caller runs it eagerly.
    bool record(Lane& ln, int32_t nq, uint32_t cap_min, Recorded& out) {
        if (hipStreamBeginCapture(ln.s, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        const int rc = enqueue(ln, nq, cap_min);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ln.s, &g);
        hipGraphExec_t exec = nullptr;
        bool ok = rc == MESSI_OK && ec == hipSuccess && g &&
                  hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            (void)hipGetLastError();
            clear_error();
            if (exec) (void)hipGraphExecDestroy(exec);
            return false;
        }
        out.exec = exec;
        out.gen = workspace_generation(ix, ln.s);
        return true;
    }

    int launch(Lane& ln) {
        const int L = ix->len;
        const int32_t nq = (int32_t)ln.batch.size();
        int32_t kmax = 1;
        for (int32_t i = 0; i < nq; ++i) {
            std::memcpy(ln.h_q + (size_t)i * L, ln.batch[i].q.data(), sizeof(float) * L);
            ln.h_k[i] = ln.batch[i].k;
            kmax = std::max(kmax, ln.batch[i].k);
        }
        ln.kmax = kmax;
        ln.mode = ln.batch[0].fp32 ? MESSI_MODE_FP32 : mode;
        // a lone query on an index with a fine summary: the FP32 search, whose
        // one-query scan bounds members by their fine summary (64 bytes) before
        // any row, where the row-filtered scan reads a 512-byte BF16 row
        if (ln.mode == MESSI_MODE_BF16 && nq == 1 && row_filter && ix->wf > 0) ln.mode = MESSI_MODE_FP32;
        if (ln.mode == MESSI_MODE_BF16 && nq > 1 && f32_filter && bf16_overflow > 0.5) {
            if (++fp32_batches_since % 256 != 0) ln.mode = MESSI_MODE_FP32;
        }
        *ln.h_err = 0;
        // a retry after an overflow: 16 times the lane's slots per retry, a
        // transient excess over the budget (the lane drops it afterwards)
        uint32_t cap_min = 0;
        if (ln.batch[0].fp32 && ln.batch[0].grow > 0)
            cap_min = (uint32_t)std::min<uint64_t>((uint64_t)lane_cap << (4 * ln.batch[0].grow), 1ull << 28);
        ln.cap_min = cap_min;
        const Shape shape{nq, kmax, ln.mode, cap_min};
        bool replayed = false, recorded = false;
        if (use_graphs) {
            auto it = ln.graphs.find(shape);
            if (it != ln.graphs.end() && it->second.gen != workspace_generation(ix, ln.s)) {
                // the workspace moved since the recording: drop every graph of the lane
                for (auto& kv : ln.graphs) drop_graph(kv.second);
                ln.graphs.clear();
                ln.seen.clear();
                it = ln.graphs.end();
            }
            if (it == ln.graphs.end() && ln.seen.count(shape) && ln.graphs.size() < kMaxGraphsPerLane) {
                Recorded r;
                if (record(ln, nq, cap_min, r)) {
                    it = ln.graphs.emplace(shape, r).first;
                    recorded = true;
                }
            }
            if (it != ln.graphs.end()) {
                MESSI_HIP_TRY(hipGraphLaunch(it->second.exec, ln.s));
                replayed = !recorded;
            }
        }
        if (!replayed && !recorded) {
            MESSI_TRY(enqueue(ln, nq, cap_min));
            ln.seen.insert(shape);
        }
        MESSI_HIP_TRY(hipEventRecord(ln.done, ln.s));
        ln.busy = true;
        // (this thread alone grows the lanes' workspaces)
        size_t dev_bytes = 0;
        for (const Lane& l : lanes) dev_bytes += workspace_device_bytes(ix, l.s) + l.staging_bytes();
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.device_bytes = (int64_t)dev_bytes;
            stats.batches += 1;
            if (ln.mode == MESSI_MODE_BF16) stats.bf16_batches += 1;
            if (row_filter_path(ix, ln.mode, nq, !row_filter) || (nq == 1 && row_filter && mode == MESSI_MODE_BF16))
                stats.row_filter += 1;
            if (recorded) stats.graphs_recorded += 1;
            if (replayed) stats.graph_replays += 1;
            if (!recorded && !replayed) stats.eager_launches += 1;
        }
        return MESSI_OK;
    }

    // A finished batch: per query, its own status decides.  A query whose
    // buffers overflowed goes back to the head of the queue to be answered
    // alone in FP32 mode (from a BF16 batch), or alone with a 16 times larger
    // candidate buffer (twice at most); every other query gets its result.
    // launch_status != MESSI_OK (the launch or the stream failed) applies to all.
    void complete(Lane& ln, int launch_status) {
        const double t = now_ms();
        std::vector<messi_result*> out;
        std::vector<Pending> redo;
        int64_t fallbacks = 0;
        out.reserve(ln.batch.size());
        for (size_t i = 0; i < ln.batch.size(); ++i) {
            const int status = launch_status != MESSI_OK ? launch_status : query_error_code(ln.h_status[i]);
            if (status == MESSI_EOVERFLOW && (!ln.batch[i].fp32 || ln.batch[i].grow < 2)) {
                Pending p = std::move(ln.batch[i]);
                fallbacks += 1;
                if (!p.fp32) {
                    // alone in FP32 mode; with a larger buffer only if it was
                    // alone in FP32 mode already
                    p.fp32 = true;
                    p.grow = ln.mode == MESSI_MODE_FP32 && ln.batch.size() == 1 ? 1 : 0;
                } else {
                    ++p.grow;
                }
                redo.push_back(std::move(p));
                continue;
            }
            messi_result* r = new messi_result();
            std::memset(r, 0, sizeof(*r));
            r->tag = ln.batch[i].tag;
            r->k = ln.batch[i].k;
            r->status = status;
            r->t_submit_ms = ln.batch[i].t_submit;
            r->t_done_ms = t;
            if (status == MESSI_OK) {
                for (int j = 0; j < r->k; ++j) {
                    r->idx[j] = ln.h_idx[i * (size_t)ln.kmax + j];
                    r->dist[j] = ln.h_dist[i * (size_t)ln.kmax + j];
                }
            }
            out.push_back(r);
        }
        if (ln.mode == MESSI_MODE_BF16 && ln.batch.size() > 1 && launch_status == MESSI_OK)
            bf16_overflow = 0.75 * bf16_overflow + 0.25 * (double)fallbacks / (double)ln.batch.size();
        ln.batch.clear();
        ln.busy = false;
        // a retry's larger candidate buffer goes back; the lane's graphs hold
        // its address, and every shape runs eagerly once more (which sizes the
        // workspace again) before it is recorded
        if (ln.cap_min > lane_cap) {
            if (trim_candidates(ix, ln.s, lane_cap) != MESSI_OK) {
                (void)hipGetLastError();
                clear_error();
            }
            for (auto& kv : ln.graphs) drop_graph(kv.second);
            ln.graphs.clear();
            ln.seen.clear();
        }
        ln.cap_min = 0;
        size_t dev_bytes = eng.S ? workspace_device_bytes(ix, eng.s) : 0;
        for (const Lane& l : lanes) dev_bytes += workspace_device_bytes(ix, l.s) + l.staging_bytes();
        std::lock_guard<std::mutex> lk(mu);
        stats.device_bytes = (int64_t)dev_bytes;
        stats.requeued += fallbacks;
        for (auto* r : out) ready.push_back(r);
        for (auto it = redo.rbegin(); it != redo.rend(); ++it) pending.push_front(std::move(*it));
    }

    // ---- the slot engine ----------------------------------------------------
    int engine_enqueue() { return slot_step_enqueue(ix, eng.s, eng.S, eng.io); }

    bool engine_record() {
        if (hipStreamBeginCapture(eng.s, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        const int rc = engine_enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(eng.s, &g);
        hipGraphExec_t exec = nullptr;
        bool ok = rc == MESSI_OK && ec == hipSuccess && g &&
                  hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            (void)hipGetLastError();
            clear_error();
            if (exec) (void)hipGraphExecDestroy(exec);
            return false;
        }
        eng.step.exec = exec;
        eng.step.gen = workspace_generation(ix, eng.s);
        return true;
    }

    // One step: the recorded graph when it still matches the workspace, else
    // the step's operations (and a new recording for the next step).
    int engine_launch() {
        bool recorded = false, replayed = false;
        if (use_graphs) {
            if (eng.step.exec && eng.step.gen != workspace_generation(ix, eng.s)) drop_graph(eng.step);
            if (!eng.step.exec) recorded = engine_record();
            if (eng.step.exec) {
                MESSI_HIP_TRY(hipGraphLaunch(eng.step.exec, eng.s));
                replayed = !recorded;
            }
        }
        if (!recorded && !replayed) MESSI_TRY(engine_enqueue());
        MESSI_HIP_TRY(hipEventRecord(eng.done, eng.s));
        eng.busy = true;
        size_t dev_bytes = workspace_device_bytes(ix, eng.s);
        for (const Lane& l : lanes) dev_bytes += workspace_device_bytes(ix, l.s) + l.staging_bytes();
        std::lock_guard<std::mutex> lk(mu);
        stats.device_bytes = (int64_t)dev_bytes;
        stats.slot_steps += 1;
        stats.batches += 1;
        stats.bf16_batches += 1;
        if (recorded) stats.graphs_recorded += 1;
        if (replayed) stats.graph_replays += 1;
        if (!recorded && !replayed) stats.eager_launches += 1;
        return MESSI_OK;
    }

    // After a step: every slot it finished posts its result (or, after a
    // buffer overflow, goes back to the queue to be answered alone in FP32).
    void engine_collect(int launch_status) {
        const double t = now_ms();
        std::vector<messi_result*> out;
        std::vector<Pending> redo;
        for (int32_t q = 0; q < eng.S; ++q) {
            eng.h_ctl[q] = 0;
            if (!eng.used[q]) continue;
            if (launch_status == MESSI_OK && eng.h_phase[q] != kSlotDone) continue;  // still searching
            const int status = launch_status != MESSI_OK ? launch_status : query_error_code(eng.h_status[q]);
            Pending& p = eng.held[q];
            eng.used[q] = 0;
            --eng.n_used;
            if (status == MESSI_EOVERFLOW) {
                p.fp32 = true;
                p.grow = 0;
                redo.push_back(std::move(p));
                continue;
            }
            messi_result* r = new messi_result();
            std::memset(r, 0, sizeof(*r));
            r->tag = p.tag;
            r->k = p.k;
            r->status = status;
            r->t_submit_ms = p.t_submit;
            r->t_done_ms = t;
            if (status == MESSI_OK) {
                for (int j = 0; j < r->k; ++j) {
                    r->idx[j] = eng.h_idx[(size_t)q * MESSI_MAX_K + j];
                    r->dist[j] = eng.h_dist[(size_t)q * MESSI_MAX_K + j];
                }
            }
            out.push_back(r);
        }
        eng.busy = false;
        std::lock_guard<std::mutex> lk(mu);
        stats.requeued += (int64_t)redo.size();
        for (auto* r : out) ready.push_back(r);
        for (auto it = redo.rbegin(); it != redo.rend(); ++it) pending.push_front(std::move(*it));
    }

    // Free slots take waiting queries (not the re-queued ones, which the
    // FP32 lanes answer); true if any slot is in use.
    bool engine_admit() {
        std::lock_guard<std::mutex> lk(mu);
        const int L = ix->len;
        int32_t q = 0;
        for (auto it = pending.begin(); it != pending.end() && eng.n_used < eng.S;) {
            if (it->fp32) {
                ++it;
                continue;
            }
            while (eng.used[q]) ++q;
            std::memcpy(eng.h_q + (size_t)q * L, it->q.data(), sizeof(float) * L);
            eng.h_k[q] = it->k;
            eng.h_ctl[q] = 1;
            eng.held[q] = std::move(*it);
            eng.used[q] = 1;
            ++eng.n_used;
            stats.slot_admitted += 1;
            it = pending.erase(it);
        }
        return eng.n_used > 0;
    }

    void run() {
        (void)hipSetDevice(device);
        for (;;) {
            bool progressed = false;
            for (auto& ln : lanes) {
                if (!ln.busy) continue;
                const hipError_t q = hipEventQuery(ln.done);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) (void)hipGetLastError();
                complete(ln, q == hipSuccess ? MESSI_OK : MESSI_EDEVICE);
                progressed = true;
            }
            if (eng.S && eng.busy) {
                const hipError_t q = hipEventQuery(eng.done);
                if (q != hipErrorNotReady) {
                    if (q != hipSuccess) (void)hipGetLastError();
                    engine_collect(q == hipSuccess ? MESSI_OK : MESSI_EDEVICE);
                    progressed = true;
                }
            }
            for (auto& ln : lanes) {
                if (ln.busy) continue;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    if (eng.S) {
                        // with the engine: a re-queued query, or a query alone in
                        // the queue while the engine is idle (unless batch-only)
                        for (auto it = pending.begin(); it != pending.end(); ++it)
                            if (it->fp32) {
                                ln.batch.push_back(std::move(*it));
                                pending.erase(it);
                                break;
                            }
                        if (ln.batch.empty() && row_filter && pending.size() == 1 && !eng.busy && eng.n_used == 0) {
                            ln.batch.push_back(std::move(pending.front()));
                            pending.pop_front();
                        }
                    } else {
                        // a batch, or a re-queued query on its own in FP32 mode
                        while (!pending.empty() && (int32_t)ln.batch.size() < batch) {
                            const bool alone = pending.front().fp32;
                            if (alone && !ln.batch.empty()) break;
                            ln.batch.push_back(std::move(pending.front()));
                            pending.pop_front();
                            if (alone) break;
                        }
                    }
                }
                if (ln.batch.empty()) continue;
                const int rc = launch(ln);
                if (rc != MESSI_OK) complete(ln, rc);
                progressed = true;
            }
            if (eng.S && !eng.busy && engine_admit()) {
                const int rc = engine_launch();
                if (rc != MESSI_OK) {
                    clear_error();
                    engine_collect(rc);
                }
                progressed = true;
            }
            bool any_busy = eng.busy;
            for (auto& ln : lanes) any_busy |= ln.busy;
            if (stop.load() && !any_busy) {
                std::lock_guard<std::mutex> lk(mu);
                if (pending.empty()) break;
            }
            if (!progressed) {
                // nothing could start: wait for a submission or a launch to end
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 500));
            }
        }
    }

    ~Server() {
        if (eng.s) {
            drop_graph(eng.step);
            (void)hipStreamSynchronize(eng.s);
            release_workspace(ix, eng.s);
            (void)hipStreamDestroy(eng.s);
        }
        if (eng.done) (void)hipEventDestroy(eng.done);
        for (void* p : {(void*)eng.h_ctl, (void*)eng.h_q, (void*)eng.h_k, (void*)eng.h_phase, (void*)eng.h_status,
                        (void*)eng.h_idx, (void*)eng.h_dist})
            if (p) (void)hipHostFree(p);
        for (auto& ln : lanes) {
            for (auto& kv : ln.graphs) drop_graph(kv.second);
            if (ln.s) {
                (void)hipStreamSynchronize(ln.s);
                release_workspace(ix, ln.s);
                (void)hipStreamDestroy(ln.s);
            }
            if (ln.done) (void)hipEventDestroy(ln.done);
            for (void* p : {(void*)ln.h_q, (void*)ln.h_k, (void*)ln.h_idx, (void*)ln.h_dist, (void*)ln.h_err,
                            (void*)ln.h_status})
                if (p) (void)hipHostFree(p);
        }
        for (auto* r : ready) delete r;
    }
};

// Device bytes one admitted query holds (workspace share + staging), for kmax
// results; used to turn the memory budget into slots.
static size_t bytes_per_query(const Index* ix, int32_t mode) {
    return workspace_bytes_per_query(ix, mode, kSlotCap) + sizeof(float) * ix->len +
           (sizeof(int64_t) + sizeof(float)) * MESSI_MAX_K + 256;
}

}  // namespace messi

using namespace messi;

extern "C" {

messi_server* messi_server_create(const messi_index* index, size_t budget_bytes, int32_t max_slots, int32_t mode) {
    clear_error();
    if (!index) {
        set_error(MESSI_EINVAL, "index is null");
        return nullptr;
    }
    if (max_slots < 0) {
        set_error(MESSI_EINVAL, "max_slots must be >= 0");
        return nullptr;
    }
    const int32_t flags = mode & ~0xff;
    mode &= 0xff;
    if ((mode != MESSI_MODE_FP32 && mode != MESSI_MODE_BF16) ||
        (flags & ~(MESSI_SERVER_BATCH_ONLY | MESSI_SERVER_NO_GRAPHS | MESSI_SERVER_SLOTS)) ||
        ((flags & MESSI_SERVER_SLOTS) && mode != MESSI_MODE_BF16)) {
        set_error(MESSI_EINVAL, "unknown mode");
        return nullptr;
    }
    const Index* ix = reinterpret_cast<const Index*>(index);
    if (mode == MESSI_MODE_BF16 && !ix->shadow.p) {
        set_error(MESSI_EINVAL, "BF16 serving needs an index built with bf16_shadow = 1");
        return nullptr;
    }
    // zero takes the index's options
    if (max_slots == 0) max_slots = ix->opts.max_slots;
    if (budget_bytes == 0) budget_bytes = ix->opts.budget_bytes ? (size_t)ix->opts.budget_bytes : (size_t)8 << 30;
    const bool engine = (flags & MESSI_SERVER_SLOTS) != 0;
    // Lanes of batches (up to 4); or, with MESSI_SERVER_SLOTS, the slot
    // engine and one FP32 lane of one query (lone queries and retries).
    const size_t per_q = bytes_per_query(ix, engine ? MESSI_MODE_FP32 : mode);
    const size_t per_slot = engine ? bytes_per_query(ix, MESSI_MODE_BF16) : per_q;
    // An FP32 launch of one query (FP32 mode, a lone BF16 query, a retry)
    // takes the split scan, whose segments each lane's workspace then holds:
    // they come out of the budget first, if it holds them beside one query
    // per lane (and one slot); else those launches go without.
    const size_t seg_b = split_scan_bytes(ix);
    const size_t nl_max = engine ? 1 : (size_t)std::min(4, max_slots);
    // every workspace (each lane's, the engine's) holds some bytes whatever its size
    const size_t fixed = (nl_max + (engine ? 1 : 0)) * workspace_fixed_bytes(ix);
    const size_t need1 = fixed + nl_max * (seg_b + per_q) + (engine ? per_slot : 0);
    const bool split = budget_bytes >= need1;
    size_t room = budget_bytes >= fixed ? budget_bytes - fixed : 0;
    if (split) room -= nl_max * seg_b;
    if (engine) room = room >= per_q ? room - per_q : 0;  // the FP32 lane's query
    const int64_t fit = (int64_t)(room / per_slot);
    if (fit < 1) {
        set_error(MESSI_ENOMEM, "memory budget below the need of one query (" + std::to_string(per_slot) + " bytes)");
        return nullptr;
    }
    const int32_t slots = (int32_t)std::min<int64_t>(max_slots, fit);
    Server* sv = new Server();
    sv->ix = ix;
    sv->mode = mode;
    sv->row_filter = !(flags & MESSI_SERVER_BATCH_ONLY);
    sv->use_graphs = !(flags & MESSI_SERVER_NO_GRAPHS);
    sv->split = split;
    sv->f32_filter = f32_filter_ok(ix);
    sv->device = ix->device;
    const int nl = engine ? 1 : std::min(4, slots);
    sv->batch = engine ? 1 : slots / nl;   // (lanes x batch <= slots: within the budget)
    sv->lane_cap = (uint32_t)std::min<uint64_t>((uint64_t)sv->batch * kSlotCap, 1ull << 28);
    sv->lanes.resize(nl);
    const int32_t lane_mode = engine ? MESSI_MODE_FP32 : mode;
    const int L = ix->len;
    int rc = MESSI_OK;
    for (auto& ln : sv->lanes) {
        const size_t B = (size_t)sv->batch;
        if (hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_q, sizeof(float) * B * L, 0) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_k, sizeof(int32_t) * B, 0) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_idx, sizeof(int64_t) * B * MESSI_MAX_K, 0) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_dist, sizeof(float) * B * MESSI_MAX_K, 0) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_err, sizeof(uint32_t), 0) != hipSuccess ||
            hipHostMalloc((void**)&ln.h_status, sizeof(uint32_t) * B, 0) != hipSuccess) {
            (void)hipGetLastError();
            set_error(MESSI_ENOMEM, "server: stream or pinned buffer allocation failed");
            rc = MESSI_ENOMEM;
            break;
        }
        if ((rc = ln.d_q.alloc(sizeof(float) * B * L)) != MESSI_OK) break;
        if ((rc = ln.d_k.alloc(sizeof(int32_t) * B)) != MESSI_OK) break;
        if ((rc = ln.d_idx.alloc(sizeof(int64_t) * B * MESSI_MAX_K)) != MESSI_OK) break;
        if ((rc = ln.d_dist.alloc(sizeof(float) * B * MESSI_MAX_K)) != MESSI_OK) break;
        // size the lane's workspace once: a full batch of copies of row 0, k = the maximum
        if (hipMemcpyAsync(ln.d_q.p, ix->series, sizeof(float) * L, hipMemcpyDeviceToDevice, ln.s) != hipSuccess) {
            rc = MESSI_EDEVICE;
            break;
        }
        for (size_t i = 1; i < B; ++i)
            if (hipMemcpyAsync(ln.d_q.as<float>() + i * L, ix->series, sizeof(float) * L, hipMemcpyDeviceToDevice,
                               ln.s) != hipSuccess) {
                rc = MESSI_EDEVICE;
                break;
            }
        const int32_t kw = (int32_t)std::min<int64_t>(MESSI_MAX_K, ix->n);
        for (size_t i = 0; i < B; ++i) ln.h_k[i] = kw;
        if (rc != MESSI_OK || hipMemcpyAsync(ln.d_k.p, ln.h_k, sizeof(int32_t) * B, hipMemcpyHostToDevice, ln.s) != hipSuccess) {
            rc = MESSI_EDEVICE;
            break;
        }
        *ln.h_err = 0;
        if ((rc = knn_enqueue(ix, ln.d_q.as<float>(), (int32_t)B, kw, ln.d_k.as<int32_t>(), lane_mode, ln.s,
                              ln.d_idx.as<int64_t>(), ln.d_dist.as<float>(), ln.h_err, ln.h_status, 0, false, true,
                              sv->lane_cap)) != MESSI_OK)
            break;
        // and a launch of one in FP32 (the split scan's segments)
        if (split && (rc = knn_enqueue(ix, ln.d_q.as<float>(), 1, kw, ln.d_k.as<int32_t>(), MESSI_MODE_FP32, ln.s,
                                       ln.d_idx.as<int64_t>(), ln.d_dist.as<float>(), ln.h_err, ln.h_status, 0,
                                       false, true, sv->lane_cap)) != MESSI_OK)
            break;
        if (hipStreamSynchronize(ln.s) != hipSuccess) {
            rc = MESSI_EDEVICE;
            break;
        }
    }
    if (rc == MESSI_OK && engine) {
        // the engine: mapped pinned slot arrays, its stream, and a first
        // (empty) step that sizes its workspace
        Engine& e = sv->eng;
        const size_t S = (size_t)slots;
        e.S = slots;
        e.held.resize(S);
        e.used.assign(S, 0);
        const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
        if (hipStreamCreateWithFlags(&e.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&e.h_ctl, sizeof(uint32_t) * S, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_q, sizeof(float) * S * L, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_k, sizeof(int32_t) * S, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_phase, sizeof(uint32_t) * S, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_status, sizeof(uint32_t) * S, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_idx, sizeof(int64_t) * S * MESSI_MAX_K, fl) != hipSuccess ||
            hipHostMalloc((void**)&e.h_dist, sizeof(float) * S * MESSI_MAX_K, fl) != hipSuccess) {
            (void)hipGetLastError();
            set_error(MESSI_ENOMEM, "server: engine stream or pinned buffer allocation failed");
            rc = MESSI_ENOMEM;
        }
        if (rc == MESSI_OK) {
            std::memset(e.h_ctl, 0, sizeof(uint32_t) * S);
            void* d = nullptr;
            auto dev = [&](void* h) -> void* {
                d = nullptr;
                if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) rc = MESSI_EDEVICE;
                return d;
            };
            e.io.ctl = (const uint32_t*)dev(e.h_ctl);
            e.io.q = (const float*)dev(e.h_q);
            e.io.k = (const int32_t*)dev(e.h_k);
            e.io.phase = (uint32_t*)dev(e.h_phase);
            e.io.status = (uint32_t*)dev(e.h_status);
            e.io.idx = (int64_t*)dev(e.h_idx);
            e.io.dist = (float*)dev(e.h_dist);
        }
        if (rc == MESSI_OK) rc = sv->engine_enqueue();
        if (rc == MESSI_OK && hipStreamSynchronize(e.s) != hipSuccess) rc = MESSI_EDEVICE;
    }
    if (rc != MESSI_OK) {
        const int code = last_error_code();
        delete sv;
        if (code == MESSI_OK) set_error(rc, "server creation failed");
        return nullptr;
    }
    sv->t0 = std::chrono::steady_clock::now();
    sv->worker = std::thread([sv] { sv->run(); });
    return reinterpret_cast<messi_server*>(sv);
}

int messi_server_submit(messi_server* server, const float* host_query, int32_t k, uint64_t tag) {
    clear_error();
    if (!server || !host_query) {
        set_error(MESSI_EINVAL, "null argument");
        return MESSI_EINVAL;
    }
    Server* sv = reinterpret_cast<Server*>(server);
    if (k < 1 || k > MESSI_MAX_K || (int64_t)k > sv->ix->n) {
        set_error(MESSI_EINVAL, "k must be in [1, min(n, 1024)]");
        return MESSI_EINVAL;
    }
    Pending p;
    p.q.assign(host_query, host_query + sv->ix->len);
    p.k = k;
    p.tag = tag;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pending.size() >= kMaxPending) {
            set_error(MESSI_EBUSY, "too many queries waiting");
            return MESSI_EBUSY;
        }
        p.t_submit = sv->now_ms();
        sv->pending.push_back(std::move(p));
    }
    sv->cv.notify_one();
    return MESSI_OK;
}

int messi_server_poll(messi_server* server, messi_result* out, int32_t max_out) {
    clear_error();
    if (!server || (!out && max_out > 0) || max_out < 0) {
        set_error(MESSI_EINVAL, "bad argument");
        return MESSI_EINVAL;
    }
    Server* sv = reinterpret_cast<Server*>(server);
    int32_t n = 0;
    std::lock_guard<std::mutex> lk(sv->mu);
    while (n < max_out && !sv->ready.empty()) {
        messi_result* r = sv->ready.front();
        sv->ready.pop_front();
        out[n++] = *r;
        delete r;
    }
    return n;
}

int messi_server_stats(messi_server* server, messi_server_counters* out) {
    clear_error();
    if (!server || !out) {
        set_error(MESSI_EINVAL, "null argument");
        return MESSI_EINVAL;
    }
    Server* sv = reinterpret_cast<Server*>(server);
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->lanes = (int32_t)sv->lanes.size();
    out->batch = sv->batch;
    out->slots = sv->eng.S;
    return MESSI_OK;
}

double messi_server_clock_ms(const messi_server* server) {
    if (!server) return 0.0;
    return reinterpret_cast<const Server*>(server)->now_ms();
}

void messi_server_destroy(messi_server* server) {
    if (!server) return;
    Server* sv = reinterpret_cast<Server*>(server);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->pending.clear();
    }
    sv->stop.store(true);
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    delete sv;
}

}  // extern "C"

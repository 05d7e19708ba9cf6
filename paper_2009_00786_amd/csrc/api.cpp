// C ABI of the library (include/messi.h): argument checking, error state,
// index lifecycle and host-side exports.  Device work lives in build.hip,
// query.hip, bf16.hip and server.cpp.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"

namespace messi {

namespace {
thread_local int t_code = MESSI_OK;
thread_local std::string t_msg;
}  // namespace

void set_error(int code, const std::string& msg) {
    t_code = code;
    t_msg = msg;
}
void clear_error() {
    t_code = MESSI_OK;
    t_msg.clear();
}
int last_error_code() { return t_code; }

int DevBuf::alloc(size_t n) {
    release();
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        set_error(e == hipErrorOutOfMemory ? MESSI_ENOMEM : MESSI_EDEVICE,
                  std::string("hipMalloc(") + std::to_string(n) + " bytes): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? MESSI_ENOMEM : MESSI_EDEVICE;
    }
    bytes = n;
    return MESSI_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

Index::~Index() {}

bool is_device_pointer(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int current_device_ok() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        set_error(MESSI_ENODEV, "no HIP device available");
        return MESSI_ENODEV;
    }
    return MESSI_OK;
}

static int fail(int code, const char* msg) {
    set_error(code, msg);
    return code;
}

static void fill_info(Index* ix) {
    messi_info& in = ix->info;
    in.n = ix->n;
    in.len = ix->len;
    in.segments = ix->w;
    in.card_bits = ix->b;
    in.leaf_cap = ix->cap;
    in.n_leaves = ix->n_leaves;
    in.max_leaf = ix->max_leaf;
    in.levels = ix->levels;
    in.has_bf16 = ix->shadow.p != nullptr;
    in.device_bytes = ix->device_bytes();
    in.data_absmax = ix->absmax;
    in.fine_segments = ix->wf;
    in.fine_length = ix->mf;
}

// Take over everything src holds (src keeps dst's old buffers, to be freed).
static void adopt(Index* dst, Index* src) {
    std::swap(dst->series, src->series);
    std::swap(dst->n, src->n);
    std::swap(dst->n_leaves, src->n_leaves);
    std::swap(dst->max_leaf, src->max_leaf);
    std::swap(dst->levels, src->levels);
    std::swap(dst->absmax, src->absmax);
    std::swap(dst->split_mask, src->split_mask);
    std::swap(dst->n_inner, src->n_inner);
    std::swap(dst->info, src->info);
    std::swap(dst->wf, src->wf);
    std::swap(dst->mf, src->mf);
    DevBuf* a[] = {&dst->words, &dst->pos, &dst->leaves, &dst->bp, &dst->sx, &dst->shadow, &dst->split_keys,
                   &dst->split_seg, &dst->split_claim, &dst->cwords, &dst->fwords};
    DevBuf* b[] = {&src->words, &src->pos, &src->leaves, &src->bp, &src->sx, &src->shadow, &src->split_keys,
                   &src->split_seg, &src->split_claim, &src->cwords, &src->fwords};
    for (size_t i = 0; i < sizeof(a) / sizeof(a[0]); ++i) {
        DevBuf t = std::move(*a[i]);
        *a[i] = std::move(*b[i]);
        *b[i] = std::move(t);
    }
}

}  // namespace messi

using namespace messi;

extern "C" {

int messi_last_error(char* buf, size_t len) {
    if (buf && len) {
        std::snprintf(buf, len, "%s", t_msg.c_str());
    }
    return t_code;
}

int messi_breakpoints(int32_t card_bits, float* host_out) {
    clear_error();
    if (card_bits < 1 || card_bits > 8) return fail(MESSI_EINVAL, "card_bits must be in [1, 8]");
    if (!host_out) return fail(MESSI_EINVAL, "host_out is null");
    breakpoints_as241(card_bits, host_out);
    return MESSI_OK;
}

static int check_series_args(const float* series, int64_t n, int32_t len) {
    if (n < 1 || n >= (int64_t(1) << 32)) return fail(MESSI_EINVAL, "n must be in [1, 2^32)");
    if (len < 1 || len > MESSI_MAX_LEN) return fail(MESSI_EINVAL, "len must be in [1, 1024]");
    if (!series) return fail(MESSI_EINVAL, "series is null");
    MESSI_TRY(current_device_ok());
    if (!is_device_pointer(series)) return fail(MESSI_EINVAL, "series is not a device pointer");
    return MESSI_OK;
}

int messi_znorm(float* series, int64_t n, int32_t len, void* stream) {
    clear_error();
    MESSI_TRY(check_series_args(series, n, len));
    hipStream_t s = (hipStream_t)stream;
    DevBuf flag;
    MESSI_TRY(flag.alloc(sizeof(int)));
    MESSI_HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    MESSI_TRY(znorm_device(series, n, len, s, flag.as<int>()));
    int h = 0;
    MESSI_HIP_TRY(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    if (h) return fail(MESSI_EINVAL, "series contain non-finite values");
    return MESSI_OK;
}

int messi_windows(const float* long_series, int64_t m, int32_t len, int64_t step, int32_t znorm, float* out_rows,
                  void* stream) {
    clear_error();
    if (len < 1 || len > MESSI_MAX_LEN) return fail(MESSI_EINVAL, "len must be in [1, 1024]");
    if (m < len) return fail(MESSI_EINVAL, "the long series is shorter than one window");
    if (step < 1) return fail(MESSI_EINVAL, "step must be >= 1");
    if (znorm != 0 && znorm != 1) return fail(MESSI_EINVAL, "znorm must be 0 or 1");
    const int64_t count = (m - len) / step + 1;
    if (count >= (int64_t(1) << 32)) return fail(MESSI_EINVAL, "more than 2^32 - 1 windows");
    if (!long_series || !out_rows) return fail(MESSI_EINVAL, "null pointer");
    MESSI_TRY(current_device_ok());
    if (!is_device_pointer(long_series)) return fail(MESSI_EINVAL, "long_series is not a device pointer");
    if (!is_device_pointer(out_rows)) return fail(MESSI_EINVAL, "out_rows is not a device pointer");
    const uintptr_t a0 = (uintptr_t)long_series, a1 = a0 + (uintptr_t)m * sizeof(float);
    const uintptr_t b0 = (uintptr_t)out_rows, b1 = b0 + (uintptr_t)count * (uintptr_t)len * sizeof(float);
    if (a0 < b1 && b0 < a1) return fail(MESSI_EINVAL, "out_rows overlaps long_series");
    hipStream_t s = (hipStream_t)stream;
    DevBuf flag;
    MESSI_TRY(flag.alloc(sizeof(int)));
    MESSI_HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    MESSI_TRY(windows_device(long_series, count, len, step, znorm == 1, out_rows, s, flag.as<int>()));
    int h = 0;
    MESSI_HIP_TRY(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    if (h) return fail(MESSI_EINVAL, "long_series contains non-finite values");
    return MESSI_OK;
}

// The options checked and their defaults filled in (no device call).
static int check_opts(const messi_opts* opts, messi_opts& o) {
    o = messi_opts{};
    if (opts) o = *opts;
    if (o.mode != MESSI_MODE_FP32 && o.mode != MESSI_MODE_BF16 && o.mode != MESSI_MODE_APPROX)
        return fail(MESSI_EINVAL, "opts.mode must be a MESSI_MODE_* value");
    if (o.mode == MESSI_MODE_BF16 && !o.bf16_shadow)
        return fail(MESSI_EINVAL, "opts.mode = MESSI_MODE_BF16 needs opts.bf16_shadow = 1");
    if (o.scan_chunk != 0 && o.scan_chunk != 256 && o.scan_chunk != 512 && o.scan_chunk != 1024)
        return fail(MESSI_EINVAL, "opts.scan_chunk must be 0, 256, 512 or 1024");
    if (o.max_slots < 0) return fail(MESSI_EINVAL, "opts.max_slots must be >= 0");
    if (o.znorm != 0 && o.znorm != 1) return fail(MESSI_EINVAL, "opts.znorm must be 0 or 1");
    if (o.bf16_shadow != 0 && o.bf16_shadow != 1) return fail(MESSI_EINVAL, "opts.bf16_shadow must be 0 or 1");
    if (o.scan_chunk == 0) o.scan_chunk = 512;
    if (o.max_slots == 0) o.max_slots = 256;
    if (o.row_filter_max_q == 0) o.row_filter_max_q = 1;
    return MESSI_OK;
}

messi_index* messi_build_ex(const float* series, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                            int32_t leaf_cap, const messi_opts* opts) {
    clear_error();
    if (segments < 1 || segments > MESSI_MAX_SEGMENTS) {
        fail(MESSI_EINVAL, "segments must be in [1, 16]");
        return nullptr;
    }
    if (len >= 1 && len % segments != 0) {
        fail(MESSI_EINVAL, "len must be a multiple of segments");
        return nullptr;
    }
    if (card_bits < 1 || card_bits > 8) {
        fail(MESSI_EINVAL, "card_bits must be in [1, 8]");
        return nullptr;
    }
    if (leaf_cap < 1) {
        fail(MESSI_EINVAL, "leaf_cap must be >= 1");
        return nullptr;
    }
    messi_opts o;
    if (check_opts(opts, o) != MESSI_OK) return nullptr;
    if (check_series_args(series, n, len) != MESSI_OK) return nullptr;
    Index* ix = new Index();
    if (hipGetDevice(&ix->device) != hipSuccess) ix->device = 0;
    ix->opts = o;
    ix->opts.stream = nullptr;  // the build's stream only
    int rc = build_index(ix, series, n, len, segments, card_bits, leaf_cap, o);
    if (rc == MESSI_OK && o.bf16_shadow) rc = build_bf16_shadow(ix, (hipStream_t)o.stream);
    if (rc != MESSI_OK) {
        const int code = t_code;
        const std::string msg = t_msg;
        (void)hipDeviceSynchronize();
        delete ix;
        set_error(code, msg);
        return nullptr;
    }
    fill_info(ix);
    return reinterpret_cast<messi_index*>(ix);
}

int messi_append(messi_index* index, const float* series, int64_t new_n, void* stream) {
    clear_error();
    if (!index) return fail(MESSI_EINVAL, "index is null");
    Index* ix = reinterpret_cast<Index*>(index);
    if (new_n < ix->n) return fail(MESSI_EINVAL, "new_n is below the indexed count");
    MESSI_TRY(check_series_args(series, new_n, ix->len));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != ix->device)
        return fail(MESSI_EINVAL, "the index lives on another device");
    hipStream_t s = (hipStream_t)stream;
    MESSI_HIP_TRY(hipDeviceSynchronize());  // searches on other streams are done with the old arrays
    Index* nx = new Index();
    nx->device = ix->device;
    nx->opts = ix->opts;
    messi_opts o{};
    o.stream = stream;
    const SplitTab tab{ix->split_keys.as<uint4>(), ix->split_seg.as<uint8_t>(), ix->split_claim.as<uint32_t>(),
                       ix->split_mask};
    int rc = build_index(nx, series, new_n, ix->len, ix->w, ix->b, ix->cap, o, &tab);
    if (rc == MESSI_OK && ix->shadow.p) rc = build_bf16_shadow(nx, s);
    if (rc != MESSI_OK) {
        const int code = last_error_code();
        char msg[512];
        messi_last_error(msg, sizeof msg);
        (void)hipDeviceSynchronize();
        delete nx;
        set_error(code, msg);
        return code;
    }
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    release_workspaces(ix);  // sized for the old leaf count
    adopt(ix, nx);
    fill_info(ix);
    delete nx;  // the old arrays
    return MESSI_OK;
}

messi_index* messi_build(const float* series, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                         int32_t leaf_cap) {
    return messi_build_ex(series, n, len, segments, card_bits, leaf_cap, nullptr);
}

void messi_free(messi_index* index) {
    if (!index) return;
    Index* ix = reinterpret_cast<Index*>(index);
    (void)hipDeviceSynchronize();
    release_workspaces(ix);
    release_bf16(ix);
    delete ix;
}

int messi_index_info(const messi_index* index, messi_info* out) {
    clear_error();
    if (!index || !out) return fail(MESSI_EINVAL, "null argument");
    *out = reinterpret_cast<const Index*>(index)->info;
    return MESSI_OK;
}

int messi_export_words(const messi_index* index, uint8_t* host_words) {
    clear_error();
    if (!index || !host_words) return fail(MESSI_EINVAL, "null argument");
    const Index* ix = reinterpret_cast<const Index*>(index);
    std::vector<uint8_t> w(16 * (size_t)ix->n);
    std::vector<uint32_t> p((size_t)ix->n);
    MESSI_HIP_TRY(hipMemcpy(w.data(), ix->words.p, w.size(), hipMemcpyDeviceToHost));
    MESSI_HIP_TRY(hipMemcpy(p.data(), ix->pos.p, sizeof(uint32_t) * p.size(), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < ix->n; ++j)
        std::memcpy(host_words + (size_t)p[j] * ix->w, &w[16 * (size_t)j], (size_t)ix->w);
    return MESSI_OK;
}

int messi_export_leaves(const messi_index* index, messi_leaf* host_leaves, uint32_t* host_pos) {
    clear_error();
    if (!index || !host_leaves || !host_pos) return fail(MESSI_EINVAL, "null argument");
    const Index* ix = reinterpret_cast<const Index*>(index);
    static_assert(sizeof(messi_leaf) == sizeof(Leaf), "leaf layout");
    MESSI_HIP_TRY(hipMemcpy(host_leaves, ix->leaves.p, sizeof(Leaf) * (size_t)ix->n_leaves, hipMemcpyDeviceToHost));
    MESSI_HIP_TRY(hipMemcpy(host_pos, ix->pos.p, sizeof(uint32_t) * (size_t)ix->n, hipMemcpyDeviceToHost));
    return MESSI_OK;
}

int messi_knn_ex(const messi_index* index, const float* queries, int32_t nq, const int32_t* k_per_query,
                 int32_t k_max, int32_t mode, void* stream, int64_t* out_idx, float* out_dist,
                 messi_knn_stats* stats) {
    clear_error();
    if (!index) return fail(MESSI_EINVAL, "index is null");
    const Index* ix = reinterpret_cast<const Index*>(index);
    if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
    if (k_max < 1 || k_max > MESSI_MAX_K || (int64_t)k_max > ix->n)
        return fail(MESSI_EINVAL, "k_max must be in [1, min(n, 1024)]");
    if (mode != MESSI_MODE_FP32 && mode != MESSI_MODE_BF16 && mode != MESSI_MODE_APPROX)
        return fail(MESSI_EINVAL, "unknown mode");
    if (mode == MESSI_MODE_BF16 && !ix->shadow.p)
        return fail(MESSI_EINVAL, "BF16 mode needs an index built with bf16_shadow = 1");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (nq == 0) return MESSI_OK;
    if (!queries || !out_idx || !out_dist) return fail(MESSI_EINVAL, "null pointer argument");
    if (!is_device_pointer(queries) || !is_device_pointer(out_idx) || !is_device_pointer(out_dist))
        return fail(MESSI_EINVAL, "queries / out_idx / out_dist must be device pointers");
    if (k_per_query && !is_device_pointer(k_per_query))
        return fail(MESSI_EINVAL, "k_per_query must be a device pointer");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != ix->device)
        return fail(MESSI_EINVAL, "the index lives on another device");
    if (k_per_query) {
        // every k is checked before any search work starts
        std::vector<int32_t> hk((size_t)nq);
        MESSI_HIP_TRY(hipMemcpyAsync(hk.data(), k_per_query, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost,
                                     (hipStream_t)stream));
        MESSI_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        for (int32_t q = 0; q < nq; ++q)
            if (hk[(size_t)q] < 1 || hk[(size_t)q] > k_max)
                return fail(MESSI_EINVAL, "k_per_query values must be in [1, k_max]");
    }
    return knn_device(ix, queries, nq, k_max, k_per_query, mode, (hipStream_t)stream, out_idx, out_dist, stats);
}

int messi_knn_dtw(const messi_index* index, const float* queries, int32_t nq, int32_t k, int32_t band,
                  void* stream, int64_t* out_idx, float* out_dist, messi_knn_stats* stats) {
    clear_error();
    if (!index) return fail(MESSI_EINVAL, "index is null");
    const Index* ix = reinterpret_cast<const Index*>(index);
    if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
    if (k < 1 || k > MESSI_MAX_K || (int64_t)k > ix->n) return fail(MESSI_EINVAL, "k must be in [1, min(n, 1024)]");
    if (band < 0 || band > MESSI_MAX_DTW_BAND) return fail(MESSI_EINVAL, "band must be in [0, 27]");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (nq == 0) return MESSI_OK;
    if (!queries || !out_idx || !out_dist) return fail(MESSI_EINVAL, "null pointer argument");
    if (!is_device_pointer(queries) || !is_device_pointer(out_idx) || !is_device_pointer(out_dist))
        return fail(MESSI_EINVAL, "queries / out_idx / out_dist must be device pointers");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != ix->device)
        return fail(MESSI_EINVAL, "the index lives on another device");
    return knn_dtw_device(ix, queries, nq, k, band, (hipStream_t)stream, out_idx, out_dist, stats);
}

int messi_knn(const messi_index* index, const float* queries, int32_t nq, int32_t k, int64_t* out_idx,
              float* out_dist) {
    const int32_t mode = index ? reinterpret_cast<const Index*>(index)->opts.mode : MESSI_MODE_FP32;
    return messi_knn_ex(index, queries, nq, nullptr, k, mode, nullptr, out_idx, out_dist, nullptr);
}

}  // extern "C"

// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "messi.h"

namespace messi {

constexpr int kWave = 64;
constexpr int kMaxW = 16;

// ---- error state (per thread) --------------------------------------------

void set_error(int code, const std::string& msg);
void clear_error();
int last_error_code();

struct Error {
    int code;
    std::string msg;
};

// Throw-free error propagation: every host routine returns an int code.
#define MESSI_HIP_TRY(expr)                                                                        \
    do {                                                                                           \
        hipError_t e__ = (expr);                                                                   \
        if (e__ != hipSuccess) {                                                                   \
            ::messi::set_error(e__ == hipErrorOutOfMemory ? MESSI_ENOMEM : MESSI_EDEVICE,          \
                               std::string(#expr) + ": " + hipGetErrorString(e__));                \
            return e__ == hipErrorOutOfMemory ? MESSI_ENOMEM : MESSI_EDEVICE;                      \
        }                                                                                          \
    } while (0)

#define MESSI_LAUNCH_CHECK(name)                                                                   \
    do {                                                                                           \
        hipError_t e__ = hipGetLastError();                                                        \
        if (e__ != hipSuccess) {                                                                   \
            ::messi::set_error(MESSI_EDEVICE, std::string("launch ") + name + ": " +             \
                                                  hipGetErrorString(e__));                          \
            return MESSI_EDEVICE;                                                                  \
        }                                                                                          \
    } while (0)

#define MESSI_TRY(expr)                                                                            \
    do {                                                                                           \
        int rc__ = (expr);                                                                         \
        if (rc__ != MESSI_OK) return rc__;                                                         \
    } while (0)

// ---- device buffers --------------------------------------------------------

// A device allocation, freed when the owner goes out of scope (move-only).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    int alloc(size_t n);   // frees any previous allocation first
    void release();
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Leaf record on the device (same layout as messi_leaf).
struct Leaf {
    uint8_t card[16];
    uint8_t prefix[16];
    uint32_t start;
    uint32_t count;
};
static_assert(sizeof(Leaf) == 40, "leaf layout");

// ---- the index -------------------------------------------------------------

// Row stride in bytes of the fine summaries (at most 64 segments).
constexpr int kFineStride = 64;

// A fine summary value p is stored as the 8-bit code floor((fl(p + 4) * 32)),
// clamped to [0, 255]: steps of 1/32 over [-4, 4).  Code c stands for
// [c / 32 - 4, (c + 1) / 32 - 4) (open-ended for 0 and 255); fl(p + 4) is off
// by at most 2^-22 from p + 4, which the search adds to its widening.
__host__ __device__ inline int fine_code(float p) {
    const float t = (p + 4.0f) * 32.0f;
    return (int)fminf(fmaxf(t, 0.0f), 255.0f);
}
constexpr float kFineCodeSlack = 4.76837158203125e-07f;  // 2^-21: twice the rounding of p + 4

// Fine summary of an index of segment length m: F = min(4, m) fine segments
// per segment when m is a power of two in [2, 64], else none.
inline int fine_per_segment(int m) {
    if (m < 2 || m > 64 || (m & (m - 1)) != 0) return 0;
    return m < 4 ? m : 4;
}

struct Index {
    int device = 0;
    const float* series = nullptr;  // borrowed, [n][len]
    int64_t n = 0;
    int32_t len = 0, w = 0, b = 0, cap = 0;
    int64_t n_leaves = 0, max_leaf = 0;
    int32_t levels = 0;          // split levels of the partition
    float absmax = 0.f;

    DevBuf words;   // uint4 [n]: member words in leaf order (bytes 0..w-1)
    DevBuf pos;     // uint32 [n]: series index of each member, leaf order
    DevBuf leaves;  // Leaf [n_leaves], depth-first order
    DevBuf bp;      // float [2^b - 1] breakpoints
    DevBuf sx;      // uint2 [n]: BF16 (|x| up, beta high, beta low, 0) per member, leaf order (bf16 shadow only)
    DevBuf shadow;  // bf16 [n][len] rows in leaf order (bf16 shadow only)
    // Summaries the search reads before a member's word and before its row:
    DevBuf cwords;  // uint2 [n], leaf order: the word's symbols cut to their top 4 bits, two per byte
                    //   (byte j = segment 2j in the high nibble, 2j + 1 in the low one)
    DevBuf fwords;  // uint8 [n][kFineStride], input order: symbols of the PAA over wf segments of
                    //   mf values (empty when wf == 0)
    int32_t wf = 0, mf = 0;  // fine segments and their length (wf * mf == len), 0: no fine summary
    // the partition's internal nodes and their split segments, as an
    // open-addressing table keyed by (card, prefix): appends keep these splits
    DevBuf split_keys;   // uint4 [2][slots]: card bytes, prefix bytes
    DevBuf split_seg;    // uint8 [slots]
    DevBuf split_claim;  // uint32 [slots]: 1 = slot used
    uint32_t split_mask = 0;  // slots - 1 (0: no table)
    uint32_t n_inner = 0;

    float bp_host[255];
    messi_info info{};
    messi_opts opts{};  // as given to the build, defaults filled in (search mode, budgets, scan chunk, ...)

    uint64_t device_bytes() const {
        return words.bytes + pos.bytes + leaves.bytes + bp.bytes + sx.bytes + shadow.bytes + cwords.bytes +
               fwords.bytes;
    }
    ~Index();
};

// ---- host entry points implemented per translation unit ---------------------

// breakpoints.cpp: fl32(Phi^-1(j / 2^b)) by Wichura's AS241 (PPND16).
void breakpoints_as241(int card_bits, float* out);

// build.hip
int znorm_device(float* series, int64_t n, int32_t len, hipStream_t s, int* d_flag);
// Rows r = 0 .. count - 1 of out[count][len] from src[r * step ..], z-normalised
// as znorm_device does when znorm is set.
int windows_device(const float* src, int64_t count, int32_t len, int64_t step, bool znorm, float* out,
                   hipStream_t s, int* d_flag);
// The split table of an index, as the build reads it (mask 0: none).
struct SplitTab {
    const uint4* keys;
    const uint8_t* seg;
    const uint32_t* claim;
    uint32_t mask;
};
// forced (may be null): nodes that split on a given segment whatever the
// balance (an append keeps the previous index's splits).
int build_index(Index* ix, const float* series, int64_t n, int32_t len, int32_t w, int32_t b, int32_t cap,
                const messi_opts& opts, const SplitTab* forced = nullptr);

// query.hip
// kq: device int32[nq] of per-query k (nullable: kmax for every query);
// outputs are [nq][kmax].
int knn_device(const Index* ix, const float* queries, int32_t nq, int32_t kmax, const int32_t* kq, int32_t mode,
               hipStream_t s, int64_t* out_idx, float* out_dist, messi_knn_stats* stats);
// Exact k-NN under DTW with a Sakoe-Chiba band of half-width `band`.
int knn_dtw_device(const Index* ix, const float* queries, int32_t nq, int32_t k, int32_t band, hipStream_t s,
                   int64_t* out_idx, float* out_dist, messi_knn_stats* stats);

// bf16.hip
int build_bf16_shadow(Index* ix, hipStream_t s);
void release_bf16(const Index* ix);
void release_workspaces(const Index* ix);

// util
bool is_device_pointer(const void* p);
int current_device_ok();

}  // namespace messi

// ---- device helpers ------------------------------------------------------------

namespace messi {
namespace dev {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Make one wave's LDS writes visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Order-preserving key of a non-negative or +inf float (NaN never reaches here).
__device__ __forceinline__ uint32_t fkey(float f) { return __float_as_uint(f); }

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

}  // namespace dev
}  // namespace messi

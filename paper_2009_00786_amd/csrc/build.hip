// Index construction on gfx950 (paper: Index Construction -- CalculateiSAXSummaries,
// then TreeConstruction / SplitNode), re-planned for a GPU:
//
//  1. summarise: one wave streams a 1 KB row (float4 per lane) and produces the
//     row's iSAX word and root key; z-normalisation can be fused into the same
//     pass (fp64 statistics).                                      HBM-bound.
//  2. bucket by root key: stable LSD radix sort of (key, word, pos), 8-bit
//     digits, per-tile histograms + device scan + stable scatter ranked with
//     wave ballots.  Its output is the paper's iSAX buffers, one contiguous run
//     per root child.
//  3. split levels: every node over capacity counts, per refinable segment,
//     the members whose next symbol bit is 1 (tiles of 4096 members, LDS
//     reduction, one atomic per tile and segment), picks the most balanced
//     segment, and stable-partitions its range into the 0 and 1 children
//     (ballot ranks + device scan).  A node's range is split in place, so the
//     final member order is the depth-first leaf order with members in
//     ascending series index -- the canonical layout.
//  4. finalise: ranges that ended in the second buffer are copied back, and
//     the leaf records are ordered by start through a bitmap rank.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <utility>
#include <vector>

#include "common.h"
#include "scan.h"

namespace messi {
namespace {

constexpr int kTile = 4096;
constexpr int kBlk = 256;
constexpr int kRounds = kTile / kBlk;

double inv_len_pow2(int32_t len) { return (len & (len - 1)) == 0 ? 1.0 / (double)len : 0.0; }

int launch_blocks(int64_t work, int per_block, int cap_blocks) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap_blocks) b = cap_blocks;
    return (int)b;
}

int device_cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
                  ? p.multiProcessorCount
                  : 256;
    }
    return cus;
}

// ---------------------------------------------------------------------------
// Fold-halving sums across the lanes of one series group (width T lanes, E
// consecutive elements per lane): pairs (i, i + h) for h = P/2 .. 1.  Strides
// of at least E elements are lane offsets h/E; smaller strides are inside the
// lane.  The full sum ends in the group's first lane, element 0.
// ---------------------------------------------------------------------------
template <int E>
__device__ __forceinline__ double fold_halving64(double (&v)[E], int T) {
    for (int off = T >> 1; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = __dadd_rn(v[k], __shfl_down(v[k], off, T));
    }
#pragma unroll
    for (int h = E >> 1; h >= 1; h >>= 1) {
#pragma unroll
        for (int k = 0; k < h; ++k) v[k] = __dadd_rn(v[k], v[k + h]);
    }
    return v[0];
}

// c / sigma rounded to fp32 as fl32(fl64(c / sigma)), with rs = fl64(1 / sigma):
// c * rs is within 2 fp64 ulps of the exact quotient, so unless it lies within
// a few fp64 ulps of an fp32 rounding midpoint (or outside the normal fp32
// range) it rounds to the same fp32 value; otherwise the correctly rounded
// fp64 quotient is formed.
__device__ __forceinline__ float quotient_f32(double c, double sigma, double rs) {
    const double q1 = __dmul_rn(c, rs);  // within 2 fp64 ulps of the exact quotient
    const uint64_t bits = (uint64_t)__double_as_longlong(q1);
    const int e = (int)((bits >> 52) & 0x7ff);
    const uint32_t low = (uint32_t)(bits & ((1ull << 29) - 1));  // the bits below fp32 precision
    const uint32_t half = 1u << 28;
    // normal fp32 range, and not near the point where fp32 rounding flips
    if (e >= 1023 - 126 && e <= 1023 + 127 && (low > half + 8u || low + 8u < half)) return (float)q1;
    return (float)__ddiv_rn(c, sigma);
}

struct SumArgs {
    const float* in;
    float* zout;          // z-normalised rows (may equal in); null when not normalising
    int64_t n;
    int32_t L, P, T, G;   // length, padded length, lanes per series, series per wave
    int32_t w, m, M, b;   // segments, segment length, padded segment length, bits
    const float* bp;      // 2^b - 1 breakpoints
    uint4* words;         // [n] input order
    uint16_t* keys;       // [n]
    uint32_t* absmax;     // float bits, atomicMax
    int* nonfinite;
    double inv_len_pow2;  // 1 / L when L is a power of two (s / L == s * (1 / L) then), else 0
};

// One kernel for: z-normalise only (SUM = false), summarise only (ZN = false),
// or both fused (read once, write z once).  Each wave loads R series groups
// before computing on any of them, so R row loads per lane are in flight.
template <int E, bool ZN, bool SUM, int R>
__global__ void __launch_bounds__(256) summarize_kernel(SumArgs a) {
    __shared__ float s_bp[256];
    __shared__ float s_row[4][64 * E];     // general PAA path: z values of the wave's series
    __shared__ uint8_t s_sym[4][64 * 16];  // general PAA path: symbols of the wave's series
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (SUM) {
        const int nb = (1 << a.b) - 1;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) s_bp[i] = (i < nb) ? a.bp[i] : 0.f;
        __syncthreads();
    }
    const int T = a.T, G = a.G, L = a.L;
    const int g = lane / T, t = lane % T;
    const bool fast_paa = SUM && ((a.m & (a.m - 1)) == 0) && (a.m % E == 0) && (L == a.P);
    const bool vec = (L == a.P) && (E % 4 == 0);
    const int64_t n_groups = (a.n + G - 1) / G;
    const int64_t wave_id = (int64_t)blockIdx.x * 4 + wave;
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    float amax = 0.f;
    bool bad = false;
    for (int64_t grp0 = wave_id * R; grp0 < n_groups; grp0 += n_waves * R) {
        float xs[R][E];
        // ---- loads of all R groups first
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = (grp0 + r) * G + g;
            const bool live = (grp0 + r < n_groups) && row < a.n;
            const float* src = a.in + (size_t)(live ? row : 0) * (size_t)L;
            if (vec) {
#pragma unroll
                for (int k = 0; k < E; k += 4) {
                    const float4 q = live ? *reinterpret_cast<const float4*>(src + t * E + k)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
                    xs[r][k] = q.x; xs[r][k + 1] = q.y; xs[r][k + 2] = q.z; xs[r][k + 3] = q.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int j = t * E + k;
                    xs[r][k] = (live && j < L) ? src[j] : 0.f;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = (grp0 + r) * G + g;
            const bool live = (grp0 + r < n_groups) && row < a.n;
            float* x = xs[r];
#pragma unroll
            for (int k = 0; k < E; ++k) bad |= !isfinite(x[k]);
            if (ZN) {
                double v[E];
#pragma unroll
                for (int k = 0; k < E; ++k) v[k] = (double)x[k];
                double s1 = fold_halving64<E>(v, T);
                s1 = __shfl(s1, g * T, 64);
                const double mu = a.inv_len_pow2 != 0.0 ? __dmul_rn(s1, a.inv_len_pow2) : __ddiv_rn(s1, (double)L);
                double c[E];
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int j = t * E + k;
                    c[k] = (j < L) ? __dsub_rn((double)x[k], mu) : 0.0;
                    v[k] = (j < L) ? __dmul_rn(c[k], c[k]) : 0.0;
                }
                double s2 = fold_halving64<E>(v, T);
                s2 = __shfl(s2, g * T, 64);
                const double var = a.inv_len_pow2 != 0.0 ? __dmul_rn(s2, a.inv_len_pow2) : __ddiv_rn(s2, (double)L);
                const double sigma = __dsqrt_rn(var);
                const double rs = var == 0.0 ? 0.0 : __ddiv_rn(1.0, sigma);
#pragma unroll
                for (int k = 0; k < E; ++k) x[k] = (var == 0.0) ? 0.f : quotient_f32(c[k], sigma, rs);
                if (live) {
                    float* dst = a.zout + (size_t)row * (size_t)L;
                    if (vec) {
#pragma unroll
                        for (int k = 0; k < E; k += 4)
                            *reinterpret_cast<float4*>(dst + t * E + k) = make_float4(x[k], x[k + 1], x[k + 2], x[k + 3]);
                    } else {
#pragma unroll
                        for (int k = 0; k < E; ++k)
                            if (t * E + k < L) dst[t * E + k] = x[k];
                    }
                }
            }
            if (!SUM) continue;
#pragma unroll
            for (int k = 0; k < E; ++k) amax = fmaxf(amax, live ? fabsf(x[k]) : 0.f);

            // ---- PAA: fold-halving sum of each segment, then one division by m.
            const int w = a.w, m = a.m;
            if (fast_paa) {
                float v[E];
#pragma unroll
                for (int k = 0; k < E; ++k) v[k] = x[k];
                const int seg_lanes = m / E;
                for (int off = seg_lanes >> 1; off >= 1; off >>= 1) {
#pragma unroll
                    for (int k = 0; k < E; ++k) v[k] = __fadd_rn(v[k], __shfl_down(v[k], off, T));
                }
#pragma unroll
                for (int h = E >> 1; h >= 1; h >>= 1) {
#pragma unroll
                    for (int k = 0; k < h; ++k) v[k] = __fadd_rn(v[k], v[k + h]);
                }
                // lane t holds segment t / seg_lanes when t % seg_lanes == 0; m is a
                // power of two, so the division by m is an exact scaling
                const bool seg_lane = (t % seg_lanes) == 0;
                const int seg = t / seg_lanes;
                const float p = __fmul_rn(v[0], 1.0f / (float)m);
                int s = 0;
                for (int step = 1 << (a.b - 1); step >= 1; step >>= 1)
                    if (s_bp[s + step - 1] <= p) s += step;
                if (live && seg_lane) reinterpret_cast<uint8_t*>(a.words + row)[seg] = (uint8_t)s;
                // root key: top bit of every segment's symbol, segment 0 most significant
                const uint64_t top = dev::ballot(seg_lane && ((s >> (a.b - 1)) & 1));
                if (live && t == 0) {
                    const uint64_t mine = top >> (g * T);
                    uint32_t key = 0;
                    for (int i = 0; i < w; ++i) key |= (uint32_t)((mine >> (i * seg_lanes)) & 1ull) << (w - 1 - i);
                    a.keys[row] = (uint16_t)key;
                }
            } else {
                // general path: z values to LDS, one lane per (series, segment) sums the
                // padded segment by fold-halving (pairwise over bit-reversed order).
#pragma unroll
                for (int k = 0; k < E; ++k) s_row[wave][g * a.P + t * E + k] = x[k];
                dev::wave_sync();
                for (int p = lane; p < G * w; p += 64) {
                    const int gg = p / w, seg = p % w;
                    const float* z = &s_row[wave][gg * a.P + seg * m];
                    float stack[11];
                    int depth = 0;
                    int lg = 0;
                    while ((1 << lg) < a.M) ++lg;
                    for (int q = 0; q < a.M; ++q) {
                        int j = 0;
                        for (int bit = 0; bit < lg; ++bit) j |= ((q >> bit) & 1) << (lg - 1 - bit);
                        const float val = (j < m) ? z[j] : 0.f;
                        int cnt = q + 1;
                        stack[depth++] = val;
                        while ((cnt & 1) == 0) {
                            const float hi = stack[--depth];
                            const float lo = stack[--depth];
                            stack[depth++] = __fadd_rn(lo, hi);
                            cnt >>= 1;
                        }
                    }
                    const float pval = __fdiv_rn(stack[0], (float)m);
                    int s = 0;
                    for (int step = 1 << (a.b - 1); step >= 1; step >>= 1)
                        if (s_bp[s + step - 1] <= pval) s += step;
                    s_sym[wave][gg * 16 + seg] = (uint8_t)s;
                }
                dev::wave_sync();
                if (lane < G) {
                    const int64_t r2 = (grp0 + r) * G + lane;
                    if ((grp0 + r < n_groups) && r2 < a.n) {
                        uint32_t wd[4] = {0u, 0u, 0u, 0u};
                        uint32_t key = 0;
                        for (int i = 0; i < w; ++i) {
                            const uint32_t sy = s_sym[wave][lane * 16 + i];
                            wd[i >> 2] |= sy << (8 * (i & 3));
                            key |= ((sy >> (a.b - 1)) & 1u) << (w - 1 - i);
                        }
                        a.words[r2] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                        a.keys[r2] = (uint16_t)key;
                    }
                }
                dev::wave_sync();
            }
        }
    }
    if (bad) atomicOr(a.nonfinite, 1);
    if (SUM) {
        amax = dev::wave_max(amax);
        if (lane == 0) atomicMax(a.absmax, __float_as_uint(amax));
    }
}

// ---------------------------------------------------------------------------
// z-normalisation only, for rows of more than 32 values (padded length P =
// 64 EP).  Lane l of a wave holds elements l, l + 64, ..., l + 64 (EP - 1) of
// its row, so the fold-halving levels with strides of 64 and more are
// additions inside the lane and only the last six (strides 32 .. 1) cross
// lanes, on one value.  Same fp64 statistics and the same order of additions
// as the general kernel; the quotient c / sigma is formed as c * (1 / sigma)
// and rounded to fp32 directly unless that product lies within a few fp64
// ulps of an fp32 rounding midpoint, where the correctly rounded fp64
// quotient is computed instead -- so the fp32 result is fl32(fl64(c / sigma))
// in every case.
// ---------------------------------------------------------------------------
// Row r is read from in + r * in_stride (in_stride = L for a collection; the
// window step for the windows of a long series, which overlap) and written to
// out + r * L.
// inv_len_pow2 is 1 / L when L is a power of two (then s / L and s * (1 / L)
// are the same correctly rounded value, and the product is much cheaper), else 0.
template <int EP, int R>
__global__ void __launch_bounds__(256) znorm_strided_kernel(const float* in, float* out, int64_t n, int L,
                                                            int64_t in_stride, int* nonfinite, double inv_len_pow2) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t wave_id = (int64_t)blockIdx.x * 4 + wave;
    int64_t n_waves = (int64_t)gridDim.x * 4;
    int64_t r_begin = 0, r_end = n;
    if (in_stride < L && (gridDim.x & 7) == 0) {
        // overlapping windows: blocks b, b + 8, ... run on one XCD; give each
        // XCD one contiguous eighth of the rows, so that the values its
        // windows share are read from HBM once into its own L2
        const int64_t per = (n + 7) / 8;
        r_begin = min(n, (int64_t)(blockIdx.x & 7) * per);
        r_end = min(n, r_begin + per);
        wave_id = (int64_t)(blockIdx.x >> 3) * 4 + wave;
        n_waves = (int64_t)(gridDim.x >> 3) * 4;
    }
    bool bad = false;
    for (int64_t row0 = r_begin + wave_id * R; row0 < r_end; row0 += n_waves * R) {
        float x[R][EP];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = row0 + r;
            const float* src = in + (size_t)(row < r_end ? row : r_begin) * (size_t)in_stride;
#pragma unroll
            for (int k = 0; k < EP; ++k) {
                const int j = lane + 64 * k;
                x[r][k] = (row < r_end && j < L) ? src[j] : 0.f;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = row0 + r;
            double v[EP];
#pragma unroll
            for (int k = 0; k < EP; ++k) {
                bad |= !isfinite(x[r][k]);
                v[k] = (double)x[r][k];
            }
#pragma unroll
            for (int h = EP >> 1; h >= 1; h >>= 1)
#pragma unroll
                for (int k = 0; k < h; ++k) v[k] = __dadd_rn(v[k], v[k + h]);
            double s1 = v[0];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) s1 = __dadd_rn(s1, __shfl_down(s1, off, 64));
            s1 = __shfl(s1, 0, 64);
            const double mu = inv_len_pow2 != 0.0 ? __dmul_rn(s1, inv_len_pow2) : __ddiv_rn(s1, (double)L);
            double c[EP];
#pragma unroll
            for (int k = 0; k < EP; ++k) {
                const bool in_row = lane + 64 * k < L;
                c[k] = in_row ? __dsub_rn((double)x[r][k], mu) : 0.0;
                v[k] = in_row ? __dmul_rn(c[k], c[k]) : 0.0;
            }
#pragma unroll
            for (int h = EP >> 1; h >= 1; h >>= 1)
#pragma unroll
                for (int k = 0; k < h; ++k) v[k] = __dadd_rn(v[k], v[k + h]);
            double s2 = v[0];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) s2 = __dadd_rn(s2, __shfl_down(s2, off, 64));
            s2 = __shfl(s2, 0, 64);
            const double var = inv_len_pow2 != 0.0 ? __dmul_rn(s2, inv_len_pow2) : __ddiv_rn(s2, (double)L);
            const double sigma = __dsqrt_rn(var);
            const double rs = var == 0.0 ? 0.0 : __ddiv_rn(1.0, sigma);
            if (row < r_end) {
                float* dst = out + (size_t)row * (size_t)L;
#pragma unroll
                for (int k = 0; k < EP; ++k) {
                    const int j = lane + 64 * k;
                    if (j < L) dst[j] = var == 0.0 ? 0.f : quotient_f32(c[k], sigma, rs);
                }
            }
        }
    }
    if (bad) atomicOr(nonfinite, 1);
}

// The windows of a long series copied as rows: row r = src[r * step ..
// r * step + L), one wave per row at a time.
__global__ void __launch_bounds__(256) windows_copy_kernel(const float* __restrict__ src, int64_t step, int64_t n,
                                                           int L, float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4) {
        const float* a = src + (size_t)r * (size_t)step;
        float* b = out + (size_t)r * (size_t)L;
        for (int j = lane; j < L; j += 64) b[j] = a[j];
    }
}

// ---------------------------------------------------------------------------
// Summarise, one segment per lane: lane l of a wave owns segment l % w of row
// l / w (64 / w rows per wave), keeps the segment's m values in registers and
// sums them by fold-halving there (no cross-lane traffic).  The symbol comes
// from a cell table over [-8, 8) (cells of 1/256, at most one breakpoint per
// cell): a first guess from the cell, corrected by one comparison each way.
// Word bytes of consecutive rows are consecutive lanes, so the byte stores of
// a wave are one contiguous run; the root key is a ballot of the top bits.
// ---------------------------------------------------------------------------
constexpr int kCells = 4096;

struct SegArgs {
    const float* in;
    int64_t n;
    int32_t L, w, m, b;
    const float* bp;        // 2^b - 1 breakpoints
    const uint8_t* cells;   // kCells: number of breakpoints <= -8 + c / 256
    uint8_t* words;         // [n][16] bytes, input order
    uint16_t* keys;         // [n]
    uint32_t* absmax;       // float bits, atomicMax
    int* nonfinite;
    uint8_t* fine;          // [n][kFineStride] fine summary (nullptr: none); m a power of two
};

template <int M, int R, bool VEC>
__global__ void __launch_bounds__(256) summarize_seg_kernel(SegArgs a) {
    __shared__ float s_bp[257];
    __shared__ uint8_t s_cell[kCells];
    const int A = 1 << a.b;
    for (int i = threadIdx.x; i < 257; i += blockDim.x) s_bp[i] = (i >= 1 && i < A) ? a.bp[i - 1] : 0.f;
    for (int i = threadIdx.x; i < kCells; i += blockDim.x) s_cell[i] = a.cells[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = a.w, m = a.m, L = a.L;
    const int rpw = 64 / w;                 // rows per wave
    const int r_in = lane / w, seg = lane % w;
    const bool lane_on = r_in < rpw;
    const uint32_t row_mask = (w == 32) ? 0xffffffffu : ((1u << w) - 1u);
    const int64_t n_blocks = (a.n + rpw - 1) / rpw;   // row blocks of rpw rows
    const int64_t wave_id = (int64_t)blockIdx.x * 4 + wave;
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    const float inv_m = 1.0f / (float)m;
    const bool pow2_m = (m & (m - 1)) == 0;
    // symbol of a PAA value: a first guess from its cell, corrected by one comparison each way
    auto symbol = [&](float p) -> int {
        const float cf = fminf(fmaxf(__fmul_rn(__fadd_rn(p, 8.0f), 256.0f), 0.0f), (float)(kCells - 1));
        int s = s_cell[(int)cf];
        if (s > 0 && s_bp[s] > p) --s;
        else if (s < A - 1 && s_bp[s + 1] <= p) ++s;
        return s;
    };
    uint32_t amax_bits = 0;
    for (int64_t blk0 = wave_id * R; blk0 < n_blocks; blk0 += n_waves * R) {
        float v[R][M];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = (blk0 + r) * rpw + r_in;
            const bool live = lane_on && (blk0 + r < n_blocks) && row < a.n;
            const float* src = a.in + (size_t)(live ? row : 0) * (size_t)L + (size_t)seg * m;
            if (VEC) {
#pragma unroll
                for (int k = 0; k < M; k += 4) {
                    const float4 q = live ? *reinterpret_cast<const float4*>(src + k) : make_float4(0.f, 0.f, 0.f, 0.f);
                    v[r][k] = q.x; v[r][k + 1] = q.y; v[r][k + 2] = q.z; v[r][k + 3] = q.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) v[r][k] = (live && k < m) ? src[k] : 0.f;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t row = (blk0 + r) * rpw + r_in;
            const bool live = lane_on && (blk0 + r < n_blocks) && row < a.n;
            uint32_t mx = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) mx = max(mx, __float_as_uint(v[r][k]) & 0x7fffffffu);
            amax_bits = max(amax_bits, mx);
            if (a.fine != nullptr) {
                // the fine summary (m == M here): F sub-segments of MF values,
                // each summed by fold-halving and scaled, and their 8-bit codes
                constexpr int F = M >= 4 ? 4 : M;
                constexpr int MF = M / F;
                uint32_t packed = 0;
#pragma unroll
                for (int t = 0; t < F; ++t) {
                    float f[MF];
#pragma unroll
                    for (int i = 0; i < MF; ++i) f[i] = v[r][t * MF + i];
#pragma unroll
                    for (int h = MF / 2; h >= 1; h /= 2)
#pragma unroll
                        for (int i = 0; i < h; ++i) f[i] = __fadd_rn(f[i], f[i + h]);
                    packed |= (uint32_t)fine_code(__fmul_rn(f[0], 1.0f / (float)MF)) << (8 * t);
                }
                uint8_t* dst = a.fine + (size_t)row * kFineStride + seg * F;
                if (live) {
                    if (F == 4) *reinterpret_cast<uint32_t*>(dst) = packed;
                    else if (F == 2) *reinterpret_cast<uint16_t*>(dst) = (uint16_t)packed;
                    else *dst = (uint8_t)packed;
                }
            }
            // fold-halving over the (zero-padded) segment
#pragma unroll
            for (int h = M / 2; h >= 1; h /= 2) {
#pragma unroll
                for (int k = 0; k < h; ++k) v[r][k] = __fadd_rn(v[r][k], v[r][k + h]);
            }
            const float p = pow2_m ? __fmul_rn(v[r][0], inv_m) : __fdiv_rn(v[r][0], (float)m);
            const int s = symbol(p);
            if (live) a.words[(size_t)row * 16 + seg] = (uint8_t)s;
            const uint64_t top = dev::ballot(lane_on && ((s >> (a.b - 1)) & 1));
            if (live && seg == 0) {
                const uint32_t bits = (uint32_t)(top >> (r_in * w)) & row_mask;
                a.keys[row] = (uint16_t)(__brev(bits) >> (32 - w));
            }
        }
    }
    if (amax_bits >= 0x7f800000u) atomicOr(a.nonfinite, 1);
    uint32_t mxw = amax_bits;
    for (int off = 32; off >= 1; off >>= 1) mxw = max(mxw, (uint32_t)__shfl_xor((int)mxw, off));
    if (lane == 0 && mxw < 0x7f800000u) atomicMax(a.absmax, mxw);
}

int launch_summarize_seg(const SegArgs& a, hipStream_t s) {
    int M = 1;
    while (M < a.m) M <<= 1;
    const bool vec = (a.m % 4 == 0) && (a.L % 4 == 0) && ((uintptr_t)a.in % 16 == 0);
    const int rpw = 64 / a.w;
    const int64_t n_blocks = (a.n + rpw - 1) / rpw;
    // A streaming read: few waves (two blocks per CU), each with 128 values
    // per lane (R row groups of M) in flight, beat many waves with few loads.
    const int cap = 2 * device_cu_count();
    switch (M) {
#define MESSI_SEG_CASE(MM)                                                                             \
    case MM: {                                                                                         \
        constexpr int R = (MM <= 8) ? 16 : 128 / MM;                                                   \
        const int blocks = launch_blocks(n_blocks, 4 * R, cap);                                        \
        if (vec && MM >= 4)                                                                            \
            hipLaunchKernelGGL((summarize_seg_kernel<MM, R, true>), dim3(blocks), dim3(256), 0, s, a);  \
        else                                                                                           \
            hipLaunchKernelGGL((summarize_seg_kernel<MM, R, false>), dim3(blocks), dim3(256), 0, s, a); \
        break;                                                                                         \
    }
        MESSI_SEG_CASE(1)
        MESSI_SEG_CASE(2)
        MESSI_SEG_CASE(4)
        MESSI_SEG_CASE(8)
        MESSI_SEG_CASE(16)
        MESSI_SEG_CASE(32)
        MESSI_SEG_CASE(64)
#undef MESSI_SEG_CASE
        default:
            set_error(MESSI_EINVAL, "segment length above 64 takes the general path");
            return MESSI_EINVAL;
    }
    MESSI_LAUNCH_CHECK("summarize_seg");
    return MESSI_OK;
}

// Cell table: cells[c] = number of breakpoints <= -8 + c / 256 (host).
void cell_table(const float* bp, int card_bits, uint8_t* cells) {
    const int nb = (1 << card_bits) - 1;
    for (int c = 0; c < kCells; ++c) {
        const float x = -8.0f + (float)c / 256.0f;
        int cnt = 0;
        for (int j = 0; j < nb; ++j) cnt += bp[j] <= x;
        cells[c] = (uint8_t)cnt;
    }
}

// ---------------------------------------------------------------------------
// Fine summary on its own (builds whose summarise pass does not produce it:
// z-normalisation fused into the summary): one thread per (row, fine
// segment) of MF values, summed by fold-halving and scaled, and its code.
// ---------------------------------------------------------------------------
template <int MF>
__global__ void __launch_bounds__(256) fine_kernel(const float* __restrict__ in, int64_t n, int L, int wf,
                                                   uint8_t* __restrict__ fine) {
    const int64_t total = n * (int64_t)wf;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = id / wf;
        const int j = (int)(id - row * wf);
        const float* src = in + (size_t)row * (size_t)L + (size_t)j * MF;
        float f[MF];
#pragma unroll
        for (int i = 0; i < MF; ++i) f[i] = src[i];
#pragma unroll
        for (int h = MF / 2; h >= 1; h /= 2)
#pragma unroll
            for (int i = 0; i < h; ++i) f[i] = __fadd_rn(f[i], f[i + h]);
        fine[(size_t)row * kFineStride + j] = (uint8_t)fine_code(__fmul_rn(f[0], 1.0f / (float)MF));
    }
}

int launch_fine(const float* in, int64_t n, int L, int wf, int mf, uint8_t* fine, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n * wf + 255) / 256, 16 * (int64_t)device_cu_count());
    switch (mf) {
#define MESSI_FINE_CASE(MM) \
    case MM: hipLaunchKernelGGL(fine_kernel<MM>, dim3(blocks), dim3(256), 0, s, in, n, L, wf, fine); break;
        MESSI_FINE_CASE(1)
        MESSI_FINE_CASE(2)
        MESSI_FINE_CASE(4)
        MESSI_FINE_CASE(8)
        MESSI_FINE_CASE(16)
#undef MESSI_FINE_CASE
        default:
            set_error(MESSI_EINVAL, "fine segments of more than 16 values are not built");
            return MESSI_EINVAL;
    }
    MESSI_LAUNCH_CHECK("fine");
    return MESSI_OK;
}

// Coarse words in leaf order: each symbol cut to its top min(b, 4) bits (a
// shift by sh = b - min(b, 4)), segments 2j and 2j + 1 in byte j.
__global__ void __launch_bounds__(256) coarse_kernel(const uint4* __restrict__ words, int64_t n, int sh,
                                                     uint2* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 wv = words[i];
        const uint32_t in[4] = {wv.x, wv.y, wv.z, wv.w};
        uint32_t o[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t hi = (in[j >> 1] >> (16 * (j & 1))) & 255u;      // segment 2j
            const uint32_t lo = (in[j >> 1] >> (16 * (j & 1) + 8)) & 255u;  // segment 2j + 1
            o[j >> 2] |= (((hi >> sh) << 4) | (lo >> sh)) << (8 * (j & 3));
        }
        out[i] = make_uint2(o[0], o[1]);
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix pass over (key, word, pos), 8-bit digit at `shift`.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlk) radix_hist_kernel(const uint16_t* __restrict__ keys, int64_t n, int shift,
                                                          uint32_t* __restrict__ hist, int64_t n_tiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + (int64_t)r * kBlk + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// The tile's elements are taken a sub-tile of kSub = 1024 at a time: each is
// ranked within its digit (round, then wave, then lane order: the stable
// order), placed in LDS sorted by digit, and written from there, so that the
// elements of one digit leave the block as one contiguous run per sub-tile
// rather than a short run per round of 256.
constexpr int kSubRounds = 4;
constexpr int kSub = kSubRounds * kBlk;
static_assert(kRounds % kSubRounds == 0, "sub-tiles divide the tile");

__global__ void __launch_bounds__(kBlk) radix_scatter_kernel(const uint16_t* __restrict__ kin,
                                                             const uint4* __restrict__ win,
                                                             const uint32_t* __restrict__ pin, int64_t n, int shift,
                                                             const uint32_t* __restrict__ offs, int64_t n_tiles,
                                                             uint16_t* __restrict__ kout, uint4* __restrict__ wout,
                                                             uint32_t* __restrict__ pout) {
    __shared__ uint32_t base[256];                // digit's next global place for this tile
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint16_t woff[kSubRounds][4][256];  // place within the sub-tile's run of the digit
    __shared__ uint32_t sstart[256];              // sub-tile: start of each digit's run
    __shared__ uint32_t wsum[4];
    __shared__ uint16_t s_key[kSub];
    __shared__ uint4 s_word[kSub];
    __shared__ uint32_t s_pos[kSub];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    base[tid] = offs[(int64_t)tid * n_tiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const uint64_t lt = dev::lanemask_lt();
    for (int sub = 0; sub < kRounds / kSubRounds; ++sub) {
        const int64_t s0 = t0 + (int64_t)sub * kSub;
        if (s0 >= n) break;  // the same for every thread
        uint32_t key[kSubRounds], pv[kSubRounds];
        uint4 wv[kSubRounds];
#pragma unroll
        for (int rr = 0; rr < kSubRounds; ++rr) {
            const int64_t i = s0 + (int64_t)rr * kBlk + tid;
            const bool valid = i < n;
            key[rr] = valid ? kin[i] : 0u;
            wv[rr] = valid ? win[i] : make_uint4(0u, 0u, 0u, 0u);
            pv[rr] = valid ? (pin ? pin[i] : (uint32_t)i) : 0u;
        }
        int rank[kSubRounds];
        uint32_t acc = 0;  // thread tid: elements of digit tid in the sub-tile's rounds so far
#pragma unroll
        for (int rr = 0; rr < kSubRounds; ++rr) {
            const bool valid = s0 + (int64_t)rr * kBlk + tid < n;
            const uint32_t d = (key[rr] >> shift) & 255u;
            uint64_t peers = dev::ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool on = (d >> bit) & 1u;
                const uint64_t m = dev::ballot(valid && on);
                peers &= on ? m : ~m;
            }
            rank[rr] = dev::popc64(peers & lt);
            if (valid && (peers & lt) == 0) wcnt[wave][d] = (uint32_t)dev::popc64(peers);
            __syncthreads();
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = wcnt[w][tid];
                woff[rr][w][tid] = (uint16_t)acc;
                acc += c;
                wcnt[w][tid] = 0;
            }
            __syncthreads();
        }
        // start of each digit's run in the sub-tile: exclusive prefix of acc over digits
        uint32_t x = acc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        sstart[tid] = before + x - acc;
        const uint32_t nsub = wsum[0] + wsum[1] + wsum[2] + wsum[3];  // valid elements of the sub-tile
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < kSubRounds; ++rr) {
            if (s0 + (int64_t)rr * kBlk + tid < n) {
                const uint32_t d = (key[rr] >> shift) & 255u;
                const uint32_t slot = sstart[d] + woff[rr][wave][d] + (uint32_t)rank[rr];
                s_key[slot] = (uint16_t)key[rr];
                s_word[slot] = wv[rr];
                s_pos[slot] = pv[rr];
            }
        }
        __syncthreads();
        for (uint32_t e = tid; e < nsub; e += kBlk) {
            const uint32_t k2 = s_key[e];
            const uint32_t d = (k2 >> shift) & 255u;
            const uint32_t dst = base[d] + (e - sstart[d]);
            if (dst >= (uint64_t)n) continue;  // cannot happen with consistent offsets
            kout[dst] = (uint16_t)k2;
            wout[dst] = s_word[e];
            pout[dst] = s_pos[e];
        }
        __syncthreads();
        base[tid] += acc;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Root children: runs of equal keys in the sorted key array.
// ---------------------------------------------------------------------------
__global__ void root_runs_kernel(const uint16_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ run_start,
                                 uint32_t* __restrict__ run_end) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) run_start[k] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != k) run_end[k] = (uint32_t)i + 1;
}

struct Lists {
    Leaf* leaves;
    uint8_t* leaf_buf;
    uint32_t* n_leaves;  // counter
    Leaf* next;
    uint32_t* n_next;    // counter
    uint32_t* max_leaf;
};

__device__ void emit_child(const Leaf& c, int w, int b, int cap, int buf, Lists L) {
    if (c.count == 0) return;
    bool refinable = false;
    for (int i = 0; i < w; ++i) refinable |= c.card[i] < b;
    if (c.count <= (uint32_t)cap || !refinable) {
        const uint32_t id = atomicAdd(L.n_leaves, 1u);
        L.leaves[id] = c;
        L.leaf_buf[id] = (uint8_t)buf;
        atomicMax(L.max_leaf, c.count);
    } else {
        const uint32_t id = atomicAdd(L.n_next, 1u);
        L.next[id] = c;
    }
}

__global__ void root_nodes_kernel(const uint32_t* __restrict__ run_start, const uint32_t* __restrict__ run_end,
                                  int w, int b, int cap, int buf, Lists L) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << w)) return;
    const uint32_t e = run_end[k];
    if (e == 0) return;
    Leaf c;
    for (int i = 0; i < 16; ++i) {
        c.card[i] = (i < w) ? 1 : 0;
        c.prefix[i] = (i < w) ? (uint8_t)((k >> (w - 1 - i)) & 1u) : 0;
    }
    c.start = run_start[k];
    c.count = e - run_start[k];
    emit_child(c, w, b, cap, buf, L);
}

// ---------------------------------------------------------------------------
// Split levels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) node_tiles_kernel(const Leaf* __restrict__ nodes, int n_nodes,
                                                          uint32_t* __restrict__ tile_first,
                                                          uint32_t* __restrict__ total) {
    __shared__ uint32_t wt[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int per = (n_nodes + 1023) / 1024;
    const int b0 = t * per;
    uint32_t acc = 0;
    for (int i = b0; i < b0 + per && i < n_nodes; ++i) acc += (nodes[i].count + kTile - 1) / kTile;
    uint32_t x = acc;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wt[wave] = x;
    __syncthreads();
    uint32_t wo = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) wo += wt[w];
        tot += wt[w];
    }
    uint32_t run = wo + x - acc;
    for (int i = b0; i < b0 + per && i < n_nodes; ++i) {
        tile_first[i] = run;
        run += (nodes[i].count + kTile - 1) / kTile;
    }
    if (t == 0) {
        tile_first[n_nodes] = tot;
        *total = tot;
    }
}

__global__ void tile_node_kernel(const uint32_t* __restrict__ tile_first, int n_nodes, uint32_t n_tiles,
                                 uint32_t* __restrict__ tile_node) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    int lo = 0, hi = n_nodes - 1;  // last node with tile_first <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_first[mid] <= t) lo = mid; else hi = mid - 1;
    }
    tile_node[t] = (uint32_t)lo;
}

__device__ __forceinline__ uint32_t word_byte(const uint4& wd, int i) {
    const uint32_t v = (i < 4) ? wd.x : (i < 8) ? wd.y : (i < 12) ? wd.z : wd.w;
    return (v >> (8 * (i & 3))) & 0xFFu;
}

__global__ void __launch_bounds__(kBlk) level_count_kernel(const Leaf* __restrict__ nodes,
                                                           const uint32_t* __restrict__ tile_first,
                                                           const uint32_t* __restrict__ tile_node,
                                                           const uint4* __restrict__ words, int w, int b,
                                                           uint32_t* __restrict__ tile_cnt,
                                                           uint32_t* __restrict__ node_cnt) {
    __shared__ uint32_t part[4][16];
    const int tile = blockIdx.x;
    const uint32_t nd = tile_node[tile];
    const Leaf node = nodes[nd];
    const uint32_t start = node.start + (tile - tile_first[nd]) * kTile;
    const uint32_t end = min(start + (uint32_t)kTile, node.start + node.count);
    int shift[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) shift[i] = (i < w && node.card[i] < b) ? (b - 1 - node.card[i]) : -1;
    uint32_t cnt[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) cnt[i] = 0;
    for (uint32_t j = start + threadIdx.x; j < end; j += kBlk) {
        const uint4 wd = words[j];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (shift[i] >= 0) cnt[i] += (word_byte(wd, i) >> shift[i]) & 1u;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t s = dev::wave_sum_u32(cnt[i]);
        if (lane == 0) part[wave][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        const int i = threadIdx.x;
        const uint32_t s = part[0][i] + part[1][i] + part[2][i] + part[3][i];
        tile_cnt[(size_t)tile * 16 + i] = s;
        if (shift[i] >= 0 && s) atomicAdd(&node_cnt[(size_t)nd * 16 + i], s);
    }
}

// ---------------------------------------------------------------------------
// The split table: (card, prefix) of every internal node -> its segment, in
// open addressing with linear probing (at least twice as many slots as nodes).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void node_key(const Leaf& nd, uint4& k0, uint4& k1) {
    uint32_t v[8];
    memcpy(v, nd.card, 16);
    memcpy(v + 4, nd.prefix, 16);
    k0 = make_uint4(v[0], v[1], v[2], v[3]);
    k1 = make_uint4(v[4], v[5], v[6], v[7]);
}

__device__ __forceinline__ uint32_t key_hash(const uint4& k0, const uint4& k1) {
    const uint32_t v[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
    uint64_t h = 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < 8; ++i) {
        h ^= v[i];
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 33;
    }
    return (uint32_t)h;
}

__device__ int split_lookup(const SplitTab& t, const Leaf& nd) {
    uint4 k0, k1;
    node_key(nd, k0, k1);
    uint32_t h = key_hash(k0, k1) & t.mask;
    for (uint32_t probe = 0; probe <= t.mask; ++probe) {
        if (t.claim[h] == 0u) return -1;
        const uint4 a = t.keys[2 * (size_t)h], c = t.keys[2 * (size_t)h + 1];
        if (a.x == k0.x && a.y == k0.y && a.z == k0.z && a.w == k0.w && c.x == k1.x && c.y == k1.y &&
            c.z == k1.z && c.w == k1.w)
            return t.seg[h];
        h = (h + 1) & t.mask;
    }
    return -1;
}

// One thread per recorded internal node (its segment in `start`).
__global__ void __launch_bounds__(256) split_insert_kernel(const Leaf* __restrict__ inner, uint32_t n,
                                                           uint4* __restrict__ keys, uint8_t* __restrict__ seg,
                                                           uint32_t* __restrict__ claim, uint32_t mask) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Leaf nd = inner[i];
    uint4 k0, k1;
    node_key(nd, k0, k1);
    uint32_t h = key_hash(k0, k1) & mask;
    while (atomicCAS(&claim[h], 0u, 1u) != 0u) h = (h + 1) & mask;
    keys[2 * (size_t)h] = k0;
    keys[2 * (size_t)h + 1] = k1;
    seg[h] = (uint8_t)nd.start;
}

// After a level's choice: every node that split, with its segment in `start`.
__global__ void __launch_bounds__(256) record_inner_kernel(const Leaf* __restrict__ nodes, int n_nodes,
                                                           const uint8_t* __restrict__ node_split,
                                                           const uint8_t* __restrict__ node_seg,
                                                           Leaf* __restrict__ inner, uint32_t* __restrict__ n_inner) {
    const int nd = blockIdx.x * 256 + threadIdx.x;
    if (nd >= n_nodes || !node_split[nd]) return;
    Leaf r = nodes[nd];
    r.start = node_seg[nd];
    r.count = 0;
    inner[atomicAdd(n_inner, 1u)] = r;
}

__global__ void level_choose_kernel(const Leaf* __restrict__ nodes, int n_nodes, const uint32_t* __restrict__ node_cnt,
                                    int w, int b, int cap, int dst_buf, uint8_t* __restrict__ node_seg,
                                    uint32_t* __restrict__ node_n0, uint8_t* __restrict__ node_split, SplitTab forced,
                                    Lists L) {
    const int nd = blockIdx.x * blockDim.x + threadIdx.x;
    if (nd >= n_nodes) return;
    const Leaf node = nodes[nd];
    // a node that split before (an append) keeps its segment
    int best = forced.mask ? split_lookup(forced, node) : -1;
    uint32_t best_gap = 0, best_n1 = 0;
    if (best >= 0) {
        best_n1 = node_cnt[(size_t)nd * 16 + best];
    } else {
        for (int i = 0; i < w; ++i) {
            if (node.card[i] >= b) continue;
            const uint32_t n1 = node_cnt[(size_t)nd * 16 + i];
            const uint32_t n0 = node.count - n1;
            const uint32_t gap = n0 > n1 ? n0 - n1 : n1 - n0;
            if (best < 0 || gap < best_gap) {
                best = i;
                best_gap = gap;
                best_n1 = n1;
            }
        }
    }
    node_split[nd] = best >= 0 ? 1 : 0;
    if (best < 0) {  // nodes on the list always have a refinable segment; keep the node whole
        node_seg[nd] = 0;
        node_n0[nd] = node.count;
        emit_child(node, w, b, 0x7fffffff, dst_buf, L);
        return;
    }
    const uint32_t n0 = node.count - best_n1;
    node_seg[nd] = (uint8_t)best;
    node_n0[nd] = n0;
    Leaf c0 = node, c1 = node;
    c0.card[best] = c1.card[best] = (uint8_t)(node.card[best] + 1);
    c0.prefix[best] = (uint8_t)(node.prefix[best] * 2);
    c1.prefix[best] = (uint8_t)(node.prefix[best] * 2 + 1);
    c0.count = n0;
    c1.start = node.start + n0;
    c1.count = best_n1;
    emit_child(c0, w, b, cap, dst_buf, L);
    emit_child(c1, w, b, cap, dst_buf, L);
}

__global__ void level_zeros_kernel(const Leaf* __restrict__ nodes, const uint32_t* __restrict__ tile_first,
                                   const uint32_t* __restrict__ tile_node, uint32_t n_tiles,
                                   const uint32_t* __restrict__ tile_cnt, const uint8_t* __restrict__ node_seg,
                                   uint32_t* __restrict__ zeros) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t nd = tile_node[t];
    const Leaf node = nodes[nd];
    const uint32_t start = node.start + (t - tile_first[nd]) * kTile;
    const uint32_t end = min(start + (uint32_t)kTile, node.start + node.count);
    zeros[t] = (end - start) - tile_cnt[(size_t)t * 16 + node_seg[nd]];
}

__global__ void __launch_bounds__(kBlk) level_scatter_kernel(const Leaf* __restrict__ nodes,
                                                             const uint32_t* __restrict__ tile_first,
                                                             const uint32_t* __restrict__ tile_node,
                                                             const uint32_t* __restrict__ zscan,
                                                             const uint8_t* __restrict__ node_seg,
                                                             const uint32_t* __restrict__ node_n0, int b,
                                                             const uint4* __restrict__ win,
                                                             const uint32_t* __restrict__ pin,
                                                             uint4* __restrict__ wout, uint32_t* __restrict__ pout) {
    __shared__ uint32_t c0[4], c1[4];
    const int tile = blockIdx.x;
    const uint32_t nd = tile_node[tile];
    const Leaf node = nodes[nd];
    const uint32_t ft = tile_first[nd];
    const uint32_t start = node.start + (tile - ft) * kTile;
    const uint32_t end = min(start + (uint32_t)kTile, node.start + node.count);
    const int seg = node_seg[nd];
    const int shift = b - 1 - node.card[seg];
    const uint32_t zb = zscan[tile] - zscan[ft];           // zeros before this tile in the node
    const uint32_t ob = (tile - ft) * kTile - zb;          // ones before
    uint32_t base0 = node.start + zb;
    uint32_t base1 = node.start + node_n0[nd] + ob;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = dev::lanemask_lt();
    for (uint32_t r0 = start; r0 < end; r0 += kBlk) {
        const uint32_t j = r0 + threadIdx.x;
        const bool valid = j < end;
        uint4 wd = make_uint4(0, 0, 0, 0);
        uint32_t p = 0;
        if (valid) {
            wd = win[j];
            p = pin[j];
        }
        const bool one = valid && ((word_byte(wd, seg) >> shift) & 1u);
        const uint64_t m1 = dev::ballot(one);
        const uint64_t m0 = dev::ballot(valid && !one);
        if (lane == 0) {
            c1[wave] = (uint32_t)dev::popc64(m1);
            c0[wave] = (uint32_t)dev::popc64(m0);
        }
        __syncthreads();
        uint32_t b0w = 0, b1w = 0, t0 = 0, t1 = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w < wave) {
                b0w += c0[w];
                b1w += c1[w];
            }
            t0 += c0[w];
            t1 += c1[w];
        }
        if (valid) {
            const uint32_t dst = one ? base1 + b1w + (uint32_t)dev::popc64(m1 & lt)
                                     : base0 + b0w + (uint32_t)dev::popc64(m0 & lt);
            if (dst >= node.start && dst < node.start + node.count) {  // always true for consistent counts
                wout[dst] = wd;
                pout[dst] = p;
            }
        }
        base0 += t0;
        base1 += t1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Finalise.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlk) copy_back_kernel(const Leaf* __restrict__ leaves,
                                                         const uint8_t* __restrict__ leaf_buf, uint32_t n_leaves,
                                                         const uint4* __restrict__ wsrc,
                                                         const uint32_t* __restrict__ psrc, uint4* __restrict__ wdst,
                                                         uint32_t* __restrict__ pdst, int src_buf) {
    for (uint32_t l = blockIdx.x; l < n_leaves; l += gridDim.x) {
        if (leaf_buf[l] != src_buf) continue;
        const Leaf lf = leaves[l];
        for (uint32_t j = lf.start + threadIdx.x; j < lf.start + lf.count; j += kBlk) {
            wdst[j] = wsrc[j];
            pdst[j] = psrc[j];
        }
    }
}

__global__ void leaf_bitmap_kernel(const Leaf* __restrict__ leaves, uint32_t n_leaves, uint32_t* __restrict__ bm) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_leaves) return;
    const uint32_t s = leaves[l].start;
    atomicOr(&bm[s >> 5], 1u << (s & 31));
}

__global__ void popc_kernel(const uint32_t* __restrict__ bm, int64_t nw, uint32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) cnt[i] = __popc(bm[i]);
}

__global__ void leaf_order_kernel(const Leaf* __restrict__ leaves, uint32_t n_leaves, const uint32_t* __restrict__ bm,
                                  const uint32_t* __restrict__ rank_scan, Leaf* __restrict__ out) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_leaves) return;
    const Leaf lf = leaves[l];
    const uint32_t s = lf.start;
    const uint32_t below = (s & 31) ? (bm[s >> 5] & ((1u << (s & 31)) - 1u)) : 0u;
    const uint32_t r = rank_scan[s >> 5] + __popc(below);
    if (r < n_leaves) out[r] = lf;
}


// Lane layout of a row: E consecutive elements per lane, T lanes per series.
struct RowLayout {
    int P, E, T, G;
};

RowLayout row_layout(int L) {
    RowLayout r;
    r.P = 1;
    while (r.P < L) r.P <<= 1;
    r.E = std::min(r.P, std::max(4, r.P / 64));
    r.T = r.P / r.E;
    r.G = 64 / r.T;
    return r;
}

template <bool ZN, bool SUM>
int launch_summarize(const SumArgs& a, int E, hipStream_t s) {
    const int64_t n_groups = (a.n + a.G - 1) / a.G;
    // series groups per wave in flight: about 4 row loads of 16 B per lane
    switch (E) {
#define MESSI_SUM_CASE(EE)                                                                          \
    case EE: {                                                                                      \
        constexpr int R = (EE >= 16) ? 1 : (EE >= 8 ? 2 : 4);                                        \
        const int blocks = launch_blocks(n_groups, 4 * R, 256 * 8);                                 \
        hipLaunchKernelGGL((summarize_kernel<EE, ZN, SUM, R>), dim3(blocks), dim3(256), 0, s, a);   \
        break;                                                                                      \
    }
        MESSI_SUM_CASE(1)
        MESSI_SUM_CASE(2)
        MESSI_SUM_CASE(4)
        MESSI_SUM_CASE(8)
        MESSI_SUM_CASE(16)
#undef MESSI_SUM_CASE
        default:
            set_error(MESSI_EINVAL, "unsupported series length");
            return MESSI_EINVAL;
    }
    MESSI_LAUNCH_CHECK("summarize");
    return MESSI_OK;
}

struct Timer {
    hipStream_t s;
    hipEvent_t e[2];
    bool ok = false;
    explicit Timer(hipStream_t st) : s(st) {
        ok = hipEventCreate(&e[0]) == hipSuccess && hipEventCreate(&e[1]) == hipSuccess;
    }
    void start() { if (ok) (void)hipEventRecord(e[0], s); }
    double stop_ms() {
        if (!ok) return 0.0;
        float ms = 0.f;
        if (hipEventRecord(e[1], s) != hipSuccess || hipEventSynchronize(e[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess)
            return 0.0;
        return ms;
    }
    ~Timer() {
        if (ok) {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    }
};

}  // namespace

// ---------------------------------------------------------------------------

int windows_device(const float* src, int64_t count, int32_t len, int64_t step, bool znorm, float* out,
                   hipStream_t s, int* d_flag) {
    if (znorm && len > 32) {
        // z-normalised straight from the long series: every window's values
        // are read once from HBM and again from the caches for the overlaps
        int P = 64;
        while (P < len) P <<= 1;
        const int blocks = launch_blocks((count + 3) / 4, 4, 256 * 16);
        switch (P / 64) {
#define MESSI_WN_CASE(EP, R)                                                                                      \
    case EP:                                                                                                      \
        hipLaunchKernelGGL((znorm_strided_kernel<EP, R>), dim3(blocks), dim3(256), 0, s, src, out, count, len, step, \
                           d_flag, inv_len_pow2(len));                                                                               \
        break;
            MESSI_WN_CASE(1, 8)
            MESSI_WN_CASE(2, 4)
            MESSI_WN_CASE(4, 4)
            MESSI_WN_CASE(8, 2)
            MESSI_WN_CASE(16, 1)
#undef MESSI_WN_CASE
            default: break;
        }
        MESSI_LAUNCH_CHECK("windows");
        return MESSI_OK;
    }
    const int blocks = launch_blocks((count + 3) / 4, 4, 256 * 16);
    hipLaunchKernelGGL(windows_copy_kernel, dim3(blocks), dim3(256), 0, s, src, step, count, len, out);
    MESSI_LAUNCH_CHECK("windows_copy");
    // short windows: z-normalised in place by the collection kernel
    if (znorm) return znorm_device(out, count, len, s, d_flag);
    return MESSI_OK;
}

int znorm_device(float* series, int64_t n, int32_t len, hipStream_t s, int* d_flag) {
    if (len > 32) {
        int P = 64;
        while (P < len) P <<= 1;
        // Reading and rewriting every row in place moves as many bytes as a
        // copy; what sets its rate is the number of loads in flight over the
        // chip.  A wide grid (up to 128 blocks of 4 waves per CU, each wave R
        // rows at a time) measured 4.79 TB/s over 16M rows of 256, within 5%
        // of a plain float4 copy there (5.05 TB/s); 4096 blocks of 4-row waves
        // gave 4.37.
        switch (P / 64) {
#define MESSI_ZN_CASE(EP, R)                                                                                  \
    case EP: {                                                                                                \
        const int blocks = launch_blocks(n, 4 * R, 256 * 128);                                                \
        hipLaunchKernelGGL((znorm_strided_kernel<EP, R>), dim3(blocks), dim3(256), 0, s, series, series, n, len, \
                           (int64_t)len, d_flag, inv_len_pow2(len));                                                             \
        break;                                                                                                \
    }
            MESSI_ZN_CASE(1, 8)
            MESSI_ZN_CASE(2, 4)
            MESSI_ZN_CASE(4, 2)
            MESSI_ZN_CASE(8, 2)
            MESSI_ZN_CASE(16, 1)
#undef MESSI_ZN_CASE
            default: break;
        }
        MESSI_LAUNCH_CHECK("znorm");
        return MESSI_OK;
    }
    RowLayout r = row_layout(len);
    SumArgs a{};
    a.in = series;
    a.zout = series;
    a.inv_len_pow2 = inv_len_pow2(len);
    a.n = n;
    a.L = len;
    a.P = r.P;
    a.T = r.T;
    a.G = r.G;
    a.nonfinite = d_flag;
    return launch_summarize<true, false>(a, r.E, s);
}

int build_index(Index* ix, const float* series, int64_t n, int32_t len, int32_t w, int32_t b, int32_t cap,
                const messi_opts& opts, const SplitTab* forced) {
    hipStream_t s = (hipStream_t)opts.stream;
    ix->series = series;
    ix->n = n;
    ix->len = len;
    ix->w = w;
    ix->b = b;
    ix->cap = cap;
    breakpoints_as241(b, ix->bp_host);
    const int nb = (1 << b) - 1;
    MESSI_TRY(ix->bp.alloc(sizeof(float) * 256));
    MESSI_HIP_TRY(hipMemcpyAsync(ix->bp.p, ix->bp_host, sizeof(float) * nb, hipMemcpyHostToDevice, s));

    const auto t_begin = std::chrono::steady_clock::now();
    Timer tm(s);

    // ---- buffers
    DevBuf W[2], P[2], K[2], misc;
    for (int i = 0; i < 2; ++i) {
        MESSI_TRY(W[i].alloc(sizeof(uint4) * (size_t)n));
        MESSI_TRY(P[i].alloc(sizeof(uint32_t) * (size_t)n));
        MESSI_TRY(K[i].alloc(sizeof(uint16_t) * (size_t)n));
    }
    // misc: [0] nonfinite, [1] absmax bits, [2] n_leaves, [3] n_next, [4] max_leaf, [5] total tiles,
    // [6] internal nodes recorded
    MESSI_TRY(misc.alloc(64));
    uint32_t* cnt = misc.as<uint32_t>();
    MESSI_HIP_TRY(hipMemsetAsync(misc.p, 0, 64, s));

    // ---- 1. summarise (optionally fused with z-normalisation)
    RowLayout r = row_layout(len);
    SumArgs a{};
    a.in = series;
    a.zout = opts.znorm ? const_cast<float*>(series) : nullptr;
    a.inv_len_pow2 = inv_len_pow2(len);
    a.n = n;
    a.L = len;
    a.P = r.P;
    a.T = r.T;
    a.G = r.G;
    a.w = w;
    a.m = len / w;
    a.M = 1;
    while (a.M < a.m) a.M <<= 1;
    a.b = b;
    a.bp = ix->bp.as<float>();
    a.words = W[0].as<uint4>();
    a.keys = K[0].as<uint16_t>();
    a.absmax = cnt + 1;
    a.nonfinite = reinterpret_cast<int*>(cnt + 0);
    if (w < 16) MESSI_HIP_TRY(hipMemsetAsync(W[0].p, 0, sizeof(uint4) * (size_t)n, s));
    // Segments of at most 64 values take the segment summariser; a build that
    // also z-normalises runs the z-normalisation kernel first (the same z
    // values as the general kernel's fused pass, which takes more than twice
    // as long as the two passes together: 31 against 13.5 ms for 20M rows of 256).
    const bool seg_path = a.m <= 64;
    // the fine summary: F sub-segments per segment (none unless m is a power of two in [2, 64])
    const int fF = fine_per_segment(a.m);
    ix->wf = fF ? w * fF : 0;
    ix->mf = fF ? a.m / fF : 0;
    ix->fwords.release();
    if (ix->wf) MESSI_TRY(ix->fwords.alloc((size_t)kFineStride * (size_t)n));
    DevBuf cells;
    if (seg_path) {
        uint8_t hc[kCells];
        cell_table(ix->bp_host, b, hc);
        MESSI_TRY(cells.alloc(kCells));
        MESSI_HIP_TRY(hipMemcpyAsync(cells.p, hc, kCells, hipMemcpyHostToDevice, s));
    }
    if (seg_path && opts.znorm) {
        tm.start();
        MESSI_TRY(znorm_device(const_cast<float*>(series), n, len, s, reinterpret_cast<int*>(cnt + 0)));
        ix->info.ms_znorm = tm.stop_ms();
    }
    tm.start();
    if (opts.znorm && !seg_path) {
        MESSI_TRY((launch_summarize<true, true>(a, r.E, s)));
    } else if (seg_path) {
        SegArgs sa{};
        sa.in = series;
        sa.n = n;
        sa.L = len;
        sa.w = w;
        sa.m = a.m;
        sa.b = b;
        sa.bp = ix->bp.as<float>();
        sa.cells = cells.as<uint8_t>();
        sa.words = reinterpret_cast<uint8_t*>(W[0].p);
        sa.keys = K[0].as<uint16_t>();
        sa.absmax = cnt + 1;
        sa.nonfinite = reinterpret_cast<int*>(cnt + 0);
        sa.fine = ix->wf ? ix->fwords.as<uint8_t>() : nullptr;
        MESSI_TRY(launch_summarize_seg(sa, s));
    } else {
        MESSI_TRY((launch_summarize<false, true>(a, r.E, s)));
    }
    ix->info.ms_summarize = tm.stop_ms();
    uint32_t flags[2];
    MESSI_HIP_TRY(hipMemcpyAsync(flags, cnt, sizeof(flags), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    if (flags[0]) {
        set_error(MESSI_EINVAL, "series contain non-finite values");
        return MESSI_EINVAL;
    }
    memcpy(&ix->absmax, &flags[1], sizeof(float));
    if (ix->wf && !seg_path) {
        // the summarise pass that ran does not write the fine summary: a pass of its own
        tm.start();
        MESSI_TRY(launch_fine(series, n, len, ix->wf, ix->mf, ix->fwords.as<uint8_t>(), s));
        ix->info.ms_summarize += tm.stop_ms();
    }

    // ---- 2. bucket by root key (stable LSD radix, 8-bit digits)
    tm.start();
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    DevBuf hist, scr;
    MESSI_TRY(hist.alloc(sizeof(uint32_t) * 256 * (size_t)n_tiles));
    int cur = 0;
    const int passes = (w + 7) / 8;
    {
        const int64_t hn = 256 * n_tiles;
        const size_t need = std::max(scan_scratch_words(hn), scan_scratch_words((n + 31) / 32)) + 16;
        MESSI_TRY(scr.alloc(sizeof(uint32_t) * need));
    }
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)n_tiles), dim3(kBlk), 0, s, K[cur].as<uint16_t>(), n,
                           shift, hist.as<uint32_t>(), n_tiles);
        MESSI_LAUNCH_CHECK("radix_hist");
        MESSI_TRY(scan_exclusive(hist.as<uint32_t>(), hist.as<uint32_t>(), 256 * n_tiles, scr.as<uint32_t>(), nullptr,
                                 s));
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)n_tiles), dim3(kBlk), 0, s, K[cur].as<uint16_t>(),
                           W[cur].as<uint4>(), pass == 0 ? nullptr : P[cur].as<uint32_t>(), n, shift,
                           hist.as<uint32_t>(), n_tiles, K[cur ^ 1].as<uint16_t>(), W[cur ^ 1].as<uint4>(),
                           P[cur ^ 1].as<uint32_t>());
        MESSI_LAUNCH_CHECK("radix_scatter");
        cur ^= 1;
    }
    hist.release();

    // root runs -> first nodes / leaves
    const uint32_t n_keys = 1u << w;
    DevBuf runs, leaves_raw, leaf_buf, nodes[2], node_cnt, node_seg, node_n0, tile_first, tile_node, tile_cnt, zeros;
    DevBuf node_split, inner;
    size_t inner_cap = 0, inner_ub = 0;  // recorded internal nodes: capacity, upper bound so far
    const SplitTab no_tab{nullptr, nullptr, nullptr, 0u};
    const SplitTab ftab = forced ? *forced : no_tab;
    MESSI_TRY(runs.alloc(sizeof(uint32_t) * 2 * n_keys));
    MESSI_HIP_TRY(hipMemsetAsync(runs.p, 0, sizeof(uint32_t) * 2 * n_keys, s));
    hipLaunchKernelGGL(root_runs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, K[cur].as<uint16_t>(), n,
                       runs.as<uint32_t>(), runs.as<uint32_t>() + n_keys);
    MESSI_LAUNCH_CHECK("root_runs");
    // Leaves: at most n.  Nodes per level: at most n / (cap + 1) + 1 (each holds > cap).
    MESSI_TRY(leaves_raw.alloc(sizeof(Leaf) * (size_t)n));
    MESSI_TRY(leaf_buf.alloc((size_t)n));
    const int64_t max_nodes = n / ((int64_t)cap + 1) + 2;
    const int64_t max_nodes2 = max_nodes;
    for (int i = 0; i < 2; ++i) MESSI_TRY(nodes[i].alloc(sizeof(Leaf) * (size_t)max_nodes2));
    Lists lists;
    lists.leaves = leaves_raw.as<Leaf>();
    lists.leaf_buf = leaf_buf.as<uint8_t>();
    lists.n_leaves = cnt + 2;
    lists.n_next = cnt + 3;
    lists.max_leaf = cnt + 4;
    lists.next = nodes[0].as<Leaf>();
    hipLaunchKernelGGL(root_nodes_kernel, dim3((n_keys + 255) / 256), dim3(256), 0, s, runs.as<uint32_t>(),
                       runs.as<uint32_t>() + n_keys, w, b, cap, cur, lists);
    MESSI_LAUNCH_CHECK("root_nodes");
    uint32_t n_nodes = 0;
    MESSI_HIP_TRY(hipMemcpyAsync(&n_nodes, cnt + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    runs.release();
    ix->info.ms_bucket = tm.stop_ms();

    // ---- 3. split levels
    tm.start();
    const int64_t max_tiles = n_tiles + max_nodes2 + 1;
    MESSI_TRY(node_cnt.alloc(sizeof(uint32_t) * 16 * (size_t)max_nodes2));
    MESSI_TRY(node_seg.alloc((size_t)max_nodes2));
    MESSI_TRY(node_n0.alloc(sizeof(uint32_t) * (size_t)max_nodes2));
    MESSI_TRY(node_split.alloc((size_t)max_nodes2));
    MESSI_TRY(tile_first.alloc(sizeof(uint32_t) * ((size_t)max_nodes2 + 1)));
    MESSI_TRY(tile_node.alloc(sizeof(uint32_t) * (size_t)max_tiles));
    MESSI_TRY(tile_cnt.alloc(sizeof(uint32_t) * 16 * (size_t)max_tiles));
    MESSI_TRY(zeros.alloc(sizeof(uint32_t) * (size_t)max_tiles));
    int levels = 0;
    // One level-synchronous split loop; the current level's nodes start in nodes[0].
    auto run_levels = [&](uint32_t nn, int cap_lvl, Lists lst, int& lv) -> int {
        int nsel = 0;
        while (nn > 0) {
            Leaf* cur_nodes = nodes[nsel].as<Leaf>();
            hipLaunchKernelGGL(node_tiles_kernel, dim3(1), dim3(1024), 0, s, cur_nodes, (int)nn,
                               tile_first.as<uint32_t>(), cnt + 5);
            MESSI_LAUNCH_CHECK("node_tiles");
            uint32_t tiles = 0;
            MESSI_HIP_TRY(hipMemcpyAsync(&tiles, cnt + 5, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            MESSI_HIP_TRY(hipMemsetAsync(node_cnt.p, 0, sizeof(uint32_t) * 16 * (size_t)nn, s));
            MESSI_HIP_TRY(hipMemsetAsync(cnt + 3, 0, sizeof(uint32_t), s));
            MESSI_HIP_TRY(hipStreamSynchronize(s));
            hipLaunchKernelGGL(tile_node_kernel, dim3((tiles + 255) / 256), dim3(256), 0, s,
                               tile_first.as<uint32_t>(), (int)nn, tiles, tile_node.as<uint32_t>());
            MESSI_LAUNCH_CHECK("tile_node");
            hipLaunchKernelGGL(level_count_kernel, dim3(tiles), dim3(kBlk), 0, s, cur_nodes,
                               tile_first.as<uint32_t>(), tile_node.as<uint32_t>(), W[cur].as<uint4>(), w, b,
                               tile_cnt.as<uint32_t>(), node_cnt.as<uint32_t>());
            MESSI_LAUNCH_CHECK("level_count");
            lst.next = nodes[nsel ^ 1].as<Leaf>();
            hipLaunchKernelGGL(level_choose_kernel, dim3((nn + 255) / 256), dim3(256), 0, s, cur_nodes, (int)nn,
                               node_cnt.as<uint32_t>(), w, b, cap_lvl, cur ^ 1, node_seg.as<uint8_t>(),
                               node_n0.as<uint32_t>(), node_split.as<uint8_t>(), ftab, lst);
            MESSI_LAUNCH_CHECK("level_choose");
            // record the nodes that split (kept for later appends)
            if (inner_ub + nn > inner_cap) {
                size_t ncap = std::max<size_t>(1024, 2 * (inner_ub + nn));
                DevBuf grown;
                MESSI_TRY(grown.alloc(sizeof(Leaf) * ncap));
                if (inner_ub) MESSI_HIP_TRY(hipMemcpyAsync(grown.p, inner.p, sizeof(Leaf) * inner_ub,
                                                           hipMemcpyDeviceToDevice, s));
                MESSI_HIP_TRY(hipStreamSynchronize(s));
                inner = std::move(grown);
                inner_cap = ncap;
            }
            hipLaunchKernelGGL(record_inner_kernel, dim3((nn + 255) / 256), dim3(256), 0, s, cur_nodes, (int)nn,
                               node_split.as<uint8_t>(), node_seg.as<uint8_t>(), inner.as<Leaf>(), cnt + 6);
            MESSI_LAUNCH_CHECK("record_inner");
            inner_ub += nn;
            hipLaunchKernelGGL(level_zeros_kernel, dim3((tiles + 255) / 256), dim3(256), 0, s, cur_nodes,
                               tile_first.as<uint32_t>(), tile_node.as<uint32_t>(), tiles, tile_cnt.as<uint32_t>(),
                               node_seg.as<uint8_t>(), zeros.as<uint32_t>());
            MESSI_LAUNCH_CHECK("level_zeros");
            MESSI_TRY(scan_exclusive(zeros.as<uint32_t>(), zeros.as<uint32_t>(), tiles, scr.as<uint32_t>(), nullptr,
                                     s));
            hipLaunchKernelGGL(level_scatter_kernel, dim3(tiles), dim3(kBlk), 0, s, cur_nodes,
                               tile_first.as<uint32_t>(), tile_node.as<uint32_t>(), zeros.as<uint32_t>(),
                               node_seg.as<uint8_t>(), node_n0.as<uint32_t>(), b, W[cur].as<uint4>(),
                               P[cur].as<uint32_t>(), W[cur ^ 1].as<uint4>(), P[cur ^ 1].as<uint32_t>());
            MESSI_LAUNCH_CHECK("level_scatter");
            MESSI_HIP_TRY(hipMemcpyAsync(&nn, cnt + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            MESSI_HIP_TRY(hipStreamSynchronize(s));
            cur ^= 1;
            nsel ^= 1;
            ++lv;
            if (lv > 16 * 8 + 2) {
                set_error(MESSI_EDEVICE, "leaf partition did not terminate");
                return MESSI_EDEVICE;
            }
        }
        return MESSI_OK;
    };
    MESSI_TRY(run_levels(n_nodes, cap, lists, levels));

    uint32_t hc[3];
    MESSI_HIP_TRY(hipMemcpyAsync(hc, cnt + 2, sizeof(hc), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    const uint32_t n_leaves = hc[0];
    ix->max_leaf = hc[2];
    const int fin = 0;  // final buffer index
    hipLaunchKernelGGL(copy_back_kernel, dim3(launch_blocks(n_leaves, 1, 65536)), dim3(kBlk), 0, s,
                       leaves_raw.as<Leaf>(), leaf_buf.as<uint8_t>(), n_leaves, W[1 - fin].as<uint4>(),
                       P[1 - fin].as<uint32_t>(), W[fin].as<uint4>(), P[fin].as<uint32_t>(), 1 - fin);
    MESSI_LAUNCH_CHECK("copy_back");
    cur = fin;
    ix->info.ms_split = tm.stop_ms();
    node_cnt.release(); node_seg.release(); node_n0.release(); tile_first.release(); tile_node.release();
    tile_cnt.release(); zeros.release(); nodes[0].release(); nodes[1].release(); node_split.release();

    // the split table of the new index (read by the next append)
    {
        uint32_t n_inner = 0;
        MESSI_HIP_TRY(hipMemcpyAsync(&n_inner, cnt + 6, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        uint32_t slots = 16;
        while (slots < 2u * n_inner) slots <<= 1;
        MESSI_TRY(ix->split_keys.alloc(sizeof(uint4) * 2 * (size_t)slots));
        MESSI_TRY(ix->split_seg.alloc((size_t)slots));
        MESSI_TRY(ix->split_claim.alloc(sizeof(uint32_t) * (size_t)slots));
        MESSI_HIP_TRY(hipMemsetAsync(ix->split_claim.p, 0, sizeof(uint32_t) * (size_t)slots, s));
        if (n_inner)
            hipLaunchKernelGGL(split_insert_kernel, dim3((n_inner + 255) / 256), dim3(256), 0, s, inner.as<Leaf>(),
                               n_inner, ix->split_keys.as<uint4>(), ix->split_seg.as<uint8_t>(),
                               ix->split_claim.as<uint32_t>(), slots - 1);
        MESSI_LAUNCH_CHECK("split_insert");
        ix->split_mask = slots - 1;
        ix->n_inner = n_inner;
        inner.release();
    }

    // ---- 4. finalise: leaves ordered by start
    tm.start();
    const int64_t nw = (n + 31) / 32;
    DevBuf bm, rank;
    MESSI_TRY(bm.alloc(sizeof(uint32_t) * (size_t)nw));
    MESSI_TRY(rank.alloc(sizeof(uint32_t) * (size_t)nw));
    MESSI_HIP_TRY(hipMemsetAsync(bm.p, 0, sizeof(uint32_t) * (size_t)nw, s));
    hipLaunchKernelGGL(leaf_bitmap_kernel, dim3((n_leaves + 255) / 256), dim3(256), 0, s, leaves_raw.as<Leaf>(),
                       n_leaves, bm.as<uint32_t>());
    MESSI_LAUNCH_CHECK("leaf_bitmap");
    hipLaunchKernelGGL(popc_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, bm.as<uint32_t>(), nw,
                       rank.as<uint32_t>());
    MESSI_LAUNCH_CHECK("popc");
    MESSI_TRY(scan_exclusive(rank.as<uint32_t>(), rank.as<uint32_t>(), nw, scr.as<uint32_t>(), nullptr, s));
    MESSI_TRY(ix->leaves.alloc(sizeof(Leaf) * (size_t)n_leaves));
    hipLaunchKernelGGL(leaf_order_kernel, dim3((n_leaves + 255) / 256), dim3(256), 0, s, leaves_raw.as<Leaf>(),
                       n_leaves, bm.as<uint32_t>(), rank.as<uint32_t>(), ix->leaves.as<Leaf>());
    MESSI_LAUNCH_CHECK("leaf_order");
    MESSI_TRY(ix->cwords.alloc(sizeof(uint2) * (size_t)n));
    hipLaunchKernelGGL(coarse_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 16 * (int64_t)device_cu_count())),
                       dim3(256), 0, s, W[fin].as<uint4>(), n, b - std::min(b, 4), ix->cwords.as<uint2>());
    MESSI_LAUNCH_CHECK("coarse");
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    ix->info.ms_finalize = tm.stop_ms();

    // keep the final arrays, drop the rest
    ix->words = std::move(W[fin]);
    ix->pos = std::move(P[fin]);
    ix->n_leaves = n_leaves;
    ix->levels = levels;
    const auto t_end = std::chrono::steady_clock::now();
    ix->info.ms_total = std::chrono::duration<double, std::milli>(t_end - t_begin).count();
    return MESSI_OK;
}

}  // namespace messi

// Batched BF16 filter on the matrix cores, with a rounding bound that keeps the
// search exact, then a compensated fp32 recheck of the survivors.
//
// For a batch of queries, the (query, leaf) pairs that survive the leaf bound
// are grouped by leaf.  A block stages a leaf's queries in LDS as BF16 rows
// (the A operand); each of its waves holds the BF16 rows of 32 of the leaf's
// members in registers (the B operand), so a member row is read from HBM once
// per leaf and round whatever the number of queries that visit the leaf.
// For every (query q, member x) the filter evaluates
//     f = |q|^2 + |x|^2 - 2 s,   s = sum_j bf16(q_j) bf16(x_j)  (fp32 accumulation)
// and may discard x for q only if f - E(q, x) > U_q, where E bounds |f - D| for
// the exact squared distance D = |q - x|^2:
//   - operand rounding to BF16 (unit roundoff u_b = 2^-8), by Cauchy-Schwarz:
//       |sum bf16(q_j) bf16(x_j) - q.x| <= (2 u_b + u_b^2) |q| |x|
//   - fp32 accumulation in any order and rounding (u = 2^-23):
//       <= gamma_{K-1} (1 + u_b)^2 |q| |x|,   gamma_n = n u / (1 - n u)
//   - the norms are fp32 roundings of fp64 sums, and the remaining operations
//     round once each: covered by relative slacks of 2^-20 on |q|^2, |x|^2, U.
// The filter kernel folds this test into its MFMA chain (one extra k-step, see
// there), so the whole drop decision is one compare per (query, member).  A
// discarded member has D > U_q >= the k-th true distance, so it is not an
// answer.  Survivors get a Neumaier-compensated fp32 distance (relative error
// ~3 u32), which feeds the same candidate/bound logic as the fp32 scan; the
// final order uses the canonical fp64 distance.
#include <algorithm>
#include <cmath>
#include <vector>

#include "query.h"

namespace messi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Ends of the filter rounds in each query's leaf order: a first bound from the
// query's best leaves, a tighter one over the next few hundred, then the rest.
// With a batch of queries nearly every leaf is visited in every later round,
// so a round costs a pass over most of the BF16 rows: few rounds.
constexpr uint32_t kRoundEnds[] = {16u, 0xffffffffu, 0xffffffffu};
// The FP32 filter's rounds when its batch is wide.  Its test is tight, so
// the members a round appends are those within the query's bound at the
// round's start.  When the leaf bounds of many of the batch's queries keep
// more than a quarter of the leaves (data with many near-equal distances),
// growing rounds keep those bounds close to the k-th distance and the
// candidate buffers small.  Otherwise the batch takes the BF16 filter's two
// rounds: fewer rounds share more reads of a leaf's rows among the queries.
constexpr uint32_t kRoundEndsF32[] = {16u, 128u, 1024u, 8192u, 0xffffffffu};

// Queries whose ordered leaves exceed a quarter of all leaves, into *count.
__global__ void __launch_bounds__(256) wide_count_kernel(QArgs a, uint32_t* count) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    uint32_t w = 0;
    if (q < a.nq && a.qs[q].err == 0) w = (uint64_t)a.qs[q].nsurv * 4 > (uint64_t)a.nL ? 1u : 0u;
    const unsigned long long b = __ballot(w != 0);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (uint32_t)__popcll(b));
}

__global__ void word_clear_kernel(uint32_t* p) { *p = 0; }

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t vload(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

// Directed roundings for non-negative values: largest fp32 / BF16 value not
// above x, smallest BF16 value not below x.
__device__ __forceinline__ float f32_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}
__device__ __forceinline__ uint16_t bf16_down(float x) { return (uint16_t)(__float_as_uint(x) >> 16); }
__device__ __forceinline__ uint16_t bf16_up(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u >> 16) + ((u & 0xFFFFu) ? 1u : 0u));
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
constexpr uint16_t kBf16MinusOne = 0xBF80u;

// The constants of the filter's test for rows padded to Lp (see the filter).
struct BfConsts {
    double c1p;  // coefficient of |q||x|
    double g;    // member-side slack
    double h;    // query-side slack
};

BfConsts bf_consts(int Lp) {
    const double ub = std::ldexp(1.0, -8), u = std::ldexp(1.0, -23);
    const double nu = (double)(Lp + 32 - 1) * u;  // terms accumulated: Lp products + the extra k-step
    const double gamma = nu / (1.0 - nu);
    const double c1 = 4.0 * ub + 2.0 * ub * ub + 2.0 * gamma * (1.0 + ub) * (1.0 + ub);
    BfConsts k;
    k.c1p = c1 * (1.0 + 2.0 * gamma + std::ldexp(1.0, -18));
    k.g = gamma + std::ldexp(1.0, -20) + std::ldexp(1.0, -22);
    k.h = std::ldexp(1.0, -20) + std::ldexp(1.0, -22);
    return k;
}

// ---------------------------------------------------------------------------
// build: BF16 rows in leaf order (zero-padded to a multiple of 32) and, per
// member, the BF16 terms of the filter's extra k-step: |x| rounded up and
// beta = (1 - g) |x|^2 as a sum of two BF16 values rounded down (|x|^2 summed
// in fp64).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) shadow_kernel(const float* __restrict__ series, const uint32_t* __restrict__ pos,
                                                     int64_t n, int L, int Lp, double one_minus_g,
                                                     uint16_t* __restrict__ shadow, uint2* __restrict__ sx) {
    const int lane = threadIdx.x & 63;
    const bool vec = (L % 4) == 0;
    for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.x * 4) {
        const float* x = series + (size_t)pos[j] * L;
        double acc = 0.0;
        for (int e0 = lane * 4; e0 < Lp; e0 += 256) {
            float v[4];
            if (vec && e0 + 3 < L) {
                const float4 f = *reinterpret_cast<const float4*>(x + e0);
                v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = (e0 + i < L) ? x[e0 + i] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) acc += (double)v[i] * (double)v[i];
            const uint32_t lo = (uint32_t)bf16_rne(v[0]) | ((uint32_t)bf16_rne(v[1]) << 16);
            const uint32_t hi = (uint32_t)bf16_rne(v[2]) | ((uint32_t)bf16_rne(v[3]) << 16);
            *reinterpret_cast<uint2*>(shadow + (size_t)j * Lp + e0) = make_uint2(lo, hi);
        }
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) {
            const uint16_t rx = bf16_up((float)sqrt(acc) * 1.0000001192092896f);  // |x|, from above
            const double beta = one_minus_g * acc;
            const uint16_t bh = bf16_down(f32_down(beta));
            const uint16_t bl = bf16_down(f32_down(beta - (double)bf16_value(bh)));
            sx[j] = make_uint2((uint32_t)rx | ((uint32_t)bh << 16), (uint32_t)bl);
        }
    }
}

// ---------------------------------------------------------------------------
// query side
// ---------------------------------------------------------------------------
struct BfArgs {
    int32_t Lp, ksteps;
    const uint16_t* shadow;
    const uint2* sx;        // [n] member terms of the extra k-step
    const uint16_t* qb;     // [nq][Lp] bf16 queries, doubled
    const float2* qnorm;    // [nq] (|q|^2, |q|)
    const uint4* qx;        // [nq] query terms of the extra k-step
    const uint32_t* leaf_cnt;
    const uint32_t* leaf_off;
    const uint32_t* leaf_q;
    const uint32_t* leaf_act;  // the round's leaves with at least one query
    uint2* pairs;           // (query, member position)
    uint32_t* npairs;       // round counters: survivors, next active leaf, active leaves, slots
    uint32_t pairs_cap;
    int32_t qc;             // queries of a leaf staged in LDS at a time (multiple of 16)
    float one_minus_h;      // 1 - h, rounded down
    float f32_c;            // FP32 filter: slack per unit of |q|^2 + |x|^2
};

// Per query: 2 q in BF16 (an exact doubling of the rounded q), |q|^2 and |q|
// from fp64, and the extra k-step (c1' |q| rounded up, -1, -1, 0, ...) that
// meets the member's (|x|, beta_hi, beta_lo, 0, ...).
__global__ void __launch_bounds__(256) qprep_bf16_kernel(const float* __restrict__ queries, int L, int Lp, float c1p,
                                                         uint16_t* __restrict__ qb, float2* __restrict__ qnorm,
                                                         uint4* __restrict__ qx) {
    __shared__ double s_part[4];
    const int q = blockIdx.x;
    const float* row = queries + (size_t)q * L;
    double acc = 0.0;
    for (int e = threadIdx.x; e < Lp; e += 256) {
        const float v = (e < L) ? row[e] : 0.f;
        acc += (double)v * (double)v;
        qb[(size_t)q * Lp + e] = bf16_rne(2.0f * v);
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        const float rq = (float)sqrt(t);
        qnorm[q] = make_float2((float)t, rq);
        // c1' |q| from above: one ulp over the rounded product, then BF16 up
        const float cq = __uint_as_float(__float_as_uint(c1p * (rq * 1.0000001192092896f)) + 1u);
        qx[q] = make_uint4((uint32_t)bf16_up(cq) | ((uint32_t)kBf16MinusOne << 16), (uint32_t)kBf16MinusOne, 0u, 0u);
    }
}

// Positions [t0, t1) of every query's leaf order whose bound does not exceed
// the query's current U take part in a round.  For the serving engine's slots
// each active slot has its own window instead.
__device__ __forceinline__ void round_window(const QArgs& a, int q, uint32_t& t0, uint32_t& t1) {
    if (a.win) {
        if (a.phase && a.phase[q] != kSlotActive) {
            t0 = t1 = 0;
            return;
        }
        t0 = a.win[3 * q];
        t1 = a.win[3 * q + 1];
    }
}

__device__ __forceinline__ bool round_leaf(const QArgs& a, int q, uint32_t t, uint32_t t1, uint32_t& leaf) {
    const QState& st = a.qs[q];
    if (t >= t1 || t >= st.nsurv || st.err) return false;
    leaf = a.order[(size_t)q * a.nL + t];
    const float U = __uint_as_float(vload(&st.U));
    return !(a.lb[(size_t)q * a.nL + leaf] * (1.0f - kRhoLb) > U);
}

// The round's counters: [0] filter survivors, [1] next active leaf of the
// filter, [2] active leaves, [3] query slots handed out; and for the call,
// [4] the most queries any leaf had in a round (cleared by the first round).
// Words, not a memset, so that the whole round can be recorded in a graph.
__global__ void __launch_bounds__(256) round_reset_kernel(uint32_t* __restrict__ leaf_cnt, uint32_t nL,
                                                          uint32_t* __restrict__ ctr, int first) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nL; i += gridDim.x * 256) leaf_cnt[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < (first ? 5 : 4)) ctr[threadIdx.x] = 0;
}

// Count the queries of every leaf; the first query to reach a leaf appends it
// to the round's list of active leaves.
__global__ void __launch_bounds__(256) leaf_count_kernel(QArgs a, uint32_t t0, uint32_t t1,
                                                         uint32_t* __restrict__ leaf_cnt,
                                                         uint32_t* __restrict__ leaf_act, uint32_t* __restrict__ ctr) {
    const int q = blockIdx.y;
    round_window(a, q, t0, t1);
    for (uint32_t t = t0 + blockIdx.x * 256 + threadIdx.x; t < t1; t += gridDim.x * 256) {
        uint32_t leaf;
        if (round_leaf(a, q, t, t1, leaf) && atomicAdd(&leaf_cnt[leaf], 1u) == 0u)
            leaf_act[atomicAdd(&ctr[2], 1u)] = leaf;
    }
}

// Each active leaf takes a contiguous run of query slots (runs in no
// particular order) and resets its fill cursor.
__global__ void __launch_bounds__(256) leaf_offsets_kernel(const uint32_t* __restrict__ leaf_cnt,
                                                           const uint32_t* __restrict__ leaf_act,
                                                           uint32_t* __restrict__ leaf_off,
                                                           uint32_t* __restrict__ leaf_cur, uint32_t* __restrict__ ctr) {
    const uint32_t nact = ctr[2];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nact; i += gridDim.x * 256) {
        const uint32_t leaf = leaf_act[i];
        leaf_off[leaf] = atomicAdd(&ctr[3], leaf_cnt[leaf]);
        leaf_cur[leaf] = 0;
        atomicMax(&ctr[4], leaf_cnt[leaf]);
    }
}

__global__ void __launch_bounds__(256) leaf_scatter_kernel(QArgs a, uint32_t t0, uint32_t t1,
                                                           const uint32_t* __restrict__ leaf_off,
                                                           uint32_t* __restrict__ leaf_cur,
                                                           uint32_t* __restrict__ leaf_q, size_t leafq_cap) {
    const int q = blockIdx.y;
    round_window(a, q, t0, t1);
    for (uint32_t t = t0 + blockIdx.x * 256 + threadIdx.x; t < t1; t += gridDim.x * 256) {
        uint32_t leaf;
        if (round_leaf(a, q, t, t1, leaf)) {
            const size_t at = (size_t)leaf_off[leaf] + atomicAdd(&leaf_cur[leaf], 1u);
            if (at < leafq_cap) leaf_q[at] = (uint32_t)q;
        }
    }
}

// ---------------------------------------------------------------------------
// The filter.  s = MFMA sum of BF16 products, with the fp32 accumulation of
// K = Lp + 32 terms in any order and rounding (u = 2^-23, gamma = gamma_{K-1})
// covered; |q~.x~ - q.x| <= (2 u_b + u_b^2) |q||x| for the BF16-rounded rows.
// The query's A row is 2 q~ followed by the extra k-step (c~, -1, -1, 0, ...),
// the member's B row is x~ followed by (r~x, b_hi, b_lo, 0, ...), where
//   c~ >= c1' |q|,  r~x >= |x|,  b_hi + b_lo <= beta = (1 - g) |x|^2,
//   c1 = 4 u_b + 2 u_b^2 + 2 gamma (1 + u_b)^2,  c1' = c1 (1 + 2 gamma + 2^-18),
//   g = gamma + 2^-20 + 2^-22,
// so one MFMA chain yields acc ~ 2 q~.x~ + c~ r~x - b_hi - b_lo.  A member is
// dropped for a query iff acc < alpha = fl(fl((1 - h) |q|^2) - fl(U (1 + 2^-20))),
// h = 2^-20 + 2^-22.  That drop is exact: with the accumulation error at most
// gamma (2 (1 + u_b)^2 |q||x| + c~ r~x + beta),
//   D = |q|^2 + |x|^2 - 2 q.x  >=  |q|^2 + |x|^2 - acc + c~ r~x (1 - gamma)
//       - c1 |q||x| - (1 - g) |x|^2 - gamma beta
//     >  U (1 + 2^-20) + (h - 2^-23) |q|^2 + (g - gamma - 2^-23) |x|^2 - err(alpha)
//     >= U,
// because c~ r~x (1 - gamma) covers c1 |q||x| (norms are fp32 roundings of
// fp64 sums, within 2^-23), and a drop needs acc > -(|q|^2 + 2|x|^2) (1.01),
// so U < 2.02 (|q|^2 + |x|^2) and the roundings of alpha stay below the 2^-20
// slacks.  The test costs one compare per (query, member).
//
// Work: blocks of kFWaves waves (one block per CU) take leaves from a shared
// counter.  For a leaf, up to QC of its queries (BF16 rows) are staged in LDS
// once; each wave holds the BF16 rows of 32 members in registers (two
// 16-member B fragments per 32-wide k-step) and streams 16-query A fragments
// from LDS, every A fragment feeding two mfma_f32_16x16x32_bf16, two query
// tiles interleaved.  Two fragments per wave keep a wave at about 150
// registers, so twelve waves fit a CU: the filter waits on memory, and the
// extra waves hide more of it than four fragments per wave save in LDS reads.
// Rows longer than 256 values are taken 8 k-steps of B at a time.
// ---------------------------------------------------------------------------
constexpr int kFWaves = 12;
constexpr int kFThreads = 64 * kFWaves;
constexpr int kFFrags = 2;                 // 16-member B fragments per wave
constexpr int kFQT = 2;                    // 16-query A tiles per step
constexpr int kFMem = 16 * kFFrags;        // members per wave
constexpr int kFTile = kFWaves * kFMem;    // members per block step
constexpr int kFKC = 8;                    // k-steps of B held at a time

__device__ __forceinline__ bf16x8 member_extra(const uint2* sx, uint32_t pos, bool valid, int kb) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (valid && kb == 0) {
        const uint2 t = sx[pos];
        v = make_uint4(t.x, t.y, 0u, 0u);
    }
    return __builtin_bit_cast(bf16x8, v);
}

__global__ void __launch_bounds__(kFThreads) bf16_filter_kernel(QArgs a, BfArgs bf) {
    extern __shared__ __align__(16) uint8_t s_raw[];
    const int QC = bf.qc, Lp = bf.Lp, ks = bf.ksteps, lda = Lp + 8;
    uint16_t* s_a = reinterpret_cast<uint16_t*>(s_raw);
    float* s_alpha = reinterpret_cast<float*>(s_raw + (size_t)QC * lda * 2);
    uint4* s_qx = reinterpret_cast<uint4*>(s_alpha + QC);
    uint32_t* s_qid = reinterpret_cast<uint32_t*>(s_qx + QC);
    __shared__ uint32_t s_leaf;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kb = lane >> 4;
    const float h1 = bf.one_minus_h;
    unsigned long long c_eval = 0, c_bytes = 0;
    const uint32_t nact = bf.npairs[2];
    for (;;) {
        __syncthreads();  // every wave is done with the previous leaf's LDS
        if (tid == 0) s_leaf = atomicAdd(&bf.npairs[1], 1u);
        __syncthreads();
        const uint32_t li = s_leaf;
        if (li >= nact) break;
        const uint32_t leaf = bf.leaf_act[li];
        const uint32_t cntq = bf.leaf_cnt[leaf];
        const Leaf lf = a.leaves[leaf];
        const uint32_t qoff = bf.leaf_off[leaf];
        for (uint32_t qc0 = 0; qc0 < cntq; qc0 += QC) {
            const int nqc = (int)min((uint32_t)QC, cntq - qc0);
            const int nrows = (nqc + 15) & ~15;
            if (qc0 > 0) __syncthreads();
            // ---- stage the chunk's queries: ids and per-query terms, then the
            // BF16 rows (rows past nqc are zero), eight 16-byte loads in flight
            // per thread
            for (int r = tid; r < nrows; r += kFThreads) {
                if (r < nqc) {
                    const uint32_t q = bf.leaf_q[qoff + qc0 + r];
                    const float2 qn = bf.qnorm[q];
                    const float U = __uint_as_float(vload(&a.qs[q].U));
                    s_qid[r] = q;
                    s_qx[r] = bf.qx[q];
                    s_alpha[r] = __fsub_rn(__fmul_rn(h1, qn.x), __fmul_rn(U, 1.00000095367431640625f));
                } else {
                    s_qid[r] = 0xffffffffu;
                    s_qx[r] = make_uint4(0, 0, 0, 0);
                    s_alpha[r] = -__uint_as_float(0x7f800000u);
                }
            }
            __syncthreads();
            const int chunks = Lp / 8;  // 16-byte pieces per row
            const int total = nrows * chunks;
            for (int base = 0; base < total; base += 8 * kFThreads) {
                uint4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + u * kFThreads + tid;
                    v[u] = make_uint4(0, 0, 0, 0);
                    if (idx < total) {
                        const uint32_t q = s_qid[idx / chunks];
                        if (q != 0xffffffffu)
                            v[u] = *reinterpret_cast<const uint4*>(bf.qb + (size_t)q * Lp + 8 * (idx % chunks));
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + u * kFThreads + tid;
                    if (idx < total) *reinterpret_cast<uint4*>(&s_a[(idx / chunks) * lda + 8 * (idx % chunks)]) = v[u];
                }
            }
            __syncthreads();
            // ---- members: each wave kFMem of every kFTile
            const bool pf = ks <= kFKC;  // the whole row fits the B registers
            for (uint32_t mt0 = 0; mt0 < lf.count; mt0 += kFTile) {
                const uint32_t mb = mt0 + wave * kFMem;
                if (mb >= lf.count) continue;  // this wave has no members in the tile
                uint32_t mpos[kFFrags];
                bool mval[kFFrags];
                bf16x8 bfrag[kFFrags][kFKC], bx[kFFrags];
#pragma unroll
                for (int f = 0; f < kFFrags; ++f) {
                    const uint32_t mi = mb + f * 16 + col;
                    mval[f] = mi < lf.count;
                    mpos[f] = lf.start + (mval[f] ? mi : 0u);
                    if (mval[f] && kb == 0) c_bytes += (uint64_t)Lp * 2 + 8;
                    bx[f] = member_extra(bf.sx, mpos[f], mval[f], kb);
                    if (pf) {
#pragma unroll
                        for (int st = 0; st < kFKC; ++st) {
                            uint4 v = make_uint4(0, 0, 0, 0);
                            if (st < ks && mval[f])
                                v = *reinterpret_cast<const uint4*>(bf.shadow + (size_t)mpos[f] * Lp + 32 * st + 8 * kb);
                            bfrag[f][st] = __builtin_bit_cast(bf16x8, v);
                        }
                    }
                }
                for (int qg0 = 0; qg0 < nqc; qg0 += 16 * kFQT) {
                    const int ntile = min(kFQT, (nqc - qg0 + 15) / 16);
                    floatx4 acc[kFQT][kFFrags];
#pragma unroll
                    for (int t = 0; t < kFQT; ++t)
#pragma unroll
                        for (int f = 0; f < kFFrags; ++f) acc[t][f] = floatx4{0.f, 0.f, 0.f, 0.f};
                    const uint16_t* arow = &s_a[(qg0 + col) * lda + 8 * kb];
                    for (int kc = 0; kc < ks; kc += kFKC) {
                        // B for these k-steps (rows of at most kFKC k-steps have it already)
                        if (!pf) {
#pragma unroll
                            for (int f = 0; f < kFFrags; ++f)
#pragma unroll
                                for (int st = 0; st < kFKC; ++st) {
                                    uint4 v = make_uint4(0, 0, 0, 0);
                                    if (kc + st < ks && mval[f])
                                        v = *reinterpret_cast<const uint4*>(bf.shadow + (size_t)mpos[f] * Lp +
                                                                            32 * (kc + st) + 8 * kb);
                                    bfrag[f][st] = __builtin_bit_cast(bf16x8, v);
                                }
                        }
                        // k-step by k-step over the query tiles: every A fragment
                        // feeds kFFrags MFMAs, kFQT * kFFrags chains interleave
#pragma unroll
                        for (int st = 0; st < kFKC; ++st) {
                            if (kc + st < ks) {
                                bf16x8 af[kFQT];
#pragma unroll
                                for (int t = 0; t < kFQT; ++t)
                                    if (t < ntile)
                                        af[t] = __builtin_bit_cast(
                                            bf16x8, *reinterpret_cast<const uint4*>(arow + 16 * t * lda + 32 * (kc + st)));
#pragma unroll
                                for (int t = 0; t < kFQT; ++t) {
                                    if (t < ntile) {
#pragma unroll
                                        for (int f = 0; f < kFFrags; ++f)
                                            acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bfrag[f][st],
                                                                                                acc[t][f], 0, 0, 0);
                                    }
                                }
                            }
                        }
                    }
                    // the extra k-step: c~ r~x - b_hi - b_lo
                    {
                        bf16x8 ax[kFQT];
#pragma unroll
                        for (int t = 0; t < kFQT; ++t)
                            if (t < ntile)
                                ax[t] = __builtin_bit_cast(bf16x8, kb == 0 ? s_qx[qg0 + 16 * t + col] : make_uint4(0, 0, 0, 0));
#pragma unroll
                        for (int t = 0; t < kFQT; ++t) {
                            if (t < ntile) {
#pragma unroll
                                for (int f = 0; f < kFFrags; ++f)
                                    acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax[t], bx[f], acc[t][f], 0, 0, 0);
                            }
                        }
                    }
                    // ---- the test; acc[t][f][i] is query row qg0 + 16 t + 4 kb + i, member col of fragment f
#pragma unroll
                    for (int t = 0; t < kFQT; ++t) {
                        if (t >= ntile) continue;
                        const int r0 = qg0 + 16 * t + 4 * kb;  // this lane's 4 query rows
                        const float4 al4 = *reinterpret_cast<const float4*>(&s_alpha[r0]);
                        const float alv[4] = {al4.x, al4.y, al4.z, al4.w};
                        int nvalid = 0;
#pragma unroll
                        for (int f = 0; f < kFFrags; ++f) nvalid += (int)mval[f];
                        c_eval += (uint32_t)(min(4, max(0, nqc - r0)) * nvalid);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (r0 + i >= nqc) continue;  // padding rows of the last tile
#pragma unroll
                            for (int f = 0; f < kFFrags; ++f) {
                                if (mval[f] && !(acc[t][f][i] < alv[i])) {
                                    const uint32_t slot = atomicAdd(bf.npairs, 1u);
                                    const uint32_t q = s_qid[r0 + i];
                                    if (slot < bf.pairs_cap) {
                                        bf.pairs[slot] = make_uint2(q, mpos[f]);
                                    } else {
                                        // this query lost a pair: its answer is redone by the fp32
                                        // path (the final kernel raises the call's flag)
                                        if (a.qs[q].err == 0) a.qs[q].err = 5;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    if (a.counters) {
        for (int off = 32; off >= 1; off >>= 1) {
            c_eval += __shfl_xor(c_eval, off);
            c_bytes += __shfl_xor(c_bytes, off);
        }
        if (lane == 0 && c_eval) {
            atomicAdd(&a.counters->distance, c_eval);
            atomicAdd(&a.counters->bytes, c_bytes);
        }
    }
}

// Neumaier-compensated fp32 sum helpers (explicit roundings, no contraction).
__device__ __forceinline__ void neumaier_add(float& s, float& c, float y) {
    const float t = __fadd_rn(s, y);
    if (fabsf(s) >= fabsf(y))
        c = __fadd_rn(c, __fadd_rn(__fsub_rn(s, t), y));
    else
        c = __fadd_rn(c, __fadd_rn(__fsub_rn(y, t), s));
    s = t;
}

__device__ __forceinline__ void two_sum_merge(float& s, float& c, float s2, float c2) {
    const float t = __fadd_rn(s, s2);
    const float bp = __fsub_rn(t, s);
    const float e = __fadd_rn(__fsub_rn(s, __fsub_rn(t, bp)), __fsub_rn(s2, bp));
    c = __fadd_rn(__fadd_rn(c, c2), e);
    s = t;
}

// 16 lanes per (query, member) pair, 4 pairs per wave.
// ---------------------------------------------------------------------------
// The FP32 filter: the same leaf-major rounds as the BF16 filter, on the fp32
// rows themselves (no shadow) with the fp32 matrix instruction
// mfma_f32_16x16x4_f32, for batches whose BF16 margin is too wide to prune
// (short rows, many near-equal distances) or calls in FP32 mode.
//   acc = q.x accumulated in fp32 in any order: |acc - q.x| <= gamma_L |q||x|
//   <= gamma_L (|q|^2 + |x|^2) / 2; |q|^2 is the fp32 rounding of an fp64
//   sum, |x|^2 an fp32 sum of squares (error <= gamma_{L+1} |x|^2), and the
//   test's own three roundings add at most 3u (|q|^2 + |x|^2 + 2|acc|).  So
//     D >= (|q|^2 + |x|^2 - 2 acc) - c (|q|^2 + |x|^2) - 8u |acc|,
//   c = (4 (L + 2) + 8) u (u = 2^-23, as for the BF16 filter), and a member
//   is dropped for a query only when that lower bound exceeds U (1 + 2^-20):
//   the drop is exact, and survivors are rechecked as BF16 survivors are.
// Layout: the 16x16x4 instruction takes A[i][k] from lane 16k + i and B[k][j]
// from lane 16k + j, and leaves D[4k' + r][j] in lane 16k' + j.  The k index
// of the product is permuted: k-step s, sub-index k covers element k E + s of
// the row (E = Lq / 4), so each lane holds one contiguous quarter of its
// member's row (float4 loads) and reads one contiguous quarter of a query row
// from LDS.  F 16-member fragments per wave, QT 16-query tiles per pass.
// ---------------------------------------------------------------------------
template <int E, int F>
__global__ void __launch_bounds__(kFThreads) f32_filter_kernel(QArgs a, BfArgs bf) {
    extern __shared__ __align__(16) uint8_t s_raw[];
    constexpr int QT = 2;
    constexpr int Lq = 4 * E, lda = Lq + 4;  // padded rows: a tile's 16 rows start in different banks
    const int QC = bf.qc, L = a.L;
    float* s_q = reinterpret_cast<float*>(s_raw);
    float* s_thr = s_q + (size_t)QC * lda;  // U (1 + 2^-20) of the query when staged
    float* s_qn = s_thr + QC;               // |q|^2
    uint32_t* s_qid = reinterpret_cast<uint32_t*>(s_qn + QC);
    __shared__ uint32_t s_leaf;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kb = lane >> 4;
    const float cq = bf.f32_c, ca = 8.0f * 1.1920928955078125e-07f;
    unsigned long long c_eval = 0, c_bytes = 0;
    const uint32_t nact = bf.npairs[2];
    for (;;) {
        __syncthreads();  // every wave is done with the previous leaf's LDS
        if (tid == 0) s_leaf = atomicAdd(&bf.npairs[1], 1u);
        __syncthreads();
        const uint32_t li = s_leaf;
        if (li >= nact) break;
        const uint32_t leaf = bf.leaf_act[li];
        const uint32_t cntq = bf.leaf_cnt[leaf];
        const Leaf lf = a.leaves[leaf];
        const uint32_t qoff = bf.leaf_off[leaf];
        for (uint32_t qc0 = 0; qc0 < cntq; qc0 += QC) {
            const int nqc = (int)min((uint32_t)QC, cntq - qc0);
            const int nrows = (nqc + 15) & ~15;
            if (qc0 > 0) __syncthreads();
            for (int r = tid; r < nrows; r += kFThreads) {
                if (r < nqc) {
                    const uint32_t q = bf.leaf_q[qoff + qc0 + r];
                    s_qid[r] = q;
                    s_qn[r] = bf.qnorm[q].x;
                    s_thr[r] = __fmul_rn(__uint_as_float(vload(&a.qs[q].U)), 1.00000095367431640625f);
                } else {
                    s_qid[r] = 0xffffffffu;
                    s_qn[r] = 0.f;
                    s_thr[r] = -__uint_as_float(0x7f800000u);
                }
            }
            __syncthreads();
            // the rows, 16 bytes at a time (values past L and rows past nqc are zero)
            constexpr int chunks = Lq / 4;
            const int total = nrows * chunks;
            for (int idx = tid; idx < total; idx += kFThreads) {
                const int r = idx / chunks, c4 = 4 * (idx % chunks);
                const uint32_t q = s_qid[r];
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (q != 0xffffffffu && c4 < L) v = *reinterpret_cast<const float4*>(a.queries + (size_t)q * L + c4);
                *reinterpret_cast<float4*>(&s_q[r * lda + c4]) = v;
            }
            __syncthreads();
            for (uint32_t mt0 = 0; mt0 < lf.count; mt0 += kFWaves * 16 * F) {
                const uint32_t mb = mt0 + wave * 16 * F;
                if (mb >= lf.count) continue;
                float b[F][E];
                float xn[F];
                bool mval[F];
                uint32_t mpos[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t mi = mb + f * 16 + col;
                    mval[f] = mi < lf.count;
                    mpos[f] = lf.start + (mval[f] ? mi : 0u);
                    const float* row = a.series + (size_t)a.pos[mpos[f]] * L + kb * E;
#pragma unroll
                    for (int j = 0; j < E; j += 4) {
                        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (mval[f] && kb * E + j < L) v = *reinterpret_cast<const float4*>(row + j);
                        b[f][j] = v.x;
                        b[f][j + 1] = v.y;
                        b[f][j + 2] = v.z;
                        b[f][j + 3] = v.w;
                    }
                    if (mval[f] && kb == 0) c_bytes += (uint64_t)L * 4;
                    float sq = 0.f;
#pragma unroll
                    for (int j = 0; j < E; ++j) sq = fmaf(b[f][j], b[f][j], sq);
                    sq += __shfl_xor(sq, 16);
                    sq += __shfl_xor(sq, 32);
                    xn[f] = sq;
                }
                for (int qg0 = 0; qg0 < nqc; qg0 += 16 * QT) {
                    const int ntile = min(QT, (nqc - qg0 + 15) / 16);
                    floatx4 acc[QT][F];
#pragma unroll
                    for (int t = 0; t < QT; ++t)
#pragma unroll
                        for (int f = 0; f < F; ++f) acc[t][f] = floatx4{0.f, 0.f, 0.f, 0.f};
                    const float* arow = &s_q[(qg0 + col) * lda + kb * E];
#pragma unroll
                    for (int j = 0; j < E; j += 4) {
                        float4 av[QT];
#pragma unroll
                        for (int t = 0; t < QT; ++t)
                            av[t] = t < ntile ? *reinterpret_cast<const float4*>(arow + t * 16 * lda + j)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                        for (int t = 0; t < QT; ++t) {
                            if (t < ntile) {
#pragma unroll
                                for (int f = 0; f < F; ++f) {
                                    acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].x, b[f][j], acc[t][f], 0, 0, 0);
                                    acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].y, b[f][j + 1], acc[t][f], 0, 0, 0);
                                    acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].z, b[f][j + 2], acc[t][f], 0, 0, 0);
                                    acc[t][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].w, b[f][j + 3], acc[t][f], 0, 0, 0);
                                }
                            }
                        }
                    }
                    // acc[t][f][r]: query row qg0 + 16 t + 4 kb + r, member col of fragment f
#pragma unroll
                    for (int t = 0; t < QT; ++t) {
                        if (t >= ntile) continue;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int qi = qg0 + 16 * t + 4 * kb + r;
                            if (qi >= nqc) continue;
                            const float thr = s_thr[qi], qn = s_qn[qi];
#pragma unroll
                            for (int f = 0; f < F; ++f) {
                                if (!mval[f]) continue;
                                ++c_eval;
                                const float ac = acc[t][f][r];
                                const float sn = __fadd_rn(qn, xn[f]);
                                const float est = __fsub_rn(sn, __fadd_rn(ac, ac));
                                const float slack = __fadd_rn(__fmul_rn(cq, sn), __fmul_rn(ca, fabsf(ac)));
                                if (!(__fsub_rn(est, slack) > thr)) {
                                    const uint32_t slot = atomicAdd(bf.npairs, 1u);
                                    const uint32_t q = s_qid[qi];
                                    if (slot < bf.pairs_cap) {
                                        bf.pairs[slot] = make_uint2(q, mpos[f]);
                                    } else {
                                        if (a.qs[q].err == 0) a.qs[q].err = 5;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    if (a.counters) {
        for (int off = 32; off >= 1; off >>= 1) {
            c_eval += __shfl_xor(c_eval, off);
            c_bytes += __shfl_xor(c_bytes, off);
        }
        if (lane == 0) {
            atomicAdd(&a.counters->distance, c_eval);
            atomicAdd(&a.counters->bytes, c_bytes);
        }
    }
}

__global__ void __launch_bounds__(256) bf16_recheck_kernel(QArgs a, BfArgs bf) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    const uint32_t np = min(*bf.npairs, bf.pairs_cap);
    const int L = a.L;
    unsigned long long c_re = 0, c_bytes = 0;
    const uint32_t stride = gridDim.x * 16;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 4; base < np; base += stride) {
        const uint32_t pi = base + quarter;
        uint2 pr = make_uint2(0, 0);
        if (pi < np) pr = bf.pairs[pi];
        // a pair outside the call's queries or the collection is never followed
        const bool act = pi < np && pr.x < (uint32_t)a.nq && (int64_t)pr.y < a.n;
        if (!act) pr = make_uint2(0, 0);
        const uint32_t gidx = a.pos[pr.y];
        const float* x = a.series + (size_t)gidx * L;
        const float* qr = a.queries + (size_t)pr.x * L;
        float s = 0.f, c = 0.f;
        if (act) {
            for (int j = ql; j < L; j += 16) {
                const float d = __fsub_rn(qr[j], x[j]);
                neumaier_add(s, c, __fmul_rn(d, d));
            }
        }
        for (int off = 8; off >= 1; off >>= 1) {
            const float s2 = __shfl_xor(s, off, 16), c2 = __shfl_xor(c, off, 16);
            two_sum_merge(s, c, s2, c2);
        }
        float d = __fadd_rn(s, c);
        d = __shfl(d, quarter * 16, 64);
        if (act && ql == 0) {
            ++c_re;
            c_bytes += (uint64_t)L * 4;
            QState& st = a.qs[pr.x];
            const float U = __uint_as_float(vload(&st.U));
            if (d * (1.0f - kRhoEd) <= U) {
                const uint32_t slot = atomicAdd(&st.ncand, 1u);
                if (slot < a.cap) {
                    a.cand[(size_t)pr.x * a.cap + slot] = Cand{d, gidx};
                } else {
                    if (st.err == 0) st.err = 2;  // the final kernel raises the call's flag
                }
                if (st.k == 1) atomicMin(&st.U, __float_as_uint(d * (1.0f + 2.0f * kRhoEd)));
            }
        }
    }
    if (a.counters) {
        for (int off = 32; off >= 1; off >>= 1) {
            c_re += __shfl_xor(c_re, off);
            c_bytes += __shfl_xor(c_bytes, off);
        }
        if (lane == 0 && c_re) {
            atomicAdd(&a.counters->recheck, c_re);
            atomicAdd(&a.counters->bytes, c_bytes);
        }
    }
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t p;
            if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        }
    }
    return cus;
}

}  // namespace

// ---------------------------------------------------------------------------

int build_bf16_shadow(Index* ix, hipStream_t s) {
    const int Lp = (ix->len + 31) / 32 * 32;
    MESSI_TRY(ix->shadow.alloc(sizeof(uint16_t) * (size_t)ix->n * Lp));
    MESSI_TRY(ix->sx.alloc(sizeof(uint2) * (size_t)ix->n));
    hipEvent_t e0, e1;
    MESSI_HIP_TRY(hipEventCreate(&e0));
    MESSI_HIP_TRY(hipEventCreate(&e1));
    MESSI_HIP_TRY(hipEventRecord(e0, s));
    const int64_t waves = (ix->n + 3) / 4;
    const unsigned blocks = (unsigned)std::min<int64_t>(waves, (int64_t)device_cus() * 16);
    const BfConsts kc = bf_consts(Lp);
    hipLaunchKernelGGL(shadow_kernel, dim3(blocks), dim3(256), 0, s, ix->series, ix->pos.as<uint32_t>(), ix->n,
                       ix->len, Lp, 1.0 - kc.g, ix->shadow.as<uint16_t>(), ix->sx.as<uint2>());
    MESSI_LAUNCH_CHECK("shadow");
    MESSI_HIP_TRY(hipEventRecord(e1, s));
    MESSI_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    MESSI_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ix->info.ms_shadow = ms;
    return MESSI_OK;
}

void release_bf16(const Index* ix) { (void)ix; }

int bf16_row_prep(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s) {
    const int L = ix->len;
    const int Lp = (L + 31) / 32 * 32;
    const int nq = a.nq;
    if (ws->qb.bytes < sizeof(uint16_t) * (size_t)nq * Lp || ws->qnorm.bytes < sizeof(float2) * (size_t)nq ||
        ws->qx.bytes < sizeof(uint4) * (size_t)nq) {
        MESSI_TRY(growth_sync(s));
        ws->bf_nq = 0;  // the batched filter's buffers are sized again on its next call
        ++ws->gen;
        MESSI_TRY(ws->grow(ix, ws->qb, sizeof(uint16_t) * (size_t)nq * Lp));
        MESSI_TRY(ws->grow(ix, ws->qnorm, sizeof(float2) * (size_t)nq));
        MESSI_TRY(ws->grow(ix, ws->qx, sizeof(uint4) * (size_t)nq));
    }
    const BfConsts kc = bf_consts(Lp);
    a.shadow = ix->shadow.as<uint16_t>();
    a.sx = ix->sx.as<uint2>();
    a.qb = ws->qb.as<uint16_t>();
    a.qnorm = ws->qnorm.as<float2>();
    a.qx = ws->qx.as<uint4>();
    a.Lp = Lp;
    a.one_minus_h = std::nextafter((float)(1.0 - kc.h), 0.0f);
    hipLaunchKernelGGL(qprep_bf16_kernel, dim3(nq), dim3(256), 0, s, a.queries, L, Lp,
                       std::nextafter((float)kc.c1p, 1.0f), ws->qb.as<uint16_t>(), ws->qnorm.as<float2>(),
                       ws->qx.as<uint4>());
    MESSI_LAUNCH_CHECK("qprep_bf16");
    return MESSI_OK;
}

namespace {

// The filter's buffers in the workspace (for a.nq queries) and its arguments.
// FP32 filter instance for rows of L values: E = Lq / 4 floats per lane.
int f32_filter_e(int L) { return L <= 32 ? 8 : L <= 64 ? 16 : L <= 128 ? 32 : 64; }

const void* f32_filter_fn(int E) {
    switch (E) {
        case 8: return (const void*)f32_filter_kernel<8, 2>;
        case 16: return (const void*)f32_filter_kernel<16, 2>;
        case 32: return (const void*)f32_filter_kernel<32, 2>;
        default: return (const void*)f32_filter_kernel<64, 1>;
    }
}

int bf16_setup(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s, BfArgs& bf, size_t& filter_lds,
               bool f32 = false) {
    const int L = ix->len;
    const int Lp = (L + 31) / 32 * 32;
    const int nq = a.nq;
    const size_t nL = (size_t)ix->n_leaves;
    const size_t leafq_cap = (size_t)nq * nL;
    const size_t pairs_cap = bf16_pairs_cap(nq);
    if (ws->bf_nq < nq || ws->bf_pairs_cap < pairs_cap || ws->bf_leafq_cap < leafq_cap) {
        MESSI_TRY(growth_sync(s));
        // not valid until every buffer is in place (a failed allocation leaves its buffer empty)
        ws->bf_nq = 0;
        ws->bf_pairs_cap = ws->bf_leafq_cap = 0;
        ++ws->gen;
        MESSI_TRY(ws->grow(ix, ws->qb, sizeof(uint16_t) * (size_t)nq * Lp));
        MESSI_TRY(ws->grow(ix, ws->qnorm, sizeof(float2) * (size_t)nq));
        MESSI_TRY(ws->grow(ix, ws->qx, sizeof(uint4) * (size_t)nq));
        MESSI_TRY(ws->grow(ix, ws->leaf_cnt, sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->grow(ix, ws->leaf_off, sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->grow(ix, ws->leaf_cur, sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->grow(ix, ws->leaf_q, sizeof(uint32_t) * leafq_cap));
        MESSI_TRY(ws->grow(ix, ws->pairs, sizeof(uint2) * pairs_cap));
        MESSI_TRY(ws->grow(ix, ws->npairs, sizeof(uint32_t) * 8));
        MESSI_TRY(ws->grow(ix, ws->leaf_act, sizeof(uint32_t) * (nL + 1)));
        ws->bf_nq = nq;
        ++ws->gen;
        ws->bf_pairs_cap = pairs_cap;
        ws->bf_leafq_cap = leafq_cap;
    }
    const BfConsts kc = bf_consts(Lp);
    bf = BfArgs{};
    bf.Lp = Lp;
    bf.ksteps = Lp / 32;
    bf.shadow = ix->shadow.as<uint16_t>();
    bf.sx = ix->sx.as<uint2>();
    bf.qb = ws->qb.as<uint16_t>();
    bf.qnorm = ws->qnorm.as<float2>();
    bf.qx = ws->qx.as<uint4>();
    bf.leaf_cnt = ws->leaf_cnt.as<uint32_t>();
    bf.leaf_off = ws->leaf_off.as<uint32_t>();
    bf.leaf_q = ws->leaf_q.as<uint32_t>();
    bf.pairs = ws->pairs.as<uint2>();
    bf.npairs = ws->npairs.as<uint32_t>();
    bf.pairs_cap = (uint32_t)pairs_cap;
    bf.one_minus_h = std::nextafter((float)(1.0 - kc.h), 0.0f);
    bf.leaf_act = ws->leaf_act.as<uint32_t>();
    // queries staged per leaf: as many as the LDS of one block holds (at most 256)
    int lds_max = 65536;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device);
    const int E = f32_filter_e(L);
    // BF16: row, alpha, extra k-step, id; FP32: padded fp32 row, bound, |q|^2, id
    const size_t row_bytes = f32 ? (size_t)(4 * E + 4) * 4 + 12 : (size_t)(Lp + 8) * 2 + 24;
    int qc = (int)std::min<size_t>(256, (size_t)(lds_max - 1024) / row_bytes) / 16 * 16;
    if (qc < 16) qc = 16;
    bf.qc = qc;
    ws->bf_stage_queries = qc;
    filter_lds = (size_t)qc * row_bytes;
    if (f32) {
        const double u = std::ldexp(1.0, -23);
        bf.f32_c = (float)((4.0 * (L + 2) + 8.0) * u);
    }
    MESSI_HIP_TRY(hipFuncSetAttribute(f32 ? f32_filter_fn(E) : (const void*)bf16_filter_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)filter_lds));

    return MESSI_OK;
}

}  // namespace

bool f32_filter_ok(const Index* ix) {
    return ix->len % 4 == 0 && ix->len <= 256 && (uintptr_t)ix->series % 16 == 0;
}

int bf16_scan(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s, bool timing, bool f32, bool probe) {
    const int L = ix->len;
    const int Lp = (L + 31) / 32 * 32;
    const int nq = a.nq;
    const size_t nL = (size_t)ix->n_leaves;
    const size_t leafq_cap = (size_t)nq * nL;
    BfArgs bf;
    size_t filter_lds = 0;
    MESSI_TRY(bf16_setup(ix, a, ws, s, bf, filter_lds, f32));
    const BfConsts kc = bf_consts(Lp);
    hipLaunchKernelGGL(qprep_bf16_kernel, dim3(nq), dim3(256), 0, s, a.queries, L, Lp,
                       std::nextafter((float)kc.c1p, 1.0f), ws->qb.as<uint16_t>(), ws->qnorm.as<float2>(),
                       ws->qx.as<uint4>());
    MESSI_LAUNCH_CHECK("qprep_bf16");
    const int cus = device_cus();
    // events around the filter and recheck launches of every round (timing only)
    std::vector<hipEvent_t> evs;
    auto mark = [&]() -> int {
        if (!timing) return MESSI_OK;
        hipEvent_t e;
        MESSI_HIP_TRY(hipEventCreate(&e));
        MESSI_HIP_TRY(hipEventRecord(e, s));
        evs.push_back(e);
        return MESSI_OK;
    };
    int rounds_run = 0;
    // Rounds over ranges of each query's leaf order (kRoundEnds); after each
    // round every query's bound is refreshed from its candidates, so later
    // rounds are filtered tighter.
    uint64_t t1 = 0;
    // the FP32 filter: growing rounds for a wide batch (see kRoundEndsF32);
    // without probe (a launch that may be recorded in a graph: no waiting)
    // the batch counts as wide
    bool wide = f32;
    if (f32 && probe) {
        uint32_t* cnt = ws->npairs.as<uint32_t>() + 6;
        hipLaunchKernelGGL(word_clear_kernel, dim3(1), dim3(1), 0, s, cnt);
        MESSI_LAUNCH_CHECK("word_clear");
        hipLaunchKernelGGL(wide_count_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, a, cnt);
        MESSI_LAUNCH_CHECK("wide_count");
        MESSI_HIP_TRY(hipMemcpyAsync(ws->h_err + 1, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        wide = (uint64_t)ws->h_err[1] * 4 > (uint64_t)nq;
    }
    for (int round = 0; t1 < (uint64_t)nL; ++round) {
        const uint64_t t0 = t1;
        t1 = std::min<uint64_t>(wide ? kRoundEndsF32[std::min(round, 4)] : kRoundEnds[std::min(round, 2)], (uint64_t)nL);
        const unsigned tbr = (unsigned)((t1 - t0 + 255) / 256);
        const uint32_t r0 = (uint32_t)t0, r1 = (uint32_t)t1;
        hipLaunchKernelGGL(round_reset_kernel, dim3((unsigned)std::min<size_t>((nL + 255) / 256, 1024)), dim3(256), 0,
                           s, ws->leaf_cnt.as<uint32_t>(), (uint32_t)nL, ws->npairs.as<uint32_t>(), round == 0);
        MESSI_LAUNCH_CHECK("round_reset");
        hipLaunchKernelGGL(leaf_count_kernel, dim3(tbr, nq), dim3(256), 0, s, a, r0, r1, ws->leaf_cnt.as<uint32_t>(),
                           ws->leaf_act.as<uint32_t>(), ws->npairs.as<uint32_t>());
        MESSI_LAUNCH_CHECK("leaf_count");
        hipLaunchKernelGGL(leaf_offsets_kernel, dim3((unsigned)std::min<size_t>((nL + 255) / 256, 256)), dim3(256), 0,
                           s, ws->leaf_cnt.as<uint32_t>(), ws->leaf_act.as<uint32_t>(), ws->leaf_off.as<uint32_t>(),
                           ws->leaf_cur.as<uint32_t>(), ws->npairs.as<uint32_t>());
        MESSI_LAUNCH_CHECK("leaf_offsets");
        hipLaunchKernelGGL(leaf_scatter_kernel, dim3(tbr, nq), dim3(256), 0, s, a, r0, r1,
                           ws->leaf_off.as<uint32_t>(), ws->leaf_cur.as<uint32_t>(), ws->leaf_q.as<uint32_t>(),
                           leafq_cap);
        MESSI_LAUNCH_CHECK("leaf_scatter");
        MESSI_TRY(mark());
        if (f32) {
            switch (f32_filter_e(L)) {
                case 8: hipLaunchKernelGGL((f32_filter_kernel<8, 2>), dim3(cus), dim3(kFThreads), filter_lds, s, a, bf); break;
                case 16: hipLaunchKernelGGL((f32_filter_kernel<16, 2>), dim3(cus), dim3(kFThreads), filter_lds, s, a, bf); break;
                case 32: hipLaunchKernelGGL((f32_filter_kernel<32, 2>), dim3(cus), dim3(kFThreads), filter_lds, s, a, bf); break;
                default: hipLaunchKernelGGL((f32_filter_kernel<64, 1>), dim3(cus), dim3(kFThreads), filter_lds, s, a, bf); break;
            }
            MESSI_LAUNCH_CHECK("f32_filter");
        } else {
            hipLaunchKernelGGL(bf16_filter_kernel, dim3(cus), dim3(kFThreads), filter_lds, s, a, bf);
            MESSI_LAUNCH_CHECK("bf16_filter");
        }
        MESSI_TRY(mark());
        hipLaunchKernelGGL(bf16_recheck_kernel, dim3(cus * 8), dim3(256), 0, s, a, bf);
        MESSI_LAUNCH_CHECK("bf16_recheck");
        MESSI_TRY(mark());
        MESSI_TRY(refresh_bounds(a, s));
        ++rounds_run;
    }
    ws->bf_rounds = rounds_run;
    ws->bf_ms_filter = ws->bf_ms_recheck = 0;
    ws->bf_max_leaf_q = 0;
    if (timing) {
        uint32_t ctr[8];
        MESSI_HIP_TRY(hipMemcpyAsync(ctr, ws->npairs.p, sizeof(ctr), hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->bf_max_leaf_q = (int)ctr[4];
        for (size_t i = 0; i + 2 < evs.size(); i += 3) {
            float f = 0, r = 0;
            MESSI_HIP_TRY(hipEventElapsedTime(&f, evs[i], evs[i + 1]));
            MESSI_HIP_TRY(hipEventElapsedTime(&r, evs[i + 1], evs[i + 2]));
            ws->bf_ms_filter += f;
            ws->bf_ms_recheck += r;
        }
        for (auto e : evs) (void)hipEventDestroy(e);
    }
    return MESSI_OK;
}

// One filter round of the serving engine's slots: each slot in kSlotActive
// over its own window of its leaf order (a.win), the (query, leaf) pairs of
// all of them grouped by leaf as in a batch round.  The BF16 query rows are
// prepared for every slot (a slot admitted in this step among them).
int bf16_slot_round(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s) {
    const int L = ix->len;
    const int Lp = (L + 31) / 32 * 32;
    const int nq = a.nq;
    const size_t nL = (size_t)ix->n_leaves;
    BfArgs bf;
    size_t filter_lds = 0;
    MESSI_TRY(bf16_setup(ix, a, ws, s, bf, filter_lds));
    const BfConsts kc = bf_consts(Lp);
    hipLaunchKernelGGL(qprep_bf16_kernel, dim3(nq), dim3(256), 0, s, a.queries, L, Lp,
                       std::nextafter((float)kc.c1p, 1.0f), ws->qb.as<uint16_t>(), ws->qnorm.as<float2>(),
                       ws->qx.as<uint4>());
    MESSI_LAUNCH_CHECK("qprep_bf16");
    hipLaunchKernelGGL(round_reset_kernel, dim3((unsigned)std::min<size_t>((nL + 255) / 256, 1024)), dim3(256), 0, s,
                       ws->leaf_cnt.as<uint32_t>(), (uint32_t)nL, ws->npairs.as<uint32_t>(), 1);
    MESSI_LAUNCH_CHECK("round_reset");
    // 16 blocks per slot stride over its window
    hipLaunchKernelGGL(leaf_count_kernel, dim3(16, nq), dim3(256), 0, s, a, 0u, 0u, ws->leaf_cnt.as<uint32_t>(),
                       ws->leaf_act.as<uint32_t>(), ws->npairs.as<uint32_t>());
    MESSI_LAUNCH_CHECK("leaf_count");
    hipLaunchKernelGGL(leaf_offsets_kernel, dim3((unsigned)std::min<size_t>((nL + 255) / 256, 256)), dim3(256), 0, s,
                       ws->leaf_cnt.as<uint32_t>(), ws->leaf_act.as<uint32_t>(), ws->leaf_off.as<uint32_t>(),
                       ws->leaf_cur.as<uint32_t>(), ws->npairs.as<uint32_t>());
    MESSI_LAUNCH_CHECK("leaf_offsets");
    hipLaunchKernelGGL(leaf_scatter_kernel, dim3(16, nq), dim3(256), 0, s, a, 0u, 0u, ws->leaf_off.as<uint32_t>(),
                       ws->leaf_cur.as<uint32_t>(), ws->leaf_q.as<uint32_t>(), (size_t)nq * nL);
    MESSI_LAUNCH_CHECK("leaf_scatter");
    const int cus = device_cus();
    hipLaunchKernelGGL(bf16_filter_kernel, dim3(cus), dim3(kFThreads), filter_lds, s, a, bf);
    MESSI_LAUNCH_CHECK("bf16_filter");
    hipLaunchKernelGGL(bf16_recheck_kernel, dim3(cus * 8), dim3(256), 0, s, a, bf);
    MESSI_LAUNCH_CHECK("bf16_recheck");
    return MESSI_OK;
}

}  // namespace messi

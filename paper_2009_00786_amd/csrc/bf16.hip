// Batched BF16 filter on the matrix cores, with a rounding bound that keeps the
// search exact, then a compensated fp32 recheck of the survivors.
//
// For a batch of queries, the (query, leaf) pairs that survive the leaf bound
// are grouped by leaf.  A wave holds the BF16 rows of 16 members of a leaf in
// registers (the B operand) and streams 16-query tiles of the leaf's queries
// from LDS (the A operand) through mfma_f32_16x16x32_bf16, so a member row is
// read from HBM once per leaf whatever the number of queries that visit it.
// For every (query q, member x) it forms
//     f = fl(fl(|q|^2 + |x|^2) - 2 s),   s = sum_j bf16(q_j) bf16(x_j) (fp32 accumulation)
// and discards x for q only if f - E(q, x) > U_q, where E bounds |f - D| for the
// exact squared distance D = |q - x|^2:
//   - operand rounding to BF16 (unit roundoff u_b = 2^-8):
//       |sum bf16(q_j) bf16(x_j) - q.x| <= (2 u_b + u_b^2) |q| |x|   (Cauchy-Schwarz)
//   - fp32 accumulation of L exact products in any order, u = 2^-23 so that
//     non-nearest or unknown rounding inside the unit is covered:
//       <= gamma_{L-1} (1 + u_b)^2 |q| |x|,   gamma_n = n u / (1 - n u)
//   - the squared norms are fp32 roundings of fp64 sums (u32 = 2^-24 each), and
//     the final add and subtract round once each:
//       <= 3 u32 (|q|^2 + |x|^2) + 2 u32 (|q| + |x|)^2
//   so E = (4 u_b + 2 u_b^2 + 2 gamma_{L-1} (1 + u_b)^2) |q||x| + 3 u32 (|q|^2 + |x|^2)
//          + 2 u32 (|q| + |x|)^2, evaluated in fp32 and scaled by (1 + 2^-20).
// A discarded member has D >= f - E > U_q >= the k-th true distance, so it is
// not an answer.  Survivors get a Neumaier-compensated fp32 distance (relative
// error ~3 u32), which feeds the same candidate/bound logic as the fp32 scan;
// the final order uses the canonical fp64 distance.
#include <algorithm>
#include <cmath>
#include <vector>

#include "query.h"
#include "scan.h"

namespace messi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kKS = 8;             // K-steps of 32 held in registers (rows up to 256)
constexpr uint32_t kFirstRound = 8;  // leaf positions per query in the first round

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t vload(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

// ---------------------------------------------------------------------------
// build: BF16 rows in leaf order (zero-padded to a multiple of 32) and the
// fp32 squared norm and norm of every member, from fp64 sums.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) shadow_kernel(const float* __restrict__ series, const uint32_t* __restrict__ pos,
                                                     int64_t n, int L, int Lp, uint16_t* __restrict__ shadow,
                                                     float2* __restrict__ norms) {
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
        if (lane == 0) norms[j] = make_float2((float)acc, (float)sqrt(acc));
    }
}

// ---------------------------------------------------------------------------
// query side
// ---------------------------------------------------------------------------
struct BfArgs {
    int32_t Lp, ksteps;
    const uint16_t* shadow;
    const float2* norms;
    const uint16_t* qb;     // [nq][Lp] bf16 queries
    const float2* qnorm;    // [nq] (|q|^2, |q|)
    const uint32_t* leaf_cnt;
    const uint32_t* leaf_off;
    const uint32_t* leaf_q;
    uint2* pairs;           // (query, member position)
    uint32_t* npairs;
    uint32_t pairs_cap;
    float c1;               // coefficient of |q||x| in E (rounded up)
};

__global__ void __launch_bounds__(256) qprep_bf16_kernel(const float* __restrict__ queries, int L, int Lp,
                                                         uint16_t* __restrict__ qb, float2* __restrict__ qnorm) {
    __shared__ double s_part[4];
    const int q = blockIdx.x;
    const float* row = queries + (size_t)q * L;
    double acc = 0.0;
    for (int e = threadIdx.x; e < Lp; e += 256) {
        const float v = (e < L) ? row[e] : 0.f;
        acc += (double)v * (double)v;
        qb[(size_t)q * Lp + e] = bf16_rne(v);
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        qnorm[q] = make_float2((float)t, (float)sqrt(t));
    }
}

// Positions [t0, t1) of every query's leaf order whose bound does not exceed
// the query's current U take part in a round.
__device__ __forceinline__ bool round_leaf(const QArgs& a, int q, uint32_t t, uint32_t t1, uint32_t& leaf) {
    const QState& st = a.qs[q];
    if (t >= t1 || t >= st.nsurv || st.err) return false;
    leaf = a.order[(size_t)q * a.nL + t];
    const float U = __uint_as_float(vload(&st.U));
    return !(a.lb[(size_t)q * a.nL + leaf] * (1.0f - kRhoLb) > U);
}

__global__ void __launch_bounds__(256) leaf_count_kernel(QArgs a, uint32_t t0, uint32_t t1,
                                                         uint32_t* __restrict__ leaf_cnt) {
    const int q = blockIdx.y;
    const uint32_t t = t0 + blockIdx.x * 256 + threadIdx.x;
    uint32_t leaf;
    if (round_leaf(a, q, t, t1, leaf)) atomicAdd(&leaf_cnt[leaf], 1u);
}

__global__ void __launch_bounds__(256) leaf_scatter_kernel(QArgs a, uint32_t t0, uint32_t t1,
                                                           const uint32_t* __restrict__ leaf_off,
                                                           uint32_t* __restrict__ leaf_cur,
                                                           uint32_t* __restrict__ leaf_q, size_t leafq_cap) {
    const int q = blockIdx.y;
    const uint32_t t = t0 + blockIdx.x * 256 + threadIdx.x;
    uint32_t leaf;
    if (round_leaf(a, q, t, t1, leaf)) {
        const size_t at = (size_t)leaf_off[leaf] + atomicAdd(&leaf_cur[leaf], 1u);
        if (at < leafq_cap) leaf_q[at] = (uint32_t)q;
    }
}

// One block per leaf at a time (persistent, static stride over leaves); wave w
// owns members w*16 .. w*16+15 of every 64-member tile of the leaf.
__global__ void __launch_bounds__(256) bf16_filter_kernel(QArgs a, BfArgs bf) {
    constexpr int kMaxLp = MESSI_MAX_LEN;
    __shared__ uint16_t s_a[16 * (kMaxLp + 8)];
    __shared__ float s_U[16], s_nq[16], s_rq[16];
    __shared__ uint32_t s_qid[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kb = lane >> 4;
    const int Lp = bf.Lp, ks = bf.ksteps, lda = Lp + 8;
    const bool resident = ks <= kKS;
    const float u32 = 5.9604644775390625e-08f;
    unsigned long long c_eval = 0, c_pass = 0, c_bytes = 0;
    for (int leaf = blockIdx.x; leaf < a.nL; leaf += gridDim.x) {
        const uint32_t cntq = bf.leaf_cnt[leaf];
        if (cntq == 0) continue;
        const Leaf lf = a.leaves[leaf];
        const uint32_t qoff = bf.leaf_off[leaf];
        for (uint32_t mt0 = 0; mt0 < lf.count; mt0 += 64) {
            const uint32_t mi = mt0 + wave * 16 + col;
            const bool mvalid = mi < lf.count;
            const uint32_t mpos = lf.start + (mvalid ? mi : 0u);
            const uint16_t* brow = bf.shadow + (size_t)mpos * Lp;
            bf16x8 bfrag[kKS];
            if (resident) {
#pragma unroll
                for (int st = 0; st < kKS; ++st) {
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (st < ks && mvalid) v = *reinterpret_cast<const uint4*>(brow + 32 * st + 8 * kb);
                    bfrag[st] = __builtin_bit_cast(bf16x8, v);
                }
            }
            const float2 xn = mvalid ? bf.norms[mpos] : make_float2(0.f, 0.f);
            if (mvalid && kb == 0) c_bytes += (uint64_t)Lp * 2 + 8;
            for (uint32_t qt0 = 0; qt0 < cntq; qt0 += 16) {
                __syncthreads();  // previous tile's readers are done
                const int chunks = Lp / 8;  // 16-byte chunks per row
                for (int idx = tid; idx < 16 * chunks; idx += 256) {
                    const int r = idx / chunks, c = idx % chunks;
                    const uint32_t qi = qt0 + r;
                    uint4 v = make_uint4(0, 0, 0, 0);
                    if (qi < cntq) {
                        const uint32_t q = bf.leaf_q[qoff + qi];
                        v = *reinterpret_cast<const uint4*>(bf.qb + (size_t)q * Lp + 8 * c);
                    }
                    *reinterpret_cast<uint4*>(&s_a[r * lda + 8 * c]) = v;
                }
                if (tid < 16) {
                    const uint32_t qi = qt0 + tid;
                    if (qi < cntq) {
                        const uint32_t q = bf.leaf_q[qoff + qi];
                        const float2 qn = bf.qnorm[q];
                        s_qid[tid] = q;
                        s_nq[tid] = qn.x;
                        s_rq[tid] = qn.y;
                        s_U[tid] = __uint_as_float(vload(&a.qs[q].U));
                    } else {
                        s_qid[tid] = 0xffffffffu;
                    }
                }
                __syncthreads();
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                if (resident) {
#pragma unroll
                    for (int st = 0; st < kKS; ++st) {
                        if (st < ks) {
                            const bf16x8 af =
                                __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&s_a[col * lda + 32 * st + 8 * kb]));
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfrag[st], acc, 0, 0, 0);
                        }
                    }
                } else {
                    for (int s0 = 0; s0 < ks; s0 += kKS) {
#pragma unroll
                        for (int st = 0; st < kKS; ++st) {
                            uint4 v = make_uint4(0, 0, 0, 0);
                            if (s0 + st < ks && mvalid) v = *reinterpret_cast<const uint4*>(brow + 32 * (s0 + st) + 8 * kb);
                            bfrag[st] = __builtin_bit_cast(bf16x8, v);
                        }
#pragma unroll
                        for (int st = 0; st < kKS; ++st) {
                            if (s0 + st < ks) {
                                const bf16x8 af = __builtin_bit_cast(
                                    bf16x8, *reinterpret_cast<const uint4*>(&s_a[col * lda + 32 * (s0 + st) + 8 * kb]));
                                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfrag[st], acc, 0, 0, 0);
                            }
                        }
                    }
                }
                // acc[i] = s for query row 4 kb + i and member col
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 4 * kb + i;
                    const uint32_t q = s_qid[r];
                    if (q != 0xffffffffu && mvalid) {
                        ++c_eval;
                        const float nq = s_nq[r], rq = s_rq[r];
                        const float f = __fsub_rn(__fadd_rn(nq, xn.x), __fmul_rn(2.0f, acc[i]));
                        const float rs = __fadd_rn(rq, xn.y);
                        const float E = (bf.c1 * (rq * xn.y) + 3.0f * u32 * (nq + xn.x) + 2.0f * u32 * (rs * rs)) *
                                        (1.0f + 9.5367431640625e-07f);
                        const float margin = __fsub_rn(f, E);
                        if (!(margin * (1.0f - 2.384185791015625e-07f) > s_U[r])) {
                            const uint32_t slot = atomicAdd(bf.npairs, 1u);
                            if (slot < bf.pairs_cap) {
                                bf.pairs[slot] = make_uint2(q, mpos);
                            } else {
                                // this query lost a pair: its answer is redone by the fp32 path
                                a.qs[q].err = 5;
                                atomicOr(a.err_any, 16u);
                            }
                            ++c_pass;
                        }
                    }
                }
            }
        }
    }
    if (a.counters) {
        for (int off = 32; off >= 1; off >>= 1) {
            c_eval += __shfl_xor(c_eval, off);
            c_pass += __shfl_xor(c_pass, off);
            c_bytes += __shfl_xor(c_bytes, off);
        }
        if (lane == 0) {
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
__global__ void __launch_bounds__(256) bf16_recheck_kernel(QArgs a, BfArgs bf) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    const uint32_t np = min(*bf.npairs, bf.pairs_cap);
    const int L = a.L;
    unsigned long long c_re = 0, c_bytes = 0;
    const uint32_t stride = gridDim.x * 16;
    for (uint32_t base = (blockIdx.x * 4 + wave) * 4; base < np; base += stride) {
        const uint32_t pi = base + quarter;
        const bool act = pi < np;
        uint2 pr = make_uint2(0, 0);
        if (act) pr = bf.pairs[pi];
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
                    st.err = 2;
                    atomicOr(a.err_any, 2u);
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
        if (lane == 0) {
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
    MESSI_TRY(ix->norms.alloc(sizeof(float2) * (size_t)ix->n));
    hipEvent_t e0, e1;
    MESSI_HIP_TRY(hipEventCreate(&e0));
    MESSI_HIP_TRY(hipEventCreate(&e1));
    MESSI_HIP_TRY(hipEventRecord(e0, s));
    const int64_t waves = (ix->n + 3) / 4;
    const unsigned blocks = (unsigned)std::min<int64_t>(waves, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(shadow_kernel, dim3(blocks), dim3(256), 0, s, ix->series, ix->pos.as<uint32_t>(), ix->n,
                       ix->len, Lp, ix->shadow.as<uint16_t>(), ix->norms.as<float2>());
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

int bf16_scan(const Index* ix, QArgs& a, Workspace* ws, hipStream_t s, bool timing) {
    const int L = ix->len;
    const int Lp = (L + 31) / 32 * 32;
    const int nq = a.nq;
    const size_t nL = (size_t)ix->n_leaves;
    const size_t leafq_cap = (size_t)nq * nL;
    const size_t pairs_cap = std::min<size_t>((size_t)nq * 16384, (size_t)1 << 28);
    if (ws->bf_nq < nq || ws->bf_pairs_cap < pairs_cap || ws->bf_leafq_cap < leafq_cap) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        MESSI_TRY(ws->qb.alloc(sizeof(uint16_t) * (size_t)nq * Lp));
        MESSI_TRY(ws->qnorm.alloc(sizeof(float2) * (size_t)nq));
        MESSI_TRY(ws->leaf_cnt.alloc(sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->leaf_off.alloc(sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->leaf_cur.alloc(sizeof(uint32_t) * (nL + 1)));
        MESSI_TRY(ws->leaf_q.alloc(sizeof(uint32_t) * leafq_cap));
        MESSI_TRY(ws->pairs.alloc(sizeof(uint2) * pairs_cap));
        MESSI_TRY(ws->npairs.alloc(sizeof(uint32_t) * 4));
        MESSI_TRY(ws->scan_scr.alloc(sizeof(uint32_t) * scan_scratch_words((int64_t)nL + 1)));
        ws->bf_nq = nq;
        ws->bf_pairs_cap = pairs_cap;
        ws->bf_leafq_cap = leafq_cap;
    }
    // coefficient of |q||x| in the bound, rounded up
    const double ub = std::ldexp(1.0, -8), u = std::ldexp(1.0, -23);
    const double nu = (double)(Lp - 1) * u;
    const double gamma = nu / (1.0 - nu);
    const double c1 = 4.0 * ub + 2.0 * ub * ub + 2.0 * gamma * (1.0 + ub) * (1.0 + ub);
    BfArgs bf{};
    bf.Lp = Lp;
    bf.ksteps = Lp / 32;
    bf.shadow = ix->shadow.as<uint16_t>();
    bf.norms = ix->norms.as<float2>();
    bf.qb = ws->qb.as<uint16_t>();
    bf.qnorm = ws->qnorm.as<float2>();
    bf.leaf_cnt = ws->leaf_cnt.as<uint32_t>();
    bf.leaf_off = ws->leaf_off.as<uint32_t>();
    bf.leaf_q = ws->leaf_q.as<uint32_t>();
    bf.pairs = ws->pairs.as<uint2>();
    bf.npairs = ws->npairs.as<uint32_t>();
    bf.pairs_cap = (uint32_t)pairs_cap;
    bf.c1 = (float)(c1 * (1.0 + 1e-6));

    hipLaunchKernelGGL(qprep_bf16_kernel, dim3(nq), dim3(256), 0, s, a.queries, L, Lp, ws->qb.as<uint16_t>(),
                       ws->qnorm.as<float2>());
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
    // Rounds over geometrically growing ranges of each query's leaf order
    // (8, 64, 512, ... positions); after each round every query's bound is
    // refreshed from its candidates, so later rounds are filtered tighter.
    for (uint64_t t0 = 0, t1 = kFirstRound; t0 < (uint64_t)nL; t0 = t1, t1 = t1 * 8u) {
        if (t1 > (uint64_t)nL) t1 = (uint64_t)nL;
        const unsigned tbr = (unsigned)((t1 - t0 + 255) / 256);
        const uint32_t r0 = (uint32_t)t0, r1 = (uint32_t)t1;
        MESSI_HIP_TRY(hipMemsetAsync(ws->leaf_cnt.p, 0, sizeof(uint32_t) * (nL + 1), s));
        MESSI_HIP_TRY(hipMemsetAsync(ws->leaf_cur.p, 0, sizeof(uint32_t) * (nL + 1), s));
        MESSI_HIP_TRY(hipMemsetAsync(ws->npairs.p, 0, sizeof(uint32_t) * 4, s));
        hipLaunchKernelGGL(leaf_count_kernel, dim3(tbr, nq), dim3(256), 0, s, a, r0, r1, ws->leaf_cnt.as<uint32_t>());
        MESSI_LAUNCH_CHECK("leaf_count");
        MESSI_TRY(scan_exclusive(ws->leaf_cnt.as<uint32_t>(), ws->leaf_off.as<uint32_t>(), (int64_t)nL,
                                 ws->scan_scr.as<uint32_t>(), nullptr, s));
        hipLaunchKernelGGL(leaf_scatter_kernel, dim3(tbr, nq), dim3(256), 0, s, a, r0, r1,
                           ws->leaf_off.as<uint32_t>(), ws->leaf_cur.as<uint32_t>(), ws->leaf_q.as<uint32_t>(),
                           leafq_cap);
        MESSI_LAUNCH_CHECK("leaf_scatter");
        MESSI_TRY(mark());
        hipLaunchKernelGGL(bf16_filter_kernel, dim3(cus * 4), dim3(256), 0, s, a, bf);
        MESSI_LAUNCH_CHECK("bf16_filter");
        MESSI_TRY(mark());
        hipLaunchKernelGGL(bf16_recheck_kernel, dim3(cus * 8), dim3(256), 0, s, a, bf);
        MESSI_LAUNCH_CHECK("bf16_recheck");
        MESSI_TRY(mark());
        MESSI_TRY(refresh_bounds(a, s));
        ++rounds_run;
    }
    ws->bf_rounds = rounds_run;
    ws->bf_ms_filter = ws->bf_ms_recheck = 0;
    if (timing) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
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

}  // namespace messi

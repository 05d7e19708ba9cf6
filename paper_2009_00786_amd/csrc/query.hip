// Exact k-NN search on gfx950 (paper: Query Answering -- ExactSearch, approxSearch,
// SearchWorker, TraverseRootSubtree, ProcessQueue, CalculateRealDistance),
// re-planned for a GPU:
//
//  prep        query PAA, norm, region widening, state reset          (1 block / query)
//  leaf_lb     lower bound of every leaf against the query PAA, from per-segment
//              tables in LDS; the argmin leaf is the approximate-search leaf
//  approx      squared distances to that leaf's members -> first upper bound U
//              on the k-th distance (the paper's initial BSF)
//  order       the leaves whose bound does not exceed U, counting-sorted into
//              1024 bound bins: the ascending order the priority queues deliver
//  scan        the members of the ordered leaves, as one list cut into chunks
//              of 1024, are shared out evenly over the query's blocks (block j
//              takes chunks j, j + G, ...), so the grid advances through the
//              order together; a leaf whose bound exceeds the current U is
//              skipped and, once a chunk starts in a bin wholly above U, the
//              block stops; inside a leaf each member's own word gives a
//              second bound (LDS table lookups) and only the survivors' rows
//              are read, 16 lanes per row, abandoning a distance as soon as
//              its partial sum exceeds U; U lives in device memory (atomicMin
//              for k = 1; for k > 1 from a histogram of candidate distances)
//  fixup       k > 1: U from the exact k-th candidate, candidates compacted;
//              if the candidate buffer overflowed, its k-th becomes U and the
//              scan runs once more from that bound
//  final       candidates within the final U get the canonical fp64 distance and
//              are ordered by (distance, index); the first k are the answer
//
// Exactness: every prune compares a quantity that is provably below the true
// squared distance with an upper bound on the k-th true squared distance.
//  * Regions are widened by delta = 2 (lg m + 1) 2^-24 A_data + 2 (m + 1) 2^-24 A_q,
//    which covers the fp32 PAA error of both the data words (fold-halving sums)
//    and the query (sequential sums), so the bound stays below the exact
//    distance (Keogh's PAA bound + containment of the exact segment mean).
//  * fp32 distances d have relative error below 2^-16 (at most a few dozen
//    roundings of non-negative terms), so U = up(d_k (1 + 2^-15)) exceeds the
//    true k-th distance; a candidate is kept iff d (1 - 2^-16) <= U, a partial
//    sum abandons iff p (1 - 2^-16) > U, a bound prunes iff b (1 - 2^-12) > U.
//  * The final order uses the canonical fp64 distance, so the returned indices
//    are those of the brute-force definition whatever the visiting order.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "query.h"
#include "scan.h"

namespace messi {
namespace {

constexpr int kScanThreads = 256;
// scan variants: Euclidean; Euclidean with the BF16 row filter; LB_Keogh for DTW
constexpr int kScanEd = 0, kScanRowFilter = 1, kScanDtw = 2;
constexpr int kEdBatch = 32;  // survivors gathered before a round of distances
// the row filter runs while U > kRowFilterTau |q|^2 (about twice its rounding
// bound for |x| = |q|)
constexpr float kRowFilterTau = 0.03f;

__device__ __forceinline__ uint32_t vload(const uint32_t* p) {
    return __atomic_load_n(p, __ATOMIC_RELAXED);
}

__device__ __forceinline__ float upper_u(float d) { return d * (1.0f + 2.0f * kRhoEd); }

// --------------------------------------------------------------------------
// leaf bounds (with the query summary folded in)
// --------------------------------------------------------------------------
constexpr int kLeafBlock = 256;  // leaves per block of the bound kernels

// Query summary, computed by every block that needs it: PAA (sequential
// fp32 sums of each segment, one division), squared norm, largest |value|,
// finiteness, and the region widening delta.  The bounds take per segment an
// interval [plo, phi] of the query side: the PAA value for ED; under DTW the
// smallest and largest value of the query's LB_Keogh envelope over the
// segment (exact: minima and maxima of query values).  The intervals stay in
// LDS (s_red[8 + i] and s_red[24 + i]): indexed by a run-time segment, a
// register copy would live in scratch memory.
struct QSum {
    float norm2, amax, delta;
    bool bad;
};

__device__ void query_summary(const QArgs& a, const float* row, float* s_q, float* s_red, int* s_bad, QSum& out) {
    if (threadIdx.x == 0) *s_bad = 0;
    __syncthreads();
    float n2 = 0.f, amax = 0.f;
    bool bad = false;
    for (int j = threadIdx.x; j < a.L; j += 256) {
        const float v = row[j];
        s_q[j] = v;
        bad |= !isfinite(v);
        n2 = fmaf(v, v, n2);
        amax = fmaxf(amax, fabsf(v));
    }
    if (bad) *s_bad = 1;
    n2 = dev::wave_sum(n2);
    amax = dev::wave_max(amax);
    if ((threadIdx.x & 63) == 0) {
        s_red[threadIdx.x >> 6] = n2;
        s_red[4 + (threadIdx.x >> 6)] = amax;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        const int i = threadIdx.x;
        float lo = 0.f, hi = 0.f;
        if (i < a.w && a.band < 0) {
            float s = 0.f;
            for (int j = 0; j < a.m; ++j) s += s_q[i * a.m + j];
            lo = hi = s / (float)a.m;
        } else if (i < a.w) {
            // the envelope over segment i: every query value within band of it
            const int t0 = max(0, i * a.m - a.band), t1 = min(a.L - 1, (i + 1) * a.m - 1 + a.band);
            lo = hi = s_q[t0];
            for (int t = t0 + 1; t <= t1; ++t) {
                lo = fminf(lo, s_q[t]);
                hi = fmaxf(hi, s_q[t]);
            }
        }
        s_red[8 + i] = lo;
        s_red[24 + i] = hi;
    }
    __syncthreads();
    out.norm2 = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    out.amax = fmaxf(fmaxf(s_red[4], s_red[5]), fmaxf(s_red[6], s_red[7]));
    const float u = 5.9604644775390625e-08f;  // 2^-24
    out.delta = 1.01f * (2.f * (float)(a.lg_m + 1) * u * a.absmax_data + 2.f * (float)(a.m + 1) * u * out.amax);
    out.bad = *s_bad != 0;
}

// Every leaf's lower bound against the query PAA, from per-segment tables in
// LDS; each block also leaves its smallest and largest bound for the next
// kernel.  Block 0 of each query initialises the query's search state (and
// block 0 of query 0 the call's error flags and counters).
__global__ void __launch_bounds__(256) leaf_lb_kernel(QArgs a, int32_t k, const int32_t* __restrict__ kq,
                                                      uint32_t kstride) {
    __shared__ float s_lo[16 * 257];
    __shared__ float s_hi[16 * 257];
    __shared__ float s_q[MESSI_MAX_LEN];
    __shared__ float s_red[40];
    __shared__ int s_bad;
    __shared__ unsigned long long s_min[4];
    __shared__ uint32_t s_max[4];
    __shared__ float s_bp[256];
    const int q = blockIdx.y;
    if (slot_off(a, q, kSlotAdmit)) return;
    const int A = 1 << a.b;
    // this thread's first leaf, in flight while the query summary is formed
    const int l0 = blockIdx.x * kLeafBlock + threadIdx.x;
    Leaf lf0{};
    if (l0 < a.nL) lf0 = a.leaves[l0];
    if (threadIdx.x < A - 1) s_bp[threadIdx.x] = a.bp[threadIdx.x];
    QSum qs;
    query_summary(a, a.queries + (size_t)q * a.L, s_q, s_red, &s_bad, qs);
    if (blockIdx.x == 0) {
        QState& st = a.qs[q];
        if (threadIdx.x < 16) {
            st.paa[threadIdx.x] = s_red[8 + threadIdx.x];
            st.paa_hi[threadIdx.x] = s_red[24 + threadIdx.x];
        }
        if (threadIdx.x == 0) {
            st.norm2 = qs.norm2;
            st.delta = qs.delta;
            st.qamax = qs.amax;
            st.skip_start = 0xffffffffu;
            st.U = 0x7f800000u;  // +inf until the first bound
            st.ncand = 0;
            st.nmemb = 0;
            st.nsurv = 0;
            st.ovf = 0;
            st.rerun = 0;
            st.hbase = 0;
            st.lbmax = 0;
            st.argmin = ~0ull;
            st.range = 0.f;
            st.k = kq ? kq[q] : k;
            st.err = qs.bad ? 1u : 0u;
            st.active = 1;
            st.kstride = kstride;
            if (q == 0) {
                for (int i = 0; i < 4; ++i) a.err_any[i] = 0;
                if (a.counters) *a.counters = QCounters{};
            }
        }
        for (int i = threadIdx.x; i < kNB; i += 256) {
            a.bins[(size_t)q * kNB + i] = 0;
            a.mbins[(size_t)q * kNB + i] = 0;
            a.cursor[(size_t)q * kNB + i] = 0;
        }
        for (int i = threadIdx.x; i < kHistBins; i += 256) a.hist[(size_t)q * kHistBins + i] = 0;
    }
    for (int i = 0; i < a.w; ++i) {
        const float pl = s_red[8 + i], ph = s_red[24 + i];
        for (int c = threadIdx.x; c <= A; c += 256) {
            float tl = 0.f, th = 0.f;
            if (c > 0 && c < A) {
                const float lo = s_bp[c - 1] - qs.delta;
                const float hi = s_bp[c - 1] + qs.delta;
                if (ph < lo) tl = (lo - ph) * (lo - ph);
                if (pl > hi) th = (pl - hi) * (pl - hi);
            }
            s_lo[i * 257 + c] = tl;
            s_hi[i * 257 + c] = th;
        }
    }
    __syncthreads();
    unsigned long long best = ~0ull;
    uint32_t mx = 0;
    const float mf = (float)a.m;
    auto bound = [&](const Leaf& lf, int l) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < a.w) {
                const int sh = a.b - lf.card[i];
                const int lo = (int)lf.prefix[i] << sh;
                const int hi = ((int)lf.prefix[i] + 1) << sh;
                s += s_lo[i * 257 + lo] + s_hi[i * 257 + hi];
            }
        }
        const float lbv = s * mf;
        a.lb[(size_t)q * a.nL + l] = lbv;
        const unsigned long long key = ((unsigned long long)__float_as_uint(lbv) << 32) | (uint32_t)l;
        best = key < best ? key : best;
        mx = max(mx, __float_as_uint(lbv));
    };
    // leaves blockIdx.x * 256 + threadIdx.x, stepping over the query's blocks
    if (l0 < a.nL) bound(lf0, l0);
    for (int l = l0 + gridDim.x * kLeafBlock; l < a.nL; l += gridDim.x * kLeafBlock) {
        const Leaf lf = a.leaves[l];  // a register copy (a reference would read every byte from memory)
        bound(lf, l);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        s_min[threadIdx.x >> 6] = best;
        s_max[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b0 = s_min[0];
        uint32_t m0 = s_max[0];
        for (int w = 1; w < 4; ++w) {
            b0 = s_min[w] < b0 ? s_min[w] : b0;
            m0 = max(m0, s_max[w]);
        }
        a.lbpart[(size_t)q * gridDim.x + blockIdx.x] = LbPart{b0, m0, 0u};
    }
}

// --------------------------------------------------------------------------
// approximate search: distances to the members of the smallest-bound leaf
// --------------------------------------------------------------------------
// The members evaluated: the argmin leaf, extended into the depth-first
// neighbouring leaves (contiguous in the member arrays) until at least k
// members, so that the first bound is finite.  The exact search extends it
// to at least a.approx_min members: the neighbouring leaves share most of
// the word, and a few more rows give a tighter first bound, so fewer leaves
// are scanned (2048 members: 2% more queries/s at 100M x 256).
__device__ __forceinline__ void approx_range(const QArgs& a, uint32_t leaf, int32_t k, uint32_t& r0,
                                             uint32_t& cnt) {
    const Leaf lf = a.leaves[leaf];
    cnt = min(max(lf.count, max((uint32_t)k, a.approx_min)), (uint32_t)kApproxMax);
    cnt = (uint32_t)min((int64_t)cnt, a.n);
    r0 = (uint32_t)min((int64_t)lf.start, a.n - (int64_t)cnt);
}

// k-th smallest (1-based) of n non-negative floats by a 4-pass radix select
// (block of 256 threads).  Returns +inf when n < k.
template <class Getter>
__device__ float block_kth(Getter get, uint32_t n, uint32_t k, uint32_t* s_hist, uint32_t* s_bcast) {
    if (n < k) return __uint_as_float(0x7f800000u);
    if (k == 1) {
        // the smallest key: one block reduction instead of four passes
        uint32_t m = 0xffffffffu;
        for (uint32_t i = threadIdx.x; i < n; i += 256) m = min(m, __float_as_uint(get(i)));
        for (int off = 32; off >= 1; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
        if ((threadIdx.x & 63) == 0) s_hist[threadIdx.x >> 6] = m;
        __syncthreads();
        m = min(min(s_hist[0], s_hist[1]), min(s_hist[2], s_hist[3]));
        __syncthreads();
        return __uint_as_float(m);
    }
    uint32_t prefix = 0, mask = 0, kk = k;
    for (int pass = 3; pass >= 0; --pass) {
        const int shift = 8 * pass;
        s_hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += 256) {
            const uint32_t key = __float_as_uint(get(i));
            if ((key & mask) == prefix) atomicAdd(&s_hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        {
            // the digit whose inclusive running count first reaches kk
            const uint32_t c = s_hist[threadIdx.x];
            uint32_t x = c;
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            __syncthreads();
            if (lane == 63) s_hist[256 + wave] = x;  // wave totals after the counts
            __syncthreads();
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += s_hist[256 + w];
            const uint32_t incl = before + x, excl = incl - c;
            if (excl < kk && incl >= kk) {
                s_bcast[0] = threadIdx.x;
                s_bcast[1] = kk - excl;
            }
        }
        __syncthreads();
        prefix |= s_bcast[0] << shift;
        mask |= 255u << shift;
        kk = s_bcast[1];
        __syncthreads();
    }
    return __uint_as_float(prefix);
}

// The smallest and largest leaf bound, from the leaf-bound kernel's per-block
// partials (every thread of the block gets both).
__device__ void lb_extremes(const QArgs& a, int q, uint32_t nlb, unsigned long long* s_min, uint32_t* s_max,
                            unsigned long long& best, uint32_t& mx) {
    best = ~0ull;
    mx = 0;
    for (uint32_t i = threadIdx.x; i < nlb; i += 256) {
        const LbPart p = a.lbpart[(size_t)q * nlb + i];
        best = p.key < best ? p.key : best;
        mx = max(mx, p.mx);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        s_min[threadIdx.x >> 6] = best;
        s_max[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
        best = s_min[w] < best ? s_min[w] : best;
        mx = max(mx, s_max[w]);
    }
}

// Distances to the approximate leaf's members.
__global__ void __launch_bounds__(256) approx_ed_kernel(QArgs a, uint32_t nlb) {
    __shared__ float s_q[MESSI_MAX_LEN];
    __shared__ unsigned long long s_min[4];
    __shared__ uint32_t s_max[4];
    const int q = blockIdx.y;
    if (slot_off(a, q, kSlotAdmit)) return;
    const QState& st = a.qs[q];
    if (st.err) return;
    for (int j = threadIdx.x; j < a.L; j += 256) s_q[j] = a.queries[(size_t)q * a.L + j];
    unsigned long long best;
    uint32_t mx;
    lb_extremes(a, q, nlb, s_min, s_max, best, mx);
    uint32_t r0, cnt;
    approx_range(a, (uint32_t)(best & 0xffffffffull), st.k, r0, cnt);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    const bool vec = (a.L & 3) == 0 && ((uintptr_t)a.series & 15u) == 0;
    for (uint32_t r = gw; r < cnt; r += gridDim.x * 4) {
        const float* x = a.series + (size_t)a.pos[r0 + r] * a.L;
        float s = 0.f;
        if (vec) {
            for (int j = lane * 4; j < a.L; j += 256) {
                const float4 v = *reinterpret_cast<const float4*>(x + j);
                const float d0 = s_q[j] - v.x, d1 = s_q[j + 1] - v.y, d2 = s_q[j + 2] - v.z, d3 = s_q[j + 3] - v.w;
                s = fmaf(d0, d0, s);
                s = fmaf(d1, d1, s);
                s = fmaf(d2, d2, s);
                s = fmaf(d3, d3, s);
            }
        } else {
            for (int j = lane; j < a.L; j += 64) {
                const float d = s_q[j] - x[j];
                s = fmaf(d, d, s);
            }
        }
        s = dev::wave_sum(s);
        if (lane == 0) a.approx_d[(size_t)q * kApproxMax + r] = s;
    }
}

// The k-th of those distances: the first upper bound U0 (the paper's initial
// best-so-far); with the smallest and largest leaf bound.  Block-wide: every
// thread gets the result, and every block that computes it gets the same.
struct FirstBound {
    unsigned long long best;  // (bound bits << 32) | leaf of the smallest leaf bound
    uint32_t mx;              // largest leaf bound (float bits)
    float U0;
    // the bound range mapped onto the order's bins
    __device__ float range() const {
        const float r = isinf(U0) ? __uint_as_float(mx) : U0;
        return r > 0.f ? r : 1e-30f;
    }
};

struct FirstBoundSmem {
    unsigned long long s_min[4];
    uint32_t s_max[4];
    uint32_t s_hist[256 + 4];
    uint32_t s_b[2];
};

__device__ FirstBound first_bound(const QArgs& a, int q, int32_t k, uint32_t nlb, FirstBoundSmem& sm) {
    FirstBound f;
    lb_extremes(a, q, nlb, sm.s_min, sm.s_max, f.best, f.mx);
    uint32_t r0, cnt;
    approx_range(a, (uint32_t)(f.best & 0xffffffffull), k, r0, cnt);
    const float* d = a.approx_d + (size_t)q * kApproxMax;
    const float kth = block_kth([&](uint32_t i) { return d[i]; }, cnt, (uint32_t)k, sm.s_hist, sm.s_b);
    f.U0 = isinf(kth) ? kth : upper_u(kth);
    return f;
}

// The members evaluated for the first bound only set it; their leaf stays in
// the order and is scanned like any other, so every candidate is appended
// exactly once per pass.
__device__ void store_first_bound(QState& st, const FirstBound& f) {
    st.argmin = f.best;
    st.lbmax = f.mx;
    st.U = __float_as_uint(f.U0);
    st.hbase = (int32_t)(__float_as_uint(f.U0) >> 16) - (kHistBins - 2);
    st.range = f.range();
}

// Approximate mode: the first bound into the query's state (the exact
// searches form it inside the bin-histogram kernel instead).
__global__ void __launch_bounds__(256) approx_select_kernel(QArgs a, uint32_t nlb) {
    __shared__ FirstBoundSmem sm;
    const int q = blockIdx.x;
    QState& st = a.qs[q];
    if (st.err) return;
    const FirstBound f = first_bound(a, q, st.k, nlb, sm);
    if (threadIdx.x == 0) store_first_bound(st, f);
}

// Approximate mode: the evaluated members of the first leaf whose distance is
// within the first bound are the candidates; the final kernel orders them.
__global__ void __launch_bounds__(256) approx_cands_kernel(QArgs a, uint32_t nlb) {
    __shared__ unsigned long long s_min[4];
    __shared__ uint32_t s_max[4];
    const int q = blockIdx.x;
    QState& st = a.qs[q];
    if (st.err) return;
    unsigned long long best;
    uint32_t mx;
    lb_extremes(a, q, nlb, s_min, s_max, best, mx);
    uint32_t r0, cnt;
    approx_range(a, (uint32_t)(best & 0xffffffffull), st.k, r0, cnt);
    const float U = __uint_as_float(st.U);
    const float* d = a.approx_d + (size_t)q * kApproxMax;
    for (uint32_t r = threadIdx.x; r < cnt; r += 256) {
        const float dv = d[r];
        if (dv * (1.0f - kRhoEd) <= U) {
            const uint32_t slot = atomicAdd(&st.ncand, 1u);
            if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{dv, a.pos[r0 + r]};
            else if (st.err == 0) st.err = 2;
        }
    }
}

// --------------------------------------------------------------------------
// order: counting sort of the surviving leaves into bound bins
// --------------------------------------------------------------------------
// Candidate-distance histogram bin of d (top 16 float bits, from hbase).
__device__ __forceinline__ uint32_t hist_bin(float d, int32_t hbase) {
    const int32_t b = (int32_t)(__float_as_uint(d) >> 16) - hbase;
    return (uint32_t)min(max(b, 0), kHistBins - 1);
}

__device__ __forceinline__ int bin_of(float lbv, float range) {
    const float f = lbv / range * (float)kNB;
    if (!(f >= 0.f)) return 0;
    return f >= (float)(kNB - 1) ? kNB - 1 : (int)f;
}

__device__ __forceinline__ bool leaf_kept(float lbv, float U0) { return !(lbv * (1.0f - kRhoLb) > U0); }

// Leaves and members per bound bin.  Every block first forms the first bound
// (the same in each; block 0 stores it for the later kernels): one launch
// fewer on the query's critical path.
__global__ void __launch_bounds__(256) bin_hist_kernel(QArgs a, uint32_t nlb) {
    __shared__ uint32_t h[kNB];
    __shared__ uint32_t hm[kNB];
    __shared__ FirstBoundSmem sm;
    const int q = blockIdx.y;
    if (slot_off(a, q, kSlotAdmit)) return;
    QState& st = a.qs[q];
    if (st.err) return;
    for (int i = threadIdx.x; i < kNB; i += 256) {
        h[i] = 0;
        hm[i] = 0;
    }
    const FirstBound f = first_bound(a, q, st.k, nlb, sm);
    if (blockIdx.x == 0 && threadIdx.x == 0) store_first_bound(st, f);
    if (blockIdx.x == 0 && a.skip_approx) {
        // The first bound's members are exactly one leaf (the one of smallest
        // bound, of at least k and at most kApproxMax members): their fp32
        // distances, already computed, go to the candidates here (those within
        // the first bound), and the scan's first pass skips the leaf.
        const uint32_t leaf = (uint32_t)(f.best & 0xffffffffull);
        const Leaf lf = a.leaves[leaf];
        uint32_t r0, cnt;
        approx_range(a, leaf, st.k, r0, cnt);
        if (r0 == lf.start && cnt == lf.count && !isinf(f.U0)) {
            const float* d = a.approx_d + (size_t)q * kApproxMax;
            const int32_t hb = (int32_t)(__float_as_uint(f.U0) >> 16) - (kHistBins - 2);  // as store_first_bound
            for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
                const float di = d[i];
                if (di * (1.0f - kRhoEd) <= f.U0) {
                    const uint32_t slot = atomicAdd(&st.ncand, 1u);
                    if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{di, a.pos[r0 + i]};
                    else st.ovf = 1;
                    if (st.k > 1) atomicAdd(&a.hist[(size_t)q * kHistBins + hist_bin(di, hb)], 1u);
                }
            }
            if (threadIdx.x == 0) st.skip_start = lf.start;
        }
    }
    __syncthreads();
    const float U0 = f.U0, range = f.range();
    for (int l = blockIdx.x * kLeafBlock + threadIdx.x; l < a.nL; l += gridDim.x * kLeafBlock) {
        const float lbv = a.lb[(size_t)q * a.nL + l];
        if (leaf_kept(lbv, U0)) {
            const int bn = bin_of(lbv, range);
            atomicAdd(&h[bn], 1u);
            atomicAdd(&hm[bn], a.leaves[l].count);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNB; i += 256)
        if (h[i]) {
            atomicAdd(&a.bins[(size_t)q * kNB + i], h[i]);
            atomicAdd(&a.mbins[(size_t)q * kNB + i], hm[i]);
        }
}

// Place every kept leaf at its position in the bin order.  Every block first
// takes the exclusive prefix sums of the leaf and member counts per bin (4
// consecutive bins per thread; the same in each block, and block 0 stores the
// totals): the bins' first positions and member offsets.  Within a bin one
// 64-bit atomic on its fill counter hands out the position and the member
// offset together, so member offsets increase with the position; the leaf
// whose member range holds the first member of a scan chunk records itself as
// that chunk's first position.
__global__ void __launch_bounds__(256) bin_scatter_kernel(QArgs a) {
    __shared__ uint32_t s_pos[kNB], s_moff[kNB];
    __shared__ uint32_t s_tmp[4];
    const int q = blockIdx.y;
    if (slot_off(a, q, kSlotAdmit)) return;
    QState& st = a.qs[q];
    if (st.err) return;
    {
        constexpr int kPer = kNB / 256;
        uint32_t v[kPer], vm[kPer], sv = 0, svm = 0;
        for (int i = 0; i < kPer; ++i) {
            v[i] = a.bins[(size_t)q * kNB + threadIdx.x * kPer + i];
            vm[i] = a.mbins[(size_t)q * kNB + threadIdx.x * kPer + i];
            sv += v[i];
            svm += vm[i];
        }
        uint32_t tot, totm;
        uint32_t ex = block_exclusive_scan(sv, s_tmp, tot);
        __syncthreads();
        uint32_t exm = block_exclusive_scan(svm, s_tmp, totm);
        for (int i = 0; i < kPer; ++i) {
            s_pos[threadIdx.x * kPer + i] = ex;
            s_moff[threadIdx.x * kPer + i] = exm;
            ex += v[i];
            exm += vm[i];
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st.nsurv = tot;
            st.nmemb = totm;
            if (a.counters) atomicAdd(&a.counters->kept, (unsigned long long)tot);
        }
        __syncthreads();
    }
    const float U0 = __uint_as_float(st.U), range = st.range;
    for (int l = blockIdx.x * kLeafBlock + threadIdx.x; l < a.nL; l += gridDim.x * kLeafBlock) {
        const float lbv = a.lb[(size_t)q * a.nL + l];
        if (!leaf_kept(lbv, U0)) continue;
        const Leaf lf = a.leaves[l];
        const int bn = bin_of(lbv, range);
        const unsigned long long old = atomicAdd(&a.cursor[(size_t)q * kNB + bn], (1ull << 32) | lf.count);
        const uint32_t t = s_pos[bn] + (uint32_t)(old >> 32), moff = s_moff[bn] + (uint32_t)old;
        if (t < (uint32_t)a.nL) {
            a.order[(size_t)q * a.nL + t] = (uint32_t)l;
            a.rec[(size_t)q * a.nL + t] = OrdRec{lf.start, lf.count, lbv, moff};
            const uint64_t end = (uint64_t)moff + lf.count;
            for (uint64_t c = ((uint64_t)moff + a.chunk - 1) / a.chunk; c * a.chunk < end; ++c)
                if (c < a.max_chunks) a.chunk_first[(size_t)q * a.max_chunks + c] = t;
        }
    }
}

// --------------------------------------------------------------------------
// scan: persistent blocks over the ordered (query, leaf) positions
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t word_byte(const uint4& wd, int i) {
    const uint32_t v = (i < 4) ? wd.x : (i < 8) ? wd.y : (i < 12) ? wd.z : wd.w;
    return (v >> (8 * (i & 3))) & 0xFFu;
}

// ---- candidate bookkeeping -------------------------------------------------
// For k > 1 the bound is the k-th smallest candidate distance.  During the scan
// it comes from a histogram of the candidate distances binned by their top 16
// float bits (128 bins per octave below the first bound): every candidate in
// the bins up to the one where the running count reaches k lies below that
// bin's upper edge, so the edge bounds the k-th distance from above.  Between
// kernels the exact k-th is taken from the candidate buffer itself.
// Distance from x to the envelope [lo, up] (0 inside it): one LB_Keogh term.
__device__ __forceinline__ float keogh_gap(float x, float up, float lo) {
    return x > up ? x - up : (x < lo ? lo - x : 0.f);
}

// acc + the dot product of 8 BF16 pairs, one fused multiply-add per pair (the
// products of two BF16 values are exact in fp32, so each step rounds once).
__device__ __forceinline__ float bf16_dot8(const uint4& x, const uint4& y, float acc) {
    const uint32_t xv[4] = {x.x, x.y, x.z, x.w}, yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc = fmaf(__uint_as_float(xv[i] << 16), __uint_as_float(yv[i] << 16), acc);
        acc = fmaf(__uint_as_float(xv[i] & 0xffff0000u), __uint_as_float(yv[i] & 0xffff0000u), acc);
    }
    return acc;
}


// Lower U from the histogram (block-wide; call from every thread).
__device__ void hist_refresh(const QArgs& a, int q, QState& st, uint32_t* s_tmp, float* s_Ublk) {
    const uint32_t* h = a.hist + (size_t)q * kHistBins;
    constexpr int kPer = kHistBins / 256;
    const int t = threadIdx.x;
    uint32_t v[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        v[i] = vload(h + t * kPer + i);
        sum += v[i];
    }
    uint32_t total;
    const uint32_t excl = block_exclusive_scan(sum, s_tmp, total);
    const uint32_t k = (uint32_t)st.k;
    if (total >= k && excl < k && excl + sum >= k) {
        uint32_t c = excl, b = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            if (c < k && c + v[i] >= k) b = t * kPer + i;
            c += v[i];
        }
        const int32_t e = (int32_t)b + 1 + st.hbase;  // upper edge of bin b, as float bits >> 16
        if (b < (uint32_t)(kHistBins - 1) && e > 0 && e < 0x7f80) {
            const uint32_t ub = __float_as_uint(upper_u(__uint_as_float((uint32_t)e << 16)));
            atomicMin(&st.U, ub);
            atomicMin(reinterpret_cast<uint32_t*>(s_Ublk), ub);
        }
    }
}

// Between kernels (every slot written): for k > 1 set U from the exact k-th
// candidate distance, then drop the candidates that can no longer be answers
// (d (1 - rho) > U), compacting the list in place.  One block per query.
__device__ void refresh_compact(QArgs& a, int q, QState& st, uint32_t* s_hist, uint32_t* s_b, uint32_t* s_tmp) {
    const uint32_t n = min(st.ncand, a.cap);
    Cand* c = a.cand + (size_t)q * a.cap;
    if (st.k > 1) {
        const float kth = block_kth([&](uint32_t i) { return c[i].d; }, n, (uint32_t)st.k, s_hist, s_b);
        if (threadIdx.x == 0 && !isinf(kth) && !isnan(kth))
            atomicMin(&st.U, __float_as_uint(kth * (1.0f + 2.0f * a.rho_d)));
    }
    __syncthreads();
    const float U = __uint_as_float(st.U);
    uint32_t out = 0;
    for (uint32_t r0 = 0; r0 < n; r0 += 256) {
        const uint32_t i = r0 + threadIdx.x;
        Cand e{0.f, 0u};
        bool keep = false;
        if (i < n) {
            e = c[i];
            keep = e.d * (1.0f - a.rho_d) <= U;
        }
        uint32_t total;
        const uint32_t o = block_exclusive_scan(keep ? 1u : 0u, s_tmp, total);  // all reads of this chunk done
        if (keep) c[out + o] = e;
        out += total;
        __syncthreads();
    }
    if (threadIdx.x == 0 && st.ncand <= a.cap) st.ncand = out;
}

__global__ void __launch_bounds__(256) refresh_kernel(QArgs a) {
    __shared__ uint32_t s_hist[256 + 4];
    __shared__ uint32_t s_b[2];
    __shared__ uint32_t s_tmp[4];
    const int q = blockIdx.x;
    if (slot_off(a, q, kSlotActive)) return;
    QState& st = a.qs[q];
    if (st.err) return;
    refresh_compact(a, q, st, s_hist, s_b, s_tmp);
}

// After scan pass `pass` (2: between the rounds of pass 0).  If the candidate buffer overflowed, the cap
// candidates it holds are exact distances of distinct series, so their k-th is
// a valid bound: take it, empty the buffer and the histogram, and let the
// second pass rescan from that much tighter bound.  A second overflow means
// more than cap candidates lie within rounding of the k-th distance (massive
// duplication) and is reported.  Otherwise (k > 1) tighten and compact.
__global__ void __launch_bounds__(256) fixup_kernel(QArgs a, int pass) {
    __shared__ uint32_t s_hist[256 + 4];
    __shared__ uint32_t s_b[2];
    __shared__ uint32_t s_tmp[4];
    const int q = blockIdx.x;
    QState& st = a.qs[q];
    if (st.err) return;
    if (pass == 1 && !st.rerun) return;
    if (st.ovf && pass == 2) {
        // between the two rounds of a split scan: tighten U from the full
        // buffer's k-th but keep it (and the overflow) for the end of pass 0
        const Cand* c = a.cand + (size_t)q * a.cap;
        const float kth = block_kth([&](uint32_t i) { return c[i].d; }, a.cap, (uint32_t)st.k, s_hist, s_b);
        if (threadIdx.x == 0 && !isinf(kth) && !isnan(kth)) atomicMin(&st.U, __float_as_uint(upper_u(kth)));
        return;
    }
    if (st.ovf) {
        if (pass == 1) {
            if (threadIdx.x == 0) {
                st.err = 2;
                atomicOr(a.err_any, 2u);
            }
            return;
        }
        const Cand* c = a.cand + (size_t)q * a.cap;
        const float kth = block_kth([&](uint32_t i) { return c[i].d; }, a.cap, (uint32_t)st.k, s_hist, s_b);
        for (int i = threadIdx.x; i < kHistBins; i += 256) a.hist[(size_t)q * kHistBins + i] = 0;
        if (threadIdx.x == 0) {
            if (!isinf(kth) && !isnan(kth)) atomicMin(&st.U, __float_as_uint(upper_u(kth)));
            st.ncand = 0;
            st.ovf = 0;
            st.rerun = 1;
            if (a.counters) atomicAdd(&a.counters->reruns, 1ull);
        }
        return;
    }
    if (st.k > 1) refresh_compact(a, q, st, s_hist, s_b, s_tmp);
}

// ---- the ordered scan --------------------------------------------------------
// The members of the ordered leaves form one list (leaf after leaf in bound
// order); it is cut into chunks of a.chunk (<= kChunk) members and the G blocks of a query
// take chunks j, j + G, j + 2G, ...  Every block does the same amount of
// member work, and the grid still advances through the order together, so
// the best leaves are scanned first and U tightens early.  Per chunk:
//   positions  the chunk's leaves (start, bound, member offset) into LDS
//   coarse     per member: leaf bound against U, then the bound of its 8-byte
//              coarse word (every symbol cut to 4 bits, two per byte) from
//              one LDS table per byte: 8 lookups
//   word       per coarse survivor (a few percent): its 16-byte word and
//              series index, read together; the word's own bound (region
//              edges from LDS); survivors compacted into LDS
//   fine       (ED) per word survivor, its fine summary (64 bytes: the PAA
//              over 64 segments at L = 256): a tighter bound that keeps
//              about one in ten of them
//   distances  16 lanes per row, each row read whole (1 KB per pass)
//   bound      k = 1: atomicMin of U; k > 1: histogram, then U from it
// The steps are software-pipelined one chunk deep: the next chunk's leaf
// records load while this chunk's words are filtered, and its words load
// while this chunk's distances are computed, so a chunk costs about two
// dependent memory round trips (row index, row) instead of six.  The stop
// test (the chunk's first leaf lies in a bin wholly above U) is taken when
// a chunk is prefetched.
// Pass 1 runs only for queries whose candidate buffer overflowed in pass 0.
// With SH (BF16 mode, few queries) a survivor's 512-byte BF16 row in leaf
// order (L = 256) is tested first, with the same exact drop rule as the
// matrix-core filter: the test is acc < alpha for
//     acc = sum 2 q~_j x~_j + c~ r~x - b_hi - b_lo    (fp32, any order)
//     alpha = fl(fl((1 - h) |q|^2) - fl(U (1 + 2^-20))),
// which implies D > U, so a dropped member is not an answer.  Only the rows
// that pass read their fp32 row for the distance the FP32 scan computes.  The
// test runs while U exceeds rf_tau |q|^2: once U is of the order of the
// rounding bound (about 4 |q||x| 2^-8) it would drop little.
// Four waves per SIMD (four blocks per CU, which the LDS also allows): the
// scan is bound by memory latency, so resident waves matter more than the
// couple of registers this spills.  The row-filtered variant runs three, with
// no spills: its BF16 pass keeps twice the rows in flight per wave.
template <bool VEC, int pass, int MODE>
__global__ void __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(MODE == kScanRowFilter ? 3 : 4)))
scan_kernel(QArgs a) {
    constexpr bool SH = MODE == kScanRowFilter;
    constexpr bool DTW = MODE == kScanDtw;
    constexpr int kPer = kChunk / kScanThreads;
    __shared__ float s_C[8 * 256];           // coarse bound: per byte value of byte j, its two segments' terms
    __shared__ float2 s_rb[256];             // each symbol's region widened by the query's delta (lo, hi)
    __shared__ float s_plo[16], s_phi[16];   // the query's interval per segment
    // the query; with SH none (the rare fp32 rows read it from L2); with DTW
    // its envelope, upper then lower
    __shared__ float s_q[SH ? 1 : DTW ? 2 * MESSI_MAX_LEN : MESSI_MAX_LEN];
    __shared__ uint32_t s_surv[kChunk + kEdBatch];  // series indices waiting for their distance
    __shared__ uint32_t s_pbase[kChunk];  // word index of the chunk's member 0 if it were in this leaf
    __shared__ float s_plb[kChunk];
    __shared__ uint16_t s_pm[kChunk];     // first chunk-relative member of each leaf (0 for the first)
    __shared__ uint32_t s_cf[64];         // first order position of this block's next 64 chunks
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_flag, s_app, s_stop;
    __shared__ float s_Ublk;  // block's view of U: refreshed each chunk, lowered by its own finds
    __shared__ uint4 s_qb[SH ? MESSI_MAX_LEN / 8 : 1];  // row filter: 2 q in BF16
    __shared__ uint4 s_qx;                              // row filter: the query's extra k-step
    __shared__ float s_q2h, s_tau;                      // row filter: fl((1 - h) |q|^2), rf_tau |q|^2
    __shared__ uint32_t s_rck[SH ? kChunk + kEdBatch : 1];  // row filter: series indices that passed
    __shared__ uint32_t s_nrck;
    __shared__ uint32_t s_ntodo;  // DTW: entries in this block's segment of the waiting list
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    const int nq = a.nq;
    const int L = a.L;
    const int nchunk = (L + 63) / 64;
    const int B = gridDim.x;
    int q0, qstep, j, G;
    if (nq <= B) {
        q0 = blockIdx.x % nq;
        qstep = nq;
        j = blockIdx.x / nq;
        G = (B - q0 + nq - 1) / nq;
    } else {
        q0 = blockIdx.x;
        qstep = B;
        j = 0;
        G = 1;
    }
    uint32_t c_scanned = 0, c_bounded = 0, c_dist = 0, c_abandon = 0, c_bytes = 0;  // this thread's share
    uint32_t c_rck = 0, c_bft = 0, c_wordb = 0;
    const int npc = SH ? (a.Lp >> 3) : 0;  // 16-byte pieces of a BF16 row
    // optional per-block phase timing, kept by thread 0 in LDS: control,
    // member filter, distances, last mark, start
    __shared__ unsigned long long s_t[5];
    const bool timing = a.prof != nullptr;
    if (timing && tid == 0) {
        s_t[0] = s_t[1] = s_t[2] = 0;
        s_t[4] = s_t[3] = wall_clock64();
    }
    auto tick = [&](int slot) {
        if (timing && tid == 0) {
            const unsigned long long now = wall_clock64();
            s_t[slot] += now - s_t[3];
            s_t[3] = now;
        }
    };
    bool worked = false;
    for (int q = q0; q < nq; q += qstep) {
        QState& st = a.qs[q];
        if (tid == 0) {
            s_flag = (st.err != 0 || st.nsurv == 0 || (pass == 1 && st.rerun == 0)) ? 1u : 0u;
            s_Ublk = __uint_as_float(0x7f800000u);
            s_nrck = 0;
            s_ntodo = 0;
        }
        __syncthreads();
        const bool skip = s_flag != 0;
        __syncthreads();
        if (skip) continue;
        worked = true;
        const uint32_t nsurv = st.nsurv;
        const uint64_t nmemb = st.nmemb;
        const int k = st.k;
        const float range = st.range;
        // this call's chunks of the query's order: [chunk_lo, chunk_hi)
        const uint64_t nch = min((nmemb + a.chunk - 1) / a.chunk, (uint64_t)a.chunk_hi);
        const uint64_t jb = (uint64_t)a.chunk_lo + (uint64_t)j;
        const uint32_t ncb = nch > jb ? (uint32_t)((nch - jb + G - 1) / G) : 0u;
        if (ncb == 0) continue;
        if (timing && tid == 0) s_t[3] = wall_clock64();
        {
            const int A = 1 << a.b;
            const float delta = st.delta;
            const float mf = (float)a.m;
            const float inf = __uint_as_float(0x7f800000u);
            for (int c = tid; c < A; c += kScanThreads)
                s_rb[c] = make_float2(c > 0 ? a.bp[c - 1] - delta : -inf, c < A - 1 ? a.bp[c] + delta : inf);
            if (tid < 16) {
                s_plo[tid] = st.paa[tid];
                s_phi[tid] = st.paa_hi[tid];
            }
            // byte j of a coarse word: coarse symbols of segments 2j (high
            // nibble) and 2j + 1; coarse symbol c covers the symbols
            // [c << csh, (c + 1) << csh)
            for (int idx = tid; idx < 8 * 256; idx += kScanThreads) {
                const int j = idx >> 8, byte = idx & 255;
                float t = 0.f;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = 2 * j + h;
                    const int c = h == 0 ? byte >> 4 : byte & 15;
                    if (i < a.w) {
                        const int s0 = c << a.csh, s1 = (c + 1) << a.csh;
                        const float pl = st.paa[i], ph = st.paa_hi[i];
                        float d = 0.f;
                        if (s0 > 0 && s0 < A) {
                            const float lo = a.bp[s0 - 1] - delta;
                            if (ph < lo) d = lo - ph;
                        }
                        if (s1 < A) {
                            const float hi = a.bp[s1 - 1] + delta;
                            if (pl > hi) d = pl - hi;
                        }
                        t += mf * (d * d);
                    }
                }
                s_C[idx] = t;
            }
            if (DTW) {
                // the query's LB_Keogh envelope (dtw_env_kernel)
                const float* eg = a.env + (size_t)q * 2 * L;
                for (int jj = tid; jj < L; jj += kScanThreads) {
                    s_q[jj] = eg[jj];
                    s_q[MESSI_MAX_LEN + jj] = eg[L + jj];
                }
            } else if (!SH) {
                for (int jj = tid; jj < L; jj += kScanThreads) s_q[jj] = a.queries[(size_t)q * L + jj];
            }
            if (SH) {
                const uint4* qb4 = reinterpret_cast<const uint4*>(a.qb) + (size_t)q * npc;
                for (int jj = tid; jj < npc; jj += kScanThreads) s_qb[jj] = qb4[jj];
                if (tid == 0) {
                    const float2 qn = a.qnorm[q];
                    s_qx = a.qx[q];
                    s_q2h = __fmul_rn(a.one_minus_h, qn.x);
                    s_tau = a.rf_tau * qn.x;
                }
            }
        }
        const uint32_t* cfq = a.chunk_first + (size_t)q * a.max_chunks;
        const OrdRec* recq = a.rec + (size_t)q * a.nL;
        // chunk starts of chunks i0 .. i0 + 63 of this block (call from every thread)
        auto load_cf = [&](uint32_t i0) {
            if (tid < 64 && i0 + tid < ncb) s_cf[tid] = cfq[jb + (uint64_t)(i0 + tid) * G];
            __syncthreads();
        };
        // The leaves of chunk c, from the order record `r` this thread loaded
        // (position t0 + tid, valid if r_ok), into the LDS position arrays;
        // returns how many leaves the chunk spans.  Call from every thread.
        auto commit_positions = [&](uint64_t c, uint32_t t0, const OrdRec& r, bool r_ok, float Uc) -> uint32_t {
            const uint64_t cbeg = c * a.chunk;
            auto put = [&](uint32_t p, const OrdRec& rr) {
                s_pbase[p] = rr.start + (uint32_t)cbeg - rr.moff;  // modulo 2^32
                s_pm[p] = (uint64_t)rr.moff > cbeg ? (uint16_t)(rr.moff - (uint32_t)cbeg) : (uint16_t)0;
                s_plb[p] = rr.lb;
                if ((uint64_t)rr.moff >= cbeg && !(rr.lb * (1.0f - kRhoLb) > Uc)) ++c_scanned;
            };
            bool inc = r_ok && (uint64_t)r.moff < cbeg + a.chunk;
            if (inc) put(tid, r);
            int cnt = __syncthreads_count(inc);
            uint32_t np = (uint32_t)cnt;
            // the included leaves are a prefix of the positions from t0; a chunk
            // of many small leaves needs more than one round of records
            for (uint32_t b0 = kScanThreads; cnt == kScanThreads && b0 < a.chunk; b0 += kScanThreads) {
                const uint32_t t = t0 + b0 + tid;
                inc = false;
                if (t < nsurv) {
                    const OrdRec r2 = recq[t];
                    inc = (uint64_t)r2.moff < cbeg + a.chunk;
                    if (inc) put(b0 + tid, r2);
                }
                cnt = __syncthreads_count(inc);
                np += (uint32_t)cnt;
            }
            return np;
        };
        // bins ascend along the order: once a chunk's first leaf lies in a bin
        // wholly above U, so does every later chunk
        auto chunk_stops = [&](float Uc) -> bool {
            const float lb0 = s_plb[0];
            const float low = (float)bin_of(lb0, range) * (range / (float)kNB);
            return lb0 * (1.0f - kRhoLb) > Uc && low * (1.0f - 2.0f * kRhoLb) > Uc;
        };
        // Member f of the chunk whose leaves are in the LDS position arrays:
        // its leaf (the last one starting at or before f) and word index.
        auto member_leaf = [&](uint32_t np, uint32_t f) -> int {
            int lo = 0, hi = (int)np - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((uint32_t)s_pm[mid] <= f) lo = mid;
                else hi = mid - 1;
            }
            return lo;
        };
        // This thread's members of a chunk: leaf bound against U, then the coarse word.
        auto issue_words = [&](uint32_t np, uint32_t clen, float Uc, uint2* cw) -> uint32_t {
            uint32_t live = 0;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const uint32_t f = r * kScanThreads + tid;
                uint32_t mp = 0;
                if (f < clen) {
                    const int lf = member_leaf(np, f);
                    if (!(s_plb[lf] * (1.0f - kRhoLb) > Uc)) {
                        live |= 1u << r;
                        mp = s_pbase[lf] + f;
                    }
                }
                cw[r] = (live & (1u << r)) ? a.cwords[mp] : make_uint2(0, 0);
            }
            return live;
        };
        auto chunk_len = [&](uint64_t c) -> uint32_t {
            return (uint32_t)min((uint64_t)a.chunk, nmemb - c * a.chunk);
        };

        // ---- prologue: chunk 0 of this block
        uint32_t nacc = 0;  // survivors gathered in s_surv (the same in every thread)
        load_cf(0);
        if (tid == 0) {
            s_Ublk = fminf(s_Ublk, __uint_as_float(vload(&st.U)));
            s_stop = vload(&st.ovf);
        }
        uint32_t t0n = s_cf[0];
        OrdRec rn{0u, 0u, 0.f, 0u};
        bool rn_ok = t0n + tid < nsurv;
        if (rn_ok) rn = recq[t0n + tid];
        __syncthreads();
        float Uc = s_Ublk;
        uint32_t np = commit_positions(jb, t0n, rn, rn_ok, Uc);
        if (np == 0 || s_stop || chunk_stops(Uc)) continue;
        uint2 cw[kPer];
        uint32_t live = issue_words(np, chunk_len(jb), Uc, cw);
        tick(0);
        for (uint32_t i = 0;; ++i) {
            const uint64_t c = jb + (uint64_t)i * G;
            bool more = i + 1 < ncb;
            // ---- next chunk's leaf records, in flight during this chunk's filter
            if (more && ((i + 1) & 63u) == 0) load_cf(i + 1);
            if (more) {
                t0n = s_cf[(i + 1) & 63u];
                rn_ok = t0n + tid < nsurv;
                if (rn_ok) rn = recq[t0n + tid];
            }
            // ---- filter this chunk: each member's coarse word bound
            const float Uf = s_Ublk;
            uint32_t bmask = 0;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                if (live & (1u << r)) {
                    float sum = 0.f;
#pragma unroll
                    for (int j2 = 0; j2 < 8; ++j2) {
                        const uint32_t half = j2 < 4 ? cw[r].x : cw[r].y;
                        sum += s_C[j2 * 256 + ((half >> (8 * (j2 & 3))) & 255u)];
                    }
                    if (!(sum * (1.0f - kRhoLb) > Uf)) bmask |= 1u << r;
                    ++c_bounded;
                }
            }
            // ---- the coarse survivors' words and series indices (with SH the
            // leaf-order position: the BF16 row's index), read together
            uint4 wd[kPer];
            uint32_t gi[kPer];
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                gi[r] = 0;
                wd[r] = make_uint4(0, 0, 0, 0);
                if (bmask & (1u << r)) {
                    // the chunk's leaves are still in LDS (the next chunk's are committed below)
                    const uint32_t f = r * kScanThreads + tid;
                    const uint32_t mp = s_pbase[member_leaf(np, f)] + f;
                    wd[r] = a.words[mp];
                    gi[r] = SH ? mp : a.pos[mp];
                }
            }
            // ---- each coarse survivor's own word bound
            uint32_t keepmask = 0, nkeep = 0;
            const float mseg = (float)a.m;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                if (bmask & (1u << r)) {
                    float sum = 0.f;
#pragma unroll
                    for (int i2 = 0; i2 < 16; ++i2) {
                        if (i2 < a.w) {
                            const float2 rg = s_rb[word_byte(wd[r], i2)];
                            const float pl = s_plo[i2], ph = s_phi[i2];
                            const float d = ph < rg.x ? rg.x - ph : (pl > rg.y ? pl - rg.y : 0.f);
                            sum += mseg * (d * d);
                        }
                    }
                    if (!(sum * (1.0f - kRhoLb) > Uf)) {
                        keepmask |= 1u << r;
                        ++nkeep;
                    }
                    ++c_wordb;
                }
            }
            uint32_t total;
            uint32_t o = nacc + block_exclusive_scan(nkeep, s_tmp, total);
#pragma unroll
            for (int r = 0; r < kPer; ++r)
                if (keepmask & (1u << r)) s_surv[o++] = gi[r];
            nacc += total;
            tick(1);
            // every thread has placed its survivors (reading this chunk's
            // leaves) before the next chunk's leaves overwrite them
            __syncthreads();
            // ---- next chunk's positions (the barrier also publishes s_surv)
            if (tid == 0) {
                s_Ublk = fminf(s_Ublk, __uint_as_float(vload(&st.U)));
                s_stop = vload(&st.ovf);
                s_app = 0;
            }
            uint32_t npn = 0;
            if (more) npn = commit_positions(c + G, t0n, rn, rn_ok, s_Ublk);
            else __syncthreads();
            Uc = s_Ublk;
            // this pass overflowed (it is redone from a tighter bound), or the
            // next chunk lies wholly above U
            if (s_stop) break;
            if (more && (npn == 0 || chunk_stops(Uc))) more = false;
            uint2 cwn[kPer];
            uint32_t liven = 0;
            if (more) liven = issue_words(npn, chunk_len(c + G), Uc, cwn);
            tick(0);
            // distances wait until a batch of survivors has gathered (or the
            // block's last chunk), so each round of row loads is well filled
            const bool run_ed = !more || nacc >= (uint32_t)kEdBatch;
            if (run_ed) {
            uint32_t nsv = nacc;
            nacc = 0;
            // With SH the list holds leaf-order positions.  While U is large
            // their BF16 rows are tested first, 8 lanes per row and 8 rows per
            // wave at a time (twice the rows in flight of the fp32 pass), and
            // the series indices of the rows that pass go to s_rck.
            bool from_rck = false;
            if (SH && s_Ublk > s_tau) {
                // nothing lowers s_Ublk before the distances below: one value for the block
                const float alpha = __fsub_rn(s_q2h, __fmul_rn(s_Ublk, 1.00000095367431640625f));
                const int g8 = lane >> 3, l8 = lane & 7;
                for (uint32_t base = wave * 8; base < nsv; base += 32) {
                    const uint32_t si = base + g8;
                    const bool act = si < nsv;
                    const uint32_t mp = act ? s_surv[si] : 0u;
                    const uint4* xr = reinterpret_cast<const uint4*>(a.shadow) + (size_t)mp * npc;
                    float bacc = 0.f;
                    for (int c0 = 0; c0 < npc; c0 += 32) {
                        uint4 xv[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int c = c0 + t * 8 + l8;
                            xv[t] = (act && c < npc) ? xr[c] : make_uint4(0u, 0u, 0u, 0u);
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int c = c0 + t * 8 + l8;
                            if (c < npc) bacc = bf16_dot8(s_qb[c], xv[t], bacc);
                        }
                    }
                    if (act && l8 == 0) {
                        const uint2 e = a.sx[mp];
                        bacc = bf16_dot8(s_qx, make_uint4(e.x, e.y, 0u, 0u), bacc);
                    }
                    bacc += __shfl_xor(bacc, 4, 8);
                    bacc += __shfl_xor(bacc, 2, 8);
                    bacc += __shfl_xor(bacc, 1, 8);
                    if (act) {
                        c_bytes += 2u * ((uint32_t)npc * 16u + 8u);  // 8 lanes of the row (the sum is taken / 16)
                        if (l8 == 0) {
                            ++c_dist;
                            ++c_bft;
                            if (!(bacc < alpha)) {
                                ++c_rck;
                                s_rck[atomicAdd(&s_nrck, 1u)] = a.pos[mp];
                            }
                        }
                    }
                }
                __syncthreads();
                nsv = s_nrck;
                from_rck = true;
            }
            // ---- distances: 16 lanes per row, the whole row per pass
            const float* qv = SH ? a.queries + (size_t)q * L : s_q;
            uint32_t appended = 0;
            for (uint32_t base = wave * 4; base < nsv; base += 16) {
                const uint32_t si = base + quarter;
                const bool act = si < nsv;
                uint32_t gidx = act ? (from_rck ? s_rck[si] : s_surv[si]) : 0u;
                if (SH && !from_rck && act) gidx = a.pos[gidx];  // a leaf-order position
                bool alive = act;
                const float* row = a.series + (size_t)gidx * L;
                float acc = 0.f;
                for (int g = 0; g < nchunk; g += 4) {
                    if (alive) {
                        if (VEC) {
                            float4 x[4];
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
                                const int j0 = (g + cc) * 64 + ql * 4;
                                x[cc] = (g + cc < nchunk && j0 < L) ? *reinterpret_cast<const float4*>(row + j0)
                                                                    : make_float4(0.f, 0.f, 0.f, 0.f);
                            }
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
                                const int j0 = (g + cc) * 64 + ql * 4;
                                if (g + cc < nchunk && j0 < L) {
                                    const float4 y = *reinterpret_cast<const float4*>(qv + j0);
                                    float d0, d1, d2, d3;
                                    if (DTW) {
                                        const float4 lw = *reinterpret_cast<const float4*>(qv + MESSI_MAX_LEN + j0);
                                        d0 = keogh_gap(x[cc].x, y.x, lw.x);
                                        d1 = keogh_gap(x[cc].y, y.y, lw.y);
                                        d2 = keogh_gap(x[cc].z, y.z, lw.z);
                                        d3 = keogh_gap(x[cc].w, y.w, lw.w);
                                    } else {
                                        d0 = y.x - x[cc].x;
                                        d1 = y.y - x[cc].y;
                                        d2 = y.z - x[cc].z;
                                        d3 = y.w - x[cc].w;
                                    }
                                    acc = fmaf(d0, d0, acc);
                                    acc = fmaf(d1, d1, acc);
                                    acc = fmaf(d2, d2, acc);
                                    acc = fmaf(d3, d3, acc);
                                }
                            }
                        } else {
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const int jj = (g + cc) * 64 + ql * 4 + e;
                                    if (g + cc < nchunk && jj < L) {
                                        const float d = DTW ? keogh_gap(row[jj], qv[jj], qv[MESSI_MAX_LEN + jj])
                                                            : qv[jj] - row[jj];
                                        acc = fmaf(d, d, acc);
                                    }
                                }
                            }
                        }
                    }
                    float p = acc;
                    p += __shfl_xor(p, 8, 16);
                    p += __shfl_xor(p, 4, 16);
                    p += __shfl_xor(p, 2, 16);
                    p += __shfl_xor(p, 1, 16);
                    p = __shfl(p, quarter * 16, 64);  // one value per row on every lane of the row
                    if (alive) c_bytes += (uint64_t)min(4, nchunk - g) * 256u;
                    if (g + 4 < nchunk) {
                        // one U for the whole wave (other waves may lower it meanwhile)
                        const float Un = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_Ublk)));
                        if (alive && p * (1.0f - kRhoEd) > Un) {
                            alive = false;
                            if (ql == 0) ++c_abandon;
                        }
                    } else {
                        acc = p;  // the full distance
                    }
                }
                if (act && ql == 0 && !(SH && from_rck)) ++c_dist;
                if (DTW) {
                    // LB_Keogh within the bound: the series waits for its DTW, in
                    // this block's own segment of the list (a counter in LDS: one
                    // counter for the whole grid would serialise the appends)
                    if (alive && ql == 0 && !(acc * (1.0f - kRhoEd) > s_Ublk)) {
                        const uint32_t slot = atomicAdd(&s_ntodo, 1u);
                        if (slot < a.todo_seg)
                            a.todo[(size_t)q * a.todo_cap + (size_t)j * a.todo_seg + slot] = Cand{acc, gidx};
                        else
                            st.ovf = 1;
                    }
                } else if (alive && ql == 0) {
                    const float d = acc;
                    if (d * (1.0f - kRhoEd) <= s_Ublk) {
                        const uint32_t slot = atomicAdd(&st.ncand, 1u);
                        if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{d, gidx};
                        else st.ovf = 1;
                        ++appended;
                        if (k == 1) {
                            const uint32_t ub = __float_as_uint(upper_u(d));
                            atomicMin(&st.U, ub);
                            atomicMin(reinterpret_cast<uint32_t*>(&s_Ublk), ub);
                        } else {
                            atomicAdd(&a.hist[(size_t)q * kHistBins + hist_bin(d, st.hbase)], 1u);
                        }
                    }
                }
            }
            if (k > 1 && appended) atomicAdd(&s_app, appended);
            __syncthreads();
            if (SH && tid == 0) s_nrck = 0;  // every thread has read it
            tick(2);
            if (k > 1 && s_app) hist_refresh(a, q, st, s_tmp, &s_Ublk);
            __syncthreads();
            }
            if (!more) break;
            np = npn;
            live = liven;
#pragma unroll
            for (int r = 0; r < kPer; ++r) cw[r] = cwn[r];
        }
        __syncthreads();
        if (DTW && tid == 0) a.todo_cnt[(size_t)q * a.todo_nseg + j] = min(s_ntodo, a.todo_seg);
    }
    if (timing && tid == 0 && (pass == 0 || worked)) {
        // pass 0 writes the block's times; a second pass adds its own
        unsigned long long* pr = a.prof + (size_t)blockIdx.x * 4;
        const unsigned long long v[4] = {s_t[0], s_t[1], s_t[2], wall_clock64() - s_t[4]};
        // pass 0 of a call starts the sums (DTW rounds after the first add to them)
        const bool first = pass == 0 && a.chunk_lo == 0;
        for (int i = 0; i < 4; ++i) pr[i] = (first ? 0ull : pr[i]) + v[i];
    }
    if (a.blk_cnt) {
        // per-block totals in plain stores (the host adds them up): same-address
        // atomics from every block at once would serialise at the end of the grid
        __shared__ unsigned long long s_cnt[4][kBlkCnt];
        // bytes: rows, 8 per coarse word, 16 per word (+ 4 for the series
        // index, read with it unless SH), the fine summary's 16-byte pieces
        unsigned long long v[kBlkCnt] = {c_scanned, c_bounded, c_dist, c_abandon,
                                         (unsigned long long)c_bytes / 16 + (unsigned long long)c_bounded * 8ull +
                                             (unsigned long long)c_wordb * (SH ? 16ull : 20ull),
                                         c_rck, c_bft, c_wordb, 0ull};
        for (int i = 0; i < kBlkCnt; ++i)
            for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off);
        if (lane == 0)
            for (int i = 0; i < kBlkCnt; ++i) s_cnt[wave][i] = v[i];
        __syncthreads();
        if (tid < kBlkCnt && (pass == 0 || worked)) {
            const unsigned long long t = s_cnt[0][tid] + s_cnt[1][tid] + s_cnt[2][tid] + s_cnt[3][tid];
            unsigned long long* p = a.blk_cnt + (size_t)blockIdx.x * kBlkCnt + tid;
            *p = (pass == 0 && a.chunk_lo == 0 ? 0ull : *p) + t;
        }
    }
}

// ---- the flat Euclidean scan ---------------------------------------------------
// The same ordered member list and chunks as scan_kernel, but a chunk is the
// work of one wave, and the waves of a block share only the query's tables:
// no barrier between chunks.  Wave i of a query's W waves takes chunks i,
// i + W, i + 2W, ...  (W is thousands: the first pass over the chunks runs
// on every wave at once, the later ones after U has tightened.)  Per chunk:
//   records    the chunk's leaves (one per lane, 64 at a time)
//   coarse     per member: its leaf's bound against U, then its coarse word
//              (8 bytes) against the coarse table; survivors' leaf-order
//              positions into the wave's list in LDS (ballot compaction)
//   word       per listed member, its word and series index read together,
//              the word's bound; survivors' series indices kept in the list
//   fine       per listed series, its fine summary (4 lanes per series)
//   distances  16 lanes per row, early abandoning; k = 1: atomicMin of U;
//              k > 1: candidate buffer and histogram, U from the histogram
// Each stage compacts the list in place: a round writes only below the
// entries it has read.  Only the member loads are many per lane; the later
// stages touch a few percent of the members each.
constexpr int kFlatList = kChunk;  // list entries per wave: a chunk's members at most
constexpr int kFlatIssue = 8;      // coarse words in flight per lane
constexpr uint32_t kSplitFirst = 64;  // chunks of the split scan's first round
// words in flight per lane in the refine kernel's word stage: each is a chain
// of two dependent gathers (segment entry, then word and series index), and
// one chain per lane with more waves resident ran fastest (refine kernel
// 54.5 us per query at 100M x 256, against 55.7, 60.2, 64.6 and 79.3 us with
// 2, 3, 4 and 8 chains per lane)
constexpr int kWordIssue = 1;

// Lower U from the histogram of candidate distances (one wave).
__device__ void wave_hist_refresh(const QArgs& a, int q, QState& st, float& U) {
    const uint32_t* h = a.hist + (size_t)q * kHistBins;
    constexpr int kPer = kHistBins / 64;
    const int lane = threadIdx.x & 63;
    uint32_t sum = 0;
#pragma unroll 8
    for (int i = 0; i < kPer; ++i) sum += vload(h + lane * kPer + i);
    // exclusive prefix over the lanes
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    const uint32_t excl = incl - sum;
    const uint32_t k = (uint32_t)st.k;
    if (excl < k && incl >= k) {
        uint32_t c = excl, b = 0;
        for (int i = 0; i < kPer; ++i) {
            const uint32_t v = vload(h + lane * kPer + i);
            if (c < k && c + v >= k) {
                b = lane * kPer + i;
                break;
            }
            c += v;
        }
        const int32_t e = (int32_t)b + 1 + st.hbase;  // upper edge of bin b, as float bits >> 16
        if (b < (uint32_t)(kHistBins - 1) && e > 0 && e < 0x7f80) {
            const uint32_t ub = __float_as_uint(upper_u(__uint_as_float((uint32_t)e << 16)));
            atomicMin(&st.U, ub);
        }
    }
    U = fminf(U, __uint_as_float(vload(&st.U)));
}

template <bool VEC, int pass>
__global__ void __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4)))
flat_scan_kernel(QArgs a) {
    __shared__ float s_C[8 * 256];
    __shared__ float2 s_rb[256];
    __shared__ float2 s_rf[256];
    __shared__ float s_plo[16], s_phi[16];
    __shared__ float s_pf[64];
    __shared__ float s_bp[256];
    __shared__ __align__(16) float s_q[MESSI_MAX_LEN];
    __shared__ uint32_t s_list[kScanThreads / 64][kFlatList];
    __shared__ OrdRec s_rec[kScanThreads / 64][64];  // per wave: a window of the chunk's leaves
    __shared__ uint32_t s_flag;
    __shared__ unsigned long long s_t0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4, ql = lane & 15;
    const uint64_t lt_mask = dev::lanemask_lt();
    uint32_t* list = s_list[wave];
    OrdRec* wrec = s_rec[wave];
    const int nq = a.nq;
    const int L = a.L;
    const int nchunk = (L + 63) / 64;
    const int B = gridDim.x;
    constexpr int kWaves = kScanThreads / 64;
    int q0, qstep, j, G;
    if (nq <= B) {
        q0 = blockIdx.x % nq;
        qstep = nq;
        j = blockIdx.x / nq;
        G = (B - q0 + nq - 1) / nq;
    } else {
        q0 = blockIdx.x;
        qstep = B;
        j = 0;
        G = 1;
    }
    const bool timing = a.prof != nullptr;
    if (timing && tid == 0) s_t0 = wall_clock64();
    uint32_t c_scanned = 0, c_bounded = 0, c_dist = 0, c_abandon = 0, c_wordb = 0, c_fine = 0;
    unsigned long long c_rowb = 0;
    bool worked = false;
    for (int q = q0; q < nq; q += qstep) {
        QState& st = a.qs[q];
        if (tid == 0) s_flag = (st.err != 0 || st.nsurv == 0 || (pass == 1 && st.rerun == 0)) ? 1u : 0u;
        __syncthreads();
        const bool skip = s_flag != 0;
        __syncthreads();
        if (skip) continue;
        worked = true;
        const uint32_t nsurv = st.nsurv;
        const uint64_t nmemb = st.nmemb;
        const int k = st.k;
        const float range = st.range;
        const uint64_t nch = min((nmemb + a.chunk - 1) / a.chunk, (uint64_t)a.chunk_hi);
        const bool fine = a.fwords != nullptr;
        // ---- the query's tables: the breakpoints, the query's summary and
        // the query itself are read into LDS first (one load per thread),
        // then the tables are computed from LDS
        {
            const int A = 1 << a.b;
            const float inf = __uint_as_float(0x7f800000u);
            for (int c = tid; c < A - 1; c += kScanThreads) s_bp[c] = a.bp[c];
            if (tid < 16) {
                s_plo[tid] = st.paa[tid];
                s_phi[tid] = st.paa_hi[tid];
            }
            for (int jj = tid; jj < L; jj += kScanThreads) s_q[jj] = a.queries[(size_t)q * L + jj];
            const float delta = st.delta;
            const float qamax = st.qamax;
            __syncthreads();
            const float mf = (float)a.m;
            for (int c = tid; c < A; c += kScanThreads)
                s_rb[c] = make_float2(c > 0 ? s_bp[c - 1] - delta : -inf, c < A - 1 ? s_bp[c] + delta : inf);
            for (int idx = tid; idx < 8 * 256; idx += kScanThreads) {
                const int j2 = idx >> 8, byte = idx & 255;
                float t = 0.f;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = 2 * j2 + h;
                    const int c = h == 0 ? byte >> 4 : byte & 15;
                    if (i < a.w) {
                        const int s0 = c << a.csh, s1 = (c + 1) << a.csh;
                        const float pl = s_plo[i], ph = s_phi[i];
                        float d = 0.f;
                        if (s0 > 0 && s0 < A) {
                            const float lo = s_bp[s0 - 1] - delta;
                            if (ph < lo) d = lo - ph;
                        }
                        if (s1 < A) {
                            const float hi = s_bp[s1 - 1] + delta;
                            if (pl > hi) d = pl - hi;
                        }
                        t += mf * (d * d);
                    }
                }
                s_C[idx] = t;
            }
            if (fine) {
                const float u = 5.9604644775390625e-08f;  // 2^-24
                const float df = 1.01f * (2.f * (float)(a.lg_mf + 1) * u * a.absmax_data +
                                          2.f * (float)(a.mf + 1) * u * qamax) + kFineCodeSlack;
                for (int c = tid; c < 256; c += kScanThreads)
                    s_rf[c] = make_float2(c > 0 ? (float)c * 0.03125f - 4.0f - df : -inf, c < 255 ? (float)(c + 1) * 0.03125f - 4.0f + df : inf);
                for (int jj = tid; jj < a.wf; jj += kScanThreads) {
                    float sum = 0.f;
                    for (int i = 0; i < a.mf; ++i) sum += s_q[jj * a.mf + i];
                    s_pf[jj] = sum / (float)a.mf;
                }
            }
            __syncthreads();
        }
        const uint32_t* cfq = a.chunk_first + (size_t)q * a.max_chunks;
        const OrdRec* recq = a.rec + (size_t)q * a.nL;
        const uint64_t WG = (uint64_t)G * kWaves;
        const float mseg = (float)a.m;
        float U = __uint_as_float(vload(&st.U));
        // Round t of this wave takes chunk t W + i for even t and
        // t W + W - 1 - i for odd t (a snake over the order): the wave that
        // takes one of the first, heaviest chunks of a round takes one of the
        // last, lightest of the next.  The first chunk's leaf position and
        // records load now, each later one's while its predecessor is filtered.
        const uint64_t wi = (uint64_t)j * kWaves + wave;
        auto chunk_of = [&](uint64_t t) -> uint64_t {
            return (uint64_t)a.chunk_lo + t * WG + ((t & 1) ? WG - 1 - wi : wi);
        };
        uint64_t rt = 0;
        uint64_t c = chunk_of(0);
        uint32_t tw_n = c < nch ? cfq[c] : 0u;
        OrdRec r_n{0u, 0u, 0.f, 0xffffffffu};
        if (c < nch && tw_n + lane < nsurv) r_n = recq[tw_n + lane];
        for (; (uint64_t)a.chunk_lo + rt * WG < nch; c = chunk_of(++rt)) {
            if (c >= nch) continue;  // the last round's chunks end before this wave's place
            if (vload(&st.ovf)) break;  // this pass overflowed: it is redone from a tighter bound
            U = fminf(U, __uint_as_float(vload(&st.U)));
            const uint64_t cbeg = c * a.chunk;
            const uint64_t cend = min(cbeg + a.chunk, nmemb);
            uint32_t tw = tw_n;  // the order position of the chunk's first leaf
            OrdRec r = r_n;
            const uint64_t cn = chunk_of(rt + 1);
            if (cn < nch) tw_n = cfq[cn];
            uint32_t n1 = 0;
            bool stop = false;
            // ---- coarse: a window of up to 64 of the chunk's leaves at a time
            for (bool first = true;; first = false) {
                if (!first) {
                    r = OrdRec{0u, 0u, 0.f, 0xffffffffu};
                    if (tw + lane < nsurv) r = recq[tw + lane];
                }
                const bool rin = tw + lane < nsurv && (uint64_t)r.moff < cend;
                const uint32_t nin = (uint32_t)__popcll(__ballot(rin));  // a prefix of the lanes
                wrec[lane] = r;
                dev::wave_sync();
                if (first) {
                    // bins ascend along the order: a chunk whose first leaf lies
                    // in a bin wholly above U ends this wave's part of the order
                    const float lb0 = wrec[0].lb;
                    const float low = (float)bin_of(lb0, range) * (range / (float)kNB);
                    if (lb0 * (1.0f - kRhoLb) > U && low * (1.0f - 2.0f * kRhoLb) > U) {
                        stop = true;
                        break;
                    }
                }
                if (rin && (uint64_t)r.moff >= cbeg && !(r.lb * (1.0f - kRhoLb) > U)) ++c_scanned;
                const uint64_t wbeg = max(cbeg, (uint64_t)wrec[0].moff);
                const OrdRec rl = wrec[nin - 1];
                const uint64_t wend = min(cend, (uint64_t)rl.moff + (uint64_t)rl.count);
                // Each member's leaf: with at most four leaves in the window their
                // ends, bases (start - member offset, mod 2^32) and bounds sit in
                // scalar registers and a member picks its leaf by comparisons;
                // otherwise a walk over the window's records in LDS.
                const bool few = nin <= 4;
                uint32_t e_s[4], b_s[4];
                float l_s[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    e_s[t] = (uint32_t)__builtin_amdgcn_readlane((int)(r.moff + r.count), t);
                    b_s[t] = (uint32_t)__builtin_amdgcn_readlane((int)(r.start - r.moff), t);
                    l_s[t] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.lb), t));
                }
                const uint32_t wb = (uint32_t)wbeg, we = (uint32_t)wend;
                int p = 0;  // the walk's leaf in the window (advances with the lane's members)
                for (uint32_t g0 = wb; g0 < we; g0 += 64 * kFlatIssue) {
                    uint2 cw[kFlatIssue];
                    uint32_t mpv[kFlatIssue];
                    uint32_t live = 0;
#pragma unroll
                    for (int i = 0; i < kFlatIssue; ++i) {
                        const uint32_t g = g0 + (uint32_t)i * 64 + lane;
                        cw[i] = make_uint2(0u, 0u);
                        mpv[i] = 0;
                        if (g < we) {
                            uint32_t bs;
                            float lbv;
                            if (few) {
                                bs = b_s[0];
                                lbv = l_s[0];
#pragma unroll
                                for (int t = 1; t < 4; ++t)
                                    if (t < (int)nin && g >= e_s[t - 1]) {
                                        bs = b_s[t];
                                        lbv = l_s[t];
                                    }
                            } else {
                                while (p + 1 < (int)nin && wrec[p + 1].moff <= g) ++p;
                                const OrdRec rp = wrec[p];
                                bs = rp.start - rp.moff;
                                lbv = rp.lb;
                            }
                            if (!(lbv * (1.0f - kRhoLb) > U)) {
                                live |= 1u << i;
                                mpv[i] = bs + g;
                                cw[i] = a.cwords[mpv[i]];
                            }
                        }
                    }
                    // the next chunk's records, in flight while this chunk is filtered
                    if (first && g0 == wb) {
                        r_n = OrdRec{0u, 0u, 0.f, 0xffffffffu};
                        if (cn < nch && tw_n + lane < nsurv) r_n = recq[tw_n + lane];
                    }
#pragma unroll
                    for (int i = 0; i < kFlatIssue; ++i) {
                        bool keep = false;
                        if (live & (1u << i)) {
                            float sum = 0.f;
#pragma unroll
                            for (int j2 = 0; j2 < 8; ++j2) {
                                const uint32_t half = j2 < 4 ? cw[i].x : cw[i].y;
                                sum += s_C[j2 * 256 + ((half >> (8 * (j2 & 3))) & 255u)];
                            }
                            keep = !(sum * (1.0f - kRhoLb) > U);
                            ++c_bounded;
                        }
                        const uint64_t bal = __ballot(keep);
                        if (keep) list[n1 + __popcll(bal & lt_mask)] = mpv[i];
                        n1 += (uint32_t)__popcll(bal);
                    }
                }
                if (nin < 64 || wend >= cend) break;
                tw += 64;
                dev::wave_sync();  // every lane is done with this window's records
            }
            if (stop) break;
            dev::wave_sync();
            // ---- word: each listed member's word and series index, read
            // together, kWordIssue per lane in flight
            constexpr int kWordIssue = 4;
            uint32_t n2 = 0;
            for (uint32_t e0 = 0; e0 < n1; e0 += 64 * kWordIssue) {
                uint4 wd[kWordIssue];
                uint32_t gi[kWordIssue];
#pragma unroll
                for (int t = 0; t < kWordIssue; ++t) {
                    const uint32_t e = e0 + (uint32_t)t * 64 + lane;
                    wd[t] = make_uint4(0u, 0u, 0u, 0u);
                    gi[t] = 0;
                    if (e < n1) {
                        const uint32_t mp = list[e];
                        wd[t] = a.words[mp];
                        gi[t] = a.pos[mp];
                    }
                }
#pragma unroll
                for (int t = 0; t < kWordIssue; ++t) {
                    const uint32_t e = e0 + (uint32_t)t * 64 + lane;
                    bool keep = false;
                    if (e < n1) {
                        float sum = 0.f;
#pragma unroll
                        for (int i2 = 0; i2 < 16; ++i2) {
                            if (i2 < a.w) {
                                const float2 rg = s_rb[word_byte(wd[t], i2)];
                                const float pl = s_plo[i2], ph = s_phi[i2];
                                const float d = ph < rg.x ? rg.x - ph : (pl > rg.y ? pl - rg.y : 0.f);
                                sum += mseg * (d * d);
                            }
                        }
                        keep = !(sum * (1.0f - kRhoLb) > U);
                        ++c_wordb;
                    }
                    const uint64_t bal = __ballot(keep);
                    if (keep) list[n2 + __popcll(bal & lt_mask)] = gi[t];
                    n2 += (uint32_t)__popcll(bal);
                }
            }
            dev::wave_sync();
            // ---- fine: 4 lanes per series, 16 series per round, kFineIssue
            // rounds in flight
            constexpr int kFineIssue = 4;
            uint32_t n3 = n2;
            // with at most half a list of word survivors, each fine survivor's
            // bound is kept in the list's upper half (for the best-first rows)
            const bool keep_lb = fine && n2 <= (uint32_t)(kFlatList / 2);
            float* llb = reinterpret_cast<float*>(list + kFlatList / 2);
            if (fine && n2) {
                n3 = 0;
                const int g4 = lane >> 2, l4 = lane & 3;
                const float mfine = (float)a.mf;
                const bool part = l4 * 16 < a.wf;
                for (uint32_t e0 = 0; e0 < n2; e0 += 16 * kFineIssue) {
                    uint4 fv[kFineIssue];
                    uint32_t gx[kFineIssue];
#pragma unroll
                    for (int t = 0; t < kFineIssue; ++t) {
                        const uint32_t e = e0 + (uint32_t)t * 16 + g4;
                        fv[t] = make_uint4(0u, 0u, 0u, 0u);
                        gx[t] = 0;
                        if (e < n2) {
                            gx[t] = list[e];
                            if (part)
                                fv[t] = *reinterpret_cast<const uint4*>(a.fwords + (size_t)gx[t] * kFineStride +
                                                                        l4 * 16);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < kFineIssue; ++t) {
                        if (e0 + (uint32_t)t * 16 >= n2) break;  // the rest of the batch is empty
                        const uint32_t e = e0 + (uint32_t)t * 16 + g4;
                        const bool act = e < n2;
                        float acc = 0.f;
#pragma unroll
                        for (int tt = 0; tt < 16; ++tt) {
                            const int jf = l4 * 16 + tt;
                            if (jf < a.wf) {
                                const float2 rg = s_rf[word_byte(fv[t], tt)];
                                const float pv = s_pf[jf];
                                const float d = pv < rg.x ? rg.x - pv : (pv > rg.y ? pv - rg.y : 0.f);
                                acc = fmaf(d, d, acc);
                            }
                        }
                        acc += __shfl_xor(acc, 1, 4);
                        acc += __shfl_xor(acc, 2, 4);
                        const float lbf = acc * mfine;
                        const bool keep = act && l4 == 0 && !(lbf * (1.0f - kRhoLb) > U);
                        if (act && l4 == 0) ++c_fine;
                        const uint64_t bal = __ballot(keep);
                        if (keep) {
                            const uint32_t o = n3 + (uint32_t)__popcll(bal & lt_mask);
                            list[o] = gx[t];
                            if (keep_lb) llb[o] = lbf;
                        }
                        n3 += (uint32_t)__popcll(bal);
                    }
                }
                dev::wave_sync();
            }
            // ---- distances: 16 lanes per row, 4 rows per round; U stays one
            // value across the wave (a row's 16 lanes must agree on abandoning)
            uint32_t appended = 0;
            auto rows = [&](uint32_t eb, uint32_t ee) {
            for (uint32_t e0 = eb; e0 < ee; e0 += 4) {
                float Unew = U;
                const uint32_t e = e0 + quarter;
                const bool act = e < ee;
                const uint32_t gidx = act ? list[e] : 0u;
                bool alive = act;
                const float* row = a.series + (size_t)gidx * L;
                float acc = 0.f;
                for (int g = 0; g < nchunk; g += 4) {
                    if (alive) {
                        if (VEC) {
                            float4 x[4];
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
                                const int j0 = (g + cc) * 64 + ql * 4;
                                x[cc] = (g + cc < nchunk && j0 < L) ? *reinterpret_cast<const float4*>(row + j0)
                                                                    : make_float4(0.f, 0.f, 0.f, 0.f);
                            }
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
                                const int j0 = (g + cc) * 64 + ql * 4;
                                if (g + cc < nchunk && j0 < L) {
                                    const float4 y = *reinterpret_cast<const float4*>(s_q + j0);
                                    const float d0 = y.x - x[cc].x, d1 = y.y - x[cc].y;
                                    const float d2 = y.z - x[cc].z, d3 = y.w - x[cc].w;
                                    acc = fmaf(d0, d0, acc);
                                    acc = fmaf(d1, d1, acc);
                                    acc = fmaf(d2, d2, acc);
                                    acc = fmaf(d3, d3, acc);
                                }
                            }
                        } else {
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
                                for (int e2 = 0; e2 < 4; ++e2) {
                                    const int jj = (g + cc) * 64 + ql * 4 + e2;
                                    if (g + cc < nchunk && jj < L) {
                                        const float d = s_q[jj] - row[jj];
                                        acc = fmaf(d, d, acc);
                                    }
                                }
                            }
                        }
                    }
                    float pp = acc;
                    pp += __shfl_xor(pp, 8, 16);
                    pp += __shfl_xor(pp, 4, 16);
                    pp += __shfl_xor(pp, 2, 16);
                    pp += __shfl_xor(pp, 1, 16);
                    pp = __shfl(pp, quarter * 16, 64);
                    if (alive && ql == 0) c_rowb += (uint64_t)min(4, nchunk - g) * 256u;
                    if (g + 4 < nchunk) {
                        if (alive && pp * (1.0f - kRhoEd) > U) {
                            alive = false;
                            if (ql == 0) ++c_abandon;
                        }
                    } else {
                        acc = pp;  // the full distance
                    }
                }
                if (act && ql == 0) ++c_dist;
                if (alive && ql == 0 && acc * (1.0f - kRhoEd) <= U) {
                    const float d = acc;
                    const uint32_t slot = atomicAdd(&st.ncand, 1u);
                    if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{d, gidx};
                    else st.ovf = 1;
                    ++appended;
                    if (k == 1) {
                        const uint32_t ub = __float_as_uint(upper_u(d));
                        atomicMin(&st.U, ub);
                        Unew = fminf(Unew, __uint_as_float(ub));
                    } else {
                        atomicAdd(&a.hist[(size_t)q * kHistBins + hist_bin(d, st.hbase)], 1u);
                    }
                }
                for (int off = 32; off >= 1; off >>= 1) Unew = fminf(Unew, __shfl_xor(Unew, off));
                U = Unew;
            }
            };
            if (keep_lb && k == 1 && n3 > 4) {
                // Best first: the series of smallest fine bound alone (the fine
                // bound is close to the distance, so that row usually sets U
                // near its final value), then the others that its U leaves.
                float bl = __uint_as_float(0x7f800000u);
                uint32_t be = 0;
                for (uint32_t e = lane; e < n3; e += 64)
                    if (llb[e] < bl) {
                        bl = llb[e];
                        be = e;
                    }
                for (int off = 32; off >= 1; off >>= 1) {
                    const float ob = __shfl_xor(bl, off);
                    const uint32_t oe = __shfl_xor(be, off);
                    if (ob < bl || (ob == bl && oe < be)) {
                        bl = ob;
                        be = oe;
                    }
                }
                dev::wave_sync();
                if (lane == 0) {
                    const uint32_t t0 = list[0];
                    const float f0 = llb[0];
                    list[0] = list[be];
                    llb[0] = llb[be];
                    list[be] = t0;
                    llb[be] = f0;
                }
                dev::wave_sync();
                rows(0, 1);
                uint32_t nk = 0;
                for (uint32_t e0 = 1; e0 < n3; e0 += 64) {
                    const uint32_t e = e0 + lane;
                    uint32_t gv = 0;
                    float fv = 0.f;
                    bool keep = false;
                    if (e < n3) {
                        gv = list[e];
                        fv = llb[e];
                        keep = !(fv * (1.0f - kRhoLb) > U);
                    }
                    const uint64_t bal = __ballot(keep);
                    if (keep) {
                        const uint32_t o = nk + (uint32_t)__popcll(bal & lt_mask);
                        list[o] = gv;
                        llb[o] = fv;
                    }
                    nk += (uint32_t)__popcll(bal);
                }
                dev::wave_sync();
                rows(0, nk);
            } else {
                rows(0, n3);
            }
            if (k > 1 && __ballot(appended != 0)) wave_hist_refresh(a, q, st, U);
            dev::wave_sync();  // the list is refilled by the next chunk
        }
        __syncthreads();  // the tables are rebuilt for the block's next query
    }
    if (timing && tid == 0 && (pass == 0 || worked)) {
        unsigned long long* pr = a.prof + (size_t)blockIdx.x * 4;
        const unsigned long long v[4] = {0ull, 0ull, 0ull, wall_clock64() - s_t0};
        const bool first = pass == 0 && a.chunk_lo == 0;
        for (int i = 0; i < 4; ++i) pr[i] = (first ? 0ull : pr[i]) + v[i];
    }
    if (a.blk_cnt) {
        __shared__ unsigned long long s_cnt[kWaves][kBlkCnt];
        const unsigned long long fine_b = 16ull * (unsigned long long)((a.wf + 15) / 16);
        unsigned long long v[kBlkCnt] = {c_scanned, c_bounded, c_dist, c_abandon,
                                         c_rowb + (unsigned long long)c_bounded * 8ull +
                                             (unsigned long long)c_wordb * 20ull +
                                             (unsigned long long)c_fine * fine_b,
                                         0ull, 0ull, c_wordb, c_fine};
        for (int i = 0; i < kBlkCnt; ++i)
            for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off);
        if (lane == 0)
            for (int i = 0; i < kBlkCnt; ++i) s_cnt[wave][i] = v[i];
        __syncthreads();
        if (tid < kBlkCnt && (pass == 0 || worked)) {
            unsigned long long t = 0;
            for (int w2 = 0; w2 < kWaves; ++w2) t += s_cnt[w2][tid];
            unsigned long long* pp = a.blk_cnt + (size_t)blockIdx.x * kBlkCnt + tid;
            *pp = (pass == 0 && a.chunk_lo == 0 ? 0ull : *pp) + t;
        }
    }
}


// ---- the split Euclidean scan -------------------------------------------------
// For calls of few queries the flat scan runs as two kernels.  The first
// streams the coarse words (8 bytes per member) and bounds them; it is light
// on registers, so more of its waves fit a CU and more member reads are in
// flight.  It stores the coarse survivors (member positions) of chunk c at
// the chunk's own place in a[q].seg (a chunk's members at most, so it cannot
// overflow) and their count in segcnt.  The second takes the survivors of a
// block's chunks as one list: their words and series indices (read together,
// 64 per wave and round) and the word bound, the fine bound of the word
// survivors (4 lanes per series), then distances; a heavy chunk's survivors
// are shared by the block's waves.  U comes from the first bound (and, in
// the second kernel, from the distances as they are found).

// Block-wide: the query's coarse table and word regions (as the flat scan's).
__device__ void coarse_word_tables(const QArgs& a, const QState& st, float* s_bp, float* s_plo, float* s_phi,
                                   float2* s_rb, float* s_C) {
    const int tid = threadIdx.x;
    const int A = 1 << a.b;
    const float inf = __uint_as_float(0x7f800000u);
    for (int c = tid; c < A - 1; c += blockDim.x) s_bp[c] = a.bp[c];
    if (tid < 16) {
        s_plo[tid] = st.paa[tid];
        s_phi[tid] = st.paa_hi[tid];
    }
    const float delta = st.delta;
    __syncthreads();
    const float mf = (float)a.m;
    for (int c = tid; c < A; c += blockDim.x)
        s_rb[c] = make_float2(c > 0 ? s_bp[c - 1] - delta : -inf, c < A - 1 ? s_bp[c] + delta : inf);
    for (int idx = tid; idx < 8 * 256; idx += blockDim.x) {
        const int j2 = idx >> 8, byte = idx & 255;
        float t = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * j2 + h;
            const int c = h == 0 ? byte >> 4 : byte & 15;
            if (i < a.w) {
                const int s0 = c << a.csh, s1 = (c + 1) << a.csh;
                const float pl = s_plo[i], ph = s_phi[i];
                float d = 0.f;
                if (s0 > 0 && s0 < A) {
                    const float lo = s_bp[s0 - 1] - delta;
                    if (ph < lo) d = lo - ph;
                }
                if (s1 < A) {
                    const float hi = s_bp[s1 - 1] + delta;
                    if (pl > hi) d = pl - hi;
                }
                t += mf * (d * d);
            }
        }
        s_C[idx] = t;
    }
    __syncthreads();
}

// The occupancy request of 6 is not met (LDS allows five blocks per CU), but
// it makes the register allocator stay at 99 VGPRs with no spills; that ran
// 0.123 ms per query against 0.137 ms with a request of 5 (96 VGPRs and
// three spilled) and 0.133 ms with 4 (117 VGPRs).
template <int pass>
__global__ void __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(6)))
flat_coarse_kernel(QArgs a) {
    __shared__ float s_C[8 * 256];
    __shared__ float2 s_rb[256];
    __shared__ float s_plo[16], s_phi[16];
    __shared__ float s_bp[256];
    __shared__ OrdRec s_rec[kScanThreads / 64][64];
    __shared__ uint32_t s_flag;
    constexpr int kWaves = kScanThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = dev::lanemask_lt();
    OrdRec* wrec = s_rec[wave];
    const int nq = a.nq;
    const int B = gridDim.x;
    // one query per block (the host runs the split scan only for nq <= blocks)
    const int q = blockIdx.x % nq;
    const int j = blockIdx.x / nq;
    const int G = (B - q + nq - 1) / nq;
    uint32_t c_scanned = 0, c_bounded = 0, c_wordb = 0;
    QState& st = a.qs[q];
    if (tid == 0) s_flag = (st.err != 0 || st.nsurv == 0 || (pass == 1 && st.rerun == 0)) ? 1u : 0u;
    __syncthreads();
    const bool skip = s_flag != 0;
    __syncthreads();
    if (!skip) {
        const uint32_t nsurv = st.nsurv;
        const uint64_t nmemb = st.nmemb;
        const float range = st.range;
        // (this round's chunks: [chunk_lo, nch))
        const uint64_t nch = min(min((nmemb + a.chunk - 1) / a.chunk, (uint64_t)a.max_chunks), (uint64_t)a.chunk_hi);
        coarse_word_tables(a, st, s_bp, s_plo, s_phi, s_rb, s_C);
        const uint32_t* cfq = a.chunk_first + (size_t)q * a.max_chunks;
        const OrdRec* recq = a.rec + (size_t)q * a.nL;
        uint32_t* segq = a.seg + (size_t)q * a.max_chunks * a.chunk;
        uint32_t* cntq = a.segcnt + (size_t)q * a.max_chunks;
        const uint64_t WG = (uint64_t)G * kWaves;
        const float U = __uint_as_float(vload(&st.U));
        const uint32_t skip = st.skip_start;
        const uint64_t wi = (uint64_t)j * kWaves + wave;
        auto chunk_of = [&](uint64_t t) -> uint64_t {
            return (uint64_t)a.chunk_lo + t * WG + ((t & 1) ? WG - 1 - wi : wi);
        };
        uint64_t rt = 0;
        uint64_t c = chunk_of(0);
        uint32_t tw_n = c < nch ? cfq[c] : 0u;
        OrdRec r_n{0u, 0u, 0.f, 0xffffffffu};
        if (c < nch && tw_n + lane < nsurv) r_n = recq[tw_n + lane];
        bool stopped = false;  // this wave's later chunks lie beyond U: their counts are 0
        for (; (uint64_t)a.chunk_lo + rt * WG < nch; c = chunk_of(++rt)) {
            if (c >= nch) continue;
            if (stopped) {
                if (lane == 0) cntq[c] = 0;
                continue;
            }
            const uint32_t cbeg = (uint32_t)(c * a.chunk);
            const uint32_t cend = (uint32_t)min(c * a.chunk + a.chunk, nmemb);
            uint32_t tw = tw_n;
            OrdRec r = r_n;
            const uint64_t cn = chunk_of(rt + 1);
            if (cn < nch) tw_n = cfq[cn];
            // the chunk's coarse survivors (member positions) go straight to
            // its segment: at most a.chunk of them, so it cannot overflow
            uint32_t n1 = 0;
            uint32_t* segc = segq + (size_t)c * a.chunk;
            // ---- coarse: a window of up to 64 of the chunk's leaves at a time
            for (bool first = true;; first = false) {
                if (!first) {
                    r = OrdRec{0u, 0u, 0.f, 0xffffffffu};
                    if (tw + lane < nsurv) r = recq[tw + lane];
                }
                const bool rin = tw + lane < nsurv && r.moff < cend;
                const uint32_t nin = (uint32_t)__popcll(__ballot(rin));
                wrec[lane] = r;
                dev::wave_sync();
                if (first) {
                    const float lb0 = wrec[0].lb;
                    const float low = (float)bin_of(lb0, range) * (range / (float)kNB);
                    if (lb0 * (1.0f - kRhoLb) > U && low * (1.0f - 2.0f * kRhoLb) > U) {
                        stopped = true;
                        break;
                    }
                }
                if (pass == 0 && r.start == skip) {
                    // the first bound's leaf: its candidates are in already
                    r.lb = __uint_as_float(0x7f800000u);
                    wrec[lane].lb = r.lb;
                }
                dev::wave_sync();
                if (rin && r.moff >= cbeg && !(r.lb * (1.0f - kRhoLb) > U)) ++c_scanned;
                const uint32_t wb = max(cbeg, wrec[0].moff);
                const OrdRec rl = wrec[nin - 1];
                const uint32_t we = (uint32_t)min((uint64_t)cend, (uint64_t)rl.moff + (uint64_t)rl.count);
                const bool few = nin <= 4;
                uint32_t e_s[4], b_s[4];
                float l_s[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    e_s[t] = (uint32_t)__builtin_amdgcn_readlane((int)(r.moff + r.count), t);
                    b_s[t] = (uint32_t)__builtin_amdgcn_readlane((int)(r.start - r.moff), t);
                    l_s[t] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.lb), t));
                }
                int p = 0;
                for (uint32_t g0 = wb; g0 < we; g0 += 64 * kFlatIssue) {
                    uint2 cw[kFlatIssue];
                    uint32_t mpv[kFlatIssue];
                    uint32_t live = 0;
#pragma unroll
                    for (int i = 0; i < kFlatIssue; ++i) {
                        const uint32_t g = g0 + (uint32_t)i * 64 + lane;
                        cw[i] = make_uint2(0u, 0u);
                        mpv[i] = 0;
                        if (g < we) {
                            uint32_t bs;
                            float lbv;
                            if (few) {
                                bs = b_s[0];
                                lbv = l_s[0];
#pragma unroll
                                for (int t = 1; t < 4; ++t)
                                    if (t < (int)nin && g >= e_s[t - 1]) {
                                        bs = b_s[t];
                                        lbv = l_s[t];
                                    }
                            } else {
                                while (p + 1 < (int)nin && wrec[p + 1].moff <= g) ++p;
                                const OrdRec rp = wrec[p];
                                bs = rp.start - rp.moff;
                                lbv = rp.lb;
                            }
                            if (!(lbv * (1.0f - kRhoLb) > U)) {
                                live |= 1u << i;
                                mpv[i] = bs + g;
                                cw[i] = a.cwords[mpv[i]];
                            }
                        }
                    }
                    if (first && g0 == wb) {
                        r_n = OrdRec{0u, 0u, 0.f, 0xffffffffu};
                        if (cn < nch && tw_n + lane < nsurv) r_n = recq[tw_n + lane];
                    }
#pragma unroll
                    for (int i = 0; i < kFlatIssue; ++i) {
                        bool keep = false;
                        if (live & (1u << i)) {
                            float sum = 0.f;
#pragma unroll
                            for (int j2 = 0; j2 < 8; ++j2) {
                                const uint32_t half = j2 < 4 ? cw[i].x : cw[i].y;
                                sum += s_C[j2 * 256 + ((half >> (8 * (j2 & 3))) & 255u)];
                            }
                            keep = !(sum * (1.0f - kRhoLb) > U);
                            ++c_bounded;
                        }
                        const uint64_t bal = __ballot(keep);
                        if (keep) segc[n1 + __popcll(bal & lt_mask)] = mpv[i];
                        n1 += (uint32_t)__popcll(bal);
                    }
                }
                if (nin < 64 || we >= cend) break;
                tw += 64;
                dev::wave_sync();
            }
            if (stopped) {
                if (lane == 0) cntq[c] = 0;
                continue;
            }
            if (lane == 0) cntq[c] = n1;
        }
    }
    if (a.blk_cnt) {
        __shared__ unsigned long long s_cnt[kWaves][3];
        unsigned long long v[3] = {c_scanned, c_bounded, c_wordb};
        for (int i = 0; i < 3; ++i)
            for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off);
        if (lane == 0)
            for (int i = 0; i < 3; ++i) s_cnt[wave][i] = v[i];
        __syncthreads();
        if (tid < kBlkCnt) {
            // slots of the statistics: scanned, coarse-bounded, word-bounded (0 here: the
            // refine kernel adds it), bytes (8 per coarse word)
            unsigned long long t = 0;
            if (tid == 0 || tid == 1 || tid == 4 || tid == 7)
                for (int w2 = 0; w2 < kWaves; ++w2) {
                    const unsigned long long sc = s_cnt[w2][0], cb = s_cnt[w2][1], wbn = s_cnt[w2][2];
                    t += tid == 0 ? sc : tid == 1 ? cb : tid == 7 ? wbn : cb * 8ull + wbn * 20ull;
                }
            unsigned long long* pp = a.blk_cnt + (size_t)blockIdx.x * kBlkCnt + tid;
            *pp = (pass == 0 && a.chunk_lo == 0 ? 0ull : *pp) + t;
        }
    }
}

// One wave's distances for the series list[eb, ee) (16 lanes per row, 4 rows
// per round; U one value across the wave): k = 1 lowers U with each
// distance; k > 1 appends to the candidate buffer and the histogram.
template <bool VEC>
__device__ void wave_rows(const QArgs& a, QState& st, int q, int k, const uint32_t* list, uint32_t eb, uint32_t ee,
                          const float* s_q, float& U, uint32_t& appended, uint32_t& c_dist, uint32_t& c_abandon,
                          unsigned long long& c_rowb) {
    const int lane = threadIdx.x & 63;
    const int quarter = lane >> 4, ql = lane & 15;
    const int L = a.L;
    const int nchunk = (L + 63) / 64;
    for (uint32_t e0 = eb; e0 < ee; e0 += 4) {
        float Unew = U;
        const uint32_t e = e0 + quarter;
        const bool act = e < ee;
        const uint32_t gidx = act ? list[e] : 0u;
        bool alive = act;
        const float* row = a.series + (size_t)gidx * L;
        float acc = 0.f;
        for (int g = 0; g < nchunk; g += 4) {
            if (alive) {
                if (VEC) {
                    float4 x[4];
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) {
                        const int j0 = (g + cc) * 64 + ql * 4;
                        x[cc] = (g + cc < nchunk && j0 < L) ? *reinterpret_cast<const float4*>(row + j0)
                                                            : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) {
                        const int j0 = (g + cc) * 64 + ql * 4;
                        if (g + cc < nchunk && j0 < L) {
                            const float4 y = *reinterpret_cast<const float4*>(s_q + j0);
                            const float d0 = y.x - x[cc].x, d1 = y.y - x[cc].y;
                            const float d2 = y.z - x[cc].z, d3 = y.w - x[cc].w;
                            acc = fmaf(d0, d0, acc);
                            acc = fmaf(d1, d1, acc);
                            acc = fmaf(d2, d2, acc);
                            acc = fmaf(d3, d3, acc);
                        }
                    }
                } else {
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
                        for (int e2 = 0; e2 < 4; ++e2) {
                            const int jj = (g + cc) * 64 + ql * 4 + e2;
                            if (g + cc < nchunk && jj < L) {
                                const float d = s_q[jj] - row[jj];
                                acc = fmaf(d, d, acc);
                            }
                        }
                    }
                }
            }
            float pp = acc;
            pp += __shfl_xor(pp, 8, 16);
            pp += __shfl_xor(pp, 4, 16);
            pp += __shfl_xor(pp, 2, 16);
            pp += __shfl_xor(pp, 1, 16);
            pp = __shfl(pp, quarter * 16, 64);
            if (alive && ql == 0) c_rowb += (uint64_t)min(4, nchunk - g) * 256u;
            if (g + 4 < nchunk) {
                if (alive && pp * (1.0f - kRhoEd) > U) {
                    alive = false;
                    if (ql == 0) ++c_abandon;
                }
            } else {
                acc = pp;  // the full distance
            }
        }
        if (act && ql == 0) ++c_dist;
        if (alive && ql == 0 && acc * (1.0f - kRhoEd) <= U) {
            const float d = acc;
            const uint32_t slot = atomicAdd(&st.ncand, 1u);
            if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{d, gidx};
            else st.ovf = 1;
            ++appended;
            if (k == 1) {
                const uint32_t ub = __float_as_uint(upper_u(d));
                atomicMin(&st.U, ub);
                Unew = fminf(Unew, __uint_as_float(ub));
            } else {
                atomicAdd(&a.hist[(size_t)q * kHistBins + hist_bin(d, st.hbase)], 1u);
            }
        }
        for (int off = 32; off >= 1; off >>= 1) Unew = fminf(Unew, __shfl_xor(Unew, off));
        U = Unew;
    }
}

constexpr int kRefineList = 512;  // fine survivors a wave holds before it computes their distances
constexpr int kWordList = 512;    // word survivors a wave holds before it bounds their fine summaries

template <bool VEC, int pass>
__global__ void __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4)))
flat_refine_kernel(QArgs a) {
    __shared__ float2 s_rf[256];
    __shared__ float2 s_rb[256];
    __shared__ float s_plo[16], s_phi[16];
    __shared__ float s_pf[64];
    __shared__ float s_bp[256];
    __shared__ uint32_t s_wl[kScanThreads / 64][kWordList];
    __shared__ __align__(16) float s_q[MESSI_MAX_LEN];
    __shared__ uint32_t s_cpre[kScanThreads + 1];  // exclusive prefix of the survivor counts of a batch of chunks
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_list[kScanThreads / 64][kRefineList];
    __shared__ float s_llb[kScanThreads / 64][kRefineList];
    __shared__ uint32_t s_flag;
    constexpr int kWaves = kScanThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = dev::lanemask_lt();
    uint32_t* list = s_list[wave];
    float* llb = s_llb[wave];
    uint32_t* wl = s_wl[wave];
    const int nq = a.nq;
    const int B = gridDim.x;
    const int q = blockIdx.x % nq;
    const int j = blockIdx.x / nq;
    const int G = (B - q + nq - 1) / nq;
    const int L = a.L;
    uint32_t c_dist = 0, c_abandon = 0, c_fine = 0, c_wordb = 0;
    unsigned long long c_rowb = 0;
    QState& st = a.qs[q];
    if (tid == 0) s_flag = (st.err != 0 || st.nsurv == 0 || (pass == 1 && st.rerun == 0)) ? 1u : 0u;
    __syncthreads();
    const bool skip = s_flag != 0;
    __syncthreads();
    if (!skip) {
        const int k = st.k;
        const uint64_t nmemb = st.nmemb;
        const uint64_t nch = min(min((nmemb + a.chunk - 1) / a.chunk, (uint64_t)a.max_chunks), (uint64_t)a.chunk_hi);
        const bool fine = a.fwords != nullptr;
        const int A = 1 << a.b;
        const float inf = __uint_as_float(0x7f800000u);
        for (int c = tid; c < A - 1; c += kScanThreads) s_bp[c] = a.bp[c];
        for (int jj = tid; jj < L; jj += kScanThreads) s_q[jj] = a.queries[(size_t)q * L + jj];
        if (tid < 16) {
            s_plo[tid] = st.paa[tid];
            s_phi[tid] = st.paa_hi[tid];
        }
        const float qamax = st.qamax;
        const float delta = st.delta;
        __syncthreads();
        // each symbol's region widened by the query's delta (the word bound)
        for (int c = tid; c < A; c += kScanThreads)
            s_rb[c] = make_float2(c > 0 ? s_bp[c - 1] - delta : -inf, c < A - 1 ? s_bp[c] + delta : inf);
        if (fine) {
            // the fine regions, widened by the fp32 error of a fine PAA value of
            // data and query, and the query's fine PAA
            const float u = 5.9604644775390625e-08f;  // 2^-24
            const float df = 1.01f * (2.f * (float)(a.lg_mf + 1) * u * a.absmax_data +
                                      2.f * (float)(a.mf + 1) * u * qamax) + kFineCodeSlack;
            for (int c = tid; c < 256; c += kScanThreads)
                s_rf[c] = make_float2(c > 0 ? (float)c * 0.03125f - 4.0f - df : -inf, c < 255 ? (float)(c + 1) * 0.03125f - 4.0f + df : inf);
            for (int jj = tid; jj < a.wf; jj += kScanThreads) {
                float sum = 0.f;
                for (int i = 0; i < a.mf; ++i) sum += s_q[jj * a.mf + i];
                s_pf[jj] = sum / (float)a.mf;
            }
        }
        __syncthreads();
        const uint32_t* segq = a.seg + (size_t)q * a.max_chunks * a.chunk;
        const uint32_t* cntq = a.segcnt + (size_t)q * a.max_chunks;
        float U = __uint_as_float(vload(&st.U));
        uint32_t n3 = 0, appended = 0;
        // the distances of the wave's list, best first for k = 1
        auto flush = [&]() {
            U = fminf(U, __uint_as_float(vload(&st.U)));  // other waves' distances
            if (n3 > 4 && k == 1) {
                float bl = inf;
                uint32_t be = 0;
                for (uint32_t e = lane; e < n3; e += 64)
                    if (llb[e] < bl) {
                        bl = llb[e];
                        be = e;
                    }
                for (int off = 32; off >= 1; off >>= 1) {
                    const float ob = __shfl_xor(bl, off);
                    const uint32_t oe = __shfl_xor(be, off);
                    if (ob < bl || (ob == bl && oe < be)) {
                        bl = ob;
                        be = oe;
                    }
                }
                dev::wave_sync();
                if (lane == 0) {
                    const uint32_t t0 = list[0];
                    const float f0 = llb[0];
                    list[0] = list[be];
                    llb[0] = llb[be];
                    list[be] = t0;
                    llb[be] = f0;
                }
                dev::wave_sync();
                wave_rows<VEC>(a, st, q, k, list, 0, 1, s_q, U, appended, c_dist, c_abandon, c_rowb);
                uint32_t nk = 0;
                for (uint32_t e0 = 1; e0 < n3; e0 += 64) {
                    const uint32_t e = e0 + lane;
                    uint32_t gv = 0;
                    float fv = 0.f;
                    bool keep = false;
                    if (e < n3) {
                        gv = list[e];
                        fv = llb[e];
                        keep = !(fv * (1.0f - kRhoLb) > U);
                    }
                    const uint64_t bal = __ballot(keep);
                    if (keep) {
                        const uint32_t o = nk + (uint32_t)__popcll(bal & lt_mask);
                        list[o] = gv;
                        llb[o] = fv;
                    }
                    nk += (uint32_t)__popcll(bal);
                }
                dev::wave_sync();
                wave_rows<VEC>(a, st, q, k, list, 0, nk, s_q, U, appended, c_dist, c_abandon, c_rowb);
            } else {
                wave_rows<VEC>(a, st, q, k, list, 0, n3, s_q, U, appended, c_dist, c_abandon, c_rowb);
            }
            n3 = 0;
            dev::wave_sync();
        };
        // this block's chunks of the round, chunk_lo + j, + G, ..., kScanThreads of them at a time
        const uint64_t j0 = (uint64_t)a.chunk_lo + (uint64_t)j;
        for (uint64_t cb = 0; j0 + cb * G < nch; cb += kScanThreads) {
            const uint64_t cme = j0 + (cb + tid) * G;
            const uint32_t cnt = cme < nch ? cntq[cme] : 0u;
            uint32_t total;
            const uint32_t ex = block_exclusive_scan(cnt, s_tmp, total);
            s_cpre[tid] = ex;
            if (tid == 0) s_cpre[kScanThreads] = total;
            __syncthreads();
            // survivor e of the batch: chunk (largest i with s_cpre[i] <= e) and place in it
            auto entry = [&](uint32_t e) -> uint32_t {
                int lo = 0, hi = kScanThreads - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_cpre[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                const uint64_t cc = j0 + (cb + (uint64_t)lo) * G;
                return segq[cc * a.chunk + (e - s_cpre[lo])];
            };
            // the fine bounds of the wave's word survivors wl[0, nw) (4 lanes per
            // series, 16 series per wave and round); fine survivors to the list
            auto fine_stage = [&](uint32_t nw) {
                constexpr int kFineIssue = 2;
                const int g4 = lane >> 2, l4 = lane & 3;
                const float mfine = (float)a.mf;
                const bool part = l4 * 16 < a.wf;
                dev::wave_sync();
                for (uint32_t e0 = 0; e0 < nw; e0 += 16 * kFineIssue) {
                    uint4 fv[kFineIssue];
                    uint32_t gx[kFineIssue];
#pragma unroll
                    for (int t = 0; t < kFineIssue; ++t) {
                        const uint32_t e = e0 + (uint32_t)t * 16 + g4;
                        gx[t] = e < nw ? wl[e] : 0u;
                        fv[t] = make_uint4(0u, 0u, 0u, 0u);
                        if (e < nw && part)
                            fv[t] = *reinterpret_cast<const uint4*>(a.fwords + (size_t)gx[t] * kFineStride + l4 * 16);
                    }
#pragma unroll
                    for (int t = 0; t < kFineIssue; ++t) {
                        if (e0 + (uint32_t)t * 16 >= nw) break;
                        const uint32_t e = e0 + (uint32_t)t * 16 + g4;
                        const bool act = e < nw;
                        float acc = 0.f;
#pragma unroll
                        for (int tt = 0; tt < 16; ++tt) {
                            const int jf = l4 * 16 + tt;
                            if (jf < a.wf) {
                                const float2 rg = s_rf[word_byte(fv[t], tt)];
                                const float pv = s_pf[jf];
                                const float d = pv < rg.x ? rg.x - pv : (pv > rg.y ? pv - rg.y : 0.f);
                                acc = fmaf(d, d, acc);
                            }
                        }
                        acc += __shfl_xor(acc, 1, 4);
                        acc += __shfl_xor(acc, 2, 4);
                        const float lbf = acc * mfine;
                        const bool keep = act && l4 == 0 && !(lbf * (1.0f - kRhoLb) > U);
                        if (act && l4 == 0) ++c_fine;
                        const uint64_t bal = __ballot(keep);
                        if (keep) {
                            const uint32_t o = n3 + (uint32_t)__popcll(bal & lt_mask);
                            list[o] = gx[t];
                            llb[o] = lbf;
                        }
                        n3 += (uint32_t)__popcll(bal);
                    }
                    if (n3 > (uint32_t)(kRefineList - 16 * kFineIssue)) {
                        dev::wave_sync();
                        flush();
                    }
                }
                dev::wave_sync();
            };
            // the coarse survivors' words and series indices, read together, and
            // the word bound; word survivors to wl (or, without a fine summary,
            // straight to the distance list)
            const float mseg = (float)a.m;
            uint32_t nw = 0;
            for (uint32_t e0 = (uint32_t)wave * 64 * kWordIssue; e0 < total; e0 += kWaves * 64 * kWordIssue) {
                uint4 wd[kWordIssue];
                uint32_t gi[kWordIssue];
#pragma unroll
                for (int t = 0; t < kWordIssue; ++t) {
                    const uint32_t e = e0 + (uint32_t)t * 64 + lane;
                    wd[t] = make_uint4(0u, 0u, 0u, 0u);
                    gi[t] = 0;
                    if (e < total) {
                        const uint32_t mp = entry(e);
                        wd[t] = a.words[mp];
                        gi[t] = a.pos[mp];
                    }
                }
#pragma unroll
                for (int t = 0; t < kWordIssue; ++t) {
                    const uint32_t e = e0 + (uint32_t)t * 64 + lane;
                    bool keep = false;
                    if (e < total) {
                        float sum = 0.f;
#pragma unroll
                        for (int i2 = 0; i2 < 16; ++i2) {
                            if (i2 < a.w) {
                                const float2 rg = s_rb[word_byte(wd[t], i2)];
                                const float pl = s_plo[i2], ph = s_phi[i2];
                                const float d = ph < rg.x ? rg.x - ph : (pl > rg.y ? pl - rg.y : 0.f);
                                sum += mseg * (d * d);
                            }
                        }
                        keep = !(sum * (1.0f - kRhoLb) > U);
                        ++c_wordb;
                    }
                    const uint64_t bal = __ballot(keep);
                    if (fine) {
                        if (keep) wl[nw + (uint32_t)__popcll(bal & lt_mask)] = gi[t];
                        nw += (uint32_t)__popcll(bal);
                    } else {
                        if (keep) {
                            const uint32_t o = n3 + (uint32_t)__popcll(bal & lt_mask);
                            list[o] = gi[t];
                            llb[o] = 0.f;
                        }
                        n3 += (uint32_t)__popcll(bal);
                    }
                }
                if (fine && nw > (uint32_t)(kWordList - 64 * kWordIssue)) {
                    fine_stage(nw);
                    nw = 0;
                }
                if (!fine && n3 > (uint32_t)(kRefineList - 64 * kWordIssue)) {
                    dev::wave_sync();
                    flush();
                }
            }
            if (fine && nw) fine_stage(nw);
            __syncthreads();  // every wave is done with this batch's prefix sums
        }
        dev::wave_sync();
        if (n3) flush();
        if (k > 1 && __ballot(appended != 0)) wave_hist_refresh(a, q, st, U);
    }
    if (a.blk_cnt) {
        __shared__ unsigned long long s_cnt[kWaves][5];
        const unsigned long long fine_b = 16ull * (unsigned long long)((a.wf + 15) / 16);
        unsigned long long v[5] = {c_dist, c_abandon, c_fine, c_rowb, c_wordb};
        for (int i = 0; i < 5; ++i)
            for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off);
        if (lane == 0)
            for (int i = 0; i < 5; ++i) s_cnt[wave][i] = v[i];
        __syncthreads();
        if (tid < kBlkCnt && (tid == 2 || tid == 3 || tid == 4 || tid == 7 || tid == 8)) {
            // added to the coarse kernel's slots: distances, abandoned, bytes (rows, fine
            // summaries, words and series indices), word-bounded, fine-bounded
            unsigned long long t = 0;
            for (int w2 = 0; w2 < kWaves; ++w2)
                t += tid == 2 ? s_cnt[w2][0] : tid == 3 ? s_cnt[w2][1] : tid == 8 ? s_cnt[w2][2]
                   : tid == 7 ? s_cnt[w2][4]
                              : s_cnt[w2][3] + s_cnt[w2][2] * fine_b + s_cnt[w2][4] * 20ull;
            unsigned long long* pp = a.blk_cnt + (size_t)blockIdx.x * kBlkCnt + tid;
            *pp = (tid == 4 || a.chunk_lo != 0 ? *pp : (pass == 0 ? 0ull : *pp)) + t;
        }
    }
}

// Every query's own status (QState::err) for the caller.
__global__ void status_kernel(QArgs a, uint32_t* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.nq) out[q] = a.qs[q].err;
}

// --------------------------------------------------------------------------
// final: canonical fp64 distance of the candidates within U, ordered by (D, idx)
// --------------------------------------------------------------------------
// --------------------------------------------------------------------------
// DTW: banded dynamic time warping in registers
// --------------------------------------------------------------------------
// Squared DTW of the query against the series x under a band of half-width
// R (a template argument: one instance per band), by the textbook recurrence
//     D(i, j) = c(i, j) + min(D(i-1, j), D(i, j-1), D(i-1, j-1)),
// i indexing the query and j the series.  The rows go over j: register slot t
// (0 <= t <= 2R) of row j holds cell (j - R + t, j); going down a row, slot t
// reads the row above in slots t + 1 (same query value) and t (one query
// value back) and its left neighbour from slot t - 1 of the new row, so the
// row is updated in place in ascending t.  A row needs one value of x per
// lane; the query values are the same for every lane and come from qp, a
// copy of the query with +inf outside it (qp[j + t] = q[j - R + t]), so
// cells outside the matrix come out +inf with no test.  The x values of a
// block of kDtwRows rows are loaded during the block before.
// T = double: the canonical value, each subtraction, product and sum rounded
// once in fp64 (no fused multiply-add), equal to the plain recurrence in any
// evaluation order.  T = float: the search value, within a relative 2^-12 of
// it for L <= 1024 (each path sum is a sequential sum of at most 2L - 1
// non-negative terms, each term within 3 units of rounding).  It stops, and
// returns +inf, once a lower bound of the final value exceeds limit: after
// row j every path still has to match each x_j', j' > j, with some query
// value inside the query's envelope [el_j', eu_j'], so the final value is at
// least the row's smallest cell plus those columns' LB_Keogh terms, which
// are lbk (the row's LB_Keogh, summed by the scan) less the terms of columns
// <= j summed here.  Both sums are within 2^-13 lbk of their exact values,
// covered by a slack of 2^-12 lbk.
constexpr int kDtwRows = 4;  // rows per block of the banded DP

template <int R, typename T>
__device__ T dtw_band(const float* __restrict__ qp, const float* __restrict__ x, int L, float limit,
                      const float* __restrict__ eu = nullptr, const float* __restrict__ el = nullptr,
                      float lbk = 0.f) {
    constexpr bool F64 = sizeof(T) == 8;
    constexpr int W = 2 * R + 1;
    const T inf = (T)__builtin_huge_valf();
    // the padded query is not written during the search: read it as constant
    // memory, so its values (the same in every lane) come through scalar loads
    using const_float = const __attribute__((address_space(4))) float;
    const_float* qc = (const_float*)qp;
    T D[W];
#pragma unroll
    for (int t = 0; t < W; ++t) D[t] = t == R ? (T)0 : inf;  // the virtual cell (-1, -1) starts the path
    float pre = 0.f;
    const float slack = lbk * 2.44140625e-04f;
    float in_x[kDtwRows];
#pragma unroll
    for (int u = 0; u < kDtwRows; ++u) in_x[u] = u < L ? x[u] : 0.f;
    for (int j0 = 0; j0 < L; j0 += kDtwRows) {
        float nx[kDtwRows];
#pragma unroll
        for (int u = 0; u < kDtwRows; ++u) nx[u] = j0 + kDtwRows + u < L ? x[j0 + kDtwRows + u] : 0.f;
        // each row takes the front of in_x and moves the rest down
#pragma unroll 1
        for (int u = 0; u < kDtwRows; ++u) {
            const int j = j0 + u;
            if (j >= L) break;
            const float xj = in_x[0];
            if (!F64) {
                const float g = keogh_gap(xj, eu[j], el[j]);
                pre += g * g;
            }
            T left = inf, rowmin = inf;
#pragma unroll
            for (int t = 0; t < W; ++t) {
                const float qi = qc[j + t];
                const T above = (t + 1 < W) ? D[t + 1] : inf;
                T m = D[t] < above ? D[t] : above;
                m = left < m ? left : m;
                T v;
                if (F64) {
                    const double d = __dsub_rn((double)qi, (double)xj);
                    v = (T)__dadd_rn(__dmul_rn(d, d), (double)m);
                } else {
                    const float d = qi - xj;
                    v = (T)(d * d + (float)m);
                }
                D[t] = v;
                left = v;
                rowmin = v < rowmin ? v : rowmin;
            }
#pragma unroll
            for (int v = 0; v + 1 < kDtwRows; ++v) in_x[v] = in_x[v + 1];
            if (!F64) {
                const float rest = fmaxf(0.f, lbk - pre - slack);
                if (((float)rowmin * (1.0f - kRhoDtw) + rest) * (1.0f - 1.0e-6f) > limit) return inf;
            }
        }
#pragma unroll
        for (int u = 0; u < kDtwRows; ++u) in_x[u] = nx[u];
    }
    return D[R];
}

// The query with MESSI_MAX_DTW_BAND values of +inf on each side, after all
// the queries' envelopes in the envelope buffer (dtw_env_kernel writes it).
constexpr int kQPad = MESSI_MAX_DTW_BAND;
__device__ __forceinline__ const float* padded_query(const QArgs& a, int q) {
    return a.env + (size_t)a.nq * 2 * a.L + (size_t)q * (a.L + 2 * kQPad);
}

// Keep this wave's LDS accesses in program order for the compiler: the
// hardware performs one wave's LDS operations in the order issued, so no wait
// is needed (a wavefront-scope fence emits none).
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// LB_Keogh of the query against the candidate's envelope (the candidate-side
// bound): every warping path in the band matches q_i with some x_j,
// |i - j| <= R, and x_j lies inside [min, max] of x over [i - R, i + R]
// (clipped to the series), so the sum over i of the squared distance from q_i
// to that interval is below the DTW.  One wave computes it for one candidate.
// The row goes into LDS once, padded on each side with copies of its first
// and last value: a window that reaches past an end contains that end, so the
// copies change no window's max or min.  Each lane then takes four
// consecutive positions jb .. jb + 3, reads the 2R + 4 values their windows
// span with 16-byte reads, forms the max and min of the part the four
// windows share once, and adds each window's few other values.  R is a
// template argument, so every register index is fixed.
constexpr int kEcPad = 32;  // padding on each side of the row (>= R + 3)

// floats per wave's row buffer: a multiple of 4, so every wave's buffer
// starts on a 16-byte boundary
__host__ __device__ constexpr int ec_row_floats(int L) { return (L + 2 * kEcPad + 16 + 3) & ~3; }

// The bound once the padded row is in the wave's buffer.
template <int R>
__device__ float lb_keogh_ec_row(const float* __restrict__ q, const float* row, int L, int lane) {
    constexpr int B0 = (kEcPad - R) & ~3;           // first value read, from jb (16-byte aligned)
    constexpr int E0 = (kEcPad - R) - B0;           // where position jb - R sits among them
    constexpr int NV = (E0 + 2 * R + 4 + 3) / 4 * 4;  // values read per lane and group
    wave_order();
    float ec = 0.f;
    for (int g0 = 0; g0 < L; g0 += 256) {
        const int jb = g0 + 4 * lane;
        if (jb < L) {
            float v[NV];
#pragma unroll
            for (int t = 0; t < NV; t += 4) {
                const float4 f = *reinterpret_cast<const float4*>(row + jb + B0 + t);
                v[t] = f.x;
                v[t + 1] = f.y;
                v[t + 2] = f.z;
                v[t + 3] = f.w;
            }
            // the window of position jb + u is v[E0 + u .. E0 + u + 2R]
            float cmx = 0.f, cmn = 0.f;
            if constexpr (R >= 2) {
                // the part all four share: v[E0 + 3 .. E0 + 2R]
                cmx = cmn = v[E0 + 3];
#pragma unroll
                for (int t = E0 + 4; t <= E0 + 2 * R; ++t) {
                    cmx = fmaxf(cmx, v[t]);
                    cmn = fminf(cmn, v[t]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (jb + u < L) {
                    float mx, mn;
                    if constexpr (R >= 2) {
                        mx = cmx;
                        mn = cmn;
#pragma unroll
                        for (int t = E0 + u; t < E0 + 3; ++t) {
                            mx = fmaxf(mx, v[t]);
                            mn = fminf(mn, v[t]);
                        }
#pragma unroll
                        for (int t = E0 + 2 * R + 1; t <= E0 + 2 * R + u; ++t) {
                            mx = fmaxf(mx, v[t]);
                            mn = fminf(mn, v[t]);
                        }
                    } else {
                        mx = mn = v[E0 + u];
#pragma unroll
                        for (int t = E0 + u + 1; t <= E0 + u + 2 * R; ++t) {
                            mx = fmaxf(mx, v[t]);
                            mn = fminf(mn, v[t]);
                        }
                    }
                    const float gq = keogh_gap(q[jb + u], mx, mn);
                    ec = fmaf(gq, gq, ec);
                }
            }
        }
    }
    wave_order();  // the row buffer is reused for the next candidate
    return dev::wave_sum(ec);
}

template <int R>
__device__ float lb_keogh_ec_wave(const float* __restrict__ x, const float* __restrict__ q, float* row, int L,
                                  int lane) {
    const int RB = ec_row_floats(L);
    for (int p = lane; p < RB; p += 64) row[p] = x[min(max(p - kEcPad, 0), L - 1)];
    return lb_keogh_ec_row<R>(q, row, L, lane);
}

// Padded rows of at most kEcHeld * 64 floats (series of up to 304 values) are
// held in registers, kEcHeld per lane, so the next candidate's row can load
// while the wave bounds the current one.
constexpr int kEcHeld = 6;

__device__ __forceinline__ void ec_row_load(const float* __restrict__ x, int L, int lane, float* v) {
    const int RB = ec_row_floats(L);
#pragma unroll
    for (int k = 0; k < kEcHeld; ++k) {
        const int p = k * 64 + lane;
        v[k] = p < RB ? x[min(max(p - kEcPad, 0), L - 1)] : 0.f;
    }
}

// Block-wide: the exclusive prefix sums of a query's G segment counts (G at
// most 4096, 16 per thread) into s_off[0 .. G], s_off[G] the total, which is
// returned.  Call from every thread.
__device__ uint32_t segment_offsets(const uint32_t* cnt, uint32_t G, uint32_t* s_off, uint32_t* s_tmp) {
    const int tid = threadIdx.x;
    const int per = (int)((G + 255) / 256);
    uint32_t loc[16], sum = 0;
    for (int k2 = 0; k2 < per && k2 < 16; ++k2) {
        const uint32_t i2 = (uint32_t)tid * per + k2;
        loc[k2] = i2 < G ? cnt[i2] : 0u;
        sum += loc[k2];
    }
    uint32_t n = 0;
    uint32_t ex = block_exclusive_scan(sum, s_tmp, n);
    for (int k2 = 0; k2 < per && k2 < 16; ++k2) {
        const uint32_t i2 = (uint32_t)tid * per + k2;
        if (i2 < G) s_off[i2] = ex;
        ex += loc[k2];
    }
    if (tid == 0) s_off[G] = n;
    __syncthreads();
    return n;
}

// The segment holding entry e of the list whose offsets s_off holds: the last
// segment whose offset is <= e.
__device__ __forceinline__ uint32_t segment_of(const uint32_t* s_off, uint32_t G, uint32_t e) {
    uint32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A waiting list overflowed its segment (cannot happen: a segment holds every
// entry its writer can produce; checked anyway).
__device__ bool list_overflow(const QArgs& a, QState& st) {
    if (!st.ovf) return false;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.err = 2;
        atomicOr(a.err_any, 2u);
    }
    return true;
}

// The series of a round whose LB_Keogh is still within the bound get the
// candidate-side bound, a wave per series; those within it too go to this
// block's segment of the second list, for the DP kernel.  The waiting list's
// segments are taken as one list (prefix sums of their counts) and spread
// evenly over the blocks.  A kernel of its own: it needs few registers, so
// far more waves hide its row and LDS latency than the DP's register-bound
// occupancy allows.  Dynamic LDS: the query (L floats), the segment offsets
// (todo_nseg + 1), then, from a 16-byte boundary, per wave the padded row
// (ec_row_floats(L) floats).  One instance per band R.
template <int R>
__global__ void __launch_bounds__(256) dtw_ec_kernel(QArgs a) {
    extern __shared__ __align__(16) float s_dyn[];
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_cnt;
    const int q = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    QState& st = a.qs[q];
    if (st.err) return;
    if (list_overflow(a, st)) return;
    const int L = a.L;
    const uint32_t G = a.todo_nseg;
    float* s_q = s_dyn;
    uint32_t* s_off = reinterpret_cast<uint32_t*>(s_dyn + L);
    float* row = s_dyn + ((L + G + 1 + 3) & ~3u) + wave * ec_row_floats(L);
    const float* qg = a.queries + (size_t)q * L;
    for (int j = tid; j < L; j += 256) s_q[j] = qg[j];
    if (tid == 0) s_cnt = 0;
    const uint32_t n = segment_offsets(a.todo_cnt + (size_t)q * G, G, s_off, s_tmp);
    Cand* out = a.ec + (size_t)q * a.ec_cap + (size_t)blockIdx.x * a.ec_seg;
    const uint32_t stride = gridDim.x * 256;
    for (uint32_t base = blockIdx.x * 256; base < n; base += stride) {
        const uint32_t e = base + tid;
        Cand t{0.f, 0u};
        bool act = e < n;
        if (act) {
            const uint32_t sg = segment_of(s_off, G, e);
            t = a.todo[(size_t)q * a.todo_cap + (size_t)sg * a.todo_seg + (e - s_off[sg])];
            act = !(t.d * (1.0f - kRhoEd) > __uint_as_float(vload(&st.U)));
        }
        // a wave per candidate
        float ec = 0.f;
        uint64_t m = __ballot(act);
        if (ec_row_floats(L) <= kEcHeld * 64) {
            // the next candidate's row loads while this one is bounded
            const int RB = ec_row_floats(L);
            float nv[kEcHeld];
            int l = m ? __ffsll((long long)m) - 1 : -1;
            if (l >= 0) ec_row_load(a.series + (size_t)__shfl(t.idx, l) * L, L, lane, nv);
            while (l >= 0) {
                m &= m - 1;
                const int ln = m ? __ffsll((long long)m) - 1 : -1;
#pragma unroll
                for (int k = 0; k < kEcHeld; ++k) {
                    const int p = k * 64 + lane;
                    if (p < RB) row[p] = nv[k];
                }
                if (ln >= 0) ec_row_load(a.series + (size_t)__shfl(t.idx, ln) * L, L, lane, nv);
                const float v = lb_keogh_ec_row<R>(s_q, row, L, lane);
                if (lane == l) ec = v;
                l = ln;
            }
        } else {
            while (m) {
                const int l = __ffsll((long long)m) - 1;
                m &= m - 1;
                const uint32_t idx = __shfl(t.idx, l);
                const float v = lb_keogh_ec_wave<R>(a.series + (size_t)idx * L, s_q, row, L, lane);
                if (lane == l) ec = v;
            }
        }
        if (act && !(ec * (1.0f - kRhoEd) > __uint_as_float(vload(&st.U)))) {
            const uint32_t slot = atomicAdd(&s_cnt, 1u);
            if (slot < a.ec_seg) out[slot] = t;
            else st.ovf = 1;
        }
    }
    __syncthreads();
    if (tid == 0) a.ec_cnt[(size_t)q * gridDim.x + blockIdx.x] = min(s_cnt, a.ec_seg);
}

// The fp32 banded DTW (band R) of every series the bound kernel passed, a
// thread each (the list is compacted, so full waves run the DP), spread evenly
// over the blocks by the prefix sums of the segment counts; those within the
// bound become candidates, and for k = 1 they lower U.
template <int R>
__global__ void __launch_bounds__(256) dtw_kernel(QArgs a) {
    __shared__ float s_eu[MESSI_MAX_LEN], s_el[MESSI_MAX_LEN];
    __shared__ uint32_t s_off[4097];
    __shared__ uint32_t s_tmp[4];
    const int q = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    QState& st = a.qs[q];
    if (st.err) return;
    if (list_overflow(a, st)) return;
    const int L = a.L;
    const float* eg = a.env + (size_t)q * 2 * L;
    for (int j = tid; j < L; j += 256) {
        s_eu[j] = eg[j];
        s_el[j] = eg[L + j];
    }
    // the query values of a row are the same in every lane: read from the
    // padded copy in memory (qp[j + t] = q[j - R + t])
    const float* qp = padded_query(a, q) + (kQPad - R);
    const uint32_t G = a.ec_nseg;
    const uint32_t n = segment_offsets(a.ec_cnt + (size_t)q * G, G, s_off, s_tmp);
    unsigned long long ndtw = 0;
    const uint32_t stride = gridDim.x * 256;
    for (uint32_t e = blockIdx.x * 256 + tid; e < n; e += stride) {
        const uint32_t sg = segment_of(s_off, G, e);
        const Cand c = a.ec[(size_t)q * a.ec_cap + (size_t)sg * a.ec_seg + (e - s_off[sg])];
        const float U = __uint_as_float(vload(&st.U));
        if (c.d * (1.0f - kRhoEd) > U) continue;
        ++ndtw;
        const float d = dtw_band<R, float>(qp, a.series + (size_t)c.idx * L, L, U, s_eu, s_el, c.d);
        if (d * (1.0f - kRhoDtw) <= __uint_as_float(vload(&st.U))) {
            const uint32_t slot = atomicAdd(&st.ncand, 1u);
            if (slot < a.cap) a.cand[(size_t)q * a.cap + slot] = Cand{d, c.idx};
            if (st.k == 1) atomicMin(&st.U, __float_as_uint(d * (1.0f + 2.0f * kRhoDtw)));
        }
    }
    if (a.counters) {
        for (int off = 32; off >= 1; off >>= 1) ndtw += __shfl_xor(ndtw, off);
        if (lane == 0 && ndtw) atomicAdd(&a.counters->recheck, ndtw);
    }
}

// Once per DTW call: every query's LB_Keogh envelope, the largest and the
// smallest query value within the band of each position; and the query
// padded with +inf for the DP.
__global__ void __launch_bounds__(256) dtw_env_kernel(QArgs a) {
    const int q = blockIdx.x;
    const int L = a.L, r = a.band;
    const float* qg = a.queries + (size_t)q * L;
    float* eg = a.env + (size_t)q * 2 * L;
    float* qp = a.env + (size_t)a.nq * 2 * L + (size_t)q * (L + 2 * kQPad);
    for (int i = threadIdx.x; i < L + 2 * kQPad; i += 256)
        qp[i] = (i >= kQPad && i < L + kQPad) ? qg[i - kQPad] : __builtin_huge_valf();
    for (int j = threadIdx.x; j < L; j += 256) {
        const int t0 = max(0, j - r), t1 = min(L - 1, j + r);
        float u = qg[t0], l = u;
        for (int t = t0 + 1; t <= t1; ++t) {
            u = fmaxf(u, qg[t]);
            l = fminf(l, qg[t]);
        }
        eg[j] = u;
        eg[L + j] = l;
    }
}

// Before a DTW round: empty every query's list of waiting series.
__global__ void __launch_bounds__(256) todo_reset_kernel(QArgs a) {
    const size_t n = (size_t)a.nq * a.todo_nseg;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) a.todo_cnt[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.err_any[2] = 0;
}

// After a DTW round: count the queries whose order goes on past chunk c1 with
// a chunk that the bound does not stop (the scan's own stop rule).
__global__ void __launch_bounds__(256) dtw_active_kernel(QArgs a, uint32_t c1) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.nq) return;
    const QState& st = a.qs[q];
    if (st.err) return;
    const uint64_t nch = ((uint64_t)st.nmemb + a.chunk - 1) / a.chunk;
    if ((uint64_t)c1 >= nch) return;
    const uint32_t t0 = a.chunk_first[(size_t)q * a.max_chunks + c1];
    const float lb0 = a.rec[(size_t)q * a.nL + t0].lb;
    const float U = __uint_as_float(st.U);
    const float low = (float)bin_of(lb0, st.range) * (st.range / (float)kNB);
    if (lb0 * (1.0f - kRhoLb) > U && low * (1.0f - 2.0f * kRhoLb) > U) return;
    atomicAdd(&a.err_any[2], 1u);
}

// ---- the serving engine's slots ---------------------------------------------
constexpr uint32_t kSlotWin0 = 16;  // first window of a slot's leaf order; each later one is 4x (<= 65536)

// Admissions of the step: a slot the host marked copies its staged query and
// k from host memory and enters kSlotAdmit.
__global__ void __launch_bounds__(256) slot_begin_kernel(QArgs a, SlotIO io, float* __restrict__ qdev,
                                                         int32_t* __restrict__ kdev) {
    __shared__ uint32_t s_go;
    const int q = blockIdx.x;
    if (threadIdx.x == 0) s_go = io.ctl[q];
    __syncthreads();
    if (!s_go) return;
    for (int j = threadIdx.x; j < a.L; j += 256) qdev[(size_t)q * a.L + j] = io.q[(size_t)q * a.L + j];
    if (threadIdx.x == 0) {
        kdev[q] = io.k[q];
        a.phase[q] = kSlotAdmit;
    }
}

// After the head: an admitted slot starts its first window (or, if its query
// is not finite, goes straight to its final kernel, which reports that).
__global__ void __launch_bounds__(256) slot_activate_kernel(QArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.nq || a.phase[q] != kSlotAdmit) return;
    const QState& st = a.qs[q];
    a.win[3 * q] = 0;
    a.win[3 * q + 1] = min(kSlotWin0, st.nsurv);
    a.win[3 * q + 2] = 0;
    a.phase[q] = (st.err || st.nsurv == 0) ? kSlotFinal : kSlotActive;
}

// After the round (and the bound refresh): a slot whose order is exhausted,
// or whose next position lies in a bin wholly above U (the scan's own stop
// rule: every later leaf's bound exceeds U), is final; any other takes its
// next window.
__global__ void __launch_bounds__(256) slot_end_kernel(QArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.nq || a.phase[q] != kSlotActive) return;
    const QState& st = a.qs[q];
    const uint32_t t = a.win[3 * q + 1];
    bool stop = st.err != 0 || t >= st.nsurv;
    if (!stop) {
        const float lb0 = a.rec[(size_t)q * a.nL + t].lb;
        const float U = __uint_as_float(st.U);
        const float low = (float)bin_of(lb0, st.range) * (st.range / (float)kNB);
        stop = lb0 * (1.0f - kRhoLb) > U && low * (1.0f - 2.0f * kRhoLb) > U;
    }
    if (stop) {
        a.phase[q] = kSlotFinal;
        return;
    }
    const uint32_t r = a.win[3 * q + 2] + 1;
    const uint32_t width = kSlotWin0 << min(2u * r, 12u);
    a.win[3 * q] = t;
    a.win[3 * q + 1] = (uint32_t)min((uint64_t)t + width, (uint64_t)st.nsurv);
    a.win[3 * q + 2] = r;
}

// End of the step: final slots are done; every slot's phase (and a done
// slot's status) goes to the host.
__global__ void __launch_bounds__(256) slot_report_kernel(QArgs a, SlotIO io) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.nq) return;
    uint32_t ph = a.phase[q];
    if (ph == kSlotFinal) {
        ph = kSlotDone;
        a.phase[q] = ph;
        io.status[q] = a.qs[q].err;
    }
    io.phase[q] = ph;
}

__global__ void __launch_bounds__(256) slot_clear_kernel(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// DB = 0: Euclidean distances; DB = R + 1: DTW under band R.
template <int DB>
__global__ void __launch_bounds__(256) final_kernel(QArgs a) {
    __shared__ double s_d[kMaxFinal];
    __shared__ uint32_t s_i[kMaxFinal];
    __shared__ float s_q[MESSI_MAX_LEN];
    __shared__ uint32_t s_kept;
    const int q = blockIdx.x;
    if (slot_off(a, q, kSlotFinal)) return;
    QState& st = a.qs[q];
    if (threadIdx.x == 0) s_kept = 0;
    for (int j = threadIdx.x; j < a.L; j += 256) s_q[j] = a.queries[(size_t)q * a.L + j];
    __syncthreads();
    // the call's error flags: one bit per kind of per-query failure (with
    // host_err, a one-query call: this block is the only writer)
    auto flag = [&](uint32_t bit) {
        atomicOr(a.err_any, bit);
        if (a.host_err) *reinterpret_cast<volatile uint32_t*>(a.host_err) = bit;
    };
    if (st.err) {
        const uint32_t e = st.err;
        if (threadIdx.x == 0) flag(e == 1 ? 1u : e == 2 ? 2u : e == 3 ? 4u : e == 4 ? 8u : 16u);
        return;
    }
    const float U = __uint_as_float(st.U);
    const uint32_t nc = st.ncand;
    if (nc > a.cap) {
        if (threadIdx.x == 0) {
            st.err = 2;
            flag(2u);
        }
        return;
    }
    const Cand* c = a.cand + (size_t)q * a.cap;
    for (uint32_t i = threadIdx.x; i < nc; i += 256) {
        const Cand e = c[i];
        if (e.d * (1.0f - a.rho_d) <= U) {
            const uint32_t slot = atomicAdd(&s_kept, 1u);
            if (slot < (uint32_t)kMaxFinal) s_i[slot] = e.idx;
        }
    }
    __syncthreads();
    const uint32_t kept = s_kept;
    const int k = st.k;
    if (kept > (uint32_t)kMaxFinal || kept < (uint32_t)k) {
        if (threadIdx.x == 0) {
            st.err = kept > (uint32_t)kMaxFinal ? 3u : 4u;
            flag(kept > (uint32_t)kMaxFinal ? 4u : 8u);
        }
        return;
    }
    if constexpr (DB > 0) {
        // DTW: the canonical fp64 value of every candidate, a thread each
        for (uint32_t j = threadIdx.x; j < kept; j += 256)
            s_d[j] = dtw_band<(DB > 0 ? DB - 1 : 0), double>(padded_query(a, q) + (kQPad - (DB - 1)),
                                                            a.series + (size_t)s_i[j] * a.L, a.L, 0.f);
    } else if (kept <= 16) {
        // D64 of every candidate: the squared differences added one after
        // another in index order, each operation rounded once (no fused
        // multiply-add).
        // few candidates: each wave stages one candidate's row in LDS with a
        // coalesced load, then one lane sums it in order from LDS (while at
        // most 16 candidates are kept, s_d beyond its first 64 entries is free)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        float* stage = reinterpret_cast<float*>(s_d + 64) + wave * MESSI_MAX_LEN;
        for (uint32_t g = 0; g < kept; g += 4) {
            const uint32_t j = g + wave;
            if (j < kept) {
                const float* x = a.series + (size_t)s_i[j] * a.L;
                for (int t = lane; t < a.L; t += 64) stage[t] = x[t];
            }
            __syncthreads();
            if (j < kept && lane == 0) {
                // 16 values per round of LDS reads, so that the chain of
                // additions does not wait on each read
                double s = 0.0;
                int t0 = 0;
                for (; t0 + 16 <= a.L; t0 += 16) {
                    float xv[16], qv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        xv[u] = stage[t0 + u];
                        qv[u] = s_q[t0 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const double d = __dsub_rn((double)qv[u], (double)xv[u]);
                        s = __dadd_rn(s, __dmul_rn(d, d));
                    }
                }
                for (; t0 < a.L; ++t0) {
                    const double d = __dsub_rn((double)s_q[t0], (double)stage[t0]);
                    s = __dadd_rn(s, __dmul_rn(d, d));
                }
                s_d[j] = s;
            }
            __syncthreads();
        }
    } else {
        // many candidates: a thread per candidate, loads 16 at a time
        for (uint32_t j = threadIdx.x; j < kept; j += 256) {
            const float* x = a.series + (size_t)s_i[j] * a.L;
            double s = 0.0;
            for (int t0 = 0; t0 < a.L; t0 += 16) {
                float xv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) xv[u] = (t0 + u < a.L) ? x[t0 + u] : 0.f;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (t0 + u < a.L) {
                        const double d = __dsub_rn((double)s_q[t0 + u], (double)xv[u]);
                        s = __dadd_rn(s, __dmul_rn(d, d));
                    }
                }
            }
            s_d[j] = s;
        }
    }
    uint32_t P = 1;
    while (P < kept) P <<= 1;
    for (uint32_t j = kept + threadIdx.x; j < P; j += 256) {
        s_d[j] = __longlong_as_double(0x7ff0000000000000ll);
        s_i[j] = 0xffffffffu;
    }
    __syncthreads();
    // bitonic sort by (distance, index)
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += 256) {
                const uint32_t lo = 2 * t - (t & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const double dl = s_d[lo], dh = s_d[hi];
                const uint32_t il = s_i[lo], ih = s_i[hi];
                const bool gt = (dl > dh) || (dl == dh && il > ih);
                if (gt == up) {
                    s_d[lo] = dh;
                    s_d[hi] = dl;
                    s_i[lo] = ih;
                    s_i[hi] = il;
                }
            }
            __syncthreads();
        }
    }
    const uint32_t ks = st.kstride;
    for (int j = threadIdx.x; j < k; j += 256) {
        a.out_idx[(size_t)q * ks + j] = (int64_t)s_i[j];
        a.out_dist[(size_t)q * ks + j] = (float)__dsqrt_rn(s_d[j]);
    }
    // a query with k below the row length: the rest of its row is (-1, +inf)
    for (uint32_t j = (uint32_t)k + threadIdx.x; j < ks; j += 256) {
        a.out_idx[(size_t)q * ks + j] = -1;
        a.out_dist[(size_t)q * ks + j] = __uint_as_float(0x7f800000u);
    }
    if (threadIdx.x == 0 && a.counters) atomicAdd(&a.counters->final_cands, (unsigned long long)kept);
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
std::mutex g_ws_mu;
std::map<std::pair<const Index*, hipStream_t>, Workspace*> g_ws;

}  // namespace

// Candidate slots per query: 2^20 for a single query, 64 k (at least 2^14;
// 2^16 in BF16 mode, whose rounds append all rechecked survivors within the
// round's bound) per query of a batch.  The index's cand_cap option replaces
// the default (at least 2 k), e.g. to exercise the overflow paths.
uint32_t default_cap(const Index* ix, int32_t nq, int32_t kmax, int32_t mode) {
    const uint32_t floor_k = 2u * (uint32_t)kmax;
    if (ix->opts.cand_cap > 0)
        return std::max<uint32_t>(floor_k, std::min<uint32_t>(ix->opts.cand_cap, 1u << 30));
    if (nq == 1) return 1u << 20;
    // the batch filters (BF16, and FP32 on rows the FP32 filter takes)
    // append every member within the bound of a round: a larger buffer
    const bool batch_filter = mode == MESSI_MODE_BF16 || (mode == MESSI_MODE_FP32 && f32_filter_ok(ix));
    const uint32_t lo = batch_filter ? (1u << 16) : (1u << 14);
    return std::max<uint32_t>(lo, 64u * (uint32_t)kmax);
}

int Workspace::ensure_stats() {
    if (ev[0]) return MESSI_OK;
    for (auto& e : ev) MESSI_HIP_TRY(hipEventCreate(&e));
    MESSI_HIP_TRY(hipHostMalloc((void**)&h_counters, sizeof(QCounters), 0));
    MESSI_HIP_TRY(hipHostMalloc((void**)&h_prof, sizeof(unsigned long long) * 4 * 4096, 0));
    MESSI_HIP_TRY(hipHostMalloc((void**)&h_blk_cnt, sizeof(unsigned long long) * kBlkCnt * 4096, 0));
    return MESSI_OK;
}

size_t Workspace::device_bytes() const {
    size_t t = 0;
    for (const DevBuf* b : {&qs, &lb, &order, &rec, &chunk_first, &bins, &mbins, &cursor, &hist, &approx_d, &cand,
                            &counters, &err, &prof, &blk_cnt, &status, &lbpart, &seg, &segcnt, &slot_phase,
                            &slot_win, &slot_q, &slot_k, &todo, &env,
                            &todo_cnt,
                            &ec, &ec_cnt,
                            &qb, &qnorm, &qx, &leaf_cnt, &leaf_off, &leaf_cur, &leaf_q, &leaf_act, &pairs, &npairs})
        t += b->bytes;
    return t;
}

int Workspace::grow(const Index* ix, DevBuf& b, size_t bytes) {
    const uint64_t budget = ix->opts.budget_bytes;
    if (budget && device_bytes() - b.bytes + bytes > budget) {
        b.release();
        set_error(MESSI_ENOMEM, "search workspace of " + std::to_string(device_bytes() + bytes) +
                                    " bytes exceeds the index's budget_bytes (" + std::to_string(budget) + ")");
        return MESSI_ENOMEM;
    }
    return b.alloc(bytes);
}

Workspace::~Workspace() {
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    for (void* p : {(void*)h_counters, (void*)h_prof, (void*)h_blk_cnt, (void*)h_err, (void*)h_flag})
        if (p) (void)hipHostFree(p);
}

namespace {

uint32_t max_chunks_of(const Index* ix) {
    const int64_t ch = ix->opts.scan_chunk;
    return (uint32_t)((ix->n + ch - 1) / ch + 1);
}

}  // namespace

size_t workspace_fixed_bytes(const Index* ix) {
    const size_t nL1 = (size_t)ix->n_leaves + 1;
    return sizeof(QCounters) + sizeof(uint32_t) * 4 + sizeof(unsigned long long) * 4 * 4096 +
           sizeof(unsigned long long) * kBlkCnt * 4096 + sizeof(uint32_t) * (4 * nL1 + 8);
}

size_t split_scan_bytes(const Index* ix) {
    return sizeof(uint32_t) * (size_t)max_chunks_of(ix) * ((size_t)ix->opts.scan_chunk + 1) * (size_t)kSplitMaxQ;
}

namespace {

// split: the call may take the split scan, whose survivor segments (one slot
// per member, split_scan_bytes) the workspace then holds.  When they do not
// fit the index's budget the call goes without them (one flat scan kernel).
int get_workspace(const Index* ix, hipStream_t s, int32_t nq, uint32_t cap, bool split, Workspace** out) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace*& ws = g_ws[{ix, s}];
    if (!ws) ws = new Workspace();
    const size_t slots = (size_t)cap * (size_t)nq;
    if (ws->nq < nq || ws->nL != ix->n_leaves) {
        MESSI_TRY(growth_sync(s));
        const int32_t nqa = std::max(nq, ws->nq);
        // not valid until every buffer is in place (a failed allocation leaves its buffer empty)
        ws->nq = 0;
        ws->nL = 0;
        ++ws->gen;
        const size_t nL = (size_t)ix->n_leaves;
        const uint32_t mc = max_chunks_of(ix);
        MESSI_TRY(ws->grow(ix, ws->qs, sizeof(QState) * nqa));
        MESSI_TRY(ws->grow(ix, ws->lb, sizeof(float) * nL * nqa));
        MESSI_TRY(ws->grow(ix, ws->order, sizeof(uint32_t) * nL * nqa));
        MESSI_TRY(ws->grow(ix, ws->rec, sizeof(OrdRec) * nL * nqa));
        MESSI_TRY(ws->grow(ix, ws->chunk_first, sizeof(uint32_t) * (size_t)mc * nqa));
        MESSI_TRY(ws->grow(ix, ws->bins, sizeof(uint32_t) * kNB * nqa));
        MESSI_TRY(ws->grow(ix, ws->mbins, sizeof(uint32_t) * kNB * nqa));
        MESSI_TRY(ws->grow(ix, ws->cursor, sizeof(unsigned long long) * kNB * nqa));
        MESSI_TRY(ws->grow(ix, ws->hist, sizeof(uint32_t) * kHistBins * nqa));
        MESSI_TRY(ws->grow(ix, ws->approx_d, sizeof(float) * kApproxMax * nqa));
        MESSI_TRY(ws->grow(ix, ws->status, sizeof(uint32_t) * nqa));
        MESSI_TRY(ws->grow(ix, ws->counters, sizeof(QCounters)));
        MESSI_TRY(ws->grow(ix, ws->err, sizeof(uint32_t) * 4));
        MESSI_TRY(ws->grow(ix, ws->prof, sizeof(unsigned long long) * 4 * 4096));
        MESSI_TRY(ws->grow(ix, ws->blk_cnt, sizeof(unsigned long long) * kBlkCnt * 4096));
        MESSI_TRY(ws->grow(ix, ws->lbpart, sizeof(LbPart) * (size_t)nqa * ((nL + kLeafBlock - 1) / kLeafBlock)));
        if (!ws->h_err) MESSI_HIP_TRY(hipHostMalloc((void**)&ws->h_err, sizeof(uint32_t) * 4, 0));
        if (!ws->h_flag) {
            MESSI_HIP_TRY(hipHostMalloc((void**)&ws->h_flag, sizeof(uint32_t) * 4,
                                        hipHostMallocMapped | hipHostMallocCoherent));
            MESSI_HIP_TRY(hipHostGetDevicePointer((void**)&ws->d_flag, ws->h_flag, 0));
        }
        ws->nq = nqa;
        ws->nL = (int32_t)nL;
        ws->max_chunks = mc;
        ++ws->gen;
    }
    if (split && nq <= kSplitMaxQ && (ws->seg_nq < nq || ws->seg.bytes < sizeof(uint32_t) * (size_t)ws->max_chunks *
                                                                            (size_t)ix->opts.scan_chunk * (size_t)nq)) {
        MESSI_TRY(growth_sync(s));
        ws->seg_nq = 0;
        ++ws->gen;
        ws->seg.release();
        ws->segcnt.release();
        int rc = ws->grow(ix, ws->seg, sizeof(uint32_t) * (size_t)ws->max_chunks * (size_t)ix->opts.scan_chunk *
                                           (size_t)kSplitMaxQ);
        if (rc == MESSI_OK) rc = ws->grow(ix, ws->segcnt, sizeof(uint32_t) * (size_t)ws->max_chunks * (size_t)kSplitMaxQ);
        if (rc == MESSI_OK) {
            ws->seg_nq = kSplitMaxQ;
        } else if (rc == MESSI_ENOMEM) {
            // over the budget (or the device's memory): go without
            ws->seg.release();
            ws->segcnt.release();
            clear_error();
        } else {
            return rc;
        }
        ++ws->gen;
    }
    if (ws->cand_slots < slots) {
        MESSI_TRY(growth_sync(s));
        ws->cand_slots = 0;
        ++ws->gen;
        MESSI_TRY(ws->grow(ix, ws->cand, sizeof(Cand) * slots));
        ws->cand_slots = slots;
        ++ws->gen;
    }
    *out = ws;
    return MESSI_OK;
}

// Scan blocks: as many as can be resident at once (the passes of a variant
// share one grid, so the per-block statistics line up across passes).
int scan_grid(int mode) {
    static int grid[3] = {0, 0, 0};
    int& blocks = grid[mode];
    if (!blocks) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t p;
            if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        }
        int per = 4;
        const void* fns[3][4] = {
            {(const void*)flat_scan_kernel<true, 0>, (const void*)flat_scan_kernel<true, 1>,
             (const void*)flat_scan_kernel<false, 0>, (const void*)flat_scan_kernel<false, 1>},
            {(const void*)scan_kernel<true, 0, kScanRowFilter>, (const void*)scan_kernel<true, 1, kScanRowFilter>,
             (const void*)scan_kernel<false, 0, kScanRowFilter>, (const void*)scan_kernel<false, 1, kScanRowFilter>},
            {(const void*)scan_kernel<true, 0, kScanDtw>, (const void*)scan_kernel<false, 0, kScanDtw>, nullptr,
             nullptr}};
        for (const void* f : fns[mode]) {
            int nb = 0;
            if (f && hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kScanThreads, 0) == hipSuccess && nb > 0)
                per = std::min(per, nb);
        }
        blocks = std::min(cus * std::max(per, 1), 4096);
    }
    return blocks;
}

// Grids of the split scan's kernels: as many blocks as fit at once; the
// coarse kernel's is the larger (its per-block statistics slots cover the
// refine kernel's).
int split_grid(int which) {
    static int grid[2] = {0, 0};
    if (!grid[0]) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t p;
            if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        }
        int n1 = 0, n2 = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, (const void*)flat_coarse_kernel<0>, kScanThreads, 0) !=
                hipSuccess || n1 < 1)
            n1 = 4;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, (const void*)flat_refine_kernel<true, 0>, kScanThreads,
                                                         0) != hipSuccess || n2 < 1)
            n2 = 4;
        grid[1] = std::min(cus * n2, 4096);
        grid[0] = std::max(std::min(cus * n1, 4096), grid[1]);
    }
    return grid[which];
}

// One pass of the ordered scan in the variant the call needs (the DTW
// variant has no second pass).
// `between` (may be null): an event recorded between the split scan's kernels.
int launch_scan(const QArgs& a, bool vec, int pass, int mode, hipStream_t s, hipEvent_t between = nullptr) {
    const dim3 g(scan_grid(mode)), b(kScanThreads);
    if (mode == kScanEd && a.seg) {
        const dim3 g1(split_grid(0)), g2(split_grid(1));
        if (pass) hipLaunchKernelGGL((flat_coarse_kernel<1>), g1, b, 0, s, a);
        else hipLaunchKernelGGL((flat_coarse_kernel<0>), g1, b, 0, s, a);
        MESSI_LAUNCH_CHECK("scan_coarse");
        if (between) MESSI_HIP_TRY(hipEventRecord(between, s));
        if (vec) {
            if (pass) hipLaunchKernelGGL((flat_refine_kernel<true, 1>), g2, b, 0, s, a);
            else hipLaunchKernelGGL((flat_refine_kernel<true, 0>), g2, b, 0, s, a);
        } else {
            if (pass) hipLaunchKernelGGL((flat_refine_kernel<false, 1>), g2, b, 0, s, a);
            else hipLaunchKernelGGL((flat_refine_kernel<false, 0>), g2, b, 0, s, a);
        }
        MESSI_LAUNCH_CHECK("scan_refine");
        return MESSI_OK;
    }
    if (mode == kScanDtw) {
        if (vec) hipLaunchKernelGGL((scan_kernel<true, 0, kScanDtw>), g, b, 0, s, a);
        else hipLaunchKernelGGL((scan_kernel<false, 0, kScanDtw>), g, b, 0, s, a);
        MESSI_LAUNCH_CHECK("scan_dtw");
        return MESSI_OK;
    }
    const bool sh = mode == kScanRowFilter;
    const int v = (vec ? 4 : 0) | (pass ? 2 : 0) | (sh ? 1 : 0);
    switch (v) {
        case 0: hipLaunchKernelGGL((flat_scan_kernel<false, 0>), g, b, 0, s, a); break;
        case 1: hipLaunchKernelGGL((scan_kernel<false, 0, kScanRowFilter>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((flat_scan_kernel<false, 1>), g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL((scan_kernel<false, 1, kScanRowFilter>), g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL((flat_scan_kernel<true, 0>), g, b, 0, s, a); break;
        case 5: hipLaunchKernelGGL((scan_kernel<true, 0, kScanRowFilter>), g, b, 0, s, a); break;
        case 6: hipLaunchKernelGGL((flat_scan_kernel<true, 1>), g, b, 0, s, a); break;
        default: hipLaunchKernelGGL((scan_kernel<true, 1, kScanRowFilter>), g, b, 0, s, a); break;
    }
    if (pass) MESSI_LAUNCH_CHECK("rescan");
    else MESSI_LAUNCH_CHECK("scan");
    return MESSI_OK;
}

}  // namespace

bool row_filter_path(const Index* ix, int32_t mode, int32_t nq, bool matrix_only) {
    if (mode != MESSI_MODE_BF16 || matrix_only) return false;
    return nq <= ix->opts.row_filter_max_q;
}

int refresh_bounds(QArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(refresh_kernel, dim3(a.nq), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("refresh");
    return MESSI_OK;
}

uint64_t workspace_generation(const Index* ix, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({ix, s});
    return it == g_ws.end() ? 0 : it->second->gen;
}

int trim_candidates(const Index* ix, hipStream_t st, size_t slots) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({ix, st});
    if (it == g_ws.end() || it->second->cand_slots <= slots) return MESSI_OK;
    Workspace* ws = it->second;
    MESSI_HIP_TRY(hipStreamSynchronize(st));
    ws->cand.release();
    ws->cand_slots = 0;
    ++ws->gen;
    return MESSI_OK;
}

size_t workspace_device_bytes(const Index* ix, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({ix, st});
    return it == g_ws.end() ? 0 : it->second->device_bytes();
}

void release_workspace(const Index* ix, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({ix, st});
    if (it != g_ws.end()) {
        delete it->second;
        g_ws.erase(it);
    }
}

void release_workspaces(const Index* ix) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == ix) {
            delete it->second;
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
}

namespace {

// Arguments of one search call shared by the synchronous entry point and the server.
struct CallArgs {
    const Index* ix;
    const float* queries;
    int32_t nq, kmax;
    const int32_t* kq;  // device, per-query k (nullable: kmax for all)
    int32_t mode;
    hipStream_t s;
    int64_t* out_idx;
    float* out_dist;
    bool matrix_only = false;  // BF16: keep few queries on the matrix-core filter
    bool split = true;         // FP32, one query: the split scan when its buffers fit
    uint32_t cap_limit = 0;    // nonzero: the default candidate buffer per query is at most this
    bool probe = false;        // the call may wait on its stream mid-search (not recorded in a graph)
};

// The call's arguments that do not depend on where its workspace lives.
void fill_call_args(const CallArgs& c, uint32_t cap, QArgs& a) {
    const Index* ix = c.ix;
    a = QArgs{};
    a.series = ix->series;
    a.n = ix->n;
    a.L = ix->len;
    a.w = ix->w;
    a.m = ix->len / ix->w;
    a.b = ix->b;
    a.words = ix->words.as<uint4>();
    a.cwords = ix->cwords.as<uint2>();
    a.fwords = ix->wf ? ix->fwords.as<uint8_t>() : nullptr;
    a.wf = ix->wf;
    a.mf = ix->mf;
    {
        int lgf = 0;
        while ((1 << lgf) < ix->mf) ++lgf;
        a.lg_mf = lgf;
    }
    a.csh = ix->b - std::min(ix->b, 4);
    a.pos = ix->pos.as<uint32_t>();
    a.leaves = ix->leaves.as<Leaf>();
    a.nL = (int32_t)ix->n_leaves;
    a.bp = ix->bp.as<float>();
    a.queries = c.queries;
    a.nq = c.nq;
    a.cap = cap;
    a.absmax_data = ix->absmax;
    int lg = 0;
    while ((1 << lg) < a.m) ++lg;
    a.lg_m = lg;
    a.host_err = nullptr;
    a.out_idx = c.out_idx;
    a.out_dist = c.out_dist;
    a.band = -1;
    a.rho_d = kRhoEd;
    a.approx_min = (c.mode == MESSI_MODE_FP32 || c.mode == MESSI_MODE_BF16) ? 2048u : 0u;
    a.chunk_lo = 0;
    a.chunk_hi = 0xffffffffu;
    a.chunk = (uint32_t)ix->opts.scan_chunk;
}

int setup_call(const CallArgs& c, bool counting, Workspace** wsp, QArgs& a, uint32_t& cap, uint32_t cap_min = 0) {
    const Index* ix = c.ix;
    const int32_t nq = c.nq;
    uint32_t cap_d = default_cap(ix, nq, c.kmax, c.mode);
    if (c.cap_limit) cap_d = std::min(cap_d, std::max(c.cap_limit, 2u * (uint32_t)c.kmax));
    cap = std::max(cap_d, cap_min);
    // the approximate mode's candidates are the evaluated members of one leaf
    if (c.mode == MESSI_MODE_APPROX) cap = std::max<uint32_t>(cap, (uint32_t)kApproxMax);
    Workspace* ws = nullptr;
    MESSI_TRY(get_workspace(ix, c.s, nq, cap, c.split && c.mode == MESSI_MODE_FP32, &ws));
    *wsp = ws;
    fill_call_args(c, cap, a);
    a.qs = ws->qs.as<QState>();
    a.lb = ws->lb.as<float>();
    a.order = ws->order.as<uint32_t>();
    a.rec = ws->rec.as<OrdRec>();
    a.chunk_first = ws->chunk_first.as<uint32_t>();
    a.max_chunks = ws->max_chunks;
    a.bins = ws->bins.as<uint32_t>();
    a.mbins = ws->mbins.as<uint32_t>();
    a.cursor = ws->cursor.as<unsigned long long>();
    a.hist = ws->hist.as<uint32_t>();
    a.approx_d = ws->approx_d.as<float>();
    a.lbpart = ws->lbpart.as<LbPart>();
    a.cand = ws->cand.as<Cand>();
    a.seg = nq <= ws->seg_nq ? ws->seg.as<uint32_t>() : nullptr;
    a.skip_approx = (a.seg != nullptr && c.mode == MESSI_MODE_FP32) ? 1 : 0;
    a.segcnt = nq <= ws->seg_nq ? ws->segcnt.as<uint32_t>() : nullptr;
    a.counters = counting ? ws->counters.as<QCounters>() : nullptr;
    a.prof = counting ? ws->prof.as<unsigned long long>() : nullptr;
    a.err_any = ws->err.as<uint32_t>();
    a.blk_cnt = counting ? ws->blk_cnt.as<unsigned long long>() : nullptr;
    return MESSI_OK;
}

// Enqueue the whole search on c.s; `mark(i)` is called at the phase boundaries
// 0 (start), 2 .. 6 (first bound, order, scan, final, end) and 7 (after the
// first FP32 scan pass).
template <class Mark>
int launch_search(const CallArgs& c, QArgs& a, Workspace* ws, uint32_t cap, bool timing, Mark mark) {
    const hipStream_t s = c.s;
    const int32_t nq = c.nq;
    const Index* ix = c.ix;
    const int32_t mode = c.mode;
    // blocks per query over the leaves: one per 256 leaves for a few queries;
    // for a large batch fewer, so that the query tables each block builds are
    // not rebuilt more often than needed (about 8K blocks in all)
    const unsigned lb_blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((a.nL + kLeafBlock - 1) / kLeafBlock, (8192 + nq - 1) / nq));
    MESSI_TRY(mark(0));
    hipLaunchKernelGGL(leaf_lb_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a, c.kmax, c.kq, (uint32_t)c.kmax);
    MESSI_LAUNCH_CHECK("leaf_lb");
    MESSI_TRY(mark(2));
    hipLaunchKernelGGL(approx_ed_kernel, dim3(approx_blocks(nq), nq), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("approx_ed");
    if (mode == MESSI_MODE_APPROX) {
        hipLaunchKernelGGL(approx_select_kernel, dim3(nq), dim3(256), 0, s, a, lb_blocks);
        MESSI_LAUNCH_CHECK("approx_select");
        MESSI_TRY(mark(3));
        hipLaunchKernelGGL(approx_cands_kernel, dim3(nq), dim3(256), 0, s, a, lb_blocks);
        MESSI_LAUNCH_CHECK("approx_cands");
        MESSI_TRY(mark(4));
        MESSI_TRY(mark(7));
        MESSI_TRY(mark(5));
        hipLaunchKernelGGL(final_kernel<0>, dim3(nq), dim3(256), 0, s, a);
        MESSI_LAUNCH_CHECK("final");
        MESSI_TRY(mark(6));
        return MESSI_OK;
    }
    MESSI_TRY(mark(3));
    hipLaunchKernelGGL(bin_hist_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("bin_hist");
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("bin_scatter");
    MESSI_TRY(mark(4));
    const bool rowf = row_filter_path(ix, mode, nq, c.matrix_only);
    if (mode == MESSI_MODE_BF16 && !rowf) {
        MESSI_TRY(bf16_scan(ix, a, ws, s, timing));
    } else if (mode == MESSI_MODE_FP32 && nq > kSplitMaxQ && ws && f32_filter_ok(ix)) {
        // several queries in FP32: the leaf-major FP32 filter, one read of a
        // leaf's rows for all the queries that visit it
        MESSI_TRY(bf16_scan(ix, a, ws, s, timing, true, c.probe));
    } else {
        const bool vec = (a.L % 4 == 0) && ((uintptr_t)a.series % 16 == 0);
        if (rowf) {
            MESSI_TRY(bf16_row_prep(ix, a, ws, s));
            a.rf_tau = kRowFilterTau;
        }
        if (!rowf && a.seg && c.kmax > 1) {
            // For k > 1 the split scan runs in two rounds: the best
            // kSplitFirst chunks (the leaves of smallest bound), U from the
            // exact k-th candidate, then the rest of the order.  The second
            // round's coarse kernel bounds against that U, where one round
            // would use the first bound (the approximate leaf's k-th)
            // throughout.  For k = 1 the first bound is already close and
            // the extra launches and the serial first round cost more than
            // the bytes they save.
            const uint32_t lo = a.chunk_lo, hi = a.chunk_hi;
            a.chunk_hi = kSplitFirst;
            MESSI_TRY(launch_scan(a, vec, 0, kScanEd, s));
            hipLaunchKernelGGL(fixup_kernel, dim3(nq), dim3(256), 0, s, a, 2);
            MESSI_LAUNCH_CHECK("fixup");
            a.chunk_lo = kSplitFirst;
            a.chunk_hi = hi;
            MESSI_TRY(launch_scan(a, vec, 0, kScanEd, s, timing && ws ? ws->ev[8] : nullptr));
            a.chunk_lo = lo;
        } else {
            MESSI_TRY(launch_scan(a, vec, 0, rowf ? kScanRowFilter : kScanEd, s, timing && ws ? ws->ev[8] : nullptr));
        }
        MESSI_TRY(mark(7));
        // k > 1: exact k-th bound and compaction, and a second pass for a
        // query whose buffer overflowed (that pass exits at once otherwise).
        // With k = 1 the bound is exact already, and an overflow (which needs
        // more improving candidates than the buffer holds) is reported by the
        // final kernel and retried with a larger buffer by the caller.
        if (c.kmax > 1) {
            hipLaunchKernelGGL(fixup_kernel, dim3(nq), dim3(256), 0, s, a, 0);
            MESSI_LAUNCH_CHECK("fixup");
            MESSI_TRY(launch_scan(a, vec, 1, rowf ? kScanRowFilter : kScanEd, s));
            hipLaunchKernelGGL(fixup_kernel, dim3(nq), dim3(256), 0, s, a, 1);
            MESSI_LAUNCH_CHECK("fixup");
        }
    }
    MESSI_TRY(mark(5));
    hipLaunchKernelGGL(final_kernel<0>, dim3(nq), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("final");
    MESSI_TRY(mark(6));
    (void)ix;
    return MESSI_OK;
}

int decode_error(uint32_t err) {
    if (err & 1u) {
        set_error(MESSI_EINVAL, "queries contain non-finite values");
        return MESSI_EINVAL;
    }
    if (err & 6u) {
        set_error(MESSI_EOVERFLOW, "too many tied candidates for the candidate buffer");
        return MESSI_EOVERFLOW;
    }
    if (err & 16u) {
        set_error(MESSI_EOVERFLOW, "BF16 filter: more surviving (query, series) pairs than the pair buffer holds");
        return MESSI_EOVERFLOW;
    }
    if (err & 8u) {
        set_error(MESSI_EDEVICE, "internal error: fewer than k candidates");
        return MESSI_EDEVICE;
    }
    return MESSI_OK;
}

}  // namespace

int knn_enqueue(const Index* ix, const float* queries, int32_t nq, int32_t kmax, const int32_t* kq, int32_t mode,
                hipStream_t s, int64_t* out_idx, float* out_dist, uint32_t* host_err, uint32_t* host_status,
                uint32_t cap_min, bool matrix_only, bool split, uint32_t cap_limit) {
    CallArgs c{ix, queries, nq, kmax, kq, mode, s, out_idx, out_dist, matrix_only, split, cap_limit};
    Workspace* ws = nullptr;
    QArgs a;
    uint32_t cap = 0;
    MESSI_TRY(setup_call(c, false, &ws, a, cap, cap_min));
    MESSI_TRY(launch_search(c, a, ws, cap, false, [](int) { return MESSI_OK; }));
    MESSI_HIP_TRY(hipMemcpyAsync(host_err, a.err_any, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (host_status) {
        hipLaunchKernelGGL(status_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, a, ws->status.as<uint32_t>());
        MESSI_LAUNCH_CHECK("status");
        MESSI_HIP_TRY(hipMemcpyAsync(host_status, ws->status.p, sizeof(uint32_t) * nq, hipMemcpyDeviceToHost, s));
    }
    return MESSI_OK;
}

int slot_step_enqueue(const Index* ix, hipStream_t s, int32_t S, const SlotIO& io) {
    if (S < 1 || !ix->shadow.p) {
        set_error(MESSI_EINVAL, "serving engine: needs slots and the BF16 shadow");
        return MESSI_EINVAL;
    }
    const int32_t kmax = (int32_t)std::min<int64_t>(MESSI_MAX_K, ix->n);
    CallArgs c{ix, nullptr, S, kmax, nullptr, MESSI_MODE_BF16, s, io.idx, io.dist};
    c.split = false;
    Workspace* ws = nullptr;
    QArgs a;
    uint32_t cap = 0;
    MESSI_TRY(setup_call(c, false, &ws, a, cap));
    if (ws->slot_n < S) {
        MESSI_TRY(growth_sync(s));
        ws->slot_n = 0;
        ++ws->gen;
        MESSI_TRY(ws->grow(ix, ws->slot_phase, sizeof(uint32_t) * (size_t)S));
        MESSI_TRY(ws->grow(ix, ws->slot_win, sizeof(uint32_t) * 3 * (size_t)S));
        MESSI_TRY(ws->grow(ix, ws->slot_q, sizeof(float) * (size_t)S * ix->len));
        MESSI_TRY(ws->grow(ix, ws->slot_k, sizeof(int32_t) * (size_t)S));
        hipLaunchKernelGGL(slot_clear_kernel, dim3((S + 255) / 256), dim3(256), 0, s, ws->slot_phase.as<uint32_t>(),
                           (uint32_t)S);
        MESSI_LAUNCH_CHECK("slot_clear");
        ws->slot_n = S;
        ++ws->gen;
    }
    a.queries = ws->slot_q.as<float>();
    a.phase = ws->slot_phase.as<uint32_t>();
    a.win = ws->slot_win.as<uint32_t>();
    const unsigned lb_blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((a.nL + kLeafBlock - 1) / kLeafBlock, (8192 + S - 1) / S));
    const unsigned sb = (unsigned)((S + 255) / 256);
    hipLaunchKernelGGL(slot_begin_kernel, dim3(S), dim3(256), 0, s, a, io, ws->slot_q.as<float>(),
                       ws->slot_k.as<int32_t>());
    MESSI_LAUNCH_CHECK("slot_begin");
    hipLaunchKernelGGL(leaf_lb_kernel, dim3(lb_blocks, S), dim3(256), 0, s, a, kmax, ws->slot_k.as<int32_t>(),
                       (uint32_t)MESSI_MAX_K);
    MESSI_LAUNCH_CHECK("leaf_lb");
    hipLaunchKernelGGL(approx_ed_kernel, dim3(approx_blocks(S), S), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("approx_ed");
    hipLaunchKernelGGL(bin_hist_kernel, dim3(lb_blocks, S), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("bin_hist");
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(lb_blocks, S), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("bin_scatter");
    hipLaunchKernelGGL(slot_activate_kernel, dim3(sb), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("slot_activate");
    MESSI_TRY(bf16_slot_round(ix, a, ws, s));
    MESSI_TRY(refresh_bounds(a, s));
    hipLaunchKernelGGL(slot_end_kernel, dim3(sb), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("slot_end");
    hipLaunchKernelGGL(final_kernel<0>, dim3(S), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("final");
    hipLaunchKernelGGL(slot_report_kernel, dim3(sb), dim3(256), 0, s, a, io);
    MESSI_LAUNCH_CHECK("slot_report");
    return MESSI_OK;
}

// ---- a search whose buffers lie in one caller-provided device region ----
namespace {

// Byte offsets of a call's buffers in the region, each 256-byte aligned; the
// candidate buffers come last, so that they take whatever room is left.
struct ViewLayout {
    size_t err, qs, lb, order, rec, chunk_first, bins, mbins, cursor, hist, approx_d, lbpart, cand;
};

ViewLayout view_layout(const Index* ix, int32_t nq) {
    const size_t nL = (size_t)ix->n_leaves, q = (size_t)nq;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    ViewLayout v{};
    v.err = take(sizeof(uint32_t) * 4);
    v.qs = take(sizeof(QState) * q);
    v.lb = take(sizeof(float) * nL * q);
    v.order = take(sizeof(uint32_t) * nL * q);
    v.rec = take(sizeof(OrdRec) * nL * q);
    v.chunk_first = take(sizeof(uint32_t) * (size_t)max_chunks_of(ix) * q);
    v.bins = take(sizeof(uint32_t) * kNB * q);
    v.mbins = take(sizeof(uint32_t) * kNB * q);
    v.cursor = take(sizeof(unsigned long long) * kNB * q);
    v.hist = take(sizeof(uint32_t) * kHistBins * q);
    v.approx_d = take(sizeof(float) * kApproxMax * q);
    v.lbpart = take(sizeof(LbPart) * q * ((nL + kLeafBlock - 1) / kLeafBlock));
    v.cand = o;
    return v;
}

}  // namespace

int knn_view(const Index* ix, const float* queries, int32_t nq, int32_t k, hipStream_t s, int64_t* out_idx,
             float* out_dist, void* base, size_t bytes) {
    if (((uintptr_t)base & 255u) != 0) {
        set_error(MESSI_EINVAL, "search region must be 256-byte aligned");
        return MESSI_EINVAL;
    }
    const ViewLayout v = view_layout(ix, nq);
    const uint32_t cap0 = default_cap(ix, nq, k, MESSI_MODE_FP32);
    const size_t need = v.cand + sizeof(Cand) * (size_t)cap0 * (size_t)nq;
    if (need > bytes) {
        set_error(MESSI_ENOMEM, "the search needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                    std::to_string(bytes) + " bytes of the fixed region");
        return MESSI_ENOMEM;
    }
    // every candidate slot the region holds (at least the default buffer), so
    // an overflow, which cannot be retried with a larger buffer here, is rarer
    const size_t fit = (bytes - v.cand) / (sizeof(Cand) * (size_t)nq);
    const uint32_t cap = (uint32_t)std::min<size_t>(fit, (size_t)1 << 28);
    CallArgs c{ix, queries, nq, k, nullptr, MESSI_MODE_FP32, s, out_idx, out_dist};
    QArgs a;
    fill_call_args(c, cap, a);
    char* b = static_cast<char*>(base);
    a.err_any = reinterpret_cast<uint32_t*>(b + v.err);
    a.qs = reinterpret_cast<QState*>(b + v.qs);
    a.lb = reinterpret_cast<float*>(b + v.lb);
    a.order = reinterpret_cast<uint32_t*>(b + v.order);
    a.rec = reinterpret_cast<OrdRec*>(b + v.rec);
    a.chunk_first = reinterpret_cast<uint32_t*>(b + v.chunk_first);
    a.max_chunks = max_chunks_of(ix);
    a.bins = reinterpret_cast<uint32_t*>(b + v.bins);
    a.mbins = reinterpret_cast<uint32_t*>(b + v.mbins);
    a.cursor = reinterpret_cast<unsigned long long*>(b + v.cursor);
    a.hist = reinterpret_cast<uint32_t*>(b + v.hist);
    a.approx_d = reinterpret_cast<float*>(b + v.approx_d);
    a.lbpart = reinterpret_cast<LbPart*>(b + v.lbpart);
    a.cand = reinterpret_cast<Cand*>(b + v.cand);
    a.seg = nullptr;  // the single-kernel scan (no survivor segments)
    a.segcnt = nullptr;
    a.counters = nullptr;
    a.prof = nullptr;
    a.blk_cnt = nullptr;
    MESSI_TRY(launch_search(c, a, nullptr, cap, false, [](int) { return MESSI_OK; }));
    uint32_t err = 0;
    MESSI_HIP_TRY(hipMemcpyAsync(&err, a.err_any, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    return decode_error(err);
}

// Rounds of the DTW search: the first takes each query's first 16 chunks of
// its order (its best leaves, for a tight bound early; at most 16K members,
// so its candidates fit any query's buffer while the bound is still the
// first one), each later one eight times as many, up to kDtwRoundChunks / nq
// (at least 64).  A round costs a
// launch of each kernel and a host synchronisation whatever its size, so the
// rounds grow fast and the last ones are large (each of the two waiting
// lists then takes 8 bytes per member of a round: about 270 MB).  The
// waiting list has a segment per scan block of a query, large enough for
// every member of that block's chunks of a round, so it cannot overflow.
constexpr uint32_t kDtwRoundChunks = 32768;

// The DP and final kernels of band r (0 <= r <= MESSI_MAX_DTW_BAND): one
// instance per band, picked at run time.
template <int R>
const void* dtw_dp_fn(int r) {
    if (r == R) return (const void*)dtw_kernel<R>;
    if constexpr (R > 0) return dtw_dp_fn<R - 1>(r);
    return nullptr;
}

template <int R>
void launch_dtw_dp(int r, dim3 g, hipStream_t s, const QArgs& a) {
    if (r == R) hipLaunchKernelGGL(dtw_kernel<R>, g, dim3(256), 0, s, a);
    else if constexpr (R > 0) launch_dtw_dp<R - 1>(r, g, s, a);
}

template <int R>
void launch_dtw_ec(int r, dim3 g, size_t lds, hipStream_t s, const QArgs& a) {
    if (r == R) hipLaunchKernelGGL(dtw_ec_kernel<R>, g, dim3(256), lds, s, a);
    else if constexpr (R > 0) launch_dtw_ec<R - 1>(r, g, lds, s, a);
}

template <int R>
void launch_dtw_final(int r, dim3 g, hipStream_t s, const QArgs& a) {
    if (r == R) hipLaunchKernelGGL(final_kernel<R + 1>, g, dim3(256), 0, s, a);
    else if constexpr (R > 0) launch_dtw_final<R - 1>(r, g, s, a);
}

// Resident blocks of the DP kernel of band r over the whole device.
static int dtw_grid(int r) {
    static int grid[MESSI_MAX_DTW_BAND + 1] = {};
    int& blocks = grid[r];
    if (!blocks) {
        int dev = 0, cus = 256, nb = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t p;
            if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dtw_dp_fn<MESSI_MAX_DTW_BAND>(r), 256, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 2;
        blocks = std::min(cus * nb, 4096);
    }
    return blocks;
}

// One DTW search with a candidate buffer of at least cap_min slots per query;
// the raw error bits and the buffer size used come back for the caller's
// retry.
static int knn_dtw_once(const Index* ix, const float* queries, int32_t nq, int32_t k, int32_t band, hipStream_t s,
                        int64_t* out_idx, float* out_dist, messi_knn_stats* stats, uint32_t cap_min,
                        uint32_t* cap_used, uint32_t* err_out) {
    CallArgs c{ix, queries, nq, k, nullptr, MESSI_MODE_FP32, s, out_idx, out_dist};
    Workspace* ws = nullptr;
    QArgs a;
    uint32_t cap = 0;
    MESSI_TRY(setup_call(c, stats != nullptr, &ws, a, cap, cap_min));
    *cap_used = cap;
    const bool timing = stats != nullptr;
    if (timing) MESSI_TRY(ws->ensure_stats());
    a.band = band;
    a.rho_d = kRhoDtw;
    a.approx_min = 0;  // DTW distances are dear: the first bound takes the leaf alone
    a.chunk = kChunk;  // DTW scans (and sizes its rounds) in chunks of 1024 members
    // scan blocks per query (the scan's own split of its grid) and the segments
    const int B = scan_grid(kScanDtw);
    const uint32_t g_max = nq <= B ? (uint32_t)((B + nq - 1) / nq) : 1u;
    const uint32_t g_min = nq <= B ? (uint32_t)(B / nq) : 1u;
    const uint64_t round_max = std::max<uint64_t>(64, kDtwRoundChunks / (uint32_t)nq);
    const uint32_t seg = (uint32_t)((round_max + g_min - 1) / g_min) * a.chunk;
    const uint32_t todo_cap = g_max * seg;
    if (ws->todo_slots < (size_t)nq * todo_cap) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->todo_slots = 0;
        MESSI_TRY(ws->grow(ix, ws->todo, sizeof(Cand) * (size_t)nq * todo_cap));
        ws->todo_slots = (size_t)nq * todo_cap;
        ++ws->gen;
    }
    if (ws->todo_cnt_n < (size_t)nq * g_max) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->todo_cnt_n = 0;
        MESSI_TRY(ws->grow(ix, ws->todo_cnt, sizeof(uint32_t) * (size_t)nq * g_max));
        ws->todo_cnt_n = (size_t)nq * g_max;
        ++ws->gen;
    }
    a.todo = ws->todo.as<Cand>();
    a.todo_cap = todo_cap;
    a.todo_seg = seg;
    a.todo_nseg = g_max;
    a.todo_cnt = ws->todo_cnt.as<uint32_t>();
    // the second list: a segment per block of the bound kernel, each holding
    // every entry that block can take from the first
    const unsigned ec_blocks = (unsigned)std::max(1, std::min(4096, 2048 / std::max(1, (int)nq)));
    const uint32_t ec_seg = (uint32_t)(((uint64_t)todo_cap + (uint64_t)ec_blocks * 256 - 1) /
                                       ((uint64_t)ec_blocks * 256)) * 256u;
    const uint32_t ec_cap = ec_blocks * ec_seg;
    if (ws->ec_slots < (size_t)nq * ec_cap) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->ec_slots = 0;
        MESSI_TRY(ws->grow(ix, ws->ec, sizeof(Cand) * (size_t)nq * ec_cap));
        ws->ec_slots = (size_t)nq * ec_cap;
        ++ws->gen;
    }
    if (ws->ec_cnt_n < (size_t)nq * ec_blocks) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->ec_cnt_n = 0;
        MESSI_TRY(ws->grow(ix, ws->ec_cnt, sizeof(uint32_t) * (size_t)nq * ec_blocks));
        ws->ec_cnt_n = (size_t)nq * ec_blocks;
        ++ws->gen;
    }
    a.ec = ws->ec.as<Cand>();
    a.ec_cap = ec_cap;
    a.ec_seg = ec_seg;
    a.ec_nseg = ec_blocks;
    a.ec_cnt = ws->ec_cnt.as<uint32_t>();
    const size_t ec_lds = sizeof(float) * ((((size_t)ix->len + g_max + 1 + 3) & ~(size_t)3) +
                                           4 * (size_t)ec_row_floats(ix->len));
    const size_t env_floats = (size_t)nq * (3 * (size_t)ix->len + 2 * kQPad);  // envelopes, padded queries
    if (ws->env_floats < env_floats) {
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        ws->env_floats = 0;
        MESSI_TRY(ws->grow(ix, ws->env, sizeof(float) * env_floats));
        ws->env_floats = env_floats;
        ++ws->gen;
    }
    a.env = ws->env.as<float>();
    hipEvent_t* ev = ws->ev;
    auto mark = [&](int i) -> int {
        if (timing) MESSI_HIP_TRY(hipEventRecord(ev[i], s));
        return MESSI_OK;
    };
    const unsigned lb_blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((a.nL + kLeafBlock - 1) / kLeafBlock, (8192 + nq - 1) / nq));
    MESSI_TRY(mark(0));
    hipLaunchKernelGGL(dtw_env_kernel, dim3(nq), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("dtw_env");
    hipLaunchKernelGGL(leaf_lb_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a, k, (const int32_t*)nullptr,
                       (uint32_t)k);
    MESSI_LAUNCH_CHECK("leaf_lb");
    MESSI_TRY(mark(2));
    // the first bound: Euclidean distances to the best leaf's members (the
    // diagonal path lies in every band, so DTW <= ED)
    hipLaunchKernelGGL(approx_ed_kernel, dim3(approx_blocks(nq), nq), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("approx_ed");
    MESSI_TRY(mark(3));
    hipLaunchKernelGGL(bin_hist_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a, lb_blocks);
    MESSI_LAUNCH_CHECK("bin_hist");
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(lb_blocks, nq), dim3(256), 0, s, a);
    MESSI_LAUNCH_CHECK("bin_scatter");
    MESSI_TRY(mark(4));
    // plan the rounds from the longest order
    std::vector<QState> hq(nq);
    MESSI_HIP_TRY(hipMemcpyAsync(hq.data(), a.qs, sizeof(QState) * nq, hipMemcpyDeviceToHost, s));
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    uint64_t max_nch = 0;
    for (const QState& h : hq)
        if (!h.err) max_nch = std::max<uint64_t>(max_nch, ((uint64_t)h.nmemb + a.chunk - 1) / a.chunk);
    const bool vec = (a.L % 4 == 0) && ((uintptr_t)a.series % 16 == 0);
    // the DP kernel's blocks: as many as are resident at once (its grid-stride
    // loop gives every block the same share, so a second partial wave of
    // blocks would only add a tail)
    const unsigned dtw_blocks = (unsigned)std::max(1, dtw_grid(band) / std::max(1, nq));
    const unsigned nqb = (unsigned)((nq + 255) / 256);
    int rounds = 0;
    for (uint64_t c0 = 0, size = std::min<uint64_t>(16, round_max); c0 < max_nch;) {
        const uint64_t c1 = std::min<uint64_t>(c0 + size, max_nch);
        a.chunk_lo = (uint32_t)c0;
        a.chunk_hi = (uint32_t)c1;
        ++rounds;
        hipLaunchKernelGGL(todo_reset_kernel, dim3((unsigned)std::min<size_t>(((size_t)nq * g_max + 255) / 256, 1024)),
                           dim3(256), 0, s, a);
        MESSI_LAUNCH_CHECK("todo_reset");
        MESSI_TRY(launch_scan(a, vec, 0, kScanDtw, s));
        launch_dtw_ec<MESSI_MAX_DTW_BAND>(band, dim3(ec_blocks, nq), ec_lds, s, a);
        MESSI_LAUNCH_CHECK("dtw_ec");
        launch_dtw_dp<MESSI_MAX_DTW_BAND>(band, dim3(dtw_blocks, nq), s, a);
        MESSI_LAUNCH_CHECK("dtw");
        MESSI_TRY(refresh_bounds(a, s));
        c0 = c1;
        size = std::min<uint64_t>(8 * size, round_max);
        if (c0 >= max_nch) break;
        // stop early once no query's order goes on below its bound
        hipLaunchKernelGGL(dtw_active_kernel, dim3(nqb), dim3(256), 0, s, a, (uint32_t)c0);
        MESSI_LAUNCH_CHECK("dtw_active");
        MESSI_HIP_TRY(hipMemcpyAsync(ws->h_err, a.err_any + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        if (*ws->h_err == 0) break;
    }
    MESSI_TRY(mark(5));
    launch_dtw_final<MESSI_MAX_DTW_BAND>(band, dim3(nq), s, a);
    MESSI_LAUNCH_CHECK("final_dtw");
    MESSI_TRY(mark(6));
    MESSI_HIP_TRY(hipMemcpyAsync(ws->h_err, a.err_any, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    const int sg = scan_grid(kScanDtw);
    if (timing) {
        MESSI_HIP_TRY(hipMemcpyAsync(ws->h_counters, a.counters, sizeof(QCounters), hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipMemcpyAsync(ws->h_blk_cnt, a.blk_cnt, sizeof(unsigned long long) * kBlkCnt * sg,
                                     hipMemcpyDeviceToHost, s));
    }
    MESSI_HIP_TRY(hipStreamSynchronize(s));
    const uint32_t err = *ws->h_err;
    *err_out = err;
    if (timing) {
        QCounters hc = *ws->h_counters;
        unsigned long long word_b = 0;
        for (int bb = 0; bb < sg; ++bb) {
            const unsigned long long* h = ws->h_blk_cnt + (size_t)bb * kBlkCnt;
            hc.scanned += h[0];
            hc.bounded += h[1];
            hc.distance += h[2];
            hc.abandoned += h[3];
            hc.bytes += h[4];
            word_b += h[7];
        }
        float ms[7] = {0, 0, 0, 0, 0, 0, 0};
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[1], ev[0], ev[2]));
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[2], ev[2], ev[3]));
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[3], ev[3], ev[4]));
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[4], ev[4], ev[5]));
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[5], ev[5], ev[6]));
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[6], ev[0], ev[6]));
        *stats = messi_knn_stats{};
        stats->ms_leaf_lb = ms[1];
        stats->ms_approx = ms[2];
        stats->ms_order = ms[3];
        stats->ms_scan = ms[4];
        stats->ms_final = ms[5];
        stats->ms_total = ms[6];
        stats->leaves_total = (int64_t)ix->n_leaves * nq;
        stats->leaves_kept = (int64_t)hc.kept;
        stats->leaves_scanned = (int64_t)hc.scanned;
        stats->series_bounded = (int64_t)hc.bounded;
        stats->series_distance = (int64_t)hc.distance;
        stats->series_abandoned = (int64_t)hc.abandoned;
        stats->series_recheck = (int64_t)hc.recheck;
        stats->candidates = (int64_t)hc.final_cands;
        stats->bytes_scan = (int64_t)hc.bytes;
        stats->series_word_bounded = (int64_t)word_b;
        stats->scan_launches = rounds;
    }
    return decode_error(err);
}

// The DTW search.  For k > 1 the bound is the k-th candidate only from the
// second round on, so a round can find more candidates within the bound than
// the buffer holds; then the search runs again with a 16 times larger buffer
// (twice at most), as the Euclidean search does.
int knn_dtw_device(const Index* ix, const float* queries, int32_t nq, int32_t k, int32_t band, hipStream_t s,
                   int64_t* out_idx, float* out_dist, messi_knn_stats* stats) {
    uint32_t cap_min = 0;
    for (int tries = 0;; ++tries) {
        uint32_t cap = 0, err = 0;
        const int rc = knn_dtw_once(ix, queries, nq, k, band, s, out_idx, out_dist, stats, cap_min, &cap, &err);
        if (rc == MESSI_EOVERFLOW && (err & 2u) && !(err & 1u) && tries < 2 && cap <= (1u << 26)) {
            cap_min = cap * 16;
            continue;
        }
        return rc;
    }
}

int query_error_code(uint32_t st) {
    switch (st) {
        case 0: return MESSI_OK;
        case 1: return MESSI_EINVAL;
        case 2:
        case 3:
        case 5: return MESSI_EOVERFLOW;
        default: return MESSI_EDEVICE;
    }
}

int knn_error_code(uint32_t err) { return decode_error(err); }

size_t workspace_bytes_per_query(const Index* ix, int32_t mode, uint32_t cap) {
    const size_t nL = (size_t)ix->n_leaves;
    size_t b = sizeof(QState) + nL * (sizeof(float) + sizeof(uint32_t) + sizeof(OrdRec)) +
               sizeof(uint32_t) * (size_t)max_chunks_of(ix) + kNB * (2 * sizeof(uint32_t) + sizeof(unsigned long long)) +
               sizeof(uint32_t) * kHistBins + sizeof(float) * kApproxMax + sizeof(Cand) * (size_t)cap +
               sizeof(LbPart) * ((nL + kLeafBlock - 1) / kLeafBlock) + sizeof(uint32_t);
    if (mode == MESSI_MODE_BF16 || (mode == MESSI_MODE_FP32 && f32_filter_ok(ix)))
        b += nL * 4 + sizeof(uint2) * bf16_pairs_cap(1) + (size_t)((ix->len + 31) / 32 * 32) * 2 + 8 + 16;
    return b;
}

namespace {
// Totals of two calls' statistics (counts and times add up).
void add_stats(messi_knn_stats* t, const messi_knn_stats& u) {
    t->leaves_total += u.leaves_total;
    t->leaves_kept += u.leaves_kept;
    t->leaves_scanned += u.leaves_scanned;
    t->series_bounded += u.series_bounded;
    t->series_distance += u.series_distance;
    t->series_abandoned += u.series_abandoned;
    t->series_recheck += u.series_recheck;
    t->candidates += u.candidates;
    t->bytes_scan += u.bytes_scan;
    t->ms_total += u.ms_total;
    t->ms_prep += u.ms_prep;
    t->ms_leaf_lb += u.ms_leaf_lb;
    t->ms_approx += u.ms_approx;
    t->ms_order += u.ms_order;
    t->ms_scan += u.ms_scan;
    t->ms_final += u.ms_final;
    t->scan_launches += u.scan_launches;
    t->reruns += u.reruns;
    t->fallbacks += u.fallbacks;
    t->ms_fixup += u.ms_fixup;
    t->series_word_bounded += u.series_word_bounded;
    t->series_fine_bounded += u.series_fine_bounded;
    t->ms_scan_coarse += u.ms_scan_coarse;
}
}  // namespace

int knn_device(const Index* ix, const float* queries, int32_t nq, int32_t k, const int32_t* kq, int32_t mode,
               hipStream_t s, int64_t* out_idx, float* out_dist, messi_knn_stats* stats) {
    if (mode == MESSI_MODE_FP32 && nq > kSplitMaxQ && !f32_filter_ok(ix)) {
        // Several queries in FP32 mode on rows the FP32 filter does not take:
        // one after another, each through the one-query path.  The flat batch
        // kernel gives each query only its share of the blocks, which a hard
        // query (millions of rows within its bound) cannot afford.  Per-query errors: the first is returned, after
        // every query has been answered.
        if (stats) *stats = messi_knn_stats{};
        messi_knn_stats sub{};
        int first = MESSI_OK;
        std::string first_msg;
        for (int32_t q = 0; q < nq; ++q) {
            sub = messi_knn_stats{};
            const int rc = knn_device(ix, queries + (size_t)q * ix->len, 1, k, kq ? kq + q : nullptr, mode, s,
                                      out_idx + (size_t)q * k, out_dist + (size_t)q * k, stats ? &sub : nullptr);
            if (rc != MESSI_OK) {
                if (rc == MESSI_EDEVICE || rc == MESSI_ENOMEM) return rc;
                if (first == MESSI_OK) {
                    first = rc;
                    char buf[512];
                    messi_last_error(buf, sizeof(buf));
                    first_msg = buf;
                }
            }
            if (stats) add_stats(stats, sub);
        }
        if (first != MESSI_OK) set_error(first, first_msg);
        return first;
    }
    CallArgs c{ix, queries, nq, k, kq, mode, s, out_idx, out_dist};
    c.probe = true;  // a synchronous call
    Workspace* ws = nullptr;
    QArgs a;
    uint32_t cap = 0;
    MESSI_TRY(setup_call(c, stats != nullptr, &ws, a, cap));
    const bool timing = stats != nullptr;
    if (timing) MESSI_TRY(ws->ensure_stats());
    hipEvent_t* ev = ws->ev;
    auto mark = [&](int i) -> int {
        if (timing) MESSI_HIP_TRY(hipEventRecord(ev[i], s));
        return MESSI_OK;
    };
    uint32_t err = 0;
    QCounters hc{};
    const bool rowf = row_filter_path(ix, mode, nq, false);
    // the split Euclidean scan (few queries): its two kernels keep no block
    // timing, and its statistics slots span the coarse kernel's grid
    const bool split = mode == MESSI_MODE_FP32 && a.seg != nullptr;
    const int sg = split ? split_grid(0) : scan_grid(rowf ? kScanRowFilter : kScanEd);
    // several queries in FP32 mode on rows it takes: the leaf-major FP32 filter
    const bool f32f = mode == MESSI_MODE_FP32 && nq > kSplitMaxQ && f32_filter_ok(ix);
    const bool fp32 = (mode == MESSI_MODE_FP32 && !f32f) || rowf;  // the ordered scan runs
    const unsigned long long* hprof = nullptr;
    const unsigned long long* hcnt = nullptr;
    int32_t retries = 0;
    // one query without statistics: the final kernel stores its error bit in
    // host memory itself, which saves the read-back copy (a kernel of its own)
    const bool direct = !timing && nq == 1;
    for (;;) {
        if (direct) {
            *reinterpret_cast<volatile uint32_t*>(ws->h_flag) = 0;
            a.host_err = ws->d_flag;  // (again after a retry's set-up)
        }
        MESSI_TRY(launch_search(c, a, ws, cap, timing, mark));
        if (!direct) MESSI_HIP_TRY(hipMemcpyAsync(ws->h_err, a.err_any, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (a.counters)
            MESSI_HIP_TRY(hipMemcpyAsync(ws->h_counters, a.counters, sizeof(QCounters), hipMemcpyDeviceToHost, s));
        if (a.prof && fp32) {
            if (!split) {
                MESSI_HIP_TRY(hipMemcpyAsync(ws->h_prof, a.prof, sizeof(unsigned long long) * 4 * sg,
                                             hipMemcpyDeviceToHost, s));
                hprof = ws->h_prof;
            }
            MESSI_HIP_TRY(hipMemcpyAsync(ws->h_blk_cnt, a.blk_cnt, sizeof(unsigned long long) * kBlkCnt * sg,
                                         hipMemcpyDeviceToHost, s));
            hcnt = ws->h_blk_cnt;
        }
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        err = direct ? *reinterpret_cast<volatile uint32_t*>(ws->h_flag) : *ws->h_err;
        if (a.counters) hc = *ws->h_counters;
        // The FP32 scan's own second pass was not enough (more than cap
        // candidates below the k-th buffered distance): search again with a
        // 16 times larger candidate buffer.
        if (fp32 && (err & 2u) && !(err & 1u) && retries < 2 && cap <= (1u << 26)) {
            ++retries;
            MESSI_TRY(setup_call(c, stats != nullptr, &ws, a, cap, cap * 16));
            continue;
        }
        break;
    }
    unsigned long long bf_rows = 0, word_b = 0, fine_b = 0;
    for (int bb = 0; hcnt && bb < sg; ++bb) {
        const unsigned long long* h = hcnt + (size_t)bb * kBlkCnt;
        hc.scanned += h[0];
        hc.bounded += h[1];
        hc.distance += h[2];
        hc.abandoned += h[3];
        hc.bytes += h[4];
        hc.recheck += h[5];
        bf_rows += h[6];
        word_b += h[7];
        fine_b += h[8];
    }
    // BF16 mode and the FP32 filter: a query whose candidates or filter pairs
    // overflowed their buffers is answered again, alone, by the one-query
    // FP32 path (which reruns and grows its own buffer as needed).
    int32_t fallbacks = 0;
    if ((mode == MESSI_MODE_BF16 || f32f) && (err & (2u | 4u | 16u)) && !(err & 1u)) {
        std::vector<uint32_t> st(nq);
        hipLaunchKernelGGL(status_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, a, ws->status.as<uint32_t>());
        MESSI_LAUNCH_CHECK("status");
        MESSI_HIP_TRY(hipMemcpyAsync(st.data(), ws->status.p, sizeof(uint32_t) * nq, hipMemcpyDeviceToHost, s));
        MESSI_HIP_TRY(hipStreamSynchronize(s));
        uint32_t rest = err & ~(2u | 4u | 16u);
        for (int32_t q = 0; q < nq; ++q) {
            if (query_error_code(st[q]) != MESSI_EOVERFLOW) continue;
            ++fallbacks;
            const int rc = knn_device(ix, queries + (size_t)q * ix->len, 1, k, kq ? kq + q : nullptr,
                                      MESSI_MODE_FP32, s, out_idx + (size_t)q * k, out_dist + (size_t)q * k,
                                      nullptr);
            if (rc == MESSI_EOVERFLOW) rest |= 2u;
            else if (rc != MESSI_OK) return rc;
        }
        err = rest;
    }
    if (timing) {
        // phase 0 (query summary) runs inside the leaf-bound kernel
        float ms[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        MESSI_HIP_TRY(hipEventElapsedTime(&ms[1], ev[0], ev[2]));
        for (int i = 2; i < 6; ++i) MESSI_HIP_TRY(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
        float tot = 0.f;
        MESSI_HIP_TRY(hipEventElapsedTime(&tot, ev[0], ev[6]));
        stats->ms_prep = ms[0];
        stats->ms_leaf_lb = ms[1];
        stats->ms_approx = ms[2];
        stats->ms_order = ms[3];
        if (fp32) {
            float scan_only = 0.f;
            MESSI_HIP_TRY(hipEventElapsedTime(&scan_only, ev[4], ev[7]));
            if (split) {
                float coarse = 0.f;
                MESSI_HIP_TRY(hipEventElapsedTime(&coarse, ev[4], ev[8]));
                stats->ms_scan_coarse = coarse;
            }
            stats->ms_scan = scan_only;
            stats->ms_fixup = ms[4] - scan_only;
        } else {
            stats->ms_scan = ms[4];
        }
        stats->ms_final = ms[5];
        stats->ms_total = tot;
        stats->leaves_total = (int64_t)ix->n_leaves * nq;
        stats->leaves_kept = (int64_t)hc.kept;
        stats->leaves_scanned = (int64_t)hc.scanned;
        stats->series_bounded = (int64_t)hc.bounded;
        stats->series_distance = (int64_t)hc.distance;
        stats->series_abandoned = (int64_t)hc.abandoned;
        stats->series_recheck = (int64_t)hc.recheck;
        stats->candidates = (int64_t)hc.final_cands;
        stats->bytes_scan = (int64_t)hc.bytes;
        stats->series_word_bounded = (int64_t)word_b;
        stats->series_fine_bounded = (int64_t)fine_b;
        stats->scan_launches = (hc.reruns ? 2 : 1) + 2 * retries;
        stats->reruns = (int32_t)hc.reruns + retries;
        stats->fallbacks = fallbacks;
        if (rowf) {
            const int Lp = (ix->len + 31) / 32 * 32;
            stats->bf16_flops = (int64_t)bf_rows * 2 * Lp;
        } else if (mode == MESSI_MODE_BF16 || f32f) {
            const int Lp = (ix->len + 31) / 32 * 32;
            stats->ms_bf16_filter = ws->bf_ms_filter;
            stats->ms_bf16_recheck = ws->bf_ms_recheck;
            stats->bf16_rounds = ws->bf_rounds;
            stats->bf16_stage_queries = ws->bf_stage_queries;
            stats->bf16_max_leaf_queries = ws->bf_max_leaf_q;
            stats->bf16_flops = f32f ? 0 : (int64_t)hc.distance * 2 * Lp;
            stats->scan_launches = ws->bf_rounds;
        }
        if (hprof) {
            int rate_khz = 100000;
            (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ix->device);
            const double to_ms = 1.0 / (double)rate_khz;
            double sum[4] = {0, 0, 0, 0}, mx = 0;
            for (int bb = 0; bb < sg; ++bb) {
                for (int i = 0; i < 4; ++i) sum[i] += (double)hprof[(size_t)bb * 4 + i];
                mx = std::max(mx, (double)hprof[(size_t)bb * 4 + 3]);
            }
            stats->scan_ms_control = sum[0] / sg * to_ms;
            stats->scan_ms_filter = sum[1] / sg * to_ms;
            stats->scan_ms_distance = sum[2] / sg * to_ms;
            stats->scan_ms_block_mean = sum[3] / sg * to_ms;
            stats->scan_ms_block_max = mx * to_ms;
        }
    }
    return decode_error(err);
}

}  // namespace messi

// Device-wide exclusive prefix sum of uint32 values: per-tile sums, one block
// scanning the tile sums, then a per-tile scan with the tile's offset.
#include "scan.h"

namespace messi {
namespace {

__global__ void __launch_bounds__(kScanBlock) tile_sums_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                               uint32_t* __restrict__ sums) {
    __shared__ uint32_t tmp[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t acc = 0;
    for (int r = 0; r < kScanItems; ++r) {
        int64_t i = base + (int64_t)r * kScanBlock + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t total;
    block_exclusive_scan(acc, tmp, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block of 1024 threads: exclusive scan of `m` tile sums in place.
__global__ void __launch_bounds__(1024) scan_sums_kernel(uint32_t* __restrict__ sums, int64_t m,
                                                         uint32_t* __restrict__ total) {
    __shared__ uint32_t wt[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t per = (m + 1023) / 1024;
    const int64_t b0 = (int64_t)t * per;
    uint32_t acc = 0;
    for (int64_t i = b0; i < b0 + per && i < m; ++i) acc += sums[i];
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
    for (int64_t i = b0; i < b0 + per && i < m; ++i) {
        uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
    if (t == 0 && total) *total = tot;
}

__global__ void __launch_bounds__(kScanBlock) tile_scan_kernel(const uint32_t* __restrict__ in, uint32_t* out,
                                                               int64_t n, const uint32_t* __restrict__ sums) {
    __shared__ uint32_t tmp[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t run = sums[blockIdx.x];
    for (int r = 0; r < kScanItems; ++r) {
        int64_t i = base + (int64_t)r * kScanBlock + threadIdx.x;
        uint32_t v = (i < n) ? in[i] : 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(v, tmp, total);
        if (i < n) out[i] = run + ex;
        run += total;
    }
}

}  // namespace

size_t scan_scratch_words(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

int scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums, uint32_t* total, hipStream_t s) {
    if (n <= 0) {
        if (total) MESSI_HIP_TRY(hipMemsetAsync(total, 0, sizeof(uint32_t), s));
        return MESSI_OK;
    }
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(tile_sums_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, n, sums);
    MESSI_LAUNCH_CHECK("tile_sums");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, tiles, total);
    MESSI_LAUNCH_CHECK("scan_sums");
    hipLaunchKernelGGL(tile_scan_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, out, n, sums);
    MESSI_LAUNCH_CHECK("tile_scan");
    return MESSI_OK;
}

}  // namespace messi

// Block- and device-wide prefix sums used by the bucketing, partition and
// compaction kernels (256-thread blocks, wave64).
#pragma once

#include "common.h"

namespace messi {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;                       // items per thread per block
constexpr int kScanTile = kScanBlock * kScanItems;   // 4096

// Exclusive prefix sum of a 256-thread block.  `tmp` is __shared__ uint32_t[4].
// Returns the value's exclusive prefix; `total` receives the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    uint32_t wo = 0;
    total = 0;
    for (int w = 0; w < 4; ++w) {
        uint32_t t = tmp[w];
        if (w < wave) wo += t;
        total += t;
    }
    __syncthreads();
    return wo + x - v;
}

// out[i] = sum_{j < i} in[i] over n values (out may alias in).  `sums` is
// device scratch of scan_scratch_words(n) uint32.  If total != nullptr the
// grand total is stored there (device memory).
size_t scan_scratch_words(int64_t n);
int scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums, uint32_t* total, hipStream_t s);

}  // namespace messi

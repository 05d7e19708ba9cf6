// Device-side twin of datagen.c: the same per-element arithmetic (dg_core.h),
// compiled for gfx950 with multiply-add contraction off, so a row generated
// here is bit-identical to the same row generated on the host.  One thread
// draws one row; the row's fp64 running sum is sequential, as on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DG_FN __device__ static inline
#include "dg_core.h"

namespace {

__global__ void __launch_bounds__(64) walk_kernel(float* __restrict__ out, uint64_t seed, uint32_t stream,
                                                  uint64_t row0, int64_t nrows, int32_t len) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    float* dst = out + (size_t)r * (size_t)len;
    uint64_t row = row0 + (uint64_t)r;
    double x = 0.0;
    for (int32_t j = 0; j < len; j += 2) {
        double a, b;
        dg_gauss_pair(seed, stream, row, (uint32_t)(j / 2), &a, &b);
        x = (j == 0) ? a : x + a;
        dst[j] = (float)x;
        if (j + 1 < len) {
            x = x + b;
            dst[j + 1] = (float)x;
        }
    }
}

__global__ void __launch_bounds__(64) mixture_kernel(float* __restrict__ out, uint64_t seed, uint32_t stream,
                                                     uint64_t row0, int64_t nrows, int32_t len,
                                                     const double* __restrict__ centres, int64_t n_centres,
                                                     double sigma) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    float* dst = out + (size_t)r * (size_t)len;
    uint64_t row = row0 + (uint64_t)r;
    uint64_t c = dg_mixture_cluster(seed, stream, row, (uint64_t)n_centres);
    const double* mu = centres + (size_t)c * (size_t)len;
    for (int32_t j = 0; j < len; j += 2) {
        double a, b;
        dg_gauss_pair(seed, stream, row, (uint32_t)(j / 2), &a, &b);
        dst[j] = (float)dg_round_clip(mu[j] + sigma * a);
        if (j + 1 < len) dst[j + 1] = (float)dg_round_clip(mu[j + 1] + sigma * b);
    }
}

}  // namespace

extern "C" {

// Rows [row0, row0 + nrows) of the random-walk collection into the device
// buffer out[nrows][len].  Returns 0, or the hipError_t of the launch.
int dg_gpu_random_walks(float* out, uint64_t seed, uint32_t stream, uint64_t row0, int64_t nrows, int32_t len,
                        void* stream_handle) {
    if (nrows <= 0) return 0;
    if (!out || len < 1) return (int)hipErrorInvalidValue;
    int64_t blocks = (nrows + 63) / 64;
    hipLaunchKernelGGL(walk_kernel, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)stream_handle, out, seed,
                       stream, row0, nrows, len);
    return (int)hipGetLastError();
}

// Rows of the Gaussian-mixture collection; centres is a device buffer
// [n_centres][len] of fp64 produced by the host's dg_mixture_centres.
int dg_gpu_mixture(float* out, uint64_t seed, uint32_t stream, uint64_t row0, int64_t nrows, int32_t len,
                   const double* centres, int64_t n_centres, double sigma, void* stream_handle) {
    if (nrows <= 0) return 0;
    if (!out || !centres || len < 1 || n_centres < 1) return (int)hipErrorInvalidValue;
    int64_t blocks = (nrows + 63) / 64;
    hipLaunchKernelGGL(mixture_kernel, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)stream_handle, out, seed,
                       stream, row0, nrows, len, centres, n_centres, sigma);
    return (int)hipGetLastError();
}

}  // extern "C"

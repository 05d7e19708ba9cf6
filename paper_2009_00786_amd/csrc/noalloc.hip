// messi_knn_noalloc: the exact FP32 search of messi_knn_ex for callers that
// cannot allocate device memory.  Its buffers (per-query state, leaf bounds
// and order, chunk table, bins, histogram, first-bound distances, candidates)
// live in one array of static device memory, `scratch`, instead of the
// per-stream workspace that grows with hipMalloc.
#include <mutex>

#include "common.h"
#include "query.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MESSI_NOALLOC_SCRATCH_BYTES;

// One copy per GPU the library runs on, held until the process ends.  In host
// code `scratch` names a host-side stand-in: kernels get the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;                       // one call at a time: calls on a device share its array
void* g_scratch_ptr[kMaxDevices] = {};  // per device: the array's device address, once looked up

// The array's address on the current device (looked up on the first call
// there, with that device current).  Caller holds g_mu.
int scratch_on(int dev, void** out) {
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            messi::set_error(MESSI_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return MESSI_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MESSI_OK;
}

int fail(int code, const char* msg) {
    messi::set_error(code, msg);
    return code;
}

}  // namespace

using namespace messi;

extern "C" int messi_knn_noalloc(const messi_index* index, const float* queries, int32_t nq, int32_t k,
                                 void* stream, int64_t* out_idx, float* out_dist) {
    clear_error();
    if (!index) return fail(MESSI_EINVAL, "index is null");
    const Index* ix = reinterpret_cast<const Index*>(index);
    if (nq < 0) return fail(MESSI_EINVAL, "nq must be >= 0");
    if (k < 1 || k > MESSI_MAX_K || (int64_t)k > ix->n) return fail(MESSI_EINVAL, "k must be in [1, min(n, 1024)]");
    if (nq == 0) return MESSI_OK;
    if (!queries || !out_idx || !out_dist) return fail(MESSI_EINVAL, "null pointer argument");
    if (!is_device_pointer(queries) || !is_device_pointer(out_idx) || !is_device_pointer(out_dist))
        return fail(MESSI_EINVAL, "queries / out_idx / out_dist must be device pointers");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != ix->device)
        return fail(MESSI_EINVAL, "the index lives on another device");
    if (dev < 0 || dev >= kMaxDevices) return fail(MESSI_ENODEV, "device ordinal beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_mu);
    void* base = nullptr;
    MESSI_TRY(scratch_on(dev, &base));
    return knn_view(ix, queries, nq, k, (hipStream_t)stream, out_idx, out_dist, base, kScratchBytes);
}

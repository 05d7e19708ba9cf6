// BF16 matrix-core filter path (batched queries).
#include "common.h"

namespace messi {

int build_bf16_shadow(Index* ix, hipStream_t s) {
    (void)ix;
    (void)s;
    set_error(MESSI_EINVAL, "bf16 shadow not available in this build");
    return MESSI_EINVAL;
}

int knn_bf16(const Index* ix, const float* queries, int32_t nq, int32_t k, hipStream_t s, int64_t* out_idx,
             float* out_dist, messi_knn_stats* stats) {
    (void)ix; (void)queries; (void)nq; (void)k; (void)s; (void)out_idx; (void)out_dist; (void)stats;
    set_error(MESSI_EINVAL, "bf16 mode not available in this build");
    return MESSI_EINVAL;
}

void release_bf16(const Index* ix) { (void)ix; }

}  // namespace messi

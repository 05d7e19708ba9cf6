// Serving loop (continuous batching).
#include "common.h"

extern "C" {

messi_server* messi_server_create(const messi_index* index, size_t budget_bytes, int32_t max_slots, int32_t mode) {
    (void)index; (void)budget_bytes; (void)max_slots; (void)mode;
    messi::set_error(MESSI_EINVAL, "server not available in this build");
    return nullptr;
}
int messi_server_submit(messi_server* server, const float* host_query, int32_t k, uint64_t tag) {
    (void)server; (void)host_query; (void)k; (void)tag;
    return MESSI_EINVAL;
}
int messi_server_poll(messi_server* server, messi_result* out, int32_t max_out) {
    (void)server; (void)out; (void)max_out;
    return MESSI_EINVAL;
}
double messi_server_clock_ms(const messi_server* server) { (void)server; return 0.0; }
void messi_server_destroy(messi_server* server) { (void)server; }

}

// Serving layer (continuous batching of BKS solves).
#include "bks_internal.h"
extern "C" {
int bks_server_create(bks_ctx, const bks_server_params *, bks_server *) { return BKS_EINVAL; }
int bks_server_submit(bks_server, bks_tensor, const bks_params *, double *, double *, double *, uint64_t *) { return BKS_EINVAL; }
int bks_server_submit_coo(bks_server, int64_t, int64_t, int64_t, const int32_t *, const int32_t *, const int32_t *, const float *, const bks_params *, double *, double *, double *, uint64_t *) { return BKS_EINVAL; }
int bks_server_poll(bks_server, uint64_t, bks_result *) { return BKS_EINVAL; }
int bks_server_wait(bks_server, uint64_t, bks_result *) { return BKS_EINVAL; }
double bks_server_now(bks_server) { return 0.0; }
void bks_server_destroy(bks_server) {}
}

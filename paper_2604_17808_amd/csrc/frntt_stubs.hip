// Entry points not implemented yet.
#include "frntt_internal.hpp"
extern "C" {
int ntt_batch(frntt_ctx*, const frntt_job*, int, void*) { return FRNTT_EINVAL; }
int ntt_batch_graph(frntt_ctx*, const frntt_job*, int, void*) { return FRNTT_EINVAL; }
int frntt_tune(frntt_ctx*, int, int, int*, int*, float*, void*) { return FRNTT_EINVAL; }
int frntt_tune_save(const frntt_ctx*, const char*) { return FRNTT_EINVAL; }
int frntt_tune_load(frntt_ctx*, const char*) { return FRNTT_EINVAL; }
int frntt_server_create(frntt_server**, frntt_ctx*, size_t, int) { return FRNTT_EINVAL; }
int frntt_server_submit(frntt_server*, int, int, uint64_t, uint64_t*) { return FRNTT_EINVAL; }
int frntt_server_poll(frntt_server*, uint64_t, int*, double*) { return FRNTT_EINVAL; }
int frntt_server_result(frntt_server*, uint64_t, void*) { return FRNTT_EINVAL; }
int frntt_server_release(frntt_server*, uint64_t) { return FRNTT_EINVAL; }
int frntt_server_stats(frntt_server*, uint64_t*, uint64_t*, uint64_t*) { return FRNTT_EINVAL; }
int frntt_server_destroy(frntt_server*) { return FRNTT_EINVAL; }
}

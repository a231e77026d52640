// Request server (continuous batching): implemented in a later step.
#include "context.h"

extern "C" {
int rsl_server_create(rsl_ctx*, size_t, int, int, rsl_server**) { return RSL_EINVAL; }
int rsl_server_submit(rsl_server*, const rsl_poly*, const rsl_poly*, int, rsl_result*, uint64_t*) { return RSL_EINVAL; }
int rsl_server_poll(rsl_server*, uint64_t, int*) { return RSL_EINVAL; }
int rsl_server_wait(rsl_server*, uint64_t, int) { return RSL_EINVAL; }
int rsl_server_stats(rsl_server*, rsl_stats*) { return RSL_EINVAL; }
int rsl_server_destroy(rsl_server*) { return RSL_EINVAL; }
}

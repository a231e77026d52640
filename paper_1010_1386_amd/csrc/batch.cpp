// Batched execution of many independent problems (RSL_BATCHED).
#include "batch.h"

namespace rsl {

int run_batched(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, rsl_result* out,
                int* status, rsl_counters* cnt) {
  (void)n; (void)f; (void)g; (void)var; (void)out; (void)status; (void)cnt;
  return fail(ctx, RSL_EINVAL, "RSL_BATCHED is not available in this build");
}

void batch_release(rsl_ctx* ctx) { (void)ctx; }

}  // namespace rsl

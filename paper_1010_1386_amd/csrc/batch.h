// Batched execution of many independent problems (RSL_BATCHED).
#pragma once
#include "context.h"

namespace rsl {

int run_batched(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, rsl_result* out,
                int* status, rsl_counters* cnt);
void batch_release(rsl_ctx* ctx);

}  // namespace rsl

// Host-callable launchers of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "device.h"

namespace rsl {

// reduce -> eval+ures -> interpolation (consecutive and gapped) -> CRT, on one stream.
hipError_t launch_pipeline(const DevProblem& P, const DevTables& T, hipStream_t st);

// Stirling numbers of the first kind mod p_g for g in [g0, g0+count), rows 0..scap.
hipError_t launch_stirling_build(uint32_t* stir, int64_t sstride, const PrimeConst* pcs, int g0,
                                 int count, int scap, hipStream_t st);

}  // namespace rsl

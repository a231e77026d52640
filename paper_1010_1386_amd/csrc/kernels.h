// Host-callable launchers of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "device.h"
#include "zgcd.h"

namespace rsl {

// One launch of stage `stage` (see stages.h) over `nitems` work items, one
// block per item.  lds: dynamic LDS bytes; crt_ns: prime slots per lane of the
// CRT kernel (ceil(max primes / 64)); crt_per_block: CRT items per block
// (consecutive items of one problem share the staged constants).
hipError_t launch_stage(int stage, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                        int crt_ns, const DevTables& T, hipStream_t st, int crt_per_block = 1);

// Evaluation + univariate resultants of items that all have layout `variant`.
hipError_t launch_eval(int variant, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                       const DevTables& T, hipStream_t st);

// Pass 0, 1 or 2 of the wide CRT (t values and quotients, column sums, carries
// and output) over `nitems` items; pass 3 is pass 1 on the matrix cores.
hipError_t launch_crt_wide(int pass, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                           const DevTables& T, hipStream_t st);

// Pass 0 (reduce u, v over `nitems` items), 1 (Euclid per prime slot), 2 (pack
// the kept scaled gcds) or 3 (G and the cofactors per kept slot) of the modular gcd.
hipError_t launch_zgcd_pass(int pass, const ZgcdDesc& Z, const WorkItem* items, int nitems, const DevTables& T,
                            hipStream_t st);

// Basis change over prime groups (problems sharing a prime share the table reads).
hipError_t launch_stir_group(const DevProblem* probs, const StirGroup* groups, const StirMember* members,
                             const WorkItem* items, int nitems, size_t lds, const DevTables& T, hipStream_t st);

// Stirling numbers of the first kind mod p_g for g in [g0, g0+count), rows 0..scap.
// Segment polynomials of the basis change (stage_interp_hseg), before the stir stage.
hipError_t launch_hseg(const DevProblem* probs, const WorkItem* items, int nitems, const DevTables& T, hipStream_t st);
// Interpolation on the matrix cores: the digit planes of each (problem, slot)
// (items: problem, slot, block of 2048 positions), then the products of one
// group's columns (items: group, 64-row set, run of 16-column tiles; sub =
// tiles + 32 x the first tile's largest degree bound).  lds_bytes: the
// largest kMmColBytes + mm_operand_bytes of the items.
// which = 1: Newton coefficients into aconv; 2: the basis change into cpart.
hipError_t launch_interp_mm(int which, const DevProblem* probs, const StirGroup* groups, const StirMember* members,
                            const WorkItem* digit_items, int ndigit, const WorkItem* mm_items, int nmm,
                            int lds_bytes, const DevTables& T, hipStream_t st);
hipError_t launch_stirling_build(uint32_t* stir, int64_t sstride, const PrimeConst* pcs, int g0,
                                 int count, int scap, hipStream_t st);

// dst[t] = src[t] (or 0 when src is null) for t < n words.
hipError_t launch_copy_words(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st);
// Zero every range of a device table of n ClearRanges in one launch.
hipError_t launch_clear_ranges(const ClearRange* ranges, int n, hipStream_t st);

}  // namespace rsl

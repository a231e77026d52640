// HIP kernels of the modular resultant pipeline for gfx950 (wave64).
//
// Every stage kernel walks a host-built list of work items, one item per
// block, so that one launch per stage serves any number of problems of
// different shapes (a single problem is a batch of one).
//
//   reduce      coefficients (multi-limb) -> residues c R^2 mod p, transposed tiles
//                                                         (paper Sec. 4.1, step 1)
//   eval_ures   one lane per (prime, point): Horner evaluation at x_i and the
//               univariate resultant over Z_p             (Sec. 4.1, steps 1-2)
//   interp_conv Newton forward differences on consecutive points
//   interp_stir falling-factorial -> monomial basis (partial sums per k-chunk)
//   interp_newton divided differences on a gapped point set (bad points replaced)
//                                                         (Sec. 4.1, step 3)
//   crt         direct form with Garner fallback + radix conversion to limbs (Sec. 4.1, step 3)
//   crt_wide_*  the direct form in three passes for problems with many primes
//   stirling_build  per-prime table of Stirling numbers of the first kind
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "kernels.h"
#include "stages.h"
#include "zgcd.h"

namespace rsl {

static_assert(kCrtWaves == kCrtBlockCoeffs, "one coefficient per wave of a CRT block");

__global__ __launch_bounds__(256) void k_reduce(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  if (w.sub == 2)
    stage_reduce_words(probs[w.prob], T, w);
  else if (w.sub)
    stage_reduce_ml(probs[w.prob], T, w, lds, true);
  else
    stage_reduce(probs[w.prob], T, w, true, true);
}

template <int V>
__global__ __launch_bounds__(64) void k_eval_ures(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint4 lds4[];  // 16-byte aligned: the Horner loop reads uint4 rows
  uint32_t* lds = reinterpret_cast<uint32_t*>(lds4);
  const WorkItem w = items[blockIdx.x];
  stage_eval_variant<V>(probs[w.prob], T, w, lds);
}

hipError_t launch_eval(int variant, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                       const DevTables& T, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g(nitems), b(64);
  switch (variant) {
    case kEvBase: hipLaunchKernelGGL(k_eval_ures<kEvBase>, g, b, lds, st, probs, items, T); break;
    case kEvG2: hipLaunchKernelGGL(k_eval_ures<kEvG2>, g, b, lds, st, probs, items, T); break;
    case kEvG4: hipLaunchKernelGGL(k_eval_ures<kEvG4>, g, b, lds, st, probs, items, T); break;
    case kEvR8: hipLaunchKernelGGL(k_eval_ures<kEvR8>, g, b, lds, st, probs, items, T); break;
    case kEvR16: hipLaunchKernelGGL(k_eval_ures<kEvR16>, g, b, lds, st, probs, items, T); break;
    case kEvR24: hipLaunchKernelGGL(k_eval_ures<kEvR24>, g, b, lds, st, probs, items, T); break;
    case kEvR32: hipLaunchKernelGGL(k_eval_ures<kEvR32>, g, b, lds, st, probs, items, T); break;
    case kEvP8: hipLaunchKernelGGL(k_eval_ures<kEvP8>, g, b, lds, st, probs, items, T); break;
    case kEvP16: hipLaunchKernelGGL(k_eval_ures<kEvP16>, g, b, lds, st, probs, items, T); break;
    case kEvP24: hipLaunchKernelGGL(k_eval_ures<kEvP24>, g, b, lds, st, probs, items, T); break;
    case kEvP32: hipLaunchKernelGGL(k_eval_ures<kEvP32>, g, b, lds, st, probs, items, T); break;
    case kEvSchur: hipLaunchKernelGGL(k_eval_ures<kEvSchur>, g, b, lds, st, probs, items, T); break;
    case kEvM8: hipLaunchKernelGGL(k_eval_ures<kEvM8>, g, b, lds, st, probs, items, T); break;
    case kEvM16: hipLaunchKernelGGL(k_eval_ures<kEvM16>, g, b, lds, st, probs, items, T); break;
    case kEvM24: hipLaunchKernelGGL(k_eval_ures<kEvM24>, g, b, lds, st, probs, items, T); break;
    case kEvM32: hipLaunchKernelGGL(k_eval_ures<kEvM32>, g, b, lds, st, probs, items, T); break;
    case kEvQ8: hipLaunchKernelGGL(k_eval_ures<kEvQ8>, g, b, lds, st, probs, items, T); break;
    case kEvQ16: hipLaunchKernelGGL(k_eval_ures<kEvQ16>, g, b, lds, st, probs, items, T); break;
    case kEvQ24: hipLaunchKernelGGL(k_eval_ures<kEvQ24>, g, b, lds, st, probs, items, T); break;
    case kEvQ32: hipLaunchKernelGGL(k_eval_ures<kEvQ32>, g, b, lds, st, probs, items, T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_interp_conv(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_interp_conv(probs[w.prob], T, w, lds);
}

__global__ __launch_bounds__(256) void k_interp_stir(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_interp_stir<true>(probs[w.prob], T, w, lds);
}

__global__ __launch_bounds__(kHsegRows) void k_interp_hseg(const DevProblem* probs, const WorkItem* items, DevTables T) {
  __shared__ uint32_t lds[kHsegRows];
  const WorkItem w = items[blockIdx.x];
  stage_interp_hseg(probs[w.prob], T, w, lds);
}

hipError_t launch_hseg(const DevProblem* probs, const WorkItem* items, int nitems, const DevTables& T, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_hseg, dim3(nitems), dim3(kHsegRows), 0, st, probs, items, T);
  return hipGetLastError();
}

template <int WHICH>
__global__ __launch_bounds__(256) void k_interp_digits(const DevProblem* probs, const WorkItem* items, DevTables T) {
  const WorkItem w = items[blockIdx.x];
  stage_interp_digits<WHICH>(probs[w.prob], T, w);
}

template <int WHICH>
__global__ __launch_bounds__(256) void k_interp_mm(const DevProblem* probs, const StirGroup* groups,
                                                   const StirMember* members, const WorkItem* items, DevTables T) {
  extern __shared__ uint64_t lds8[];
  const WorkItem w = items[blockIdx.x];
  stage_interp_mm<WHICH>(probs, groups[w.prob], members, w, T, reinterpret_cast<uint8_t*>(lds8));
}

hipError_t launch_interp_mm(int which, const DevProblem* probs, const StirGroup* groups, const StirMember* members,
                            const WorkItem* digit_items, int ndigit, const WorkItem* mm_items, int nmm,
                            int lds_bytes, const DevTables& T, hipStream_t st) {
  if (ndigit > 0) {
    if (which == 1) hipLaunchKernelGGL(k_interp_digits<1>, dim3(ndigit), dim3(256), 0, st, probs, digit_items, T);
    else hipLaunchKernelGGL(k_interp_digits<2>, dim3(ndigit), dim3(256), 0, st, probs, digit_items, T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nmm <= 0) return hipSuccess;
  if (lds_bytes < kMmColBytes || lds_bytes > 65536) return hipErrorInvalidValue;
  if (which == 1)
    hipLaunchKernelGGL(k_interp_mm<1>, dim3(nmm), dim3(256), lds_bytes, st, probs, groups, members, mm_items, T);
  else
    hipLaunchKernelGGL(k_interp_mm<2>, dim3(nmm), dim3(256), lds_bytes, st, probs, groups, members, mm_items, T);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_interp_newton(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_interp_newton(probs[w.prob], T, w, lds);
}

template <int NS>
__global__ __launch_bounds__(512) void k_crt(const DevProblem* probs, const WorkItem* items, int nitems, int per,
                                             DevTables T) {
  extern __shared__ uint32_t lds[];
  // items blockIdx.x * per .. + per - 1 (one problem's items are consecutive:
  // the constants and limb table are staged again only when the problem changes)
  for (int b = 0; b < per; ++b) {
    const int idx = blockIdx.x * per + b;
    if (idx >= nitems) break;  // block-uniform
    const WorkItem w = items[idx];
    const bool fresh = b == 0 || items[idx - 1].prob != w.prob;
    if (b > 0) __syncthreads();  // the previous item's waves are done with the LDS
    stage_crt<NS>(probs[w.prob], T, w, lds, kCrtBlockCoeffs / static_cast<int>(blockDim.x >> 6), fresh);
  }
}

__global__ __launch_bounds__(256) void k_crt_wide_t(const DevProblem* probs, const WorkItem* items, DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_crt_wide_t(probs[w.prob], T, w, lds);
}

__global__ __launch_bounds__(kWideHT) void k_crt_wide_sum(const DevProblem* probs, const WorkItem* items) {
  extern __shared__ uint4 lds4[];  // 16-byte aligned: rows of t values are read as uint4
  const WorkItem w = items[blockIdx.x];
  stage_crt_wide_sum(probs[w.prob], w, reinterpret_cast<uint32_t*>(lds4));
}

__global__ __launch_bounds__(64) void k_crt_wide_fin(const DevProblem* probs, const WorkItem* items) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_crt_wide_fin(probs[w.prob], w, lds);
}

__global__ __launch_bounds__(256) void k_crt_wide_sum_mfma(const DevProblem* probs, const WorkItem* items) {
  extern __shared__ uint4 lds4[];
  const WorkItem w = items[blockIdx.x];
  stage_crt_wide_sum_mfma(probs[w.prob], w, reinterpret_cast<uint32_t*>(lds4));
}

hipError_t launch_crt_wide(int pass, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                           const DevTables& T, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g(nitems);
  switch (pass) {
    case 0: hipLaunchKernelGGL(k_crt_wide_t, g, dim3(256), lds, st, probs, items, T); break;
    case 1: hipLaunchKernelGGL(k_crt_wide_sum, g, dim3(kWideHT), lds, st, probs, items); break;
    case 2: hipLaunchKernelGGL(k_crt_wide_fin, g, dim3(64), lds, st, probs, items); break;
    case 3: hipLaunchKernelGGL(k_crt_wide_sum_mfma, g, dim3(256), lds, st, probs, items); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(kZThreads) void k_zreduce(ZgcdDesc Z, const WorkItem* items, DevTables T) {
  stage_zreduce(Z, T, items[blockIdx.x]);
}
__global__ __launch_bounds__(64) void k_zgcd(ZgcdDesc Z, DevTables T) {
  extern __shared__ uint32_t lds[];
  stage_zgcd(Z, T, blockIdx.x, lds);
}
__global__ __launch_bounds__(kZThreads) void k_zpack(ZgcdDesc Z, DevTables T) { stage_zpack(Z, T, blockIdx.x); }
__global__ __launch_bounds__(64) void k_zcof(ZgcdDesc Z, DevTables T) {
  extern __shared__ uint32_t lds[];
  stage_zcof(Z, T, blockIdx.x, lds);
}

hipError_t launch_zgcd_pass(int pass, const ZgcdDesc& Z, const WorkItem* items, int nitems, const DevTables& T,
                            hipStream_t st) {
  const dim3 b(kZThreads);
  switch (pass) {
    case 0:
      if (nitems <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_zreduce, dim3(nitems), b, 0, st, Z, items, T);
      break;
    case 1:
      if (Z.np <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_zgcd, dim3(Z.np), dim3(64), static_cast<size_t>(zgcd_lds_words(Z)) * 4, st, Z, T);
      break;
    case 2:
      if (Z.nk <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_zpack, dim3(Z.nk), b, 0, st, Z, T);
      break;
    case 3:
      if (Z.nk <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_zcof, dim3(Z.nk), dim3(64), static_cast<size_t>(zcof_lds_words(Z)) * 4, st, Z, T);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// s(k+1, j) = s(k, j-1) - k s(k, j); one block per prime, rows in LDS.
__global__ __launch_bounds__(1024) void k_stirling_build(uint32_t* stir, int64_t sstride,
                                                         const PrimeConst* pcs, int g0, int scap) {
  extern __shared__ uint32_t sm[];
  const int g = g0 + blockIdx.x;
  const PrimeConst pc = pcs[g];
  uint32_t* cur = sm;
  uint32_t* nxt = sm + (scap + 2);
  uint32_t* S = stir + static_cast<int64_t>(g) * sstride;
  if (threadIdx.x == 0) { cur[0] = pc.r1; S[0] = pc.r1; }
  __syncthreads();
  for (int k = 0; k < scap; ++k) {
    const uint32_t kt = mmul(static_cast<uint32_t>(k), pc.r2, pc.p, pc.pinv);
    const bool keep = ((k + 1) % kCkpt) == 0;  // a checkpoint row
    uint32_t* row = S + ckpt_rowoff((k + 1) / kCkpt);
    for (int j = threadIdx.x; j <= k + 1; j += 1024) {
      const uint32_t left = (j > 0) ? cur[j - 1] : 0u;
      const uint32_t mid = (j <= k) ? cur[j] : 0u;
      const uint32_t v = msubm(left, mmul(mid, kt, pc.p, pc.pinv), pc.p);
      nxt[j] = v;
      if (keep) row[j] = v;
    }
    __syncthreads();
    uint32_t* t = cur; cur = nxt; nxt = t;
  }
}

// ------------------------------------------------------------ launchers

__global__ __launch_bounds__(256) void k_interp_stir_group(const DevProblem* probs, const StirGroup* groups,
                                                           const StirMember* members, const WorkItem* items,
                                                           DevTables T) {
  extern __shared__ uint32_t lds[];
  const WorkItem w = items[blockIdx.x];
  stage_interp_stir_group(probs, groups, members, T, w, lds);
}

hipError_t launch_stir_group(const DevProblem* probs, const StirGroup* groups, const StirMember* members,
                             const WorkItem* items, int nitems, size_t lds, const DevTables& T, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_stir_group, dim3(nitems), dim3(256), lds, st, probs, groups, members,
                     items, T);
  return hipGetLastError();
}

hipError_t launch_stage(int stage, const DevProblem* probs, const WorkItem* items, int nitems, size_t lds,
                        int crt_ns, const DevTables& T, hipStream_t st, int crt_per_block) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g(nitems);
  const int per = crt_per_block > 1 ? crt_per_block : 1;
  const dim3 gc((nitems + per - 1) / per);
  switch (stage) {
    case kStageReduce: hipLaunchKernelGGL(k_reduce, g, dim3(256), lds, st, probs, items, T); break;
    case kStageEval: return hipErrorInvalidValue;  // launch_eval: one kernel per layout
    case kStageConv: hipLaunchKernelGGL(k_interp_conv, g, dim3(256), lds, st, probs, items, T); break;
    case kStageStir: hipLaunchKernelGGL(k_interp_stir, g, dim3(256), lds, st, probs, items, T); break;
    case kStageNewton: hipLaunchKernelGGL(k_interp_newton, g, dim3(1024), lds, st, probs, items, T); break;
    case kStageCrt:
      switch (crt_ns) {
        case 1: hipLaunchKernelGGL(k_crt<1>, gc, dim3(kCrtWaves * 64), lds, st, probs, items, nitems, per, T); break;
        case 2: hipLaunchKernelGGL(k_crt<2>, gc, dim3(kCrtWaves * 64), lds, st, probs, items, nitems, per, T); break;
        case 3: hipLaunchKernelGGL(k_crt<3>, gc, dim3(kCrtWaves * 64), lds, st, probs, items, nitems, per, T); break;
        case 4: hipLaunchKernelGGL(k_crt<4>, gc, dim3(kCrtWaves * 64), lds, st, probs, items, nitems, per, T); break;
        case 6:
          hipLaunchKernelGGL(k_crt<6>, gc, dim3(crt_block_waves(6) * 64), lds, st, probs, items, nitems, per, T);
          break;
        case 8:
          hipLaunchKernelGGL(k_crt<8>, gc, dim3(crt_block_waves(8) * 64), lds, st, probs, items, nitems, per, T);
          break;
        default: return hipErrorInvalidValue;
      }
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Device-to-device word copy / fill, launched as kernels so that a resident
// job's per-run resets are plain kernel nodes when the run is captured in a graph.
__global__ __launch_bounds__(256) void k_copy_words(uint32_t* dst, const uint32_t* src, size_t n) {
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += static_cast<size_t>(gridDim.x) * blockDim.x)
    dst[t] = src ? src[t] : 0u;
}

hipError_t launch_copy_words(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_copy_words, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

// Workgroup b clears part (b mod kClearSplit) of range b / kClearSplit.
constexpr int kClearSplit = 16;
__global__ __launch_bounds__(256) void k_clear_ranges(const ClearRange* ranges) {
  const ClearRange r = ranges[blockIdx.x / kClearSplit];
  const size_t stride = static_cast<size_t>(kClearSplit) * 256;
  for (size_t t = static_cast<size_t>(blockIdx.x % kClearSplit) * 256 + threadIdx.x; t < r.words; t += stride)
    r.dst[t] = 0u;
}

hipError_t launch_clear_ranges(const ClearRange* ranges, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_ranges, dim3(static_cast<unsigned>(n) * kClearSplit), dim3(256), 0, st, ranges);
  return hipGetLastError();
}

hipError_t launch_stirling_build(uint32_t* stir, int64_t sstride, const PrimeConst* pcs, int g0,
                                 int count, int scap, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stirling_build, dim3(count), dim3(1024),
                     static_cast<size_t>(2) * (scap + 2) * sizeof(uint32_t), st, stir, sstride, pcs, g0, scap);
  return hipGetLastError();
}

}  // namespace rsl

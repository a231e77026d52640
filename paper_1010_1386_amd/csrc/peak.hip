// Issue-rate microbenchmarks of the gfx950 units the resultant kernels use
// (measurement only; not called by the library).  Each kernel runs K
// independent dependency chains per lane for `iters` iterations over a grid of
// `waves_per_simd` waves on every SIMD; the host times it with HIP events and
// reports operations per second (lane operations for the vector ALU kinds,
// integer multiply-adds for the matrix-core kind).
//
//   kind 0  v_add_u32                   (one lane op per chain step, plus one xor per
//                                        iteration shared by the chains)
//   kind 1  v_mul_lo_u32
//   kind 2  32 x 32 -> 64 multiply-add  (v_mad_u64_u32)
//   kind 3  Montgomery product          (mmul: three multiplies, the final min)
//   kind 4  fused three-product update  (mmad3: the remainder-sequence step)
//   kind 5  int8 16x16x32 matrix product (v_mfma_i32_16x16x32_i8), MACs
#include <hip/hip_runtime.h>

#include <cstdint>

#include "modarith.h"

namespace rsl {
namespace {

constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void k_peak(uint32_t* sink, int iters, uint32_t p, uint32_t pinv, uint32_t seed) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (seed ^ (t * 2654435761u) ^ (c * 40503u)) % p;
  const uint32_t y = (seed * 7u + t) % p, z = (seed * 13u + 3u * t) % p;
  uint64_t acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = x[c];
  typedef int v4i __attribute__((ext_vector_type(4)));
  v4i S[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) S[c] = v4i{static_cast<int>(x[c]), 0, 0, 0};
  const long a8 = static_cast<long>(static_cast<uint64_t>(x[0]) * 0x0101010101010101ull);
  const long b8 = static_cast<long>(static_cast<uint64_t>(y) * 0x0001000100010001ull);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == 0) x[c] = x[c] + (y ^ static_cast<uint32_t>(i));  // no closed form
      else if constexpr (KIND == 1) x[c] = x[c] * y;
      else if constexpr (KIND == 2) acc[c] = static_cast<uint64_t>(static_cast<uint32_t>(acc[c])) * y + acc[c];
      else if constexpr (KIND == 3) x[c] = mmul(x[c], y, p, pinv);
      else if constexpr (KIND == 4) x[c] = mmad3(y, x[c], z, x[c], y, x[c] ^ 1u, p, pinv);
      else S[c] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a8, b8, S[c], 0, 0, 0);
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    if constexpr (KIND == 2) r ^= static_cast<uint32_t>(acc[c] ^ (acc[c] >> 32));
    else if constexpr (KIND == 5) r ^= static_cast<uint32_t>(S[c][0] ^ S[c][1] ^ S[c][2] ^ S[c][3]);
    else r ^= x[c];
  }
  if (r == 0x9E3779B9u) sink[t] = r;  // keeps the chains live; practically never taken
}

template <int KIND>
hipError_t launch_peak(int blocks, uint32_t* sink, int iters, uint32_t p, uint32_t pinv, hipStream_t st) {
  hipLaunchKernelGGL(k_peak<KIND>, dim3(blocks), dim3(256), 0, st, sink, iters, p, pinv, 12345u);
  return hipGetLastError();
}

}  // namespace
}  // namespace rsl

using namespace rsl;

// Rate of `kind` (see above) in operations per second on `device`, measured
// over `reps` timed launches after one warm-up.  cus: compute units of the
// device (the grid is cus x 4 SIMDs x waves_per_simd waves).  Returns 0 on
// success, a negative value on a HIP error or bad argument.  sink: device
// buffer of at least cus * 4 * waves_per_simd * 64 words (written almost never).
extern "C" int rsl_peak_rate(int device, int kind, int cus, int waves_per_simd, int iters, int reps,
                             uint32_t* sink, double* ops_per_s) {
  if (!ops_per_s || !sink || kind < 0 || kind > 5 || cus < 1 || waves_per_simd < 1 || iters < 1 || reps < 1)
    return -1;
  if (hipSetDevice(device) != hipSuccess) return -2;
  const uint32_t p = 1431655751u;  // the largest prime below 2^32 / 3, as in the library's table
  const PrimeConst pc = make_prime_const(p);
  const int blocks = cus * 4 * waves_per_simd / 4;  // 256-thread blocks = 4 waves each
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -2;
  auto launch = [&]() -> hipError_t {
    switch (kind) {
      case 0: return launch_peak<0>(blocks, sink, iters, p, pc.pinv, nullptr);
      case 1: return launch_peak<1>(blocks, sink, iters, p, pc.pinv, nullptr);
      case 2: return launch_peak<2>(blocks, sink, iters, p, pc.pinv, nullptr);
      case 3: return launch_peak<3>(blocks, sink, iters, p, pc.pinv, nullptr);
      case 4: return launch_peak<4>(blocks, sink, iters, p, pc.pinv, nullptr);
      default: return launch_peak<5>(blocks, sink, iters, p, pc.pinv, nullptr);
    }
  };
  int rc = 0;
  if (launch() != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) rc = -3;
  float ms = 0.f;
  if (!rc && hipEventRecord(e0, nullptr) != hipSuccess) rc = -3;
  for (int r = 0; !rc && r < reps; ++r)
    if (launch() != hipSuccess) rc = -3;
  if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = -3;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const double lanes = static_cast<double>(blocks) * 256;
  const double steps = lanes * kChains * static_cast<double>(iters) * reps;
  // a 16x16x32 product is 8192 multiply-adds per wave: 128 per lane
  const double per_step = (kind == 5) ? 128.0 : 1.0;
  *ops_per_s = steps * per_step / (ms * 1e-3);
  return 0;
}

// rsl_res_static: the synchronous single resultant without any device or
// pinned-memory allocation.  Its job (inputs, residues, values, partial sums,
// statuses, outputs) is laid out in `scratch`, a fixed device array of this
// library, instead of the context's workspace.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "context.h"
#include "job.h"
#include "kernels.h"

namespace rsl {

// The job region of rsl_res_static.  A host-side use of this name is a host
// stand-in, not a device address: every use goes through the address that
// hipGetSymbolAddress returns on the current device (scratch_on below).
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current), looked
// up once per device.
int scratch_on(rsl_ctx* ctx, int device, uint8_t** out) {
  if (device < 0 || device >= kMaxDevices) return fail(ctx, RSL_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_check(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch_ptr[device] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_ptr[device];
  return RSL_OK;
}

}  // namespace
}  // namespace rsl

using namespace rsl;

extern "C" int rsl_res_static(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts,
                              rsl_result* out) {
  if (!ctx || !out) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  const double t0 = now_ms();
  rsl_counters cnt{};
  uint8_t* base = nullptr;
  int rc = scratch_on(ctx, ctx->device, &base);
  if (rc) return rc;
  Job J;
  std::string err;
  job_plan(1, f, g, &var, opts, &J, &err);
  // host layout only: the constant tables are not grown here (that would allocate)
  rc = job_build(ctx, 1, f, g, &var, opts, &J, &err, nullptr, true, true);
  if (rc) return fail(ctx, rc, err);
  if (!J.live.empty()) {
    if (J.total > kStaticScratchBytes)
      return fail(ctx, RSL_ENOMEM, "footprint of " + std::to_string(J.total) + " bytes > the " +
                                       std::to_string(kStaticScratchBytes) + "-byte static scratch");
    if (J.need_g > ctx->npcap || J.need_E > ctx->kcap || J.need_D > ctx->scap)
      return fail(ctx, RSL_ENOMEM, "the context's constant tables do not cover this problem (an earlier "
                                   "rsl_res or rsl_batch of a problem at least this large grows them)");
    // upload image and download buffer in ordinary (pageable) host memory
    job_bind(&J, base, nullptr, false);
    J.direct_image = true;
    std::vector<uint8_t> down(J.down_bytes);
    hipStream_t st = ctx->stream;
    if ((rc = job_upload(ctx, &J, st)) || (rc = hip_check(ctx, hipEventRecord(ctx->e0, st), "event")) ||
        (rc = job_launch(ctx, &J, RSL_STAGED, st, false)) ||
        (rc = hip_check(ctx, hipEventRecord(ctx->e1, st), "event")) ||
        (rc = job_download(ctx, &J, down.data(), st)) ||
        (rc = hip_check(ctx, hipStreamSynchronize(st), "hipStreamSynchronize")))
      return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->e0, ctx->e1);
    cnt.ms_device = ms;
    rc = job_decode(ctx, J, down.data(), out, nullptr, &cnt);
  } else {
    rc = job_decode(ctx, J, nullptr, out, nullptr, &cnt);
  }
  if (rc && !err.empty() && ctx->err.empty()) ctx->err = err;
  cnt.ms_total = now_ms() - t0;
  ctx->last = cnt;
  return rc;
}

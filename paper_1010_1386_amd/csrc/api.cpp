// C-ABI entry points (include/rsl.h): contexts, tables, the plain pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "batch.h"
#include "context.h"
#include "kernels.h"

namespace rsl {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int fail(rsl_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_check(rsl_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return RSL_OK;
  if (ctx) {
    ctx->poisoned = true;
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return RSL_EDEVICE;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static void free_tables(rsl_ctx* c) {
  for (void* p : {static_cast<void*>(c->d_pc), static_cast<void*>(c->d_fact),
                  static_cast<void*>(c->d_ifact), static_cast<void*>(c->d_stir),
                  static_cast<void*>(c->d_Tg), static_cast<void*>(c->d_invM),
                  static_cast<void*>(c->d_Plimb)})
    if (p) (void)hipFree(p);
  c->d_pc = nullptr;
  c->d_fact = c->d_ifact = c->d_stir = c->d_Tg = c->d_invM = c->d_Plimb = nullptr;
  c->npcap = 0;
  c->kcap = c->scap = -1;
}

int ensure_tables(rsl_ctx* ctx, int np, int kneed, int sneed) {
  if (np <= ctx->npcap && kneed <= ctx->kcap && sneed <= ctx->scap) return RSL_OK;
  const int new_np = std::max(ctx->npcap, static_cast<int>(align_up(std::max(np, 1), 64)));
  const int new_k = std::max(ctx->kcap, static_cast<int>(align_up(kneed + 1, 256)) - 1);
  const int new_s = std::max(ctx->scap, static_cast<int>(align_up(sneed + 1, 256)) - 1);
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (rc) return rc;
  free_tables(ctx);

  const std::vector<uint32_t>& tab = prime_table(new_np);
  if (static_cast<int>(tab.size()) < new_np) return fail(ctx, RSL_EPRIMES, "prime table exhausted");
  std::vector<uint32_t> primes(tab.begin(), tab.begin() + new_np);
  std::vector<PrimeConst> pc(new_np);
  for (int g = 0; g < new_np; ++g) pc[g] = make_prime_const(primes[g]);

  // factorials and inverse factorials, Montgomery form
  const int ks = new_k + 1;
  std::vector<uint32_t> fact(static_cast<size_t>(new_np) * ks), ifact(fact.size());
  for (int g = 0; g < new_np; ++g) {
    const uint64_t p = primes[g];
    std::vector<uint64_t> f(ks);
    f[0] = 1;
    for (int t = 1; t < ks; ++t) f[t] = f[t - 1] * static_cast<uint64_t>(t) % p;
    uint64_t inv = 1, b = f[ks - 1], e = p - 2;
    while (e) {
      if (e & 1) inv = inv * b % p;
      b = b * b % p;
      e >>= 1;
    }
    std::vector<uint64_t> fi(ks);
    fi[ks - 1] = inv;
    for (int t = ks - 1; t > 0; --t) fi[t - 1] = fi[t] * static_cast<uint64_t>(t) % p;
    for (int t = 0; t < ks; ++t) {
      fact[static_cast<size_t>(g) * ks + t] = static_cast<uint32_t>((f[t] << 32) % p);
      ifact[static_cast<size_t>(g) * ks + t] = static_cast<uint32_t>((fi[t] << 32) % p);
    }
  }
  // canonical CRT tables
  const int LPg = (31 * new_np + 31) / 32 + 1;
  std::vector<uint32_t> Tg, invM, Plimb;
  crt_tables(primes, LPg, &Tg, &invM, &Plimb);

  const int64_t sstride = static_cast<int64_t>(align_up(static_cast<size_t>(new_s + 1) * (new_s + 2) / 2, 64));
  auto dmalloc = [&](void** p, size_t bytes) { return hip_check(ctx, hipMalloc(p, bytes), "hipMalloc(tables)"); };
  if ((rc = dmalloc(reinterpret_cast<void**>(&ctx->d_pc), sizeof(PrimeConst) * new_np)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_fact), fact.size() * 4)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_ifact), ifact.size() * 4)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_stir), static_cast<size_t>(new_np) * sstride * 4)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_Tg), Tg.size() * 4)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_invM), invM.size() * 4)) ||
      (rc = dmalloc(reinterpret_cast<void**>(&ctx->d_Plimb), Plimb.size() * 4))) {
    free_tables(ctx);
    return rc;
  }
  auto up = [&](void* d, const void* h, size_t bytes) {
    return hip_check(ctx, hipMemcpy(d, h, bytes, hipMemcpyHostToDevice), "hipMemcpy(tables)");
  };
  if ((rc = up(ctx->d_pc, pc.data(), sizeof(PrimeConst) * new_np)) ||
      (rc = up(ctx->d_fact, fact.data(), fact.size() * 4)) ||
      (rc = up(ctx->d_ifact, ifact.data(), ifact.size() * 4)) ||
      (rc = up(ctx->d_Tg, Tg.data(), Tg.size() * 4)) ||
      (rc = up(ctx->d_invM, invM.data(), invM.size() * 4)) ||
      (rc = up(ctx->d_Plimb, Plimb.data(), Plimb.size() * 4)))
    return rc;
  if ((rc = hip_check(ctx, launch_stirling_build(ctx->d_stir, sstride, ctx->d_pc, 0, new_np, new_s, ctx->stream),
                      "stirling build")) ||
      (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stirling build sync")))
    return rc;
  ctx->npcap = new_np;
  ctx->kcap = new_k;
  ctx->scap = new_s;
  ctx->kstride = ks;
  ctx->sstride = sstride;
  ctx->LPg = LPg;
  return RSL_OK;
}

DevTables tables_of(const rsl_ctx* ctx) {
  DevTables T{};
  T.pc = ctx->d_pc;
  T.fact = ctx->d_fact;
  T.ifact = ctx->d_ifact;
  T.stir = ctx->d_stir;
  T.sstride = ctx->sstride;
  T.kstride = ctx->kstride;
  T.kcap = ctx->kcap;
  T.scap = ctx->scap;
  T.npcap = ctx->npcap;
  return T;
}

int ensure_staging(rsl_ctx* ctx, size_t up, size_t down) {
  if (up > ctx->h_up_bytes) {
    if (ctx->h_up) (void)hipHostFree(ctx->h_up);
    ctx->h_up = nullptr;
    ctx->h_up_bytes = 0;
    size_t sz = align_up(std::max(up, static_cast<size_t>(1) << 20), 1 << 20);
    int rc = hip_check(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->h_up), sz, hipHostMallocDefault),
                       "hipHostMalloc");
    if (rc) return rc;
    ctx->h_up_bytes = sz;
  }
  if (down > ctx->h_down_bytes) {
    if (ctx->h_down) (void)hipHostFree(ctx->h_down);
    ctx->h_down = nullptr;
    ctx->h_down_bytes = 0;
    size_t sz = align_up(std::max(down, static_cast<size_t>(1) << 20), 1 << 20);
    int rc = hip_check(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->h_down), sz, hipHostMallocDefault),
                       "hipHostMalloc");
    if (rc) return rc;
    ctx->h_down_bytes = sz;
  }
  return RSL_OK;
}

Layout layout_of(const Plan& P) {
  Layout L;
  const size_t A = 256;
  L.L_in = std::max(P.f.L, P.g.L);
  const int ncoef = P.goff + (P.ny + 1) * P.rowg;
  size_t o = 0;
  L.u_coeff = o; o = align_up(o + static_cast<size_t>(ncoef) * L.L_in * 4, A);
  L.u_rdeg = o;  o = align_up(o + static_cast<size_t>(P.my + P.ny + 2) * 4, A);
  L.u_pidx = o;  o = align_up(o + static_cast<size_t>(P.np) * 4, A);
  L.u_Hm = o;    o = align_up(o + static_cast<size_t>(P.np) * 4, A);
  L.u_NH = o;    o = align_up(o + static_cast<size_t>(P.L_out) * 4, A);
  if (!P.canonical) {
    L.u_Tg = o;    o = align_up(o + static_cast<size_t>(P.np) * P.np * 4, A);
    L.u_invM = o;  o = align_up(o + static_cast<size_t>(P.np) * 4, A);
    L.u_Plimb = o; o = align_up(o + static_cast<size_t>(P.np) * P.L_out * 4, A);
  }
  L.u_status = o; o = align_up(o + static_cast<size_t>(P.np + 2) * 4, A);
  L.up_off = 0;
  L.up_bytes = o;
  const size_t np = P.np;
  L.resid = o; o = align_up(o + np * P.CS * 4, A);
  L.zval = o;  o = align_up(o + np * (P.E + 1) * 4, A);
  L.zbad = o;  o = align_up(o + np * (P.E + 1), A);
  L.aconv = o; o = align_up(o + np * (P.D + 1) * 4, A);
  L.cres = o;  o = align_up(o + np * (P.D + 1) * 4, A);
  L.out = o;
  L.out_bytes = static_cast<size_t>(P.D + 1) * P.L_out * 4;
  o = align_up(o + L.out_bytes, A);
  L.status = L.u_status;
  L.status_bytes = static_cast<size_t>(P.np + 2) * 4;
  L.total = o;
  return L;
}

void fill_upload(const Plan& P, const Layout& L, uint8_t* blob) {
  // coefficients: f tile rows 0..my (stride rowf), then g tile rows 0..ny (stride rowg),
  // sign-extended to L_in limbs
  uint32_t* c = reinterpret_cast<uint32_t*>(blob + L.u_coeff);
  const int Li = L.L_in;
  auto put = [&](const View& V, int rows, int rowstride, size_t base) {
    for (int j = 0; j < rows; ++j)
      for (int i = 0; i < rowstride; ++i) {
        uint32_t* dst = c + (base + static_cast<size_t>(j) * rowstride + i) * Li;
        if (i <= V.rdeg[j]) {
          const uint32_t* src = &V.c[(static_cast<size_t>(j) * (V.dx + 1) + i) * V.L];
          const uint32_t ext = (src[V.L - 1] >> 31) ? 0xFFFFFFFFu : 0u;
          for (int l = 0; l < Li; ++l) dst[l] = (l < V.L) ? src[l] : ext;
        } else {
          for (int l = 0; l < Li; ++l) dst[l] = 0;
        }
      }
  };
  put(P.f, P.my + 1, P.rowf, 0);
  put(P.g, P.ny + 1, P.rowg, static_cast<size_t>(P.goff));
  int* rd = reinterpret_cast<int*>(blob + L.u_rdeg);
  for (int j = 0; j <= P.my; ++j) rd[j] = P.f.rdeg[j];
  for (int j = 0; j <= P.ny; ++j) rd[P.my + 1 + j] = P.g.rdeg[j];
  std::memcpy(blob + L.u_pidx, P.pidx.data(), P.np * 4);
  std::memcpy(blob + L.u_Hm, P.Hm.data(), P.np * 4);
  std::memcpy(blob + L.u_NH, P.NH.data(), P.L_out * 4);
  if (!P.canonical) {
    std::memcpy(blob + L.u_Tg, P.Tg.data(), P.Tg.size() * 4);
    std::memcpy(blob + L.u_invM, P.invM.data(), P.invM.size() * 4);
    std::memcpy(blob + L.u_Plimb, P.Plimb.data(), P.Plimb.size() * 4);
  }
  std::memset(blob + L.u_status, 0, static_cast<size_t>(P.np + 2) * 4);
}

DevProblem dev_problem(const rsl_ctx* ctx, const Plan& P, const Layout& L, uint8_t* base) {
  DevProblem d{};
  d.my = P.my;
  d.ny = P.ny;
  d.rowf = P.rowf;
  d.rowg = P.rowg;
  d.goff = P.goff;
  d.CS = P.CS;
  d.ncoef = P.goff + (P.ny + 1) * P.rowg;
  d.L_in = L.L_in;
  d.D = P.D;
  d.E = P.E;
  d.origin = P.origin;
  d.formal = P.formal;
  d.np = P.np;
  d.L_out = P.L_out;
  uint8_t* up = base + L.up_off;
  d.coeff = reinterpret_cast<const uint32_t*>(up + L.u_coeff);
  d.rdeg = reinterpret_cast<const int*>(up + L.u_rdeg);
  d.pidx = reinterpret_cast<const int*>(up + L.u_pidx);
  d.Hm = reinterpret_cast<const uint32_t*>(up + L.u_Hm);
  d.NH = reinterpret_cast<const uint32_t*>(up + L.u_NH);
  if (P.canonical) {
    d.Tg = ctx->d_Tg;
    d.tgs = ctx->npcap;
    d.invM = ctx->d_invM;
    d.Plimb = ctx->d_Plimb;
    d.LP = ctx->LPg;
  } else {
    d.Tg = reinterpret_cast<const uint32_t*>(up + L.u_Tg);
    d.tgs = P.np;
    d.invM = reinterpret_cast<const uint32_t*>(up + L.u_invM);
    d.Plimb = reinterpret_cast<const uint32_t*>(up + L.u_Plimb);
    d.LP = P.L_out;
  }
  d.resid = reinterpret_cast<uint32_t*>(base + L.resid);
  d.zval = reinterpret_cast<uint32_t*>(base + L.zval);
  d.zbad = base + L.zbad;
  d.aconv = reinterpret_cast<uint32_t*>(base + L.aconv);
  d.cres = reinterpret_cast<uint32_t*>(base + L.cres);
  d.out = reinterpret_cast<uint32_t*>(base + L.out);
  d.status = reinterpret_cast<int*>(up + L.u_status);
  return d;
}

// Signed limbs needed by a two's complement value.
static int signed_limbs(const uint32_t* c, int L) {
  int n = L;
  while (n > 1) {
    const uint32_t top = c[n - 1], below = c[n - 2] >> 31;
    if ((top == 0u && below == 0u) || (top == 0xFFFFFFFFu && below == 1u)) --n;
    else break;
  }
  return n;
}

int decode_result(const Plan& P, const uint32_t* limbs, rsl_result* out) {
  if (!out) return RSL_EINVAL;
  int deg = -1, need = 1;
  if (!P.zero) {
    const int L = P.L_out;
    for (int k = 0; k <= P.D; ++k) {
      const uint32_t* c = limbs + static_cast<size_t>(k) * L;
      bool nz = false;
      for (int l = 0; l < L; ++l) nz |= (c[l] != 0u);
      if (nz) {
        deg = k;
        need = std::max(need, signed_limbs(c, L));
      }
    }
  }
  out->deg = deg;
  out->needed_limbs = need;
  if (deg < 0) return RSL_OK;
  if (out->limbs < need || out->cap_deg < deg || !out->coeff) return RSL_ERANGE;
  const int L = P.L_out;
  for (int k = 0; k <= deg; ++k) {
    const uint32_t* c = limbs + static_cast<size_t>(k) * L;
    const uint32_t ext = (c[L - 1] >> 31) ? 0xFFFFFFFFu : 0u;
    uint32_t* dst = out->coeff + static_cast<size_t>(k) * out->limbs;
    for (int l = 0; l < out->limbs; ++l) dst[l] = (l < L) ? c[l] : ext;
  }
  return RSL_OK;
}

// One problem on the context stream, synchronously.
static int run_plain(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts,
                     rsl_result* out, rsl_counters* cnt) {
  if (!out) return fail(ctx, RSL_EINVAL, "null result");
  Plan P;
  int rc = make_plan(f, g, var, opts, &P, &ctx->err);
  if (rc) return rc;
  cnt->problems += 1;
  if (P.zero) return decode_result(P, nullptr, out);
  if (P.np > 256) return fail(ctx, RSL_EINVAL, "more than 256 primes needed (coefficients too large)");
  if (P.E > 3800) return fail(ctx, RSL_EINVAL, "more than 3800 evaluation points needed (degree bound too large)");
  int maxg = 0;
  for (int g0 : P.pidx) maxg = std::max(maxg, g0 + 1);
  if ((rc = ensure_tables(ctx, maxg, P.E, P.D))) return rc;
  Layout L = layout_of(P);
  if (L.total > ctx->ws_bytes)
    return fail(ctx, RSL_ENOMEM, "workspace of " + std::to_string(ctx->ws_bytes) + " bytes < footprint " +
                                     std::to_string(L.total));
  if ((rc = ensure_staging(ctx, L.up_bytes, L.out_bytes + L.status_bytes))) return rc;
  fill_upload(P, L, ctx->h_up);
  DevProblem dp = dev_problem(ctx, P, L, ctx->ws);
  DevTables T = tables_of(ctx);
  hipStream_t st = ctx->stream;
  if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->ws + L.up_off, ctx->h_up, L.up_bytes, hipMemcpyHostToDevice, st),
                      "upload")) ||
      (rc = hip_check(ctx, hipEventRecord(ctx->e0, st), "event")) ||
      (rc = hip_check(ctx, launch_pipeline(dp, T, st), "launch")) ||
      (rc = hip_check(ctx, hipEventRecord(ctx->e1, st), "event")) ||
      (rc = hip_check(ctx, hipMemcpyAsync(ctx->h_down, ctx->ws + L.out, L.out_bytes, hipMemcpyDeviceToHost, st),
                      "download")) ||
      (rc = hip_check(ctx, hipMemcpyAsync(ctx->h_down + L.out_bytes, ctx->ws + L.status, L.status_bytes,
                                          hipMemcpyDeviceToHost, st), "download")) ||
      (rc = hip_check(ctx, hipStreamSynchronize(st), "hipStreamSynchronize")))
    return rc;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ctx->e0, ctx->e1);
  cnt->ms_device += ms;
  const int* status = reinterpret_cast<const int*>(ctx->h_down + L.out_bytes);
  if (status[0] & kErrTooFewGoodPoints) return fail(ctx, RSL_EPRIMES, "fewer than D+1 good points for a prime");
  cnt->pairs += static_cast<int64_t>(P.np) * (P.E + 1);
  cnt->bad_pairs += status[P.np + 1];
  cnt->bad_primes += P.bad_primes;
  for (int i = 0; i < P.np; ++i) cnt->slow_primes += status[1 + i];
  rc = decode_result(P, reinterpret_cast<const uint32_t*>(ctx->h_down), out);
  if (rc == RSL_ERANGE) return fail(ctx, rc, "result buffer too small");
  return rc;
}

}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_ctx_create(int device, void* d_workspace, size_t ws_bytes, void* stream, rsl_ctx** out) {
  if (!out || (ws_bytes && !d_workspace)) return RSL_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RSL_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return RSL_EDEVICE;
  rsl_ctx* c = new (std::nothrow) rsl_ctx();
  if (!c) return RSL_ENOMEM;
  c->device = device;
  c->ws = static_cast<uint8_t*>(d_workspace);
  c->ws_bytes = ws_bytes;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipEventCreate(&c->e0) != hipSuccess || hipEventCreate(&c->e1) != hipSuccess) {
    delete c;
    return RSL_EDEVICE;
  }
  *out = c;
  return RSL_OK;
}

int rsl_ctx_destroy(rsl_ctx* ctx) {
  if (!ctx) return RSL_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_tables(ctx);
  batch_release(ctx);
  if (ctx->h_up) (void)hipHostFree(ctx->h_up);
  if (ctx->h_down) (void)hipHostFree(ctx->h_down);
  if (ctx->e0) (void)hipEventDestroy(ctx->e0);
  if (ctx->e1) (void)hipEventDestroy(ctx->e1);
  delete ctx;
  return RSL_OK;
}

int rsl_query(const rsl_poly* f, const rsl_poly* g, int var, rsl_info* info) {
  if (!info) return RSL_EINVAL;
  Plan P;
  std::string err;
  int rc = make_plan(f, g, var, nullptr, &P, &err);
  if (rc) return rc;
  std::memset(info, 0, sizeof(*info));
  if (P.zero) {
    info->D = -1;
    info->my = P.f.dy;
    info->ny = P.g.dy;
    info->out_limbs = 1;
    return RSL_OK;
  }
  info->D = P.D;
  info->bound_bits = P.bound_bits;
  info->n_primes = P.np;
  info->n_points = P.E + 1;
  info->out_limbs = P.L_out;
  info->my = P.my;
  info->ny = P.ny;
  info->bad_primes = P.bad_primes;
  info->footprint_bytes = layout_of(P).total;
  return RSL_OK;
}

int rsl_res(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts,
            rsl_result* out) {
  if (!ctx) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  const double t0 = now_ms();
  rsl_counters cnt{};
  int rc = run_plain(ctx, f, g, var, opts, out, &cnt);
  cnt.ms_total = now_ms() - t0;
  ctx->last = cnt;
  return rc;
}

int rsl_res_y(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, rsl_result* out) {
  return rsl_res(ctx, f, g, RSL_Y, nullptr, out);
}

int rsl_res_x(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, rsl_result* out) {
  return rsl_res(ctx, f, g, RSL_X, nullptr, out);
}

int rsl_batch(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, rsl_result* out,
              int* status, int mode) {
  if (!ctx || n < 0 || (n > 0 && (!f || !g || !var || !out))) return RSL_EINVAL;
  if (mode != RSL_PLAIN && mode != RSL_BATCHED) return fail(ctx, RSL_EINVAL, "mode must be RSL_PLAIN or RSL_BATCHED");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  const double t0 = now_ms();
  rsl_counters cnt{};
  int first = RSL_OK;
  if (mode == RSL_BATCHED) {
    first = run_batched(ctx, n, f, g, var, out, status, &cnt);
  } else {
    for (int k = 0; k < n; ++k) {
      int rc = run_plain(ctx, &f[k], &g[k], var[k], nullptr, &out[k], &cnt);
      if (status) status[k] = rc;
      if (rc && !first) first = rc;
      if (rc == RSL_EDEVICE) break;
    }
  }
  cnt.ms_total = now_ms() - t0;
  ctx->last = cnt;
  return first;
}

int rsl_last_counters(rsl_ctx* ctx, rsl_counters* c) {
  if (!ctx || !c) return RSL_EINVAL;
  *c = ctx->last;
  return RSL_OK;
}

const char* rsl_strerror(int code) {
  switch (code) {
    case RSL_OK: return "ok";
    case RSL_EINVAL: return "invalid argument";
    case RSL_ERANGE: return "output buffer too small";
    case RSL_ENOMEM: return "workspace or budget smaller than the footprint";
    case RSL_EPRIMES: return "prime table exhausted";
    case RSL_EDEVICE: return "device error (context poisoned)";
    case RSL_EAGAIN: return "server queue full";
    case RSL_ETIMEDOUT: return "timed out";
    default: return "unknown error";
  }
}

const char* rsl_last_error(rsl_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char* rsl_version(void) { return "rsl 0.1 (gfx950)"; }

}  // extern "C"

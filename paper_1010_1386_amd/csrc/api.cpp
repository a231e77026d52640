// C-ABI entry points (include/rsl.h): contexts, tables, the plain pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>

#include "context.h"
#include "job.h"
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

static void reset_tables(rsl_ctx* c) {
  c->d_pc = nullptr;
  c->d_fact = c->d_ifact = c->d_stir = c->d_Tg = c->d_invM = c->d_Plimb = nullptr;
  c->npcap = 0;
  c->garner_np = 0;
  c->kcap = c->scap = -1;
}

TableLayout table_layout(int np_cap, int kcap, int scap) {
  TableLayout L{};
  const size_t A = 256;
  L.ks = kcap + 1;
  L.gnp = std::min(np_cap, kSlotCrtPrimes);
  L.LPg = (31 * L.gnp + 31) / 32 + 1;
  L.sstride = static_cast<int64_t>(align_up(static_cast<size_t>(ckpt_rowoff(scap / kCkpt + 1)), 64));
  size_t o = 0;
  L.pc = o;    o = align_up(o + sizeof(PrimeConst) * np_cap, A);
  L.fact = o;  o = align_up(o + static_cast<size_t>(np_cap) * L.ks * 4, A);
  L.ifact = o; o = align_up(o + static_cast<size_t>(np_cap) * L.ks * 4, A);
  L.stir = o;  o = align_up(o + static_cast<size_t>(np_cap) * L.sstride * 4, A);
  L.Tg = o;    o = align_up(o + static_cast<size_t>(L.gnp) * L.gnp * 4, A);
  L.invM = o;  o = align_up(o + static_cast<size_t>(L.gnp) * 4, A);
  L.Plimb = o; o = align_up(o + static_cast<size_t>(L.gnp) * L.LPg * 4, A);
  L.total = o;
  return L;
}

void table_caps(int np, int kneed, int sneed, int* np_cap, int* kcap, int* scap) {
  *np_cap = static_cast<int>(align_up(std::max(np, 1), 64));
  *kcap = static_cast<int>(align_up(std::max(kneed, 0) + 1, 256)) - 1;
  *scap = static_cast<int>(align_up(std::max(sneed, 0) + 1, 256)) - 1;
}

int workspace_taken(rsl_ctx* ctx) {
  return fail(ctx, RSL_EINVAL,
              "a server runs on this context and owns its workspace: submit the call to the server, "
              "use another context, or destroy the server first");
}

int wait_table_readers(rsl_ctx* ctx) {
  // every launch that reads the tables was issued on one of these streams
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  for (hipStream_t s : {ctx->s_up, ctx->s_comp2, ctx->s_down})
    if (!rc && s) rc = hip_check(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
  for (hipStream_t s : ctx->reader_streams)
    if (!rc) rc = hip_check(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
  return rc;
}

int ensure_tables(rsl_ctx* ctx, int np, int kneed, int sneed) {
  if (np <= ctx->npcap && kneed <= ctx->kcap && sneed <= ctx->scap) return RSL_OK;
  int cap_np, cap_k, cap_s;
  table_caps(np, kneed, sneed, &cap_np, &cap_k, &cap_s);
  const int new_np = std::max(ctx->npcap, cap_np);
  const int new_k = std::max(ctx->kcap, cap_k);
  const int new_s = std::max(ctx->scap, cap_s);
  const TableLayout L = table_layout(new_np, new_k, new_s);
  if (L.total > ctx->tab_bytes)
    return fail(ctx, RSL_ENOMEM, "the constant tables need " + std::to_string(L.total) + " bytes, the table region has " +
                                     std::to_string(ctx->tab_bytes));
  // the old tables (in the same region) may still be read by this context's
  // work in flight: wait for its streams, not for the whole device
  int rc = wait_table_readers(ctx);
  if (rc) return rc;
  reset_tables(ctx);

  size_t have = 0;
  const uint32_t* tab = prime_table(new_np, &have);
  if (static_cast<int>(have) < new_np) return fail(ctx, RSL_EPRIMES, "prime table exhausted");
  std::vector<uint32_t> primes(tab, tab + new_np);
  std::vector<PrimeConst> pc(new_np);
  for (int g = 0; g < new_np; ++g) pc[g] = make_prime_const(primes[g]);

  // factorials and inverse factorials, Montgomery form
  const int ks = L.ks;
  std::vector<uint32_t> fact(static_cast<size_t>(new_np) * ks), ifact(fact.size());
  parallel_for(new_np, 8, [&](int g) {
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
  });
  // canonical CRT tables (Garner's digits serve only the per-lane-slot CRT, so
  // they cover at most kSlotCrtPrimes primes)
  std::vector<uint32_t> Tg, invM, Plimb;
  crt_tables(std::vector<uint32_t>(primes.begin(), primes.begin() + L.gnp), L.LPg, &Tg, &invM, &Plimb);

  uint8_t* base = ctx->tab;
  auto up = [&](size_t off, const void* h, size_t bytes) {
    return hip_check(ctx, hipMemcpy(base + off, h, bytes, hipMemcpyHostToDevice), "hipMemcpy(tables)");
  };
  if ((rc = up(L.pc, pc.data(), sizeof(PrimeConst) * new_np)) || (rc = up(L.fact, fact.data(), fact.size() * 4)) ||
      (rc = up(L.ifact, ifact.data(), ifact.size() * 4)) || (rc = up(L.Tg, Tg.data(), Tg.size() * 4)) ||
      (rc = up(L.invM, invM.data(), invM.size() * 4)) || (rc = up(L.Plimb, Plimb.data(), Plimb.size() * 4)))
    return rc;
  ctx->d_pc = reinterpret_cast<PrimeConst*>(base + L.pc);
  ctx->d_fact = reinterpret_cast<uint32_t*>(base + L.fact);
  ctx->d_ifact = reinterpret_cast<uint32_t*>(base + L.ifact);
  ctx->d_stir = reinterpret_cast<uint32_t*>(base + L.stir);
  ctx->d_Tg = reinterpret_cast<uint32_t*>(base + L.Tg);
  ctx->d_invM = reinterpret_cast<uint32_t*>(base + L.invM);
  ctx->d_Plimb = reinterpret_cast<uint32_t*>(base + L.Plimb);
  if ((rc = hip_check(ctx, launch_stirling_build(ctx->d_stir, L.sstride, ctx->d_pc, 0, new_np, new_s, ctx->stream),
                      "stirling build")) ||
      (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stirling build sync"))) {
    reset_tables(ctx);
    return rc;
  }
  ctx->npcap = new_np;
  ctx->kcap = new_k;
  ctx->scap = new_s;
  ctx->kstride = ks;
  ctx->sstride = L.sstride;
  ctx->LPg = L.LPg;
  ctx->garner_np = L.gnp;
  ctx->tab_used = L.total;
  ctx->table_gen += 1;
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

static int grow_pinned(rsl_ctx* ctx, uint8_t** buf, size_t* have, size_t need) {
  if (need <= *have) return RSL_OK;
  if (*buf) (void)hipHostFree(*buf);
  *buf = nullptr;
  *have = 0;
  const size_t sz = align_up(std::max(need, static_cast<size_t>(1) << 20), 1 << 20);
  int rc = hip_check(ctx, hipHostMalloc(reinterpret_cast<void**>(buf), sz, hipHostMallocDefault), "hipHostMalloc");
  if (!rc) *have = sz;
  return rc;
}

// Contiguous ranges by estimated device work: the first range takes half a
// share (the device starts sooner), the others a full share each; a y problem
// directly followed by an x problem (a joint pair sharing its reduction) is
// never split.
static std::vector<std::pair<int, int>> chunk_ranges(const std::vector<ShapeEst>& est, const int* var, int S) {
  const int n = static_cast<int>(est.size());
  double total = 0.0;
  for (const ShapeEst& e : est) total += e.zero ? 0.0 : e.cost;
  std::vector<std::pair<int, int>> out;
  int lo = 0;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    acc += est[k].zero ? 0.0 : est[k].cost;
    const bool pair_next = k + 1 < n && var[k] == RSL_Y && var[k + 1] == RSL_X;
    const int c = static_cast<int>(out.size());
    if (c < S - 1 && !pair_next && acc >= total * (2.0 * c + 1.0) / (2.0 * S - 1.0)) {
      out.push_back({lo, k + 1});
      lo = k + 1;
    }
  }
  if (lo < n) out.push_back({lo, n});
  return out;
}

// A batch as S chunks in a pipeline: a host thread plans and lays out chunk
// c + 1 while the device runs chunk c, and chunk c is decoded while later
// chunks run.  Every chunk is a staged (or plain) job of its own, in its own
// region of the workspace (the workspace is reused after a synchronization
// when the regions do not all fit) with its own pinned staging.
static int run_chunked(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var,
                       const rsl_opts* opts, rsl_result* out, int* status, int mode, const TuneConfig* tc,
                       const std::vector<std::pair<int, int>>& ranges, const std::vector<ShapeEst>& est,
                       std::string* err, rsl_counters* cnt) {
  const int S = static_cast<int>(ranges.size());
  if (static_cast<int>(ctx->chunk_stage.size()) < S) ctx->chunk_stage.resize(S);
  for (int c = 0; c < S; ++c) {
    rsl_ctx::ChunkStage& cs = ctx->chunk_stage[c];
    if (!cs.e0 && hipEventCreate(&cs.e0) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipEventCreate");
    if (!cs.e1 && hipEventCreate(&cs.e1) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipEventCreate");
    if (!cs.e2 && hipEventCreate(&cs.e2) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipEventCreate");
    if (!cs.e3 && hipEventCreateWithFlags(&cs.e3, hipEventDisableTiming) != hipSuccess)
      return fail(ctx, RSL_EDEVICE, "hipEventCreate");
  }
  if (!ctx->s_up && hipStreamCreateWithFlags(&ctx->s_up, hipStreamNonBlocking) != hipSuccess)
    return fail(ctx, RSL_EDEVICE, "hipStreamCreate");
  if (!ctx->s_down && hipStreamCreateWithFlags(&ctx->s_down, hipStreamNonBlocking) != hipSuccess)
    return fail(ctx, RSL_EDEVICE, "hipStreamCreate");
  if (!ctx->s_comp2 && hipStreamCreateWithFlags(&ctx->s_comp2, hipStreamNonBlocking) != hipSuccess)
    return fail(ctx, RSL_EDEVICE, "hipStreamCreate");
  auto sync_all = [&]() {
    int e = hip_check(ctx, hipStreamSynchronize(ctx->s_up), "hipStreamSynchronize");
    if (!e) e = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (!e) e = hip_check(ctx, hipStreamSynchronize(ctx->s_comp2), "hipStreamSynchronize");
    if (!e) e = hip_check(ctx, hipStreamSynchronize(ctx->s_down), "hipStreamSynchronize");
    return e;
  };
  while (static_cast<int>(ctx->chunk_jobs.size()) < S) ctx->chunk_jobs.push_back(std::make_shared<Job>());
  std::vector<Job*> jobs(S);
  for (int c = 0; c < S; ++c) jobs[c] = ctx->chunk_jobs[c].get();
  std::vector<std::string> errs(S);
  std::vector<int> brc(S, RSL_OK);
  std::vector<char> ready(S, 0);
  std::mutex mu;
  std::condition_variable cv;
  double build_ms = 0.0;
  // the constant tables for the estimated shapes, before any launch (growing
  // them later would synchronize the device; a chunk that needs more still
  // grows them, correctly)
  {
    int ng = 0, nE = 0, nD = 0;
    for (const ShapeEst& e : est)
      if (!e.zero && !e.bad) {
        ng = std::max(ng, e.np_est + 2);
        nE = std::max(nE, e.E);
        nD = std::max(nD, e.D);
      }
    int rc0 = ng ? ensure_tables(ctx, std::min(ng, kMaxPrimes), nE, nD) : RSL_OK;
    if (rc0 == RSL_ENOMEM) {  // the estimate overshoots the region: each chunk grows what it needs
      ctx->err.clear();
      rc0 = RSL_OK;
    }
    if (rc0) {
      if (status)
        for (int k = 0; k < n; ++k) status[k] = rc0;
      return rc0;
    }
  }
  // producers: kProducers host threads plan and lay out the chunks, producer
  // q taking chunks q, q + kProducers, ... in order (host only; the tables
  // are grown below, on this thread).  build_ms: the time until the last
  // chunk was laid out.
  constexpr int kProducers = 2;
  const int nprod = std::min(S, kProducers);
  const double tb = now_ms();
  std::vector<std::thread> producers;
  for (int q = 0; q < nprod; ++q)
    producers.emplace_back([&, q]() {
      for (int c = q; c < S; c += nprod) {
        const int lo = ranges[c].first, hi = ranges[c].second;
        Job& J = *jobs[c];
        job_plan(hi - lo, f + lo, g + lo, var + lo, opts, &J, &errs[c]);
        brc[c] = job_build(ctx, J.n, f + lo, g + lo, var + lo, opts, &J, &errs[c], tc, true, true);
        std::lock_guard<std::mutex> lk(mu);
        ready[c] = 1;
        build_ms = std::max(build_ms, now_ms() - tb);
        cv.notify_all();
      }
    });
  hipStream_t st = ctx->stream;
  int rc = RSL_OK;
  size_t off = 0;
  int launched = 0, decoded = 0;
  double bind_ms = 0.0, dec_ms = 0.0;
  // decode launched chunks in order: those whose copies are done (block =
  // false), or all of them
  auto decode = [&](bool block) {
    while (decoded < launched) {
      const int c = decoded;
      Job& J = *jobs[c];
      const int lo = ranges[c].first;
      if (!J.live.empty()) {
        if (!block && hipEventQuery(ctx->chunk_stage[c].e2) != hipSuccess) return;
        const int e = hip_check(ctx, hipEventSynchronize(ctx->chunk_stage[c].e2), "hipEventSynchronize");
        if (e) {
          rc = rc ? rc : e;
          decoded = launched;
          return;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->chunk_stage[c].e0, ctx->chunk_stage[c].e1);
        cnt->ms_device += ms;
      }
      const double t3 = now_ms();
      std::vector<int> stc(J.n);
      const int r = job_decode(ctx, J, J.live.empty() ? nullptr : ctx->chunk_stage[c].down, out + lo, stc.data(), cnt);
      dec_ms += now_ms() - t3;
      if (status)
        for (int k = 0; k < J.n; ++k) status[lo + k] = stc[k];
      if (r && !rc) rc = r;
      ++decoded;
    }
  };
  for (int c = 0; c < S && !rc; ++c) {
    decode(false);  // while the next chunk is still being laid out
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return ready[c] != 0; });
    }
    Job& J = *jobs[c];
    if (brc[c]) { rc = brc[c]; break; }
    if (J.live.empty()) { ++launched; continue; }
    if (J.total > ctx->ws_bytes) {
      rc = fail(ctx, RSL_ENOMEM, "workspace of " + std::to_string(ctx->ws_bytes) + " bytes < footprint " +
                                     std::to_string(J.total) + " of a chunk");
      for (int k : J.live) J.pstatus[k] = RSL_ENOMEM;
      break;
    }
    if (off + J.total > ctx->ws_bytes) {  // reuse the workspace once the earlier chunks are done
      if ((rc = sync_all())) break;
      off = 0;
    }
    if ((rc = ensure_tables(ctx, J.need_g, J.need_E, J.need_D))) break;  // a no-op once grown
    rsl_ctx::ChunkStage& cs = ctx->chunk_stage[c];
    if ((rc = grow_pinned(ctx, &cs.up, &cs.up_bytes, J.up_bytes)) ||
        (rc = grow_pinned(ctx, &cs.down, &cs.down_bytes, J.down_bytes)))
      break;
    const double t1 = now_ms();
    job_bind(&J, ctx->ws + off, cs.up, mode == RSL_BATCHED);
    bind_ms += now_ms() - t1;
    off = align_up(off + J.total, 256);
    // upload on the copy stream; the kernels wait for it on a compute stream
    // (the context's stream and the second one in turn); the download waits
    // for the kernels on the other copy stream
    hipStream_t sc = (c & 1) ? ctx->s_comp2 : st;
    if ((rc = job_upload_copy(ctx, &J, ctx->s_up)) ||
        (rc = hip_check(ctx, hipEventRecord(cs.e3, ctx->s_up), "event")) ||
        (rc = hip_check(ctx, hipStreamWaitEvent(sc, cs.e3, 0), "hipStreamWaitEvent")) ||
        (rc = job_upload_clear(ctx, &J, sc)) || (rc = hip_check(ctx, hipEventRecord(cs.e0, sc), "event")) ||
        (rc = job_launch(ctx, &J, mode, sc, false)) || (rc = hip_check(ctx, hipEventRecord(cs.e1, sc), "event")) ||
        (rc = hip_check(ctx, hipStreamWaitEvent(ctx->s_down, cs.e1, 0), "hipStreamWaitEvent")) ||
        (rc = job_download(ctx, &J, cs.down, ctx->s_down)) ||
        (rc = hip_check(ctx, hipEventRecord(cs.e2, ctx->s_down), "event")))
      break;
    ++launched;
  }
  // the remaining chunks, each as soon as its copies are done
  decode(true);
  for (std::thread& t : producers) t.join();
  (void)sync_all();
  cnt->ms_build += build_ms;
  cnt->ms_bind += bind_ms;
  cnt->ms_decode += dec_ms;
  for (int c = 0; c < S; ++c)
    if (!errs[c].empty() && err->empty()) *err = errs[c];
  if (status && rc && launched < S)
    for (int c = launched; c < S; ++c)
      for (int k = ranges[c].first; k < ranges[c].second; ++k) status[k] = rc;
  return rc;
}

// Run a job laid out in the context workspace, synchronously.
static int run_in_workspace(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var,
                            const rsl_opts* opts, rsl_result* out, int* status, int mode, rsl_counters* cnt) {
  if (ctx->server) return workspace_taken(ctx);
  const double t0 = now_ms();
  std::string err;
  // shapes from the inputs alone: the schedule lookup and the chunking need no plans
  std::vector<ShapeEst> est(n);
  parallel_for(n, 32, [&](int k) { est[k] = estimate_shape(&f[k], &g[k], var[k]); });
  // RSL_AUTO: the schedule the autotuner chose for this shape bucket, else the
  // staged default; the job is laid out once, with the chosen parameters
  const TuneConfig* tc = nullptr;
  if (mode == RSL_AUTO) {
    mode = RSL_STAGED;
    auto it = ctx->tune_cache.find(tune_key_of(est));
    if (it != ctx->tune_cache.end()) {
      mode = it->second.cfg.mode;
      tc = &it->second.cfg;
    }
  }
  // large batches on the staged or plain schedule: a pipeline of chunks, so
  // that host work overlaps the device
  if (mode != RSL_BATCHED) {
    int live = 0;
    for (const ShapeEst& e : est) live += (!e.zero && !e.bad) ? 1 : 0;
    int S = live >= 384 ? 5 : live >= 192 ? 4 : live >= 96 ? 2 : 1;
    if (const char* env = std::getenv("RSL_BATCH_CHUNKS")) S = std::max(1, std::min(16, std::atoi(env)));
    if (S > 1) {
      std::vector<std::pair<int, int>> ranges = chunk_ranges(est, var, S);
      if (ranges.size() > 1) {
        cnt->ms_build += now_ms() - t0;
        int rc = run_chunked(ctx, n, f, g, var, opts, out, status, mode, tc, ranges, est, &err, cnt);
        if (rc && !err.empty() && ctx->err.empty()) ctx->err = err;
        return rc;
      }
    }
  }
  if (ctx->chunk_jobs.empty()) ctx->chunk_jobs.push_back(std::make_shared<Job>());
  Job& J = *ctx->chunk_jobs[0];
  job_plan(n, f, g, var, opts, &J, &err);
  int rc = job_build(ctx, n, f, g, var, opts, &J, &err, tc, true);
  if (rc) {  // no layout (tables, options or LDS): nothing ran
    if (status)
      for (int k = 0; k < n; ++k) status[k] = J.pstatus[k] ? J.pstatus[k] : rc;
    if (!err.empty()) ctx->err = err;
    return rc;
  }
  const double t1 = now_ms();
  cnt->ms_build += t1 - t0;
  if (!J.live.empty()) {
    if (J.total > ctx->ws_bytes) {
      const std::string m = "workspace of " + std::to_string(ctx->ws_bytes) + " bytes < footprint " +
                            std::to_string(J.total);
      for (int k : J.live) J.pstatus[k] = RSL_ENOMEM;
      if (status)
        for (int k = 0; k < n; ++k) status[k] = J.pstatus[k];
      return fail(ctx, RSL_ENOMEM, m);
    }
    if ((rc = ensure_staging(ctx, J.up_bytes, J.down_bytes))) return rc;
    // the upload image is written straight into pinned staging; only the
    // persistent launch needs its queue image
    job_bind(&J, ctx->ws, ctx->h_up, mode == RSL_BATCHED);
    const double t2 = now_ms();
    cnt->ms_bind += t2 - t1;
    hipStream_t st = ctx->stream;
    if ((rc = job_upload(ctx, &J, st)) || (rc = hip_check(ctx, hipEventRecord(ctx->e0, st), "event")) ||
        (rc = job_launch(ctx, &J, mode, st, false)) || (rc = hip_check(ctx, hipEventRecord(ctx->e1, st), "event")) ||
        (rc = job_download(ctx, &J, ctx->h_down, st)) ||
        (rc = hip_check(ctx, hipStreamSynchronize(st), "hipStreamSynchronize")))
      return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->e0, ctx->e1);
    cnt->ms_device += ms;
    cnt->ms_transfer += now_ms() - t2 - ms;
  }
  const double t3 = now_ms();
  rc = job_decode(ctx, J, ctx->h_down, out, status, cnt);
  cnt->ms_decode += now_ms() - t3;
  if (rc && !err.empty() && ctx->err.empty()) ctx->err = err;
  if (rc && rc != RSL_ERANGE && rc != RSL_EPRIMES && !err.empty()) ctx->err = err;
  return rc;
}

}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_ctx_create(int device, void* d_workspace, size_t ws_bytes, void* d_tables, size_t table_bytes, void* stream,
                   rsl_ctx** out) {
  if (!out || (ws_bytes && !d_workspace) || (d_tables && !table_bytes)) return RSL_EINVAL;
  if (!d_tables && table_bytes > ws_bytes) return RSL_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RSL_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return RSL_EDEVICE;
  rsl_ctx* c = new (std::nothrow) rsl_ctx();
  if (!c) return RSL_ENOMEM;
  c->device = device;
  c->ws = static_cast<uint8_t*>(d_workspace);
  c->ws_bytes = ws_bytes;
  if (d_tables) {  // a region of its own for the constant tables
    c->tab = static_cast<uint8_t*>(d_tables);
    c->tab_bytes = table_bytes;
  } else {  // the top table_bytes of the workspace, 256-byte aligned
    const size_t jb = (ws_bytes - table_bytes) & ~static_cast<size_t>(255);
    c->tab = c->ws + jb;
    c->tab_bytes = ws_bytes - jb;
    c->ws_bytes = jb;
  }
  c->stream = static_cast<hipStream_t>(stream);
  bool ok = hipEventCreate(&c->e0) == hipSuccess && hipEventCreate(&c->e1) == hipSuccess;
  for (int s = 0; s <= kNumStages && ok; ++s) ok = hipEventCreate(&c->ev[s]) == hipSuccess;
  if (!ok) {
    delete c;
    return RSL_EDEVICE;
  }
  // bound on a persistent-launch wave's wait for its next task
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
  double wait_ms = 10000.0;
  if (const char* env = std::getenv("RSL_QUEUE_WAIT_MS")) wait_ms = std::max(0.0, std::atof(env));
  c->queue_wait_ticks = static_cast<int64_t>(wait_ms * khz);
  if (const char* env = std::getenv("RSL_CRT_GARNER")) c->crt_garner = std::atoi(env) != 0;
  if (const char* env = std::getenv("RSL_WIDE_VALU")) c->wide_valu = std::atoi(env) != 0;
  if (const char* env = std::getenv("RSL_EVAL_HORNER")) c->eval_horner = std::atoi(env) != 0;
  *out = c;
  return RSL_OK;
}

int rsl_ctx_destroy(rsl_ctx* ctx) {
  if (!ctx) return RSL_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)wait_table_readers(ctx);
  reset_tables(ctx);
  if (ctx->h_up) (void)hipHostFree(ctx->h_up);
  if (ctx->h_down) (void)hipHostFree(ctx->h_down);
  for (rsl_ctx::ChunkStage& cs : ctx->chunk_stage) {
    if (cs.up) (void)hipHostFree(cs.up);
    if (cs.down) (void)hipHostFree(cs.down);
    if (cs.e0) (void)hipEventDestroy(cs.e0);
    if (cs.e1) (void)hipEventDestroy(cs.e1);
    if (cs.e2) (void)hipEventDestroy(cs.e2);
    if (cs.e3) (void)hipEventDestroy(cs.e3);
  }
  if (ctx->s_up) (void)hipStreamDestroy(ctx->s_up);
  if (ctx->s_down) (void)hipStreamDestroy(ctx->s_down);
  if (ctx->s_comp2) (void)hipStreamDestroy(ctx->s_comp2);
  if (ctx->e0) (void)hipEventDestroy(ctx->e0);
  if (ctx->e1) (void)hipEventDestroy(ctx->e1);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& set : ctx->evsets)
    for (hipEvent_t e : set) (void)hipEventDestroy(e);
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
  info->origin = P.origin;
  Job J;
  std::string e2;
  if (job_build(nullptr, 1, f, g, &var, nullptr, &J, &e2) == RSL_OK) {
    info->footprint_bytes = J.total;
    int cn, ck, cs;
    table_caps(J.need_g, J.need_E, J.need_D, &cn, &ck, &cs);
    info->table_bytes = table_layout(cn, ck, cs).total;
  }
  return RSL_OK;
}

int rsl_res(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts,
            rsl_result* out) {
  if (!ctx || !out) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  const double t0 = now_ms();
  rsl_counters cnt{};
  int rc = run_in_workspace(ctx, 1, f, g, &var, opts, out, nullptr, RSL_STAGED, &cnt);
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

int rsl_res_xy(rsl_ctx* ctx, const rsl_poly* f, const rsl_poly* g, const rsl_opts* opts, rsl_result* out_y,
               rsl_result* out_x) {
  if (!ctx || !f || !g || !out_y || !out_x) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  const double t0 = now_ms();
  const rsl_poly fs[2] = {*f, *f}, gs[2] = {*g, *g};
  const int var[2] = {RSL_Y, RSL_X};
  rsl_result out[2] = {*out_y, *out_x};
  rsl_counters cnt{};
  int rc = run_in_workspace(ctx, 2, fs, gs, var, opts, out, nullptr, RSL_AUTO, &cnt);
  *out_y = out[0];
  *out_x = out[1];
  cnt.ms_total = now_ms() - t0;
  ctx->last = cnt;
  return rc;
}

int rsl_batch(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, rsl_result* out,
              int* status, int mode) {
  if (!ctx || n < 0 || (n > 0 && (!f || !g || !var || !out))) return RSL_EINVAL;
  if (mode != RSL_PLAIN && mode != RSL_BATCHED && mode != RSL_STAGED && mode != RSL_AUTO)
    return fail(ctx, RSL_EINVAL, "mode must be RSL_PLAIN, RSL_BATCHED, RSL_STAGED or RSL_AUTO");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  const double t0 = now_ms();
  rsl_counters cnt{};
  int rc = run_in_workspace(ctx, n, f, g, var, nullptr, out, status, mode, &cnt);
  cnt.ms_total = now_ms() - t0;
  ctx->last = cnt;
  return rc;
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

int rsl_profile_enable(rsl_ctx* ctx, int on) {
  if (!ctx) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->profiling = on != 0;
  ctx->evused = 0;
  return RSL_OK;
}

int rsl_profile_take(rsl_ctx* ctx, double* stage_ms, int* runs) {
  if (!ctx || !stage_ms) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int s = 0; s < kNumStages; ++s) stage_ms[s] = 0.0;
  for (int r = 0; r < ctx->evused; ++r) {
    const std::vector<hipEvent_t>& ev = ctx->evsets[r];
    // the events as the run recorded them: an empty stage's end boundary is
    // its start event, recorded again where the next stage began, so the
    // stage itself reads zero and the marker time goes to the stage before
    const unsigned empty = ctx->evempty[r];
    hipEvent_t at[kNumStages + 1];
    for (int s = 0; s <= kNumStages; ++s) at[s] = (s > 0 && (empty >> (s - 1) & 1u)) ? at[s - 1] : ev[s];
    for (int s = 0; s < kNumStages; ++s) {
      if (empty >> s & 1u) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, at[s], at[s + 1]) == hipSuccess) stage_ms[s] += ms;
    }
  }
  if (runs) *runs = ctx->evused;
  ctx->evused = 0;
  return RSL_OK;
}

}  // extern "C"

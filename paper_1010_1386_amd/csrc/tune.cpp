// Resident jobs (rsl_job_*) and the schedule autotuner (rsl_job_tune, rsl_tune_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>

#include "context.h"
#include "job.h"
#include "kernels.h"
#include "persistent.h"

struct rsl_job {
  rsl::Job J;
  uint8_t* dmem = nullptr;  // the caller's device memory (rsl_job_bind), nullptr until bound
  size_t dmem_bytes = 0;
  uint8_t* hdown = nullptr;
  rsl::TuneConfig tc;       // schedule of the current layout
  int gen = -1;
  rsl_ctx* ctx = nullptr;
  // inputs, kept so that the autotuner can lay the job out again
  std::vector<std::vector<uint32_t>> fbuf, gbuf;
  std::vector<rsl_poly> f, g;
  std::vector<int> var;
  rsl_opts opts{};
  bool has_opts = false;
  // captured runs, per schedule (index = mode), valid for table generation graph_gen
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  int graph_gen[4] = {-1, -1, -1, -1};
};

namespace rsl {

static int ilog2up(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

// Shape bucket of a batch: live problems, max degree bound, max degree in the
// eliminated variable, max input limbs -- each rounded up to a power of two.
// Computed from the inputs alone (no planning), so that a batch call can look
// up its schedule before any problem is planned.
std::string tune_key(int n, const rsl_poly* f, const rsl_poly* g, const int* var) {
  std::vector<ShapeEst> est(n);
  parallel_for(n, 32, [&](int k) { est[k] = estimate_shape(&f[k], &g[k], var[k]); });
  return tune_key_of(est);
}

std::string tune_key_of(const std::vector<ShapeEst>& est) {
  int64_t live = 0, maxD = 0, maxdeg = 0, maxL = 0;
  for (const ShapeEst& e : est) {
    if (e.zero || e.bad) continue;
    ++live;
    maxD = std::max<int64_t>(maxD, e.D + 1);
    maxdeg = std::max<int64_t>(maxdeg, std::max(e.my, e.ny) + 1);
    maxL = std::max<int64_t>(maxL, e.L);
  }
  std::ostringstream os;
  os << "n" << ilog2up(std::max<int64_t>(live, 1)) << ".D" << ilog2up(maxD) << ".m" << ilog2up(maxdeg) << ".L"
     << ilog2up(maxL);
  return os.str();
}

static void release_graphs(rsl_job* j) {
  for (int m = 0; m < 4; ++m) {
    if (j->graph[m]) (void)hipGraphExecDestroy(j->graph[m]);
    j->graph[m] = nullptr;
    j->graph_gen[m] = -1;
  }
}

static void release_mem(rsl_job* j) {
  release_graphs(j);
  if (j->hdown) (void)hipHostFree(j->hdown);
  j->hdown = nullptr;
  j->gen = -1;
}

// Point the laid-out job at the caller's memory and upload its inputs.
static int bind_and_upload(rsl_ctx* ctx, rsl_job* j) {
  release_mem(j);
  if (j->J.total > j->dmem_bytes)
    return fail(ctx, RSL_ENOMEM, "the job needs " + std::to_string(j->J.total) + " device bytes, " +
                                     std::to_string(j->dmem_bytes) + " are bound");
  int rc;
  if ((rc = hip_check(ctx, hipHostMalloc(reinterpret_cast<void**>(&j->hdown),
                                         std::max<size_t>(j->J.down_bytes, 256), hipHostMallocDefault),
                      "hipHostMalloc(job)")))
    return rc;
  job_bind(&j->J, j->dmem);
  if ((rc = job_upload(ctx, &j->J, ctx->stream)) ||
      (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"))) {
    release_mem(j);
    return rc;
  }
  j->gen = ctx->table_gen;
  return RSL_OK;
}

// Lay the job out with `tc` and, when memory is bound, upload the inputs.
static int materialize(rsl_ctx* ctx, rsl_job* j, const TuneConfig& tc) {
  release_mem(j);
  j->J = Job();
  j->tc = tc;
  std::string err;
  const int n = static_cast<int>(j->f.size());
  int rc = job_build(ctx, n, j->f.data(), j->g.data(), j->var.data(), j->has_opts ? &j->opts : nullptr, &j->J,
                     &err, &tc);
  if (!err.empty()) ctx->err = err;
  if (rc) return rc;
  return j->dmem ? bind_and_upload(ctx, j) : RSL_OK;
}

static int require_bound(rsl_ctx* ctx, const rsl_job* j) {
  return j->dmem ? RSL_OK : fail(ctx, RSL_EINVAL, "the job has no device memory yet (rsl_job_bind)");
}

// Re-point the job's problems at the current constant tables if they moved.
static int job_refresh(rsl_ctx* ctx, rsl_job* j) {
  if (j->gen == ctx->table_gen) return RSL_OK;
  // (synchronous: the upload goes through the context's shared staging buffer)
  int rc = job_upload(ctx, &j->J, ctx->stream);
  if (!rc) rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (rc) return rc;
  j->gen = ctx->table_gen;
  return RSL_OK;
}

// Per-stage events of one launch (profiling).
static hipEvent_t* next_evset(rsl_ctx* ctx) {
  if (ctx->evused == static_cast<int>(ctx->evsets.size())) {
    std::vector<hipEvent_t> set(kNumStages + 1, nullptr);
    for (auto& e : set)
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->evsets.push_back(set);
    ctx->evempty.push_back(0u);
  }
  return ctx->evsets[ctx->evused++].data();
}

// Stages of the staged schedule that launch no kernel for this job.  Their
// boundary events would only time the event markers themselves, so the
// profiler folds them into the stage before (see rsl_profile_take).
static unsigned empty_stages(const Job& J) {
  unsigned m = 0u;
  if (J.items[kStageReduce].empty()) m |= 1u << kStageReduce;
  if (J.eval_ranges.empty()) m |= 1u << kStageEval;
  if (J.mm_interp) {
    if (J.dig_items.empty() && J.mm_items.empty()) m |= (1u << kStageConv) | (1u << kStageStir);
  } else {
    if (J.items[kStageConv].empty()) m |= 1u << kStageConv;
    if (J.items[kStageStir].empty() && J.sg_items.empty() && J.hseg_items.empty()) m |= 1u << kStageStir;
  }
  if (J.items[kStageNewton].empty()) m |= 1u << kStageNewton;
  if (J.items[kStageCrt].empty() && J.wide_items[0].empty() && J.wide_items[1].empty() && J.wide_items[2].empty())
    m |= 1u << kStageCrt;
  return m;
}

// Capture reset + launches of `mode` into a graph on the context stream.
static int capture(rsl_ctx* ctx, rsl_job* j, int mode) {
  if (j->graph[mode]) (void)hipGraphExecDestroy(j->graph[mode]);
  j->graph[mode] = nullptr;
  int rc;
  if ((rc = hip_check(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "begin capture")))
    return rc;
  // the staged and plain launches clear the statuses in their reduce stage
  int rc_launch = (mode == RSL_BATCHED) ? job_reset(ctx, &j->J, ctx->stream) : RSL_OK;
  if (!rc_launch) rc_launch = job_launch(ctx, &j->J, mode, ctx->stream, false);
  hipGraph_t g = nullptr;
  if ((rc = hip_check(ctx, hipStreamEndCapture(ctx->stream, &g), "end capture"))) return rc;
  if (rc_launch) {
    (void)hipGraphDestroy(g);
    return rc_launch;
  }
  rc = hip_check(ctx, hipGraphInstantiate(&j->graph[mode], g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  if (rc) return rc;
  j->graph_gen[mode] = ctx->table_gen;
  return RSL_OK;
}

static int run_job(rsl_ctx* ctx, rsl_job* j, int mode) {
  const bool graph = (mode & RSL_GRAPH) != 0;
  mode &= ~RSL_GRAPH;
  if (mode == RSL_AUTO) mode = j->J.tune.mode;
  int rc;
  if ((rc = require_bound(ctx, j)) || (rc = job_refresh(ctx, j))) return rc;
  if (graph && !ctx->profiling && !j->J.live.empty()) {
    if (j->graph_gen[mode] != ctx->table_gen && (rc = capture(ctx, j, mode))) return rc;
    return hip_check(ctx, hipGraphLaunch(j->graph[mode], ctx->stream), "graph launch");
  }
  if (mode == RSL_BATCHED && (rc = job_reset(ctx, &j->J, ctx->stream))) return rc;
  if (ctx->profiling && mode != RSL_PLAIN) {
    hipEvent_t* ev = next_evset(ctx);
    if (!ev) return fail(ctx, RSL_EDEVICE, "hipEventCreate");
    // an empty stage's end boundary reuses its start event, which is then
    // recorded again where the next stage begins (one persistent launch
    // records every boundary after its kernel: nothing to fold)
    const unsigned empty = mode == RSL_STAGED ? empty_stages(j->J) : 0u;
    ctx->evempty[ctx->evused - 1] = empty;
    for (int s = 0; s <= kNumStages; ++s)
      ctx->ev[s] = (s > 0 && (empty >> (s - 1) & 1u)) ? ctx->ev[s - 1] : ev[s];
    return job_launch(ctx, &j->J, mode, ctx->stream, true);
  }
  return job_launch(ctx, &j->J, mode, ctx->stream, false);
}

}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_job_create(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, const rsl_opts* opts,
                   int* status, rsl_job** out) {
  if (!ctx || !out || n < 0 || (n > 0 && (!f || !g || !var))) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  *out = nullptr;
  rsl_job* j = new (std::nothrow) rsl_job();
  if (!j) return RSL_ENOMEM;
  j->ctx = ctx;
  j->fbuf.resize(n);
  j->gbuf.resize(n);
  j->f.resize(n);
  j->g.resize(n);
  j->var.assign(var, var + n);
  for (int k = 0; k < n; ++k) {
    auto copy = [](const rsl_poly& p, std::vector<uint32_t>* buf, rsl_poly* dst) {
      *dst = p;
      if (p.coeff && p.dx >= 0 && p.dy >= 0 && p.limbs >= 1) {
        buf->assign(p.coeff, p.coeff + static_cast<size_t>(p.dx + 1) * (p.dy + 1) * p.limbs);
        dst->coeff = buf->data();
      }
    };
    copy(f[k], &j->fbuf[k], &j->f[k]);
    copy(g[k], &j->gbuf[k], &j->g[k]);
  }
  if (opts) {
    j->opts = *opts;
    j->has_opts = true;
  }
  // the shape bucket's cached schedule, if the autotuner has seen this shape
  TuneConfig tc;
  if (!ctx->tune_cache.empty()) {
    auto it = ctx->tune_cache.find(tune_key(n, j->f.data(), j->g.data(), j->var.data()));
    if (it != ctx->tune_cache.end()) tc = it->second.cfg;
  }
  int rc = materialize(ctx, j, tc);
  if (status)
    for (int k = 0; k < n; ++k) status[k] = k < static_cast<int>(j->J.pstatus.size()) ? j->J.pstatus[k] : rc;
  if (rc) {
    release_mem(j);
    delete j;
    return rc;
  }
  *out = j;
  return RSL_OK;
}

int rsl_job_bind(rsl_ctx* ctx, rsl_job* j, void* d_mem, size_t bytes) {
  if (!ctx || !j || j->ctx != ctx || !d_mem) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  // work of this job on the old memory may still be in flight
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (rc) return rc;
  j->dmem = static_cast<uint8_t*>(d_mem);
  j->dmem_bytes = bytes;
  if ((rc = bind_and_upload(ctx, j))) {
    j->dmem = nullptr;
    j->dmem_bytes = 0;
  }
  return rc;
}

int rsl_job_run(rsl_ctx* ctx, rsl_job* j, int mode) {
  if (!ctx || !j || j->ctx != ctx) return RSL_EINVAL;
  const int base = mode & ~RSL_GRAPH;
  if (base != RSL_PLAIN && base != RSL_BATCHED && base != RSL_STAGED && base != RSL_AUTO)
    return fail(ctx, RSL_EINVAL, "mode must be RSL_PLAIN, RSL_BATCHED, RSL_STAGED or RSL_AUTO (| RSL_GRAPH)");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  return run_job(ctx, j, mode);
}

int rsl_job_results(rsl_ctx* ctx, rsl_job* j, rsl_result* out, int* status) {
  if (!ctx || !j || j->ctx != ctx || (j->J.n > 0 && !out)) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  int rc;
  if ((rc = require_bound(ctx, j)) || (rc = job_download(ctx, &j->J, j->hdown, ctx->stream)) ||
      (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize")))
    return rc;
  rsl_counters cnt{};
  rc = job_decode(ctx, j->J, j->hdown, out, status, &cnt);
  ctx->last = cnt;
  return rc;
}

int rsl_job_info_get(const rsl_job* j, rsl_job_info* info) {
  if (!j || !info) return RSL_EINVAL;
  info->n_problems = j->J.n;
  info->n_live = static_cast<int32_t>(j->J.live.size());
  info->pairs = j->J.pairs;
  info->mulmods = j->J.mulmods;
  info->mulmods_sums_mfma = j->J.mm_sums_mfma;
  info->mulmods_valu = j->J.mm_valu;
  info->mfma_int8_macs = j->J.mfma_macs;
  info->interp_mulmods = j->J.interp_mm;
  info->device_bytes = j->J.total;
  info->upload_bytes = j->J.up_bytes;
  info->download_bytes = j->J.down_bytes;
  info->layout_mode = j->J.tune.mode;
  info->chunk_target = j->J.tune.chunk_target;
  info->grid_mult = j->J.tune.grid_mult;
  int lanes = 1;
  for (const DevProblem& d : j->J.dev) lanes = std::max(lanes, d.evk);
  info->eval_lanes = lanes;
  int mf = 0;
  for (const DevProblem& d : j->J.dev) mf += d.evmf;
  info->eval_mfma = mf;
  return RSL_OK;
}

int rsl_job_destroy(rsl_job* j) {
  if (!j) return RSL_EINVAL;
  if (j->ctx) {
    std::lock_guard<std::recursive_mutex> lk(j->ctx->mu);
    (void)hipSetDevice(j->ctx->device);
    (void)hipStreamSynchronize(j->ctx->stream);
  }
  release_mem(j);
  delete j;
  return RSL_OK;
}

int rsl_job_tune(rsl_ctx* ctx, rsl_job* j, int reps, rsl_tune_result* best) {
  if (!ctx || !j || j->ctx != ctx || reps < 1) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  int rc;
  if ((rc = require_bound(ctx, j))) return rc;
  if (j->J.live.empty()) {
    if (best) *best = rsl_tune_result{RSL_STAGED, j->J.tune.chunk_target, 1, 1, 0, 0, 0, 0, 0.0, 0.0};
    return RSL_OK;
  }
  // coordinate search: schedule x lanes per pair at the default chunking, then
  // the chunking (and the persistent grid) around the best of those
  std::vector<TuneConfig> cands;
  auto same = [](const TuneConfig& a, const TuneConfig& b) {
    return a.mode == b.mode && a.chunk_target == b.chunk_target && a.grid_mult == b.grid_mult && a.evk == b.evk &&
           a.conv_whole == b.conv_whole && a.schur == b.schur && a.interp_mm == b.interp_mm;
  };
  auto add = [&](const TuneConfig& c) {
    for (const TuneConfig& d : cands)
      if (same(c, d)) return;
    cands.push_back(c);
  };
  // first the layout the job has when it came from a cached choice (it can
  // need less memory than the default layouts, and it fits the bound memory
  // by construction); a job laid out with the defaults starts from the
  // explicit lane counts below
  if (!same(j->tc, TuneConfig{})) add(j->tc);
  for (int evk : {1, 2, 4})
    for (int mode : {RSL_STAGED, RSL_BATCHED})
      if (mode == RSL_STAGED || j->J.max_np <= kMaxSlots) add(TuneConfig{mode, 4096, 1, evk, 0, 0});
  // the Schur evaluation (one wave per pair) when every problem's shape allows
  // it and the job is small: its O(r) depth can only pay when the remainder
  // sequence's one or two lanes per pair leave most of the chip idle
  bool schur_ok = j->J.pairs <= 16384;
  for (int k : j->J.live) {
    const Plan& P = j->J.plans[k];
    schur_ok = schur_ok && P.my >= 1 && P.ny >= 1 && P.my + P.ny <= kSchurMaxR;
  }
  if (schur_ok) add(TuneConfig{RSL_STAGED, 4096, 1, 1, 0, 1});
  const size_t phase1 = cands.size();
  std::vector<uint8_t> ref;
  TuneConfig win = cands[0];
  double win_ms = 1e300, worst_ms = 0.0;
  bool any = false;
  int timed = 0;
  for (size_t ci = 0;; ++ci) {
    if (ci == phase1) {  // phase two around the winner of phase one
      if (!any) return fail(ctx, RSL_ENOMEM, "no schedule's layout fits the job's bound device memory");
      for (int target : {1024, 16384}) add(TuneConfig{win.mode, target, 1, win.evk, 0, win.schur});
      add(TuneConfig{win.mode, 4096, 1, win.evk, 1, win.schur});
      if (win.mode == RSL_BATCHED) add(TuneConfig{RSL_BATCHED, 4096, 2, win.evk, 0, 0});
      // the interpolation on the matrix cores (staged schedule)
      if (win.mode == RSL_STAGED) add(TuneConfig{RSL_STAGED, 4096, 1, win.evk, 1, win.schur, 1});
    }
    if (ci >= cands.size()) break;
    const TuneConfig tc = cands[ci];
    rc = materialize(ctx, j, tc);
    if (rc == RSL_ENOMEM) continue;  // this layout does not fit the bound memory
    if (rc) return rc;
    any = true;
    ++timed;
    // warm-up run (also the correctness check), then `reps` timed runs
    if ((rc = run_job(ctx, j, tc.mode)) || (rc = job_download(ctx, &j->J, j->hdown, ctx->stream)) ||
        (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize")))
      return rc;
    // statuses and outputs do not depend on the schedule: every candidate must
    // download the same words (alignment padding between them is not compared)
    std::vector<uint8_t> img;
    for (size_t li = 0; li < j->J.live.size(); ++li) {
      const Plan& P = j->J.plans[j->J.live[li]];
      const ProbLayout& L = j->J.lay[li];
      const uint8_t* st = j->hdown + (L.status - j->J.down_off);
      const uint8_t* out = j->hdown + (L.out - j->J.down_off);
      img.insert(img.end(), st, st + static_cast<size_t>(2 * P.np + 2) * 4);
      img.insert(img.end(), out, out + static_cast<size_t>(P.D + 1) * P.L_out * 4);
    }
    if (ref.empty()) {
      ref = img;
    } else if (img != ref) {
      size_t at = 0;
      while (at < img.size() && img[at] == ref[at]) ++at;
      return fail(ctx, RSL_EDEVICE,
                  "autotuner: candidate (mode " + std::to_string(tc.mode) + ", chunk target " +
                      std::to_string(tc.chunk_target) + ", grid x" + std::to_string(tc.grid_mult) +
                      ", lanes per pair " + std::to_string(tc.evk) + ", Schur " + std::to_string(tc.schur) +
                      ", matrix-core interpolation " + std::to_string(tc.interp_mm) +
                      ") differs from the first candidate in its statuses or outputs (byte " + std::to_string(at) +
                      " of the compared image)");
    }
    if ((rc = hip_check(ctx, hipEventRecord(ctx->e0, ctx->stream), "event"))) return rc;
    for (int r = 0; r < reps; ++r)
      if ((rc = run_job(ctx, j, tc.mode))) return rc;
    if ((rc = hip_check(ctx, hipEventRecord(ctx->e1, ctx->stream), "event")) ||
        (rc = hip_check(ctx, hipEventSynchronize(ctx->e1), "event")))
      return rc;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->e0, ctx->e1);
    const double per = ms / reps;
    worst_ms = std::max(worst_ms, per);
    if (per < win_ms) {
      win_ms = per;
      win = tc;
    }
  }
  if ((rc = materialize(ctx, j, win))) return rc;
  ctx->tune_cache[tune_key(j->J.n, j->f.data(), j->g.data(), j->var.data())] = TuneEntry{win, win_ms};
  if (best) *best = rsl_tune_result{win.mode, win.chunk_target, win.grid_mult, win.evk, win.conv_whole, win.schur,
                                    win.interp_mm, timed, win_ms, worst_ms};
  return RSL_OK;
}

int rsl_tune_save(rsl_ctx* ctx, const char* path) {
  if (!ctx || !path) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  std::ofstream os(path);
  if (!os) return fail(ctx, RSL_EINVAL, std::string("cannot write ") + path);
  for (const auto& kv : ctx->tune_cache)
    os << kv.first << " " << kv.second.cfg.mode << " " << kv.second.cfg.chunk_target << " "
       << kv.second.cfg.grid_mult << " " << kv.second.cfg.evk << " " << kv.second.cfg.conv_whole << " "
       << kv.second.cfg.schur << " " << kv.second.cfg.interp_mm << " " << kv.second.ms << "\n";
  return RSL_OK;
}

int rsl_tune_load(rsl_ctx* ctx, const char* path) {
  if (!ctx || !path) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  std::ifstream is(path);
  if (!is) return fail(ctx, RSL_EINVAL, std::string("cannot read ") + path);
  std::string line;
  while (std::getline(is, line)) {
    std::istringstream ls(line);
    std::string key;
    if (!(ls >> key)) continue;
    // key mode chunk grid evk conv_whole schur [interp_mm] ms
    std::vector<double> v;
    double x;
    while (ls >> x) v.push_back(x);
    TuneEntry e;
    if (v.size() != 7 && v.size() != 8) return fail(ctx, RSL_EINVAL, "malformed tuning cache line for " + key);
    e.cfg.mode = static_cast<int>(v[0]);
    e.cfg.chunk_target = static_cast<int>(v[1]);
    e.cfg.grid_mult = static_cast<int>(v[2]);
    e.cfg.evk = static_cast<int>(v[3]);
    e.cfg.conv_whole = static_cast<int>(v[4]);
    e.cfg.schur = static_cast<int>(v[5]);
    e.cfg.interp_mm = v.size() == 8 ? static_cast<int>(v[6]) : 0;
    e.ms = v.back();
    if ((e.cfg.mode != RSL_STAGED && e.cfg.mode != RSL_BATCHED) || e.cfg.chunk_target < 64 || e.cfg.grid_mult < 1 ||
        e.cfg.grid_mult > 8 || (e.cfg.evk != 1 && e.cfg.evk != 2 && e.cfg.evk != 4) ||
        (e.cfg.conv_whole != 0 && e.cfg.conv_whole != 1) || (e.cfg.schur != 0 && e.cfg.schur != 1) ||
        (e.cfg.schur && e.cfg.mode != RSL_STAGED) || (e.cfg.interp_mm != 0 && e.cfg.interp_mm != 1) ||
        (e.cfg.interp_mm && e.cfg.mode != RSL_STAGED))
      return fail(ctx, RSL_EINVAL, "malformed tuning cache line for " + key);
    ctx->tune_cache[key] = e;
  }
  return RSL_OK;
}

}  // extern "C"

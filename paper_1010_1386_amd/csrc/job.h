// A job: a planned batch of problems laid out in one device region, runnable
// as one pipeline per problem (plain) or one launch per stage over all
// problems (staged), or as a single persistent launch (batched).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rsl.h"
#include "context.h"
#include "device.h"
#include "plan.h"
#include "persistent.h"
#include "stages.h"

struct rsl_ctx;

namespace rsl {

// Schedule parameters chosen by the autotuner (tune.cpp).
struct ProbLayout {
  // offsets from the job base
  size_t coeff, gdeg, pidx, Hm, NH, Tg, invM, Plimb, Mi, wdir, rinv, negM, Mw, NHM, wMd, status;
  size_t out, resid, dig, zval, zbad, aconv, cpart, hseg, ydig, hdig, wT, wq, wS;
  int hseg_begin, hseg_end;        // range of Job::hseg_items
  int L_in;
  bool crt_own;  // this problem's layout holds the CRT constant block it shares
  int item_begin[kNumStages], item_end[kNumStages];
  int wide_begin[3], wide_end[3];  // ranges of Job::wide_items[pass] (wide CRT)
};

struct Job {
  int n = 0;                       // problems submitted
  std::vector<Plan> plans;         // one per problem
  std::vector<int> pstatus;        // planning status per problem (0 = ok)
  std::string plan_err;            // message of the first planning failure
  std::vector<int> live;           // problems with device work, in launch order
  std::vector<ProbLayout> lay;     // per live problem
  std::vector<DevProblem> dev;     // per live problem (pointers valid for `base`)
  std::vector<WorkItem> items[kNumStages];
  // evaluation items are ordered by layout: one launch per (variant, range)
  struct EvalRange {
    int variant, begin, end;
    size_t lds;  // dynamic LDS bytes of its launch: the most any of its problems needs
  };
  std::vector<EvalRange> eval_ranges;  // ranges of eval_staged
  std::vector<int> eval_vstart;        // first evaluation item of each layout variant (and the end)
  std::vector<WorkItem> eval_staged;   // evaluation items dealt across XCDs
  size_t evs_off = 0;
  // basis change over prime groups (staged schedule)
  std::vector<StirGroup> sgroups;
  std::vector<StirMember> smembers;
  std::vector<WorkItem> sg_items;
  size_t sg_off = 0, sm_off = 0, sgi_off = 0, sg_lds = 0;
  // segment polynomials of the basis change (before the stir stage)
  std::vector<WorkItem> hseg_items;
  size_t hseg_off = 0;
  // interpolation on the matrix cores: prime groups of (problem, slot) columns
  // (all members of a prime), the digit-plane items (problem, slot, block of
  // 2048 positions) and the product items (group, 64-row set, run of column tiles)
  bool mm_interp = false;
  std::vector<StirGroup> mgroups;
  std::vector<StirMember> mmembers;
  std::vector<WorkItem> dig_items, mm_items;
  int mm_lds[2] = {0, 0};  // dynamic LDS bytes of the two matrix-core interpolation launches
  size_t mg_off = 0, mm_off = 0, digi_off = 0, mmi_off = 0;
  // the ranges the kernels expect zeroed (a table in the upload image, cleared
  // by one launch after the upload)
  size_t clr_off = 0;
  int nclr = 0;
  // wide CRT (problems with more primes than the per-lane slots cover): items of
  // its three passes
  std::vector<WorkItem> wide_items[3];
  bool wide_mfma = false;          // the contraction (pass 1) runs on the matrix cores
  size_t wide_off[3] = {};
  size_t wide_lds[3] = {};
  size_t items_off[kNumStages] = {};
  size_t stage_lds[kNumStages] = {};
  int crt_ns = 1;
  int max_np = 0;                  // most primes of any live problem
  int need_g = 0, need_E = 0, need_D = 0;  // constant tables the job reads (primes, points, degree)
  bool any_schur = false;          // some problem evaluates by the Schur algorithm
  // live index of the partner (the same system eliminated in x) that a
  // problem's reduction also fills, -1 if none; prime slots shared
  std::vector<int> partner, pshared;
  std::vector<int> skip_reduce;     // leading prime slots a problem's partner reduces for it
  size_t probs_off = 0;
  size_t up_bytes = 0;             // [0, up_bytes) is uploaded
  size_t down_off = 0, down_bytes = 0;  // statuses + outputs, downloaded
  size_t status_off = 0, status_bytes = 0;
  // persistent launch: initial queue image (uploaded) and the live queue
  size_t qinit_off = 0, queue_off = 0, queue_bytes = 0;
  size_t q_tasks = 0, q_ready = 0, q_counters = 0;  // offsets inside a queue image
  int q_capacity = 0, q_initial = 0, q_crt_total = 0;
  size_t persist_lds = 0;
  int persist_grid = 0;
  size_t total = 0;
  uint8_t* base = nullptr;         // device region the job is laid out in
  std::vector<uint8_t> blob;       // host image of [0, up_bytes) when bound without an external image
  uint8_t* image = nullptr;        // the host image job_bind wrote (blob or the caller's pinned buffer)
  bool with_queue = true;          // the image holds the persistent queue (and is uploaded whole)
  bool direct_image = false;       // job_upload sends the image itself (pageable host memory), no staging
  int64_t pairs = 0;
  int64_t mulmods = 0;             // algorithmic work of eval + ures: Montgomery products over all pairs
  int64_t mm_sums_mfma = 0;        // of which evaluation sums on the matrix cores
  int64_t mm_valu = 0;             // of which on the vector ALUs
  int64_t mfma_macs = 0;           // int8 multiply-adds issued on the matrix cores for those sums
  int64_t interp_mm = 0;           // interpolation products: N_p (D+1)(D+2) over problems
  TuneConfig tune;                 // schedule parameters the job was laid out with
  // scratch of job_build, kept with the job so that a job object reused for
  // the next batch reuses its host memory (no fresh pages per call)
  std::vector<WorkItem> tmp_items;
  std::vector<int> tmp_a, tmp_b, tmp_c;
};

// Autotuner cache key of a batch (its shape bucket), from the inputs alone.
std::string tune_key(int n, const rsl_poly* f, const rsl_poly* g, const int* var);
std::string tune_key_of(const std::vector<ShapeEst>& est);

// Size of the fixed device array rsl_res_static lays its job out in.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;

// Plan every problem (host threads): plans, statuses, live problems.
int job_plan(int n, const rsl_poly* f, const rsl_poly* g, const int* var, const rsl_opts* opts, Job* J,
             std::string* err);
// Plan every problem (unless `planned`: J holds job_plan's result for these
// inputs) and lay the job out (host only).
// defer_tables: leave the context's constant tables alone (the caller grows them
// to need_g / need_E / need_D before binding; host work only, any thread).
int job_build(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, const rsl_opts* opts,
              Job* J, std::string* err, const TuneConfig* tc = nullptr, bool planned = false,
              bool defer_tables = false);
// Device work of a planned problem (evaluation, resultants and interpolation
// products), for balancing.
int64_t problem_cost(const Plan& P);
// Bind the job to a device region (fills device pointers and the upload image).
// image: host memory of at least up_bytes to write the upload image into (e.g.
// pinned staging; null = the job's own blob).  with_queue = false leaves out the
// persistent queue and the statuses (staged and plain runs clear the statuses
// themselves): only [0, upload_bytes()) is written and uploaded.
void job_bind(Job* J, uint8_t* base, uint8_t* image = nullptr, bool with_queue = true);
// Bytes of the image that job_upload sends.
inline size_t upload_bytes(const Job& J) { return J.with_queue ? J.up_bytes : J.qinit_off; }
// Upload the inputs (asynchronous on the stream).  The image is copied to
// `pinned` (>= up_bytes of pinned host memory that stays untouched until the
// copy is done) or to the context's staging buffer when pinned is null, unless
// it already is pinned memory bound with job_bind (then it is sent directly).
int job_upload(rsl_ctx* ctx, Job* J, hipStream_t st, uint8_t* pinned = nullptr);
// The two halves of job_upload: the copy of the image, and the clearing
// launches of the intermediate buffers the kernels expect zeroed (ordered
// after the copy; they may run on another stream that waits for it).
int job_upload_copy(rsl_ctx* ctx, Job* J, hipStream_t st, uint8_t* pinned = nullptr);
int job_upload_clear(rsl_ctx* ctx, Job* J, hipStream_t st);
// Zero the status words before a persistent run (the staged and plain launches
// clear them in their reduce stage).
int job_reset(rsl_ctx* ctx, Job* J, hipStream_t st);
// Launch the device pipeline: RSL_PLAIN (per problem), RSL_STAGED (one launch per
// stage over all problems) or RSL_BATCHED (one persistent launch).
int job_launch(rsl_ctx* ctx, Job* J, int mode, hipStream_t st, bool stage_events);
// Download statuses and outputs (asynchronous) into `host` (down_bytes).
int job_download(rsl_ctx* ctx, Job* J, uint8_t* host, hipStream_t st);
// Decode the downloaded image into the callers' results.
int job_decode(rsl_ctx* ctx, const Job& J, const uint8_t* host, rsl_result* out, int* status, rsl_counters* cnt);

}  // namespace rsl

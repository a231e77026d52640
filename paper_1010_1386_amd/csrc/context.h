// Context state shared by the C-ABI entry points, the batch planner and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rsl.h"
#include "device.h"
#include "plan.h"
#include "stages.h"

namespace rsl {
// Schedule parameters of a job layout (chosen by the autotuner).
struct TuneConfig {
  int mode = RSL_STAGED;      // RSL_STAGED or RSL_BATCHED
  int chunk_target = 4096;    // interpolation blocks to keep in flight (sets the k-/i-chunking)
  int grid_mult = 1;          // persistent launch: workgroups = grid_mult x resident capacity
  int evk = 0;                // lanes per (prime, point) pair in evaluation; 0 = from the job size
  int conv_whole = 0;         // 1: the convolution sums each coefficient whole (no i-chunks)
  int schur = 0;              // 1: evaluation by the Schur algorithm where the shape allows
  int interp_mm = 0;          // 1: interpolation on the matrix cores (staged schedule)
};
struct TuneEntry {
  TuneConfig cfg;
  double ms = 0.0;            // measured time per run of the winning schedule
};
struct Job;
}  // namespace rsl

struct rsl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  bool poisoned = false;
  std::string err;

  // constant tables (device, in the caller's table region), indexed by global prime index
  uint8_t* tab = nullptr;
  size_t tab_bytes = 0;   // size of the table region
  size_t tab_used = 0;    // bytes the current tables take
  std::vector<hipStream_t> reader_streams;  // other streams reading the tables (server lanes)
  struct rsl_server* server = nullptr;      // the server whose arena is the workspace, if any
  int npcap = 0, kcap = -1, scap = -1;
  rsl::PrimeConst* d_pc = nullptr;
  uint32_t* d_fact = nullptr;
  uint32_t* d_ifact = nullptr;
  uint32_t* d_stir = nullptr;
  int64_t sstride = 0;
  int kstride = 0;
  // canonical Garner tables for primes 0..garner_np-1
  uint32_t* d_Tg = nullptr;
  uint32_t* d_invM = nullptr;
  uint32_t* d_Plimb = nullptr;
  int LPg = 0;
  int garner_np = 0;

  // pinned host staging
  uint8_t* h_up = nullptr;
  size_t h_up_bytes = 0;
  uint8_t* h_down = nullptr;
  size_t h_down_bytes = 0;

  // pinned staging and completion events of the pipelined chunks of a batch call
  struct ChunkStage {
    uint8_t* up = nullptr;
    size_t up_bytes = 0;
    uint8_t* down = nullptr;
    size_t down_bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;  // around the device pipeline
    hipEvent_t e2 = nullptr;                // after the download
    hipEvent_t e3 = nullptr;                // after the upload
  };
  std::vector<ChunkStage> chunk_stage;
  // host state of the batch calls' jobs (one per chunk), reused from call to
  // call so that their large arrays keep their memory
  std::vector<std::shared_ptr<rsl::Job>> chunk_jobs;
  // copy streams of the pipelined batch call (created on first use, default
  // priority): uploads and downloads of one chunk overlap the kernels of another
  hipStream_t s_up = nullptr, s_down = nullptr;
  // second compute stream: consecutive chunks alternate between it and the
  // context's stream, so one chunk's kernels fill the tail of the previous one's
  hipStream_t s_comp2 = nullptr;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEvent_t ev[rsl::kNumStages + 1] = {};   // stage boundaries of the last batched launch
  std::vector<std::vector<hipEvent_t>> evsets; // per-run stage events while profiling
  std::vector<unsigned> evempty;               // per set: bit s = stage s launched nothing in that run
  int evused = 0;
  bool profiling = false;
  int table_gen = 0;                          // bumped whenever the constant tables move
  int64_t queue_wait_ticks = 0;               // persistent launch: longest wait for a task (counter ticks)
  bool crt_garner = false;                    // test hook (RSL_CRT_GARNER): CRT by Garner's digits only
  bool eval_horner = false;                   // test hook (RSL_EVAL_HORNER): register-form evaluation by Horner's rule only
  bool wide_valu = false;                     // test hook (RSL_WIDE_VALU): wide CRT contraction without matrix cores
  std::map<std::string, rsl::TuneEntry> tune_cache; // shape bucket -> best schedule
  rsl_counters last{};
  std::recursive_mutex mu;
};

namespace rsl {

// Set the context error message and return the code.
int fail(rsl_ctx* ctx, int code, const std::string& msg);
// Check a HIP status; on error poison the context.
int hip_check(rsl_ctx* ctx, hipError_t e, const char* what);

// Make sure the constant tables cover global prime indices < np, factorials up
// to kneed and Stirling rows up to sneed (RSL_ENOMEM when the table region is
// too small; a growth first waits for the context's streams).
int ensure_tables(rsl_ctx* ctx, int np, int kneed, int sneed);
// Layout of the constant tables in their region, for the given capacities.
struct TableLayout {
  size_t pc, fact, ifact, stir, Tg, invM, Plimb, total;
  int64_t sstride;
  int ks, gnp, LPg;
};
TableLayout table_layout(int np_cap, int kcap, int scap);
// Capacities ensure_tables rounds a need up to.
void table_caps(int np, int kneed, int sneed, int* np_cap, int* kcap, int* scap);
// Wait for every stream of the context that may read the tables.
int wait_table_readers(rsl_ctx* ctx);
// The error of a call that needs the workspace while a server owns it.
int workspace_taken(rsl_ctx* ctx);
DevTables tables_of(const rsl_ctx* ctx);

// Grow the pinned staging buffers.
int ensure_staging(rsl_ctx* ctx, size_t up, size_t down);

// Decode the CRT limbs of a problem into the caller's result.
int decode_result(const Plan& P, const uint32_t* limbs, rsl_result* out);

double now_ms();

}  // namespace rsl

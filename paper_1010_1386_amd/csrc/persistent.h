// Device task queue of the persistent batched launch (persistent.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "device.h"

namespace rsl {

enum : int {
  kTaskReduce = 0,
  kTaskEval = 1,
  kTaskConv = 2,
  kTaskStir = 3,
  kTaskNewton = 4,
  kTaskCrt = 5,
};

constexpr int kCrtPerTask = 8;     // coefficients per CRT task
constexpr int kMaxSlots = 256;     // primes per problem

struct Task {
  int type_prob;  // type << 24 | problem
  int slot;
  int blk;
  int sub;
};

struct QueueState {
  int head;       // next slot to pop
  int tail;       // next slot to fill
  int done;       // set when the last CRT task finishes (or on an error)
  int crt_done;   // CRT tasks finished
  int err;        // kErrQueueStall when a wave gave up waiting
  int pad[11];
};

// Dependency counters of one problem.
struct ProbCounters {
  int slots_left;
  int pad[3];
  int eval_left[kMaxSlots];
  int conv_left[kMaxSlots];
  int stir_left[kMaxSlots];
};

struct QueueDesc {
  QueueState* state;
  Task* tasks;
  int* ready;
  ProbCounters* counters;
  int capacity;
  int crt_total;
  int nprob;
  int64_t wait_ticks;  // longest wait for a queue slot, in wall-clock counter ticks
};

hipError_t launch_persistent(const DevProblem* probs, const QueueDesc& Q, const DevTables& T, int ns, int grid,
                             size_t lds, hipStream_t st);
// Resident workgroups per CU of the persistent kernel at a given LDS size.
int persistent_blocks_per_cu(int ns, size_t lds);

}  // namespace rsl

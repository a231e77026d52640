// One persistent launch for a whole batch of problems.
//
// Workgroups of one wave pop tasks from a device queue.  A task is one block
// of one stage of one problem (the same stage_* code as the staged launches);
// finishing the last task of a group enqueues the next stage's tasks:
//
//   REDUCE(p, s) -> EVAL(p, s, *)            per (problem, prime slot)
//   last EVAL(p, s, *) -> CONV(p, s, *)  if the points origin..origin+D are all usable
//                      -> NEWTON(p, s)    otherwise (gapped point set)
//   last CONV(p, s, *) -> STIR(p, s, *)
//   last STIR(p, s, *) -> NEWTON(p, s)  for a shifted origin (the shift back)
//   last STIR(p, s, *) otherwise, or NEWTON(p, s) -> slot done; last slot of p -> CRT(p, *)
//   last CRT task of the batch -> done
//
// Termination: every wave exits once the done flag is set (or on an error),
// so a wave waiting on an empty queue slot never outlives the batch.  The
// wait is bounded in wall-clock time (QueueDesc::wait_ticks of the constant
// rate counter): past it the wave records kErrQueueStall and raises the done
// flag, which ends the launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "persistent.h"
#include "stages.h"

namespace rsl {

static_assert(kCrtPerTask == kCrtBlockCoeffs, "a CRT task is one CRT block's coefficients");

// Polling load: coherent at device scope but without the cache invalidation an
// acquire implies (thousands of waiting waves must not keep invalidating the
// caches the working waves use); an acquire fence follows a successful poll.
__device__ __forceinline__ int ld_poll(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Give up the launch: mark every problem and raise the done flag.
__device__ inline void queue_abort(const QueueDesc& Q, const DevProblem* probs) {
  atomicOr(&Q.state->err, kErrQueueStall);
  for (int i = 0; i < Q.nprob; ++i) atomicOr(probs[i].status, kErrQueueStall);
  st_release(&Q.state->done, 1);
}

// Enqueue n tasks made by make(i) (i < n); called by one thread.
template <class F>
__device__ inline void enqueue(const QueueDesc& Q, const DevProblem* probs, int n, F make) {
  if (n <= 0) return;
  const int base = atomicAdd(&Q.state->tail, n);
  for (int i = 0; i < n; ++i) {
    const int s = base + i;
    if (s >= Q.capacity) {  // cannot happen with a correct capacity; fail loudly
      queue_abort(Q, probs);
      return;
    }
    Q.tasks[s] = make(i);
  }
  // one release for the task records (and everything this wave has seen),
  // then plain flag stores
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  for (int i = 0; i < n; ++i) __hip_atomic_store(&Q.ready[base + i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline Task mk(int type, int prob, int slot, int blk, int sub) {
  Task t;
  t.type_prob = (type << 24) | prob;
  t.slot = slot;
  t.blk = blk;
  t.sub = sub;
  return t;
}

template <int NS>
__global__ __launch_bounds__(64) void k_persistent(const DevProblem* probs, QueueDesc Q, DevTables T) {
  extern __shared__ uint4 lds4[];
  uint32_t* lds = reinterpret_cast<uint32_t*>(lds4);
  __shared__ Task cur;
  __shared__ int quit;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      quit = 0;
      const int s = atomicAdd(&Q.state->head, 1);
      const uint64_t t0 = wall_clock64();
      for (int polls = 1;; ++polls) {
        if (ld_poll(&Q.state->done)) { quit = 1; break; }
        if (s < Q.capacity && ld_poll(&Q.ready[s])) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          cur = Q.tasks[s];
          break;
        }
        if ((polls & 63) == 0 && static_cast<int64_t>(wall_clock64() - t0) > Q.wait_ticks) {
          queue_abort(Q, probs);
          quit = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
    if (quit) return;
    const Task t = cur;
    __syncthreads();
    const int type = t.type_prob >> 24;
    const int prob = t.type_prob & 0xFFFFFF;
    const DevProblem& P = probs[prob];
    const WorkItem w{prob, t.slot, t.blk, t.sub};
    ProbCounters* C = Q.counters + prob;
    switch (type) {
      case kTaskReduce:
        for (int b = 0; b * 64 < P.CS; ++b) stage_reduce(P, T, WorkItem{prob, t.slot, b, 0});
        break;
      case kTaskEval: stage_eval<false>(P, T, w, lds); break;
      case kTaskConv: stage_interp_conv(P, T, w, lds); break;
      case kTaskStir: stage_interp_stir<false>(P, T, w, lds); break;
      case kTaskNewton: stage_interp_newton(P, T, w, lds); break;
      case kTaskCrt: stage_crt<NS>(P, T, w, lds, kCrtPerTask); break;
      default: break;
    }
    // successors (decided by thread 0 after the block's writes are released)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (type == kTaskEval) {
      // last EVAL of the slot: choose the interpolation path (block-uniform)
      __shared__ int last;
      if (tid == 0) last = (atomicSub(&C->eval_left[t.slot], 1) == 1);
      __syncthreads();
      if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other eval blocks' flags
        const bool fast = fast_prime(P, t.slot);
        if (tid == 0) {
          if (fast) {
            const int nb = (P.D + 64) / 64;
            enqueue(Q, probs, nb * P.ncchunk,
                    [&](int i) { return mk(kTaskConv, prob, t.slot, i / P.ncchunk, i % P.ncchunk); });
          } else {
            enqueue(Q, probs, 1, [&](int) { return mk(kTaskNewton, prob, t.slot, 0, 0); });
          }
        }
      }
    } else if (tid == 0) {
      switch (type) {
        case kTaskReduce: {
          const int nb = (P.E + P.evpb) / P.evpb;
          enqueue(Q, probs, nb, [&](int i) { return mk(kTaskEval, prob, t.slot, i, 0); });
          break;
        }
        case kTaskConv:
          if (atomicSub(&C->conv_left[t.slot], 1) == 1) {
            const int nj = (P.D + 64) / 64;  // one wave: 64 columns per task
            enqueue(Q, probs, nj * P.nchunk, [&](int i) { return mk(kTaskStir, prob, t.slot, i / P.nchunk, i % P.nchunk); });
          }
          break;
        case kTaskStir:
        case kTaskNewton: {
          bool slot_done = true;
          if (type == kTaskStir) {
            slot_done = (atomicSub(&C->stir_left[t.slot], 1) == 1);
            if (slot_done && P.origin != 0) {  // the shift back from the origin first
              enqueue(Q, probs, 1, [&](int) { return mk(kTaskNewton, prob, t.slot, 0, 0); });
              slot_done = false;
            }
          }
          if (slot_done && atomicSub(&C->slots_left, 1) == 1) {
            const int nc = (P.D + kCrtPerTask) / kCrtPerTask;
            enqueue(Q, probs, nc, [&](int i) { return mk(kTaskCrt, prob, -1, i, 0); });
          }
          break;
        }
        case kTaskCrt:
          if (atomicAdd(&Q.state->crt_done, 1) == Q.crt_total - 1) st_release(&Q.state->done, 1);
          break;
        default: break;
      }
    }
  }
}

hipError_t launch_persistent(const DevProblem* probs, const QueueDesc& Q, const DevTables& T, int ns, int grid,
                             size_t lds, hipStream_t st) {
  switch (ns) {
    case 1: hipLaunchKernelGGL(k_persistent<1>, dim3(grid), dim3(64), lds, st, probs, Q, T); break;
    case 2: hipLaunchKernelGGL(k_persistent<2>, dim3(grid), dim3(64), lds, st, probs, Q, T); break;
    case 3: hipLaunchKernelGGL(k_persistent<3>, dim3(grid), dim3(64), lds, st, probs, Q, T); break;
    case 4: hipLaunchKernelGGL(k_persistent<4>, dim3(grid), dim3(64), lds, st, probs, Q, T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rsl

namespace rsl {

int persistent_blocks_per_cu(int ns, size_t lds) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ns) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<1>, 64, lds); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<2>, 64, lds); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<3>, 64, lds); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<4>, 64, lds); break;
    default: break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace rsl

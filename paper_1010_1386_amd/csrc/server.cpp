// Request server with continuous batching (rsl_server_* in include/rsl.h).
//
// Client threads submit requests (inputs are copied at submit).  A scheduler
// thread admits pending requests in FIFO order while a slot is free and the
// sum of the admitted requests' device footprints stays within the budget,
// plans the admitted group as one job laid out in a region of the context
// workspace (first-fit arena), and runs it with the staged schedule on one of
// several HIP streams ("lanes").  Requests that arrive while batches run join
// the next batch as soon as a lane, slots and memory are free, so the work of
// requests admitted at different times overlaps on the device.  A finished
// batch (its lane's event has completed) is decoded into the callers' result
// buffers and its workspace region and slots are released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.h"
#include "job.h"

namespace rsl {
namespace {

constexpr int kLanes = 3;  // batches in flight at once, one HIP stream each
// Layout of the server's batches: the interpolation sums taken whole (one
// chunk), which keeps each request's footprint -- and so the budget's share
// per request -- a few times smaller than the throughput layout of large
// batch calls; a batch of many requests has enough blocks in flight anyway.
const TuneConfig kServeLayout{RSL_STAGED, 64, 1, 0, 1, 0};
constexpr int kTablesFull = -1000;  // launch(): the table region cannot cover the group

struct Request {
  uint64_t ticket = 0;
  std::vector<uint32_t> fc, gc;
  rsl_poly f{}, g{};
  int var = RSL_Y;
  rsl_result* out = nullptr;
  Plan plan;                 // planned once, at submit; the batch layout reuses it
  size_t footprint = 0;
  double t_submit = 0.0;
  bool done = false;
  int status = RSL_OK;
};

// First-fit allocator over [0, size) of the workspace.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* h_up = nullptr;
  size_t h_up_bytes = 0;
  uint8_t* h_down = nullptr;
  size_t h_down_bytes = 0;
  bool busy = false;
  Job job;
  std::vector<std::shared_ptr<Request>> reqs;
  std::vector<rsl_result> outs;
  size_t off = 0, bytes = 0;
};

int grow_pinned(uint8_t** p, size_t* have, size_t need) {
  if (need <= *have) return RSL_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  const size_t sz = std::max<size_t>((need + (1 << 20) - 1) / (1 << 20) * (1 << 20), 1 << 20);
  if (hipHostMalloc(reinterpret_cast<void**>(p), sz, hipHostMallocDefault) != hipSuccess) return RSL_EDEVICE;
  *have = sz;
  return RSL_OK;
}

double pctl(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t i = std::min(v.size() - 1, static_cast<size_t>(q * (v.size() - 1) + 0.5));
  return v[i];
}

}  // namespace
}  // namespace rsl

struct rsl_server {
  rsl_ctx* ctx = nullptr;
  size_t budget = 0;
  int max_slots = 1;
  int max_queue = 1;
  std::mutex mu;
  std::condition_variable cv_sched;  // wakes the scheduler (submit, stop)
  std::condition_variable cv_done;   // wakes waiting clients
  std::deque<std::shared_ptr<rsl::Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<rsl::Request>> tickets;
  uint64_t next_ticket = 1;
  // planned requests not queued yet (rsl_server_plan -> rsl_server_enqueue)
  std::unordered_map<uint64_t, std::shared_ptr<rsl::Request>> planned;
  uint64_t next_handle = 1;
  bool stop = false;
  std::thread th;
  rsl::Arena arena;
  rsl::Lane lanes[rsl::kLanes];
  int slots_used = 0;
  size_t bytes_used = 0;
  int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, max_batch = 0;
  int64_t admitted_peak = 0;
  std::vector<double> lat_ms;
  double t_created = 0.0;
};

namespace rsl {
namespace {

void finish(rsl_server* S, Request& r, int status) {
  r.status = status;
  r.done = true;
  S->lat_ms.push_back(now_ms() - r.t_submit);
  S->completed += 1;
}

// Decode a finished lane and release its resources (server lock held).
void retire(rsl_server* S, Lane& ln) {
  const int n = static_cast<int>(ln.reqs.size());
  std::vector<int> st(n, RSL_OK);
  rsl_counters cnt{};
  {
    std::lock_guard<std::recursive_mutex> lk(S->ctx->mu);
    job_decode(S->ctx, ln.job, ln.h_down, ln.outs.data(), st.data(), &cnt);
  }
  for (int k = 0; k < n; ++k) {
    *ln.reqs[k]->out = ln.outs[k];
    finish(S, *ln.reqs[k], st[k]);
  }
  S->arena.release(ln.off, ln.bytes);
  S->bytes_used -= ln.bytes;
  S->slots_used -= n;
  ln.reqs.clear();
  ln.outs.clear();
  ln.job = Job();
  ln.busy = false;
  S->cv_done.notify_all();
}

// Plan the admitted group and launch it on the lane.  Called WITHOUT the
// server lock (clients keep submitting meanwhile); touches only the lane and
// the arena, which belong to the scheduler thread.  Returns RSL_ENOMEM when the
// arena has no room yet.
int launch(rsl_server* S, Lane& ln, std::vector<std::shared_ptr<Request>>& grp) {
  rsl_ctx* ctx = S->ctx;
  const int n = static_cast<int>(grp.size());
  std::vector<rsl_poly> f(n), g(n);
  std::vector<int> var(n);
  for (int k = 0; k < n; ++k) {
    f[k] = grp[k]->f;
    g[k] = grp[k]->g;
    var[k] = grp[k]->var;
  }
  // the requests' plans from submit: only the layout of the group is new
  Job J;
  J.n = n;
  J.plans.resize(n);
  J.pstatus.assign(n, 0);
  J.live.clear();
  for (int k = 0; k < n; ++k) {
    J.plans[k] = grp[k]->plan;
    if (!J.plans[k].zero) J.live.push_back(k);
  }
  std::string err;
  int rc;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    rc = job_build(ctx, n, f.data(), g.data(), var.data(), nullptr, &J, &err, &kServeLayout, /*planned=*/true);
  }
  if (rc) return rc == RSL_ENOMEM ? kTablesFull : rc;  // waiting frees no table room
  size_t off = 0;
  const size_t bytes = std::max<size_t>(J.total, 256);
  if (!S->arena.alloc(bytes, &off)) return RSL_ENOMEM;
  ln.job = std::move(J);
  ln.off = off;
  ln.bytes = bytes;
  if (grow_pinned(&ln.h_up, &ln.h_up_bytes, ln.job.up_bytes) ||
      grow_pinned(&ln.h_down, &ln.h_down_bytes, ln.job.down_bytes)) {
    S->arena.release(off, bytes);
    return RSL_EDEVICE;
  }
  // the upload image written straight into the lane's pinned staging, without
  // the persistent queue (the lane's previous upload is complete: it retired)
  job_bind(&ln.job, ctx->ws + off, ln.h_up, false);
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if ((rc = job_upload(ctx, &ln.job, ln.stream, ln.h_up)) ||
        (rc = job_launch(ctx, &ln.job, RSL_STAGED, ln.stream, false)) ||
        (rc = job_download(ctx, &ln.job, ln.h_down, ln.stream)) ||
        (rc = hip_check(ctx, hipEventRecord(ln.done, ln.stream), "event"))) {
      S->arena.release(off, bytes);
      return rc;
    }
  }
  ln.reqs = grp;
  ln.outs.resize(n);
  for (int k = 0; k < n; ++k) ln.outs[k] = *grp[k]->out;
  ln.busy = true;
  return RSL_OK;
}

// Book a launched lane in the server's accounting (server lock held).
void account(rsl_server* S, const Lane& ln) {
  const int n = static_cast<int>(ln.reqs.size());
  S->bytes_used += ln.bytes;
  S->slots_used += n;
  S->admitted_peak = std::max<int64_t>(S->admitted_peak, static_cast<int64_t>(S->bytes_used));
  S->launches += 1;
  S->max_batch = std::max<int64_t>(S->max_batch, n);
}

void scheduler(rsl_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool any_busy = false;
    for (Lane& ln : S->lanes) {
      if (ln.busy && hipEventQuery(ln.done) == hipSuccess) retire(S, ln);
      any_busy |= ln.busy;
    }
    // admission: FIFO while a lane, slots and budget allow
    for (Lane& ln : S->lanes) {
      if (ln.busy || S->pending.empty()) continue;
      std::vector<std::shared_ptr<Request>> grp;
      size_t est = 0;
      while (!S->pending.empty()) {
        const auto& r = S->pending.front();
        if (S->slots_used + static_cast<int>(grp.size()) >= S->max_slots) break;
        if (S->bytes_used + est + r->footprint > S->budget) break;
        est += r->footprint;
        grp.push_back(r);
        S->pending.pop_front();
      }
      if (grp.empty()) break;
      // plan and launch without the lock: requests arriving meanwhile queue up
      // and form the next batch
      std::vector<std::shared_ptr<Request>> back;  // returned to the queue, in order
      lk.unlock();
      int rc = launch(S, ln, grp);
      while (rc == RSL_ENOMEM && grp.size() > 1) {  // arena fragmented: shrink the group
        back.insert(back.begin(), grp.back());
        grp.pop_back();
        rc = launch(S, ln, grp);
      }
      lk.lock();
      if (rc == RSL_ENOMEM && any_busy) {  // no room yet: wait for a batch to finish
        back.insert(back.begin(), grp.front());
        grp.clear();
      }
      for (auto it = back.rbegin(); it != back.rend(); ++it) S->pending.push_front(*it);
      if (grp.empty()) break;
      if (rc) {
        if (rc == kTablesFull) rc = RSL_ENOMEM;
        for (auto& r : grp) finish(S, *r, rc);
        S->cv_done.notify_all();
        continue;
      }
      account(S, ln);
      any_busy = true;
    }
    if (S->stop && S->pending.empty() && !any_busy) break;
    if (any_busy)
      S->cv_sched.wait_for(lk, std::chrono::microseconds(20));
    else
      S->cv_sched.wait(lk, [&] { return S->stop || !S->pending.empty(); });
  }
}

}  // namespace
}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_server_create(rsl_ctx* ctx, size_t budget_bytes, int max_slots, int max_queue, rsl_server** out) {
  if (!ctx || !out || max_slots < 1 || max_queue < 1 || budget_bytes == 0) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> ctx_lk(ctx->mu);
  if (ctx->server) return fail(ctx, RSL_EINVAL, "a server already runs on this context");
  if (budget_bytes > ctx->ws_bytes) return fail(ctx, RSL_ENOMEM, "server budget exceeds the workspace");
  *out = nullptr;
  rsl_server* S = new (std::nothrow) rsl_server();
  if (!S) return RSL_ENOMEM;
  S->ctx = ctx;
  S->budget = budget_bytes;
  S->max_slots = max_slots;
  S->max_queue = max_queue;
  S->arena.reset(budget_bytes);
  S->t_created = now_ms();
  if (hipSetDevice(ctx->device) != hipSuccess) { delete S; return RSL_EDEVICE; }
  for (Lane& ln : S->lanes) {
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
      for (Lane& l2 : S->lanes) {
        if (l2.stream) (void)hipStreamDestroy(l2.stream);
        if (l2.done) (void)hipEventDestroy(l2.done);
      }
      delete S;
      return RSL_EDEVICE;
    }
  }
  // the lanes read the constant tables: a table growth waits for them too
  for (Lane& ln : S->lanes) ctx->reader_streams.push_back(ln.stream);
  ctx->server = S;
  S->th = std::thread(scheduler, S);
  *out = S;
  return RSL_OK;
}

// Plan the request (host only): sizes, footprint, admission against the
// table region.  On success *rp holds the request, not yet queued.
static int plan_request(rsl_server* S, const rsl_poly* f, const rsl_poly* g, int var,
                        std::shared_ptr<Request>* rp, rsl_info* info) {
  auto r = std::make_shared<Request>();
  auto copy = [](const rsl_poly* p, std::vector<uint32_t>* buf, rsl_poly* dst) {
    if (!p->coeff || p->dx < 0 || p->dy < 0 || p->limbs < 1) return false;
    buf->assign(p->coeff, p->coeff + static_cast<size_t>(p->dx + 1) * (p->dy + 1) * p->limbs);
    *dst = *p;
    dst->coeff = buf->data();
    return true;
  };
  if (!copy(f, &r->fc, &r->f) || !copy(g, &r->gc, &r->g) || (var != RSL_Y && var != RSL_X)) return RSL_EINVAL;
  r->var = var;
  // the one plan of this request, and its footprint from the layout of it alone
  Job J;
  std::string err;
  int rc = job_build(nullptr, 1, &r->f, &r->g, &r->var, nullptr, &J, &err, &kServeLayout);
  if (rc) return rc;
  if (J.pstatus[0]) return J.pstatus[0];
  r->footprint = std::max<size_t>(J.total, 256);
  if (info) {
    const Plan& P = J.plans[0];
    *info = rsl_info{};
    if (P.zero) {  // as rsl_query: R = 0
      info->D = -1;
      info->my = P.f.dy;
      info->ny = P.g.dy;
      info->out_limbs = 1;
    } else {
      info->D = P.D;
      info->bound_bits = P.bound_bits;
      info->n_primes = P.np;
      info->n_points = P.E + 1;
      info->out_limbs = P.L_out;
      info->my = P.my;
      info->ny = P.ny;
      info->bad_primes = P.bad_primes;
      info->origin = P.origin;
    }
    info->footprint_bytes = J.total;
  }
  {
    // the constant tables this request needs (with what the context holds) must fit the table region
    rsl_ctx* ctx = S->ctx;
    std::lock_guard<std::recursive_mutex> ctx_lk(ctx->mu);
    int cn, ck, cs;
    table_caps(J.need_g, J.need_E, J.need_D, &cn, &ck, &cs);
    const size_t tb = table_layout(std::max(cn, ctx->npcap), std::max(ck, ctx->kcap), std::max(cs, ctx->scap)).total;
    if (info) info->table_bytes = tb;
    if (tb > ctx->tab_bytes) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->rejected += 1;
      return fail(ctx, RSL_ENOMEM, "the request's constant tables need " + std::to_string(tb) +
                                       " bytes, the table region has " + std::to_string(ctx->tab_bytes));
    }
  }
  r->plan = std::move(J.plans[0]);
  *rp = std::move(r);
  return RSL_OK;
}

// Queue a planned request with its result buffer (server lock not held).
static int enqueue(rsl_server* S, std::shared_ptr<Request> r, rsl_result* out, uint64_t* ticket) {
  r->out = out;
  std::lock_guard<std::mutex> lk(S->mu);
  if (r->footprint > S->budget) {
    S->rejected += 1;
    return RSL_ENOMEM;
  }
  if (static_cast<int>(S->pending.size()) >= S->max_queue) {
    S->rejected += 1;
    return RSL_EAGAIN;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = now_ms();
  S->tickets[r->ticket] = r;
  S->pending.push_back(r);
  S->submitted += 1;
  *ticket = r->ticket;
  S->cv_sched.notify_one();
  return RSL_OK;
}

int rsl_server_submit(rsl_server* S, const rsl_poly* f, const rsl_poly* g, int var, rsl_result* out,
                      uint64_t* ticket) {
  if (!S || !f || !g || !out || !ticket) return RSL_EINVAL;
  std::shared_ptr<Request> r;
  int rc = plan_request(S, f, g, var, &r, nullptr);
  if (rc) return rc;
  return enqueue(S, std::move(r), out, ticket);
}

int rsl_server_plan(rsl_server* S, const rsl_poly* f, const rsl_poly* g, int var, rsl_info* info,
                    uint64_t* handle) {
  if (!S || !f || !g || !info || !handle) return RSL_EINVAL;
  std::shared_ptr<Request> r;
  int rc = plan_request(S, f, g, var, &r, info);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(S->mu);
  const uint64_t h = S->next_handle++;
  S->planned[h] = std::move(r);
  *handle = h;
  return RSL_OK;
}

int rsl_server_enqueue(rsl_server* S, uint64_t handle, rsl_result* out, uint64_t* ticket) {
  if (!S || !out || !ticket) return RSL_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->planned.find(handle);
    if (it == S->planned.end()) return RSL_EINVAL;
    r = std::move(it->second);
    S->planned.erase(it);
  }
  const int rc = enqueue(S, r, out, ticket);
  if (rc == RSL_EAGAIN) {  // queue full: the handle stays valid for a later enqueue
    std::lock_guard<std::mutex> lk(S->mu);
    S->planned[handle] = std::move(r);
  }
  return rc;
}

int rsl_server_poll(rsl_server* S, uint64_t ticket, int* status) {
  if (!S) return RSL_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return RSL_EINVAL;
  if (!it->second->done) return 0;
  if (status) *status = it->second->status;
  S->tickets.erase(it);
  return 1;
}

int rsl_server_wait(rsl_server* S, uint64_t ticket, int timeout_ms) {
  if (!S) return RSL_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return RSL_EINVAL;
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return RSL_ETIMEDOUT;
  }
  S->tickets.erase(ticket);
  return r->status;
}

int rsl_server_stats(rsl_server* S, rsl_stats* st) {
  if (!S || !st) return RSL_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->rejected = S->rejected;
  st->in_flight = S->submitted - S->completed;
  st->p50_ms = pctl(S->lat_ms, 0.50);
  st->p99_ms = pctl(S->lat_ms, 0.99);
  double sum = 0.0;
  for (double v : S->lat_ms) sum += v;
  st->mean_ms = S->lat_ms.empty() ? 0.0 : sum / S->lat_ms.size();
  const double el = (now_ms() - S->t_created) * 1e-3;
  st->throughput = el > 0 ? S->completed / el : 0.0;
  st->admitted_bytes_peak = S->admitted_peak;
  st->launches = S->launches;
  st->max_batch = S->max_batch;
  return RSL_OK;
}

int rsl_server_destroy(rsl_server* S) {
  if (!S) return RSL_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_sched.notify_all();
  if (S->th.joinable()) S->th.join();  // drains pending and in-flight requests
  (void)hipSetDevice(S->ctx->device);
  {
    std::lock_guard<std::recursive_mutex> ctx_lk(S->ctx->mu);
    std::vector<hipStream_t>& rs = S->ctx->reader_streams;
    for (Lane& ln : S->lanes) rs.erase(std::remove(rs.begin(), rs.end(), ln.stream), rs.end());
    S->ctx->server = nullptr;
  }
  for (Lane& ln : S->lanes) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.h_up) (void)hipHostFree(ln.h_up);
    if (ln.h_down) (void)hipHostFree(ln.h_down);
  }
  delete S;
  return RSL_OK;
}

}  // extern "C"

// Host-side stress driver for the library's planning, layout and decoding code,
// built with AddressSanitizer + UndefinedBehaviorSanitizer (or ThreadSanitizer)
// from the same sources as the library, host pass only (test infrastructure:
// no device is touched; device entry points are expected to report
// RSL_EDEVICE without a GPU).
//
// Several threads at once
//   - size problems of random shape and coefficient size through rsl_query
//     (the shared prime table grows while other threads read it),
//   - plan and lay out batches (job_plan / job_build without a context, whose
//     per-problem planning runs on the shared host pool) under every schedule
//     and lanes-per-pair choice, and estimate shapes for the schedule lookup,
//   - decode a download image of random words with job_decode (every status
//     and residue word a device could write, in range or not),
// and every thread must reach the same sizes for the same problem.
// Exit status 0 = all checks passed; a sanitizer report aborts with its own.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1010_1386_amd/csrc/job.h"

using namespace rsl;

namespace {

// SplitMix64 (Steele, Lea, Flood 2014): the driver's own seeded stream.
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int range(int lo, int hi) { return lo + static_cast<int>(next() % static_cast<uint64_t>(hi - lo + 1)); }
};

struct Poly {
  std::vector<uint32_t> w;
  rsl_poly p{};
};

// Dense bivariate polynomial of total degree <= d with `bits`-bit signed
// coefficients (limbs = bits/32 + 1), some rows and leading terms zeroed.
Poly random_poly(Rng& r, int d, int bits) {
  Poly P;
  const int L = bits / 32 + 1;
  P.p.dx = d;
  P.p.dy = d;
  P.p.limbs = L;
  P.w.assign(static_cast<size_t>(d + 1) * (d + 1) * L, 0u);
  for (int j = 0; j <= d; ++j)
    for (int i = 0; i + j <= d; ++i) {
      if (r.next() % 5 == 0) continue;
      uint32_t* c = &P.w[(static_cast<size_t>(j) * (d + 1) + i) * L];
      for (int l = 0; l < L; ++l) {
        const int lbits = std::min(32, bits - 32 * l);
        c[l] = lbits <= 0 ? 0u : static_cast<uint32_t>(r.next()) & (lbits == 32 ? ~0u : ((1u << lbits) - 1));
      }
      if (r.next() & 1) {  // negate: two's complement over all limbs
        uint64_t carry = 1;
        for (int l = 0; l < L; ++l) {
          const uint64_t v = static_cast<uint64_t>(~c[l]) + carry;
          c[l] = static_cast<uint32_t>(v);
          carry = v >> 32;
        }
      }
    }
  P.p.coeff = P.w.data();
  return P;
}

struct Problem {
  Poly f, g;
  int var;
};

std::vector<Problem> make_problems(uint64_t seed, int n, int dmax, int bmax) {
  Rng r(seed);
  std::vector<Problem> v(n);
  for (int k = 0; k < n; ++k) {
    v[k].f = random_poly(r, r.range(1, dmax), r.range(4, bmax));
    v[k].g = random_poly(r, r.range(1, dmax), r.range(4, bmax));
    v[k].var = (r.next() & 1) ? RSL_X : RSL_Y;
  }
  return v;
}

std::atomic<int> g_fail{0};

void check(bool ok, const char* what, int a = 0, int b = 0) {
  if (!ok) {
    std::fprintf(stderr, "CHECK FAILED: %s (%d, %d)\n", what, a, b);
    g_fail.fetch_add(1);
  }
}

struct Sizes {
  int rc, D, np, out_limbs;
  size_t footprint, table;
};

Sizes query(const Problem& p) {
  rsl_info info{};
  Sizes s{};
  s.rc = rsl_query(&p.f.p, &p.g.p, p.var, &info);
  s.D = info.D;
  s.np = info.n_primes;
  s.out_limbs = info.out_limbs;
  s.footprint = info.footprint_bytes;
  s.table = info.table_bytes;
  return s;
}

// One batch: plan + lay out under a schedule, then decode random words.
void layout_and_decode(const std::vector<Problem>& probs, int lo, int hi, const TuneConfig& tc, uint64_t seed,
                       size_t* total_out) {
  const int n = hi - lo;
  std::vector<rsl_poly> f(n), g(n);
  std::vector<int> var(n);
  for (int k = 0; k < n; ++k) {
    f[k] = probs[lo + k].f.p;
    g[k] = probs[lo + k].g.p;
    var[k] = probs[lo + k].var;
  }
  std::vector<ShapeEst> est(n);
  for (int k = 0; k < n; ++k) est[k] = estimate_shape(&f[k], &g[k], var[k]);
  const std::string key = tune_key_of(est);
  check(!key.empty(), "tune key");

  Job J;
  std::string err;
  job_plan(n, f.data(), g.data(), var.data(), nullptr, &J, &err);
  const int rc = job_build(nullptr, n, f.data(), g.data(), var.data(), nullptr, &J, &err, &tc, true, true);
  check(rc == RSL_OK || rc == RSL_EINVAL, "job_build", rc);
  if (rc) return;
  *total_out = J.total;
  check(J.down_off + J.down_bytes <= J.total, "download window inside the layout");
  for (size_t li = 0; li < J.live.size(); ++li) {
    const ProbLayout& L = J.lay[li];
    check(L.status >= J.down_off && L.status < J.down_off + J.down_bytes, "status in the download window");
    check(L.out >= J.down_off && L.out < J.down_off + J.down_bytes, "output in the download window");
  }
  // a download image of random words: statuses and residues the decoder must survive
  Rng r(seed);
  std::vector<uint8_t> img(std::max<size_t>(J.down_bytes, 4));
  for (size_t i = 0; i + 4 <= img.size(); i += 4) {
    const uint32_t w = static_cast<uint32_t>(r.next());
    std::memcpy(&img[i], &w, 4);
  }
  std::vector<std::vector<uint32_t>> bufs(n);
  std::vector<rsl_result> out(n);
  for (int k = 0; k < n; ++k) {
    const Sizes s = query(probs[lo + k]);
    const int cap = std::max(s.D, 0), lim = std::max(1, s.out_limbs);
    bufs[k].assign(static_cast<size_t>(cap + 1) * lim, 0u);
    out[k] = rsl_result{cap, lim, bufs[k].data(), 0, 0};
  }
  std::vector<int> st(n, 0);
  rsl_counters cnt{};
  // job_decode writes its error text into the context: give it a host-only one
  static thread_local rsl_ctx host_ctx;
  (void)job_decode(&host_ctx, J, img.data(), out.data(), st.data(), &cnt);
  for (int k = 0; k < n; ++k) {
    check(out[k].deg <= out[k].cap_deg || st[k] == RSL_ERANGE, "decoded degree within capacity", out[k].deg,
          out[k].cap_deg);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int T = argc > 1 ? std::atoi(argv[1]) : 8;
  const int N = argc > 2 ? std::atoi(argv[2]) : 96;
  // problems that need ever more primes, so that the first threads to reach
  // them grow the shared prime table while the others read it
  std::vector<Problem> probs = make_problems(12345, N, 16, 600);

  // 1. sizing from every thread at once, each in its own order
  std::vector<std::vector<Sizes>> sz(T, std::vector<Sizes>(N));
  {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        for (int i = 0; i < N; ++i) {
          const int k = (t & 1) ? N - 1 - (i + 7 * t) % N : (i + 7 * t) % N;
          sz[t][k] = query(probs[k]);
        }
      });
    for (auto& x : th) x.join();
  }
  for (int t = 1; t < T; ++t)
    for (int k = 0; k < N; ++k) {
      const Sizes &a = sz[0][k], &b = sz[t][k];
      check(a.rc == b.rc && a.D == b.D && a.np == b.np && a.out_limbs == b.out_limbs &&
                a.footprint == b.footprint && a.table == b.table,
            "the same sizes from every thread", t, k);
    }
  for (int k = 0; k < N; ++k) check(sz[0][k].rc == RSL_OK && sz[0][k].np > 0, "query", sz[0][k].rc, k);

  // 2. layouts under every schedule choice, batches planned from several threads
  const TuneConfig cfgs[] = {
      TuneConfig{RSL_STAGED, 4096, 1, 1, 0, 0}, TuneConfig{RSL_STAGED, 1024, 1, 2, 0, 0},
      TuneConfig{RSL_STAGED, 16384, 1, 4, 1, 0}, TuneConfig{RSL_BATCHED, 4096, 2, 1, 0, 0},
      TuneConfig{RSL_STAGED, 4096, 1, 1, 0, 1}, TuneConfig{RSL_STAGED, 4096, 1, 1, 1, 0, 1},
  };
  const int C = static_cast<int>(sizeof(cfgs) / sizeof(cfgs[0]));
  std::vector<size_t> totals(static_cast<size_t>(T) * C, 0);
  {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        for (int c = 0; c < C; ++c) {
          const int lo = (t * 5) % (N / 2), hi = lo + N / 2;
          layout_and_decode(probs, lo, hi, cfgs[c], 99 + t * 31 + c, &totals[static_cast<size_t>(t) * C + c]);
        }
      });
    for (auto& x : th) x.join();
  }
  // the same batch under the same schedule lays out to the same size on every thread
  for (int t = 0; t < T; ++t)
    for (int u = 0; u < T; ++u)
      if ((t * 5) % (N / 2) == (u * 5) % (N / 2))
        for (int c = 0; c < C; ++c)
          check(totals[static_cast<size_t>(t) * C + c] == totals[static_cast<size_t>(u) * C + c],
                "deterministic layout", t, u);

  // 3. device entry points without a device: errors, not crashes
  rsl_ctx* ctx = nullptr;
  const int rc = rsl_ctx_create(0, nullptr, 0, nullptr, 0, nullptr, &ctx);
  check(rc == RSL_EDEVICE && ctx == nullptr, "context creation without a device", rc);
  check(rsl_ctx_create(0, nullptr, 16, nullptr, 0, nullptr, &ctx) == RSL_EINVAL, "workspace size without pointer");

  if (g_fail.load()) {
    std::fprintf(stderr, "%d checks failed\n", g_fail.load());
    return 1;
  }
  std::printf("host driver: %d threads, %d problems, %d schedules: ok\n", T, N, C);
  return 0;
}

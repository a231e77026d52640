// Host-side planning (see plan.h).
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>

namespace rsl {

namespace {

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) {
  return static_cast<uint64_t>((static_cast<unsigned __int128>(a) * b) % m);
}
uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}

std::mutex g_prime_mu;
std::vector<uint32_t> g_primes;
std::atomic<size_t> g_prime_count{0};  // entries published (written before the count)
uint32_t g_next_candidate = 1431655765u;  // floor(2^32 / 3): every prime p of the table has 3p < 2^32

constexpr size_t kPrimeTableMax = 1u << 16;

}  // namespace

// Deterministic Miller-Rabin for n < 4,759,123,141 with bases 2, 7, 61.
bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u, 11u, 13u, 17u, 19u, 23u, 29u, 31u, 37u, 41u, 43u, 47u, 53u, 59u, 61u})
    if (n % q == 0) return n == q;
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1u) == 0) { d >>= 1; ++s; }
  for (uint32_t a : {2u, 7u, 61u}) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

const uint32_t* prime_table(size_t at_least, size_t* avail) {
  at_least = std::min(at_least, kPrimeTableMax);
  // fast path (no lock): the entries below the published count are final
  const size_t have = g_prime_count.load(std::memory_order_acquire);
  if (have > 0 && have >= at_least) {
    if (avail) *avail = have;
    return g_primes.data();
  }
  std::lock_guard<std::mutex> lk(g_prime_mu);
  // the storage is reserved once, so the table never moves: a pointer taken by
  // one planning thread stays valid while another thread extends the table
  if (g_primes.capacity() < kPrimeTableMax) g_primes.reserve(kPrimeTableMax);
  while (g_primes.size() < at_least) {
    uint32_t c = g_next_candidate;
    g_next_candidate -= 2;
    if (is_prime_u32(c)) g_primes.push_back(c);
  }
  g_prime_count.store(g_primes.size(), std::memory_order_release);
  if (avail) *avail = g_primes.size();
  return g_primes.data();
}

int make_view(const rsl_poly* f, int var, View* v, std::string* err) {
  if (!f || f->dx < 0 || f->dy < 0 || f->limbs < 1 || f->limbs > 4096) {
    *err = "invalid polynomial descriptor (null, negative degree or limbs < 1)";
    return RSL_EINVAL;
  }
  const int64_t ncoef = static_cast<int64_t>(f->dx + 1) * (f->dy + 1);
  if (ncoef > (int64_t(1) << 26)) {
    *err = "polynomial too large";
    return RSL_EINVAL;
  }
  if (!f->coeff) {
    *err = "null coefficient pointer";
    return RSL_EINVAL;
  }
  const int L = f->limbs;
  // In the eliminated variable's view, "y" is the eliminated variable.
  const int Ydim = (var == RSL_Y) ? f->dy : f->dx;
  const int Xdim = (var == RSL_Y) ? f->dx : f->dy;
  auto at = [&](int j, int i) -> const uint32_t* {  // coefficient of X^i Y^j
    int yi = (var == RSL_Y) ? j : i;   // power of the original y
    int xi = (var == RSL_Y) ? i : j;   // power of the original x
    return f->coeff + (static_cast<int64_t>(yi) * (f->dx + 1) + xi) * L;
  };
  auto nonzero = [&](const uint32_t* w) {
    for (int l = 0; l < L; ++l)
      if (w[l]) return true;
    return false;
  };
  v->L = L;
  v->dy = -1;
  v->dx = -1;
  v->tdeg = -1;
  std::vector<int> rdeg(Ydim + 1, -1);
  for (int j = 0; j <= Ydim; ++j)
    for (int i = 0; i <= Xdim; ++i)
      if (nonzero(at(j, i))) {
        rdeg[j] = i;
        v->dy = j;
        v->dx = std::max(v->dx, i);
        v->tdeg = std::max(v->tdeg, i + j);
      }
  if (v->dy < 0) {
    v->rdeg.clear();
    v->c.clear();
    return RSL_OK;
  }
  rdeg.resize(v->dy + 1);
  v->rdeg = rdeg;
  const int row = v->dx + 1;
  v->c.assign(static_cast<size_t>(v->dy + 1) * row * L, 0u);
  v->row_l1.assign(v->dy + 1, BigU());
  for (int j = 0; j <= v->dy; ++j) {
    if (v->rdeg[j] < 0) continue;
    if (var == RSL_Y) {
      // rows of the original layout are contiguous: one copy per row
      std::memcpy(&v->c[static_cast<size_t>(j) * row * L], at(j, 0), sizeof(uint32_t) * (v->rdeg[j] + 1) * L);
    } else {
      for (int i = 0; i <= v->rdeg[j]; ++i)
        std::memcpy(&v->c[(static_cast<size_t>(j) * row + i) * L], at(j, i), sizeof(uint32_t) * L);
    }
    // ||f_j||_1: at most 2^26 coefficients of at most 64 bits fit 128 bits
    if (L <= 2) {
      unsigned __int128 acc = 0;
      const uint32_t* r = &v->c[static_cast<size_t>(j) * row * L];
      for (int i = 0; i <= v->rdeg[j]; ++i) {
        const uint32_t* w = r + static_cast<size_t>(i) * L;
        if (L == 1) {
          const int64_t x = static_cast<int32_t>(w[0]);
          acc += static_cast<uint64_t>(x < 0 ? -x : x);
        } else {
          const uint64_t u = static_cast<uint64_t>(w[0]) | (static_cast<uint64_t>(w[1]) << 32);
          acc += (u >> 63) ? (~u + 1) : u;  // |INT64_MIN| = 2^63 as unsigned
        }
      }
      BigU t;
      for (int q = 0; q < 4 && acc; ++q) {
        t.d.push_back(static_cast<uint32_t>(acc));
        acc >>= 32;
      }
      v->row_l1[j] = t;
    } else {
      BigU t;
      for (int i = 0; i <= v->rdeg[j]; ++i)
        t = BigU::add(t, abs_limbs(&v->c[(static_cast<size_t>(j) * row + i) * L], L, nullptr));
      v->row_l1[j] = t;
    }
  }
  v->lc_abs.assign(v->rdeg[v->dy] + 1, BigU());
  v->lc_neg.assign(v->rdeg[v->dy] + 1, 0);
  for (int i = 0; i <= v->rdeg[v->dy]; ++i) {
    bool neg = false;
    v->lc_abs[i] = abs_limbs(&v->c[(static_cast<size_t>(v->dy) * row + i) * L], L, &neg);
    v->lc_neg[i] = neg;
  }
  return RSL_OK;
}

// The leading coefficient (a polynomial in the other variable) of V at x0,
// modulo q = 2^31 - 1: zero when x0 is a root over Z (and, rarely, when q
// divides the value).
static bool lc_zero_mod_q(const View& V, uint32_t x0) {
  const uint64_t q = 2147483647u;
  uint64_t acc = 0;
  for (size_t i = V.lc_abs.size(); i-- > 0;) {
    const uint64_t a = V.lc_abs[i].mod_small(static_cast<uint32_t>(q));
    acc = (acc * (x0 % q) + (V.lc_neg[i] ? (q - a) % q : a)) % q;
  }
  return acc == 0;
}

void crt_tables(const std::vector<uint32_t>& primes, int LP, std::vector<uint32_t>* Tg,
                std::vector<uint32_t>* invM, std::vector<uint32_t>* Plimb) {
  const int np = static_cast<int>(primes.size());
  Tg->assign(static_cast<size_t>(np) * np, 0u);
  invM->assign(np, 0u);
  Plimb->assign(static_cast<size_t>(np) * LP, 0u);
  std::vector<uint64_t> run(np, 1);  // prod_{l<j} p_l mod p_i
  BigU P(1);
  for (int j = 0; j < np; ++j) {
    const uint32_t pj = primes[j];
    for (int i = 0; i < np; ++i) {
      if (i > j) (*Tg)[static_cast<size_t>(j) * np + i] =
          static_cast<uint32_t>(((run[i] % primes[i]) << 32) % primes[i]);  // Montgomery form
    }
    // invM[j] = (prod_{l<j} p_l)^{-1} mod p_j in Montgomery form
    uint64_t inv = powmod64(run[j] % pj, pj - 2, pj);
    (*invM)[j] = static_cast<uint32_t>((inv << 32) % pj);
    std::vector<uint32_t> lim = P.limbs(LP);
    std::copy(lim.begin(), lim.end(), Plimb->begin() + static_cast<size_t>(j) * LP);
    for (int i = 0; i < np; ++i) run[i] = (run[i] * (pj % primes[i])) % primes[i];
    P = BigU::mul_small(P, pj);
  }
}

void direct_crt_tables(const std::vector<uint32_t>& primes, const BigU& M, int L, std::vector<uint32_t>* Mi,
                       std::vector<uint32_t>* wdir, std::vector<uint32_t>* rinv, std::vector<uint32_t>* negM) {
  const int np = static_cast<int>(primes.size());
  Mi->assign(static_cast<size_t>(np) * L, 0u);
  wdir->assign(np, 0u);
  rinv->assign(2 * static_cast<size_t>(np), 0u);
  for (int i = 0; i < np; ++i) {
    const uint32_t p = primes[i];
    const BigU mi = M.div_small(p);
    const std::vector<uint32_t> lim = mi.limbs(L);
    std::copy(lim.begin(), lim.end(), Mi->begin() + static_cast<size_t>(i) * L);
    const uint64_t inv = powmod64(mi.mod_small(p), p - 2, p);
    (*wdir)[i] = static_cast<uint32_t>((inv << 32) % p);  // Montgomery form
    const uint64_t r = ~static_cast<uint64_t>(0) / p;      // floor(2^64 / p), p odd
    (*rinv)[2 * i] = static_cast<uint32_t>(r);
    (*rinv)[2 * i + 1] = static_cast<uint32_t>(r >> 32);
  }
  *negM = M.neg_limbs(L);
}

namespace {

std::shared_ptr<const CrtConst> build_crt_const(const std::vector<uint32_t>& primes, bool canonical) {
  auto C = std::make_shared<CrtConst>();
  C->np = static_cast<int>(primes.size());
  BigU M(1);
  for (uint32_t p : primes) M = BigU::mul_small(M, p);
  C->L_out = std::max(1, (M.bitlen() + 31) / 32);
  BigU H = M.half();  // (M - 1) / 2, M odd
  C->Hm.resize(C->np);
  for (int i = 0; i < C->np; ++i) C->Hm[i] = H.mod_small(primes[i]);
  C->NH = H.neg_limbs(C->L_out);
  // beyond the per-lane slots the CRT takes the wide path: Y0 = sum_i t_i M_i - q M
  // with q possibly one short, so Y0 < 2M needs one limb more than M
  C->wide = C->np > kSlotCrtPrimes;
  C->Lw = C->wide ? C->L_out + 1 : C->L_out;
  if (!canonical && !C->wide) crt_tables(primes, C->L_out, &C->Tg, &C->invM, &C->Plimb);
  direct_crt_tables(primes, M, C->Lw, &C->Mi, &C->wdir, &C->rinv, &C->negM);
  if (C->wide) {
    C->Mw = M.limbs(C->Lw);
    C->NHM = BigU::add(H, M).neg_limbs(C->L_out);
  }
  return C;
}

// canonical lists by prime count; dropped whole when it holds more than kCrtCacheBytes
std::mutex g_crt_mu;
std::map<int, std::shared_ptr<const CrtConst>> g_crt;
size_t g_crt_bytes = 0;
constexpr size_t kCrtCacheBytes = size_t(512) << 20;

size_t crt_bytes(const CrtConst& C) {
  return 4 * (C.Hm.size() + C.NH.size() + C.Tg.size() + C.invM.size() + C.Plimb.size() + C.Mi.size() +
              C.wdir.size() + C.rinv.size() + C.negM.size() + C.Mw.size() + C.NHM.size());
}

}  // namespace

void plan_crt(Plan* P) {
  const uint32_t* tab = prime_table(0);
  P->np = static_cast<int>(P->pidx.size());
  P->canonical = true;
  for (int i = 0; i < P->np; ++i)
    if (P->pidx[i] != i) P->canonical = false;
  std::shared_ptr<const CrtConst> C;
  if (P->canonical) {
    std::lock_guard<std::mutex> lk(g_crt_mu);
    auto it = g_crt.find(P->np);
    if (it != g_crt.end()) C = it->second;
  }
  if (!C) {
    std::vector<uint32_t> primes(P->np);
    for (int i = 0; i < P->np; ++i) primes[i] = tab[P->pidx[i]];
    C = build_crt_const(primes, P->canonical);
    if (P->canonical) {
      std::lock_guard<std::mutex> lk(g_crt_mu);
      const size_t b = crt_bytes(*C);
      if (g_crt_bytes + b > kCrtCacheBytes) {
        g_crt.clear();
        g_crt_bytes = 0;
      }
      // a planner on another thread may have built the same list meanwhile:
      // every plan takes the cached object, so that jobs share one block
      auto ins = g_crt.emplace(P->np, C);
      if (ins.second) g_crt_bytes += b;
      else C = ins.first->second;
    }
  }
  P->crt = C;
  P->L_out = C->L_out;
  P->wide = C->wide;
  P->Lw = C->Lw;
}

namespace {

// Degrees and per-row L1 norms (double) of one input in the eliminated variable's view.
struct RowScan {
  int dy = -1, dx = -1, tdeg = -1, lcdeg = -1, L = 1;
  int64_t nterms = 0;
  double sq = 0.0;  // sum_j ||f_j||_1^2, scaled by 2^-(2 * shift)
  int shift = 0;    // values are scaled by 2^-shift so that no sum overflows a double
  bool ok = false;
  double log2_sq() const { return std::log2(std::max(sq, 1e-300)) + 2.0 * shift; }
};

RowScan scan_rows(const rsl_poly* f, int var) {
  RowScan r;
  if (!f || f->dx < 0 || f->dy < 0 || f->limbs < 1 || !f->coeff) return r;
  r.ok = true;
  const int L = f->limbs;
  r.L = L;
  const int Ydim = (var == RSL_Y) ? f->dy : f->dx;
  const int Xdim = (var == RSL_Y) ? f->dx : f->dy;
  // a value is at most 2^(32 L); scaled by 2^-shift it stays below 2^96, a row
  // sum below 2^123 and the sum of squares far from the double range's end
  r.shift = 32 * std::max(0, L - 3);
  const double one = std::ldexp(1.0, -r.shift);
  for (int j = 0; j <= Ydim; ++j) {
    double l1 = 0.0;
    int rd = -1;
    for (int i = 0; i <= Xdim; ++i) {
      const int yi = (var == RSL_Y) ? j : i, xi = (var == RSL_Y) ? i : j;
      const uint32_t* w = f->coeff + (static_cast<int64_t>(yi) * (f->dx + 1) + xi) * L;
      bool nz = false;
      for (int l = 0; l < L; ++l) nz |= w[l] != 0u;
      if (!nz) continue;
      rd = i;
      // |value| from its top three limbs (two's complement), scaled
      const bool neg = (w[L - 1] >> 31) != 0;
      double v = 0.0;
      for (int l = L - 1; l >= 0 && l >= L - 3; --l) {
        const uint32_t x = neg ? ~w[l] : w[l];
        v += std::ldexp(static_cast<double>(x), 32 * l - r.shift);
      }
      l1 += v + one;
    }
    if (rd >= 0) {
      r.dy = j;
      r.dx = std::max(r.dx, rd);
      r.tdeg = std::max(r.tdeg, rd + j);
      r.lcdeg = rd;
      r.nterms += rd + 1;
      r.sq += l1 * l1;
    }
  }
  return r;
}

}  // namespace

ShapeEst estimate_shape(const rsl_poly* f, const rsl_poly* g, int var) {
  ShapeEst e;
  const RowScan a = scan_rows(f, var), b = scan_rows(g, var);
  if (!a.ok || !b.ok || (var != RSL_Y && var != RSL_X)) {
    e.bad = true;
    return e;
  }
  e.L = std::max(a.L, b.L);
  if (a.dy < 0 || b.dy < 0) return e;
  e.zero = false;
  e.my = a.dy;
  e.ny = b.dy;
  const int64_t d1 = static_cast<int64_t>(b.dy) * a.dx + static_cast<int64_t>(a.dy) * b.dx;
  const int64_t d2 = static_cast<int64_t>(b.dy) * a.tdeg + static_cast<int64_t>(a.dy) * b.tdeg -
                     static_cast<int64_t>(a.dy) * b.dy;
  e.D = static_cast<int>(std::min<int64_t>(std::min(d1, d2), 1 << 20));
  e.E = e.D + a.lcdeg + b.lcdeg;
  const double lb2 = b.dy * std::max(a.log2_sq(), 0.0) + a.dy * std::max(b.log2_sq(), 0.0);
  e.np_est = static_cast<int>(std::ceil((lb2 / 2.0 + 1.0) / 30.99)) + 1;
  e.cost = (static_cast<double>(a.nterms + b.nterms) + static_cast<double>(a.dy) * b.dy) * e.np_est * (e.E + 1) +
           static_cast<double>(e.np_est) * (e.D + 1) * (e.D + 1);
  return e;
}

namespace {

// A fixed set of worker threads, shared by every parallel_for of the process
// (the batch pipeline runs several at once: planning on its producer thread,
// binding and decoding on the caller's).  The calling thread works on its own
// task too, so a task finishes even when every worker is busy elsewhere.
class HostPool {
 public:
  struct Task {
    const std::function<void(int)>* fn = nullptr;
    int n = 0, grain = 1;
    std::atomic<int> next{0};
    std::atomic<int> left{0};
    std::mutex m;
    std::condition_variable done;
  };

  explicit HostPool(int workers) {
    for (int t = 0; t < workers; ++t) th_.emplace_back([this] { loop(); });
  }

  void run(const std::function<void(int)>& fn, int n, int grain) {
    auto t = std::make_shared<Task>();
    t->fn = &fn;
    t->n = n;
    t->grain = grain;
    t->left.store(n);
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(t);
    }
    cv_.notify_all();
    work(*t);
    std::unique_lock<std::mutex> lk(t->m);
    t->done.wait(lk, [&] { return t->left.load() == 0; });
  }

 private:
  void work(Task& t) {
    for (;;) {
      const int b = t.next.fetch_add(t.grain);
      if (b >= t.n) break;
      const int e = std::min(t.n, b + t.grain);
      for (int i = b; i < e; ++i) (*t.fn)(i);
      if (t.left.fetch_sub(e - b) == e - b) {
        std::lock_guard<std::mutex> lk(t.m);
        t.done.notify_all();
      }
    }
  }
  void loop() {
    for (;;) {
      std::shared_ptr<Task> t;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return !q_.empty(); });
        t = q_.front();
        if (t->next.load() >= t->n) {  // exhausted: take it off the queue
          q_.pop_front();
          continue;
        }
      }
      work(*t);
    }
  }

  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::shared_ptr<Task>> q_;
  std::vector<std::thread> th_;
};

int host_threads() {
  static const int t = [] {
    int hw = static_cast<int>(std::thread::hardware_concurrency());
    if (hw <= 0) hw = 1;
    int v = std::min(hw, 16);
    if (const char* env = std::getenv("RSL_HOST_THREADS")) v = std::max(1, std::min(64, std::atoi(env)));
    return v;
  }();
  return t;
}

}  // namespace

void parallel_for(int n, int grain, const std::function<void(int)>& fn, int threads) {
  if (n <= 0) return;
  grain = std::max(1, grain);
  const int T = threads > 0 ? threads : host_threads();
  if (T <= 1 || n <= grain) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  // the workers live for the rest of the process (never destroyed: no
  // ordering problem with other static objects at exit)
  static HostPool* pool = new HostPool(host_threads() - 1);
  pool->run(fn, n, grain);
}

int make_plan(const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts, Plan* P,
              std::string* err) {
  if (var != RSL_Y && var != RSL_X) {
    *err = "var must be RSL_Y or RSL_X";
    return RSL_EINVAL;
  }
  rsl_opts o{};
  if (opts) o = *opts;
  if (o.points != RSL_POINTS_REPLACE && o.points != RSL_POINTS_FORMAL) {
    *err = "opts.points must be RSL_POINTS_REPLACE or RSL_POINTS_FORMAL";
    return RSL_EINVAL;
  }
  if (o.prime_start < 0 || o.extra_primes < 0 || o.extra_points < 0 || o.point_origin < -1 ||
      o.point_origin > (1 << 24) || o.prime_limit < 0) {
    *err = "invalid options";
    return RSL_EINVAL;
  }
  int rc = make_view(f, var, &P->f, err);
  if (rc) return rc;
  rc = make_view(g, var, &P->g, err);
  if (rc) return rc;
  P->zero = (P->f.dy < 0 || P->g.dy < 0);
  P->formal = o.points;
  P->origin = o.point_origin > 0 ? o.point_origin : 0;
  if (P->zero) return RSL_OK;

  const View &F = P->f, &G = P->g;
  const int my = F.dy, ny = G.dy, mx = F.dx, nx = G.dx, m = F.tdeg, n = G.tdeg;
  P->my = my;
  P->ny = ny;
  int64_t d1 = static_cast<int64_t>(ny) * mx + static_cast<int64_t>(my) * nx;
  int64_t d2 = static_cast<int64_t>(ny) * m + static_cast<int64_t>(my) * n - static_cast<int64_t>(my) * ny;
  int64_t D = std::min(d1, d2);
  if (D > (1 << 20)) {
    *err = "degree bound too large";
    return RSL_EINVAL;
  }
  P->D = static_cast<int>(D);
  P->s = F.rdeg[my] + G.rdeg[ny];
  P->E = P->D + P->s + o.extra_points;
  // Automatic origin (option 0): a leading coefficient that vanishes at x = 0
  // over Z makes point 0 bad for every prime, and every prime would take the
  // gapped interpolation; start instead at the first x0 in 1 .. kAutoOriginMax
  // where neither leading coefficient vanishes (the consecutive path then
  // interpolates in x - x0 and shifts back).
  constexpr uint32_t kAutoOriginMax = 16;
  if (o.point_origin == 0 && !P->formal && P->s > 0 && (lc_zero_mod_q(F, 0) || lc_zero_mod_q(G, 0)))
    for (uint32_t x0 = 1; x0 <= kAutoOriginMax; ++x0)
      if (!lc_zero_mod_q(F, x0) && !lc_zero_mod_q(G, x0)) {
        P->origin = static_cast<int>(x0);
        break;
      }

  // Hadamard bound: B^2 = (sum_j ||f_j||_1^2)^{n_y} (sum_j ||g_j||_1^2)^{m_y}.
  // Primes are taken until M^2 > 4 B^2 (M their product).  The comparison runs
  // on log2 values in double precision (relative error far below 1e-12) and
  // falls back to exact big integers only when the two sides are within a
  // safety margin of each other, so the prime count is the exact minimum.
  auto row_sq_sum = [](const View& V) {
    BigU S;
    for (int j = 0; j <= V.dy; ++j) S = BigU::add(S, BigU::mul(V.row_l1[j], V.row_l1[j]));
    return S;
  };
  const BigU Sf = row_sq_sum(F), Sg = row_sq_sum(G);
  auto log2_of = [](const BigU& a) {
    if (a.is_zero()) return 0.0;
    const int nb = a.bitlen();
    const int sh = std::max(0, nb - 64);
    const BigU t = a.shr(sh);
    uint64_t v = 0;
    for (size_t i = 0; i < t.d.size() && i < 2; ++i) v |= static_cast<uint64_t>(t.d[i]) << (32 * i);
    return std::log2(static_cast<double>(v)) + sh;
  };
  const double lb2 = ny * log2_of(Sf) + my * log2_of(Sg);  // log2(B^2)
  const double slack = 1e-3 + 1e-9 * lb2;
  BigU fourB2;  // exact 4 B^2, made on first need
  bool have_exact = false;
  auto exact_4b2 = [&]() -> const BigU& {
    if (!have_exact) {
      fourB2 = BigU::mul_small(BigU::mul(BigU::pow(Sf, ny), BigU::pow(Sg, my)), 4);
      have_exact = true;
    }
    return fourB2;
  };
  P->bound_bits = static_cast<int>((std::floor(lb2) + 2.0) / 2.0);

  // primes: largest first, skipping bad primes (p | every coefficient of lc_y f or lc_y g)
  auto lc_vanishes = [](const View& V, uint32_t p) {
    for (const BigU& a : V.lc_abs)
      if (a.mod_small(p) != 0) return false;
    return true;
  };
  const size_t limit = o.prime_limit ? static_cast<size_t>(o.prime_limit) : kPrimeTableMax;
  double lm = 0.0;  // log2(M)
  P->pidx.clear();
  P->bad_primes = 0;
  int extra_left = o.extra_primes;
  bool enough = false;
  for (size_t k = static_cast<size_t>(o.prime_start);; ++k) {
    if (k >= limit) {
      *err = "prime table exhausted";
      return RSL_EPRIMES;
    }
    size_t have = 0;
    const uint32_t* tab = prime_table(k + 1, &have);
    if (k >= have) {
      *err = "prime table exhausted";
      return RSL_EPRIMES;
    }
    uint32_t p = tab[k];
    if (lc_vanishes(F, p) || lc_vanishes(G, p)) {
      ++P->bad_primes;
      continue;
    }
    P->pidx.push_back(static_cast<int>(k));
    lm += std::log2(static_cast<double>(p));
    if (!enough) {
      const double d = 2.0 * lm - (lb2 + 2.0);  // log2(M^2) - log2(4 B^2)
      if (d > slack) {
        enough = true;
      } else if (d >= -slack) {
        BigU M(1);
        for (int i : P->pidx) M = BigU::mul_small(M, tab[i]);
        enough = BigU::cmp(BigU::mul(M, M), exact_4b2()) > 0;
      }
    }
    if (enough) {
      if (extra_left == 0) break;
      --extra_left;
    }
  }
  plan_crt(P);

  // residue tile layout
  P->rowf = F.dx + 1;
  P->rowg = G.dx + 1;
  P->goff = (my + 1) * P->rowf;
  P->CS = (P->goff + (ny + 1) * P->rowg + 3) & ~3;
  return RSL_OK;
}

}  // namespace rsl

// Host build of the kernels' per-lane arithmetic, for CPU tests of its logic
// against the oracle (test infrastructure only; not part of the library).
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>
#include "../../paper_1010_1386_amd/csrc/modarith.h"
#include "../../paper_1010_1386_amd/csrc/ures.h"
#include "../../paper_1010_1386_amd/csrc/ures_regs.h"

using namespace rsl;

namespace {

// Reusable barrier for the K lane threads of the group simulation.
struct Barrier {
  std::mutex mu;
  std::condition_variable cv;
  int n, waiting = 0, gen = 0;
  explicit Barrier(int k) : n(k) {}
  void wait() {
    std::unique_lock<std::mutex> lk(mu);
    const int g = gen;
    if (++waiting == n) {
      waiting = 0;
      ++gen;
      cv.notify_all();
    } else {
      cv.wait(lk, [&] { return gen != g; });
    }
  }
};

template <int NMAX>
int regs_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad) {
  constexpr int N = RegPoly<NMAX>::kN;
  uint32_t X[N] = {}, Y[N] = {};
  if (m > NMAX + 3 || n > NMAX + 3) return -1;
  for (int j = 0; j <= m && j < N; ++j) X[j] = mmul(A[j] % pc.p, pc.r2, pc.p, pc.pinv);
  for (int j = 0; j <= n && j < N; ++j) Y[j] = mmul(B[j] % pc.p, pc.r2, pc.p, pc.pinv);
  std::vector<uint32_t> ca(N + 64, 0), cb(N + 64, 0);
  bool bd = false;
  const uint32_t r = ures_regs<NMAX>(X, Y, m, n, pc, &bd, Column<1>{ca.data()}, Column<1>{cb.data()});
  *out = redc(r, pc.p, pc.pinv);
  *bad = bd;
  return 0;
}

// Two lane threads of the pair form: the swap is an exchange through two
// slots between barriers, as the lanes of a pair exchange registers.
template <int NMAX>
int regs2_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
              int* agree);

template <int K>
uint32_t group_run(const PrimeConst& pc, int m, int n, std::vector<uint32_t>& a, std::vector<uint32_t>& b,
                   bool* bad, int* agree) {
  Barrier bar(K);
  uint32_t r[K];
  bool bd[K];
  std::vector<std::thread> th;
  for (int l = 0; l < K; ++l)
    th.emplace_back([&, l] {
      r[l] = ures_group<K>(Column<1>{a.data()}, Column<1>{b.data()}, m, n, pc, l, &bd[l], [&] { bar.wait(); });
    });
  for (auto& t : th) t.join();
  *agree = 1;
  for (int l = 1; l < K; ++l)
    if (r[l] != r[0] || bd[l] != bd[0]) *agree = 0;
  *bad = bd[0];
  return r[0];
}

template <int NMAX>
int regs2_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
              int* agree) {
  constexpr int N2 = RegPoly2<NMAX>::kN;
  Barrier bar(2);
  uint32_t slot[2] = {0, 0};
  std::vector<uint32_t> ca(2 * N2 + 64, 0), cb(2 * N2 + 64, 0);
  uint32_t r[2];
  bool bd[2];
  std::vector<std::thread> th;
  for (int l = 0; l < 2; ++l)
    th.emplace_back([&, l] {
      uint32_t X[N2] = {}, Y[N2] = {};
      for (int k = 0; k < N2; ++k) {
        const int j = 2 * k + l;
        if (j <= m) X[k] = mmul(A[j] % pc.p, pc.r2, pc.p, pc.pinv);
        if (j <= n) Y[k] = mmul(B[j] % pc.p, pc.r2, pc.p, pc.pinv);
      }
      auto swp = [&](uint32_t v) {
        slot[l] = v;
        bar.wait();
        const uint32_t o = slot[1 - l];
        bar.wait();
        return o;
      };
      r[l] = ures_regs2<NMAX>(X, Y, m, n, l, pc, &bd[l], Column<1>{ca.data()}, Column<1>{cb.data()}, swp,
                              [&] { bar.wait(); });
    });
  for (auto& t : th) t.join();
  *agree = (r[0] == r[1] && bd[0] == bd[1]) ? 1 : 0;
  *out = redc(r[0], pc.p, pc.pinv);
  *bad = bd[0];
  return 0;
}

// The matrix-core stage's lane-pair path: the branch-free generic chain, and
// on its failure the column code from the original values.
template <int NMAX>
int regs2_gen_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
                  int* agree, int* generic) {
  constexpr int N2 = RegPoly2<NMAX>::kN;
  Barrier bar(2);
  uint32_t slot[2] = {0, 0};
  std::vector<uint32_t> ca(2 * N2 + 64, 0), cb(2 * N2 + 64, 0);
  uint32_t r[2];
  bool bd[2], okv[2];
  std::vector<std::thread> th;
  for (int l = 0; l < 2; ++l)
    th.emplace_back([&, l] {
      uint32_t X[N2] = {}, Y[N2] = {};
      auto load = [&] {
        for (int k = 0; k < N2; ++k) {
          const int j = 2 * k + l;
          X[k] = (j <= m) ? mmul(A[j] % pc.p, pc.r2, pc.p, pc.pinv) : 0u;
          Y[k] = (j <= n) ? mmul(B[j] % pc.p, pc.r2, pc.p, pc.pinv) : 0u;
        }
      };
      auto swp = [&](uint32_t v) {
        slot[l] = v;
        bar.wait();
        const uint32_t o = slot[1 - l];
        bar.wait();
        return o;
      };
      load();
      r[l] = ures_regs2_generic<NMAX>(X, Y, m, n, l, pc, &okv[l], &bd[l], swp);
      if (!okv[l]) {
        load();
        r[l] = ures2_columns<NMAX>(X, Y, m, n, l, pc, Column<1>{ca.data()}, Column<1>{cb.data()}, swp,
                                   [&] { bar.wait(); });
      }
    });
  for (auto& t : th) t.join();
  *agree = (r[0] == r[1] && bd[0] == bd[1] && okv[0] == okv[1]) ? 1 : 0;
  *out = redc(r[0], pc.p, pc.pinv);
  *bad = bd[0];
  *generic = okv[0];
  return 0;
}

// The one-lane branch-free chain, and on its failure ures_formal on columns
// from the original values (the matrix-core stage's one-lane path).
template <int NMAX>
int regs_gen_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
                 int* generic) {
  constexpr int N = RegPoly<NMAX>::kN;
  uint32_t X[N] = {}, Y[N] = {};
  auto load = [&] {
    for (int j = 0; j < N; ++j) {
      X[j] = (j <= m) ? mmul(A[j] % pc.p, pc.r2, pc.p, pc.pinv) : 0u;
      Y[j] = (j <= n) ? mmul(B[j] % pc.p, pc.r2, pc.p, pc.pinv) : 0u;
    }
  };
  load();
  bool ok = false, bd = false;
  uint32_t r = ures_regs_generic<NMAX>(X, Y, m, n, pc, &ok, &bd);
  if (!ok) {
    load();
    std::vector<uint32_t> ca(NMAX + 1, 0), cb(NMAX + 1, 0);
    for (int j = 0; j <= NMAX; ++j) {
      ca[j] = j < N ? X[j] : 0u;
      cb[j] = j < N ? Y[j] : 0u;
    }
    bool b2 = false;
    r = ures_formal(Column<1>{ca.data()}, Column<1>{cb.data()}, m, n, pc, &b2);
  }
  *out = redc(r, pc.p, pc.pinv);
  *bad = bd;
  *generic = ok;
  return 0;
}

// The general-shape one-lane path: the first division on rows, then the
// branch-free chain in registers (or the general code from the state reached).
template <int NMAX>
int regs_long_run(const PrimeConst& pc, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad) {
  std::vector<uint32_t> ra(NMAX + 2, 0), rb(NMAX + 2, 0);
  for (int j = 0; j <= m; ++j) ra[j] = mmul(A[j] % pc.p, pc.r2, pc.p, pc.pinv);
  for (int j = 0; j <= n; ++j) rb[j] = mmul(B[j] % pc.p, pc.r2, pc.p, pc.pinv);
  bool bd = false;
  const uint32_t r = ures_regs_long<NMAX>(Column<1>{ra.data()}, Column<1>{rb.data()}, m, n, pc, &bd);
  *out = redc(r, pc.p, pc.pinv);
  *bad = bd;
  return 0;
}

}  // namespace

extern "C" {

// The general-shape one-lane register form (any m, n <= nmax).
int hs_ures_regs_long(int nmax, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out,
                      int* bad) {
  PrimeConst pc = make_prime_const(p);
  if (m > nmax || n > nmax || m < 0 || n < 0) return -1;
  switch (nmax) {
    case 8: return regs_long_run<8>(pc, m, n, A, B, out, bad);
    case 16: return regs_long_run<16>(pc, m, n, A, B, out, bad);
    case 24: return regs_long_run<24>(pc, m, n, A, B, out, bad);
    case 32: return regs_long_run<32>(pc, m, n, A, B, out, bad);
    default: return -1;
  }
}

// The one-lane branch-free chain with its column restart.
int hs_ures_regs_gen(int nmax, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out,
                     int* bad, int* generic) {
  PrimeConst pc = make_prime_const(p);
  if (m > nmax || n > nmax) return -1;
  switch (nmax) {
    case 8: return regs_gen_run<8>(pc, m, n, A, B, out, bad, generic);
    case 16: return regs_gen_run<16>(pc, m, n, A, B, out, bad, generic);
    case 24: return regs_gen_run<24>(pc, m, n, A, B, out, bad, generic);
    case 32: return regs_gen_run<32>(pc, m, n, A, B, out, bad, generic);
    default: return -1;
  }
}

// The branch-free generic chain of a lane pair with its column restart.
int hs_ures_regs2_gen(int nmax, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out,
                      int* bad, int* agree, int* generic) {
  PrimeConst pc = make_prime_const(p);
  if (m > nmax || n > nmax) return -1;
  switch (nmax) {
    case 8: return regs2_gen_run<8>(pc, m, n, A, B, out, bad, agree, generic);
    case 16: return regs2_gen_run<16>(pc, m, n, A, B, out, bad, agree, generic);
    case 24: return regs2_gen_run<24>(pc, m, n, A, B, out, bad, agree, generic);
    case 32: return regs2_gen_run<32>(pc, m, n, A, B, out, bad, agree, generic);
    default: return -1;
  }
}

// The two-lanes-per-pair register form, run by two host threads.
int hs_ures_regs2(int nmax, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
                  int* agree) {
  PrimeConst pc = make_prime_const(p);
  if (m > nmax || n > nmax) return -1;
  switch (nmax) {
    case 8: return regs2_run<8>(pc, m, n, A, B, out, bad, agree);
    case 16: return regs2_run<16>(pc, m, n, A, B, out, bad, agree);
    case 24: return regs2_run<24>(pc, m, n, A, B, out, bad, agree);
    case 32: return regs2_run<32>(pc, m, n, A, B, out, bad, agree);
    default: return -1;
  }
}

// The register form (ures_regs<NMAX>) of the same resultant; m, n <= NMAX.
int hs_ures_regs(int nmax, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out,
                 int* bad) {
  PrimeConst pc = make_prime_const(p);
  if (m > nmax || n > nmax) return -1;
  switch (nmax) {
    case 8: return regs_run<8>(pc, m, n, A, B, out, bad);
    case 16: return regs_run<16>(pc, m, n, A, B, out, bad);
    case 24: return regs_run<24>(pc, m, n, A, B, out, bad);
    case 32: return regs_run<32>(pc, m, n, A, B, out, bad);
    default: return -1;
  }
}

// The K-lane group form of the same resultant, run by K host threads that
// meet at a barrier wherever the kernel's lanes synchronise.  *agree is 0 if
// the lanes finished with different results.
int hs_ures_group(int K, uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad,
                  int* agree) {
  PrimeConst pc = make_prime_const(p);
  int nm = (m > n ? m : n) + 1;
  std::vector<uint32_t> a(nm, 0), b(nm, 0);
  for (int j = 0; j <= m; ++j) a[j] = mmul(A[j] % p, pc.r2, p, pc.pinv);
  for (int j = 0; j <= n; ++j) b[j] = mmul(B[j] % p, pc.r2, p, pc.pinv);
  bool bd = false;
  uint32_t r;
  switch (K) {
    case 2: r = group_run<2>(pc, m, n, a, b, &bd, agree); break;
    case 4: r = group_run<4>(pc, m, n, a, b, &bd, agree); break;
    case 8: r = group_run<8>(pc, m, n, a, b, &bd, agree); break;
    default: return -1;
  }
  *out = redc(r, p, pc.pinv);
  *bad = bd;
  return 0;
}


// Resultant over Z_p with formal degrees (m, n) of A (m+1 coefficients) and B
// (n+1 coefficients), given and returned in normal form.
int hs_ures(uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad) {
  PrimeConst pc = make_prime_const(p);
  int nm = (m > n ? m : n) + 1;
  std::vector<uint32_t> a(nm, 0), b(nm, 0);
  for (int j = 0; j <= m; ++j) a[j] = mmul(A[j] % p, pc.r2, p, pc.pinv);
  for (int j = 0; j <= n; ++j) b[j] = mmul(B[j] % p, pc.r2, p, pc.pinv);
  bool bd = false;
  uint32_t r = ures_formal(Column<1>{a.data()}, Column<1>{b.data()}, m, n, pc, &bd);
  *out = redc(r, p, pc.pinv);
  *bad = bd;
  return 0;
}

// Horner evaluation of rows of coefficients (normal form) at x, result normal form.
int hs_eval(uint32_t p, int nrows, int rowstride, const uint32_t* coeff, const int* rdeg, uint32_t x,
            uint32_t* out) {
  PrimeConst pc = make_prime_const(p);
  std::vector<uint32_t> c(static_cast<size_t>(nrows) * rowstride);
  for (size_t i = 0; i < c.size(); ++i) c[i] = mmul(coeff[i] % p, pc.r3, p, pc.pinv);
  uint32_t xt = mmul(x % p, pc.r2, p, pc.pinv);
  std::vector<uint32_t> o(nrows);
  eval_rows(Column<1>{o.data()}, c.data(), nrows, rowstride, rdeg, xt, p, pc.pinv);
  for (int j = 0; j < nrows; ++j) out[j] = redc(o[j], p, pc.pinv);
  return 0;
}

}

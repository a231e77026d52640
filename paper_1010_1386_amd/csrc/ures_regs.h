// Univariate resultant over Z_p with the two polynomials in registers.
//
// The same division-free remainder sequence as ures_formal (ures.h), for the
// shapes that dominate: formal degrees m, n <= NMAX with |m - n| <= 1 and
// nonvanishing leading coefficients.  Every index is a compile-time constant:
// the generic division steps are unrolled for the degrees NMAX-1, ..., 1 of B
// (a lane enters the sequence at its own degree), the two coefficient arrays
// swap roles from one step to the next by construction, and no scratch memory
// is touched.  A lane whose remainder sequence leaves the generic pattern
// (a remainder of degree below deg B - 1), or whose leading coefficient
// vanishes at the point, finishes with the general code on two scratch
// columns, resuming from the state it reached.
#pragma once
#include "modarith.h"
#include "ures.h"

namespace rsl {

// Registers per polynomial: rows 0..NMAX rounded up to whole row groups of 4.
template <int NMAX>
struct RegPoly {
  static constexpr int kN = (NMAX / 4 + 1) * 4;
};

template <int N>
RSL_HD uint32_t reg_get(const uint32_t (&v)[N], int i) {
  uint32_t r = 0u;
#pragma unroll
  for (int j = 0; j < N; ++j) r = (j == i) ? v[j] : r;
  return r;
}

// One generic division with deg B = BS (compile time), deg A = BS + 1:
//   R[j] = L^2 A[j] - L lc(A) B[j-1] - lc(A~) B[j]   (j < BS), stored over A.
// Returns false (and leaves the step's scalars) when deg R < BS - 1.
template <int BS, int N>
RSL_HD bool reg_step(uint32_t (&A)[N], const uint32_t (&B)[N], uint32_t p, uint32_t pinv, uint32_t* L_out,
                     uint32_t* y_out) {
  const uint32_t L = B[BS], lcA = A[BS + 1], Ab = A[BS], Bb1 = B[BS - 1];
  const uint32_t lcAt = mmulsub(L, Ab, lcA, Bb1, p, pinv);
  const uint32_t alpha = mmul(L, L, p, pinv);
  const uint32_t beta = p - mmul(L, lcA, p, pinv);  // in [1, p]: mmad3 takes operands up to p
  const uint32_t gamma = p - lcAt;
#pragma unroll
  for (int j = 0; j < BS; ++j) A[j] = mmad3(alpha, A[j], beta, j > 0 ? B[j - 1] : 0u, gamma, B[j], p, pinv);
  *L_out = L;
  *y_out = alpha;
  return A[BS - 1] != 0u;
}

// Steps BS = HI, HI-1, ..., 1, entered at BS = b0: A is in X when BS is odd.
template <int BS, int N>
struct RegChain {
  RSL_HD static void run(uint32_t (&X)[N], uint32_t (&Y)[N], int b0, uint32_t p, uint32_t pinv, uint32_t& num,
                         uint32_t& den, uint32_t& U, bool& slow, int& f_bs, uint32_t& f_L, uint32_t& f_y) {
    if (BS <= b0 && !slow) {
      uint32_t L, y;
      const bool generic = (BS & 1) ? reg_step<BS>(X, Y, p, pinv, &L, &y) : reg_step<BS>(Y, X, p, pinv, &L, &y);
      if (generic) {  // k = 2, delta = 1: num L^2, U L^2, den U; the sign is unchanged
        num = mmul(num, y, p, pinv);
        U = mmul(U, y, p, pinv);
        den = mmul(den, U, p, pinv);
      } else {
        slow = true;
        f_bs = BS;
        f_L = L;
        f_y = y;
      }
    }
    RegChain<BS - 1, N>::run(X, Y, b0, p, pinv, num, den, U, slow, f_bs, f_L, f_y);
  }
};
template <int N>
struct RegChain<0, N> {
  RSL_HD static void run(uint32_t (&)[N], uint32_t (&)[N], int, uint32_t, uint32_t, uint32_t&, uint32_t&, uint32_t&,
                         bool&, int&, uint32_t&, uint32_t&) {}
};

// Res_{m,n}(A, B) with A's coefficients in X[0..m], B's in Y[0..n] (Montgomery
// form; zero above the degree).  m, n must be the same in every lane that
// takes part (they are per problem).  CA, CB: two scratch columns of at least
// NMAX + 1 entries used only by lanes that leave the register path.
template <int NMAX, class Col>
RSL_HD uint32_t ures_regs(uint32_t (&X)[RegPoly<NMAX>::kN], uint32_t (&Y)[RegPoly<NMAX>::kN], int m, int n,
                          const PrimeConst& pc, bool* bad, Col CA, Col CB) {
  constexpr int N = RegPoly<NMAX>::kN;
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  const uint32_t lcf = reg_get(X, m), lcg = reg_get(Y, n);
  *bad = (lcf == 0u) || (lcg == 0u);
  const bool shape_ok = m >= 1 && n >= 1 && m <= NMAX && n <= NMAX && (m - n <= 1) && (n - m <= 1);
  if (!shape_ok || *bad) {
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j <= NMAX) {
        CA[j] = X[j];
        CB[j] = Y[j];
      }
    bool b2 = false;
    return ures_formal(CA, CB, m, n, pc, &b2);
  }
  uint32_t neg = 0u;
  if (m < n) {  // Res(A, B) = (-1)^{mn} Res(B, A)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const uint32_t t = X[j];
      X[j] = Y[j];
      Y[j] = t;
    }
    neg = static_cast<uint32_t>(m * n) & 1u;
    const int t = m;
    m = n;
    n = t;
  }
  uint32_t num = one, den = one, U = one;
  bool slow = false;
  int f_a = 0, f_b = 0, f_k = 0;
  uint32_t f_L = 0, f_y = 0;
  bool r_in_x = false;  // where a frozen lane's remainder lies
  bool a_in_x = true;   // where A lies now
  int b0;
  if (m == n) {
    // first division, k = 1: R = L A - lc(A) B, then (A, B) <- (B, R)
    const uint32_t L = lcg, lcA = lcf;
#pragma unroll
    for (int j = 0; j < N; ++j) X[j] = (j < n) ? mmulsub(L, X[j], lcA, Y[j], p, pinv) : 0u;
    if (reg_get(X, n - 1) != 0u) {  // delta = 1: num L, U L, den U
      neg ^= static_cast<uint32_t>(n * n) & 1u;
      num = mmul(num, L, p, pinv);
      U = mmul(U, L, p, pinv);
      den = mmul(den, U, p, pinv);
    } else {
      slow = true;
      f_a = n;
      f_b = n;
      f_k = 1;
      f_L = L;
      f_y = L;
      r_in_x = true;
    }
    a_in_x = false;
    b0 = n - 1;
  } else {
    b0 = n;
  }
  if (!slow && b0 >= 1) {
    // the chain wants A in X exactly when the step's degree is odd
    if (a_in_x != ((b0 & 1) != 0)) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const uint32_t t = X[j];
        X[j] = Y[j];
        Y[j] = t;
      }
    }
    int f_bs = 0;
    RegChain<NMAX - 1, N>::run(X, Y, b0, p, pinv, num, den, U, slow, f_bs, f_L, f_y);
    if (slow) {
      f_a = f_bs + 1;
      f_b = f_bs;
      f_k = 2;
      r_in_x = (f_bs & 1) != 0;
    }
    // generic end: the last remainder (degree 0) is in X (step 1 is odd)
  } else if (!slow) {
    // b0 == 0: the remainder of the first division is the constant X[0]
  }
  if (!slow) {
    // B is the nonzero constant X[0] and deg A = 1: num B^1
    num = mmul(num, X[0], p, pinv);
    const uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
    return neg ? mneg(r, p) : r;
  }
  // leave the register path: remainder column R (degree < f_b - 1) and B
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (j <= NMAX) {
      CA[j] = r_in_x ? X[j] : Y[j];  // R
      CB[j] = r_in_x ? Y[j] : X[j];  // B
    }
  int c = f_b - 1;
  while (c >= 0 && CA[c] == 0u) --c;
  if (c < 0) return 0u;  // zero remainder with deg B >= 1
  neg ^= static_cast<uint32_t>(f_a * f_b) & 1u;
  const int delta = f_b - c;
  const int enum_ = f_k - 1 + delta;
  num = mmul(num, mpow(f_L, static_cast<uint32_t>(enum_), one, p, pinv), p, pinv);
  U = mmul(U, f_y, p, pinv);
  den = mmul(den, mpow(U, static_cast<uint32_t>(delta), one, p, pinv), p, pinv);
  // (A, B) <- (B, R)
  return ures_run(CB, CA, UresState{f_b, c, num, den, U, neg}, pc);
}

// The one-lane generic chain without per-step branches (as RegChain2Gen).
template <int BS, int N>
struct RegChainGen {
  RSL_HD static void run(uint32_t (&X)[N], uint32_t (&Y)[N], int b0, uint32_t p, uint32_t pinv, uint32_t& den,
                         uint32_t& U, bool& ok) {
    if (BS <= b0) {
      uint32_t L, y;
      const bool generic = (BS & 1) ? reg_step<BS>(X, Y, p, pinv, &L, &y) : reg_step<BS>(Y, X, p, pinv, &L, &y);
      ok = ok && generic;
      U = mmul(U, y, p, pinv);
      den = mmul(den, U, p, pinv);
    }
    RegChainGen<BS - 1, N>::run(X, Y, b0, p, pinv, den, U, ok);
  }
};
template <int N>
struct RegChainGen<0, N> {
  RSL_HD static void run(uint32_t (&)[N], uint32_t (&)[N], int, uint32_t, uint32_t, uint32_t&, uint32_t&, bool&) {}
};

// Res_{m,n}(A, B) with A in X, B in Y (one lane) along the generic pattern
// only; *ok as in ures_regs2_generic (on false the caller restarts from the
// original coefficients with ures_formal on columns).
template <int NMAX>
RSL_HD uint32_t ures_regs_generic(uint32_t (&X)[RegPoly<NMAX>::kN], uint32_t (&Y)[RegPoly<NMAX>::kN], int m, int n,
                                  const PrimeConst& pc, bool* ok, bool* bad) {
  constexpr int N = RegPoly<NMAX>::kN;
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  const uint32_t lcf = reg_get(X, m), lcg = reg_get(Y, n);
  *bad = (lcf == 0u) || (lcg == 0u);
  const bool shape_ok = m >= 1 && n >= 1 && m <= NMAX && n <= NMAX && (m - n <= 1) && (n - m <= 1);
  if (!shape_ok) {
    *ok = false;
    return 0u;
  }
  bool good = !*bad;
  uint32_t neg = 0u, den = one, U = one;
  if (m < n) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const uint32_t t = X[j];
      X[j] = Y[j];
      Y[j] = t;
    }
    neg = static_cast<uint32_t>(m * n) & 1u;
    const int t = m;
    m = n;
    n = t;
  }
  bool a_in_x = true;
  int b0 = n;
  if (m == n) {  // first division, k = 1: R = L A - lc(A) B
    const uint32_t L = reg_get(Y, n), lcA = reg_get(X, n);
#pragma unroll
    for (int j = 0; j < N; ++j) X[j] = (j < n) ? mmulsub(L, X[j], lcA, Y[j], p, pinv) : 0u;
    good = good && reg_get(X, n - 1) != 0u;
    neg ^= static_cast<uint32_t>(n * n) & 1u;
    U = L;
    den = L;
    a_in_x = false;
    b0 = n - 1;
  }
  if (b0 >= 1) {
    if (a_in_x != ((b0 & 1) != 0)) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const uint32_t t = X[j];
        X[j] = Y[j];
        Y[j] = t;
      }
    }
    RegChainGen<NMAX - 1, N>::run(X, Y, b0, p, pinv, den, U, good);
  }
  *ok = good;
  const uint32_t num = mmul(U, X[0], p, pinv);  // the last remainder (degree 0) is in X
  const uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
  return neg ? mneg(r, p) : r;
}

// Res_{m,n}(A, B) for the shapes with |m - n| >= 2 (one lane).  A and B are
// rows of scratch memory holding the coefficients (Montgomery form, formal
// degrees m, n); both are overwritten.  The first division -- k = |m - n| + 1
// elimination passes of the longer polynomial by the shorter -- runs on the
// rows, each pass touching only the n positions that meet the shifted divisor
// (a coefficient that joins that window late takes the powers of L it
// missed in one product).  If the remainder has the generic degree n - 1, the
// rest of the sequence runs in registers without branches (RegChainGen) from
// (B, R~); a lane that leaves the generic pattern there continues with the
// general code on the rows from the state after the first division (the rows
// are untouched by the register chain).  Vanishing leading coefficients and
// non-generic first remainders take the general code too.
template <int NMAX, class Col>
RSL_HD uint32_t ures_regs_long(Col A, Col B, int m, int n, const PrimeConst& pc, bool* bad) {
  constexpr int N = RegPoly<NMAX>::kN;
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  *bad = (A[m] == 0u) || (B[n] == 0u);
  if (*bad || m < 1 || n < 1) {
    bool b2 = false;
    return ures_formal(A, B, m, n, pc, &b2);
  }
  uint32_t neg = 0u;
  if (m < n) {  // Res(A, B) = (-1)^{mn} Res(B, A)
    Col t = A;
    A = B;
    B = t;
    neg = static_cast<uint32_t>(m * n) & 1u;
    const int ti = m;
    m = n;
    n = ti;
  }
  const int a = m, b = n, k = a - b + 1;
  const uint32_t L = B[b];
  // pass t (degree d = a - t, shift sh = d - b): A[j] <- L A[j] - lc B[j - sh]
  // for sh <= j < d; position sh joins now and takes L^(t+1)
  uint32_t Lt = L;
  for (int t = 0; t < k; ++t) {
    const int d = a - t, sh = d - b;
    const uint32_t lc = A[d];
    A[sh] = mmulsub(Lt, A[sh], lc, B[0], p, pinv);
    for (int j = sh + 1; j < d; ++j) A[j] = mmulsub(L, A[j], lc, B[j - sh], p, pinv);
    if (t + 1 < k) Lt = mmul(Lt, L, p, pinv);
  }
  const uint32_t y = Lt;  // L^k
  neg ^= static_cast<uint32_t>(a * b) & 1u;
  int c = b - 1;
  while (c >= 0 && A[c] == 0u) --c;
  if (c < 0) return 0u;  // zero remainder with deg B >= 1
  const int delta = b - c;
  if (delta != 1) {
    const uint32_t num = mpow(L, static_cast<uint32_t>(k - 1 + delta), one, p, pinv);
    const uint32_t den = mpow(y, static_cast<uint32_t>(delta), one, p, pinv);
    return ures_run(B, A, UresState{b, c, num, den, y, neg}, pc);
  }
  // (A, B) <- (B, R~) with scale num = U = den = L^k
  if (b == 1) {  // R~ is a nonzero constant: Res(B, R~) = R~^1
    const uint32_t r = mmul(mmul(y, A[0], p, pinv), minv(y, one, p, pinv), p, pinv);
    return neg ? mneg(r, p) : r;
  }
  uint32_t X[N], Y[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    X[j] = (j <= b) ? B[j] : 0u;
    Y[j] = (j < b) ? A[j] : 0u;
  }
  const int b0 = b - 1;
  if ((b0 & 1) == 0) {  // the chain wants its dividend in X exactly when the step's degree is odd
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const uint32_t t = X[j];
      X[j] = Y[j];
      Y[j] = t;
    }
  }
  uint32_t den = y, U = y;
  bool ok = true;
  RegChainGen<NMAX - 1, N>::run(X, Y, b0, p, pinv, den, U, ok);
  if (!ok) return ures_run(B, A, UresState{b, b0, y, y, y, neg}, pc);
  const uint32_t num = mmul(U, X[0], p, pinv);  // the last remainder (degree 0) is in X
  const uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
  return neg ? mneg(r, p) : r;
}

}  // namespace rsl

namespace rsl {

// The register form with two lanes per pair: lane l (0 or 1) keeps the
// coefficients j = 2k + l of each polynomial in its element k.  Swap(v)
// returns the partner lane's v (a lane-pair exchange on the device); every
// scalar of the remainder sequence is formed identically in both lanes.
template <int NMAX>
struct RegPoly2 {
  static constexpr int kN = RegPoly<NMAX>::kN / 2;  // elements per lane
};

// Coefficient j (compile time) as seen by both lanes.
template <int J, int N, class Swap>
RSL_HD uint32_t reg2_at(const uint32_t (&v)[N], int l, Swap swp) {
  const uint32_t mine = v[J >> 1];
  const uint32_t other = swp(mine);
  return (l == (J & 1)) ? mine : other;
}
// Coefficient j (uniform run-time index) as seen by both lanes.
template <int N, class Swap>
RSL_HD uint32_t reg2_get(const uint32_t (&v)[N], int j, int l, Swap swp) {
  const uint32_t mine = reg_get(v, j >> 1);
  const uint32_t other = swp(mine);
  return (l == (j & 1)) ? mine : other;
}

template <int BS, int N, class Swap>
RSL_HD bool reg2_step(uint32_t (&A)[N], const uint32_t (&B)[N], int l, uint32_t p, uint32_t pinv, Swap swp,
                      uint32_t* L_out, uint32_t* y_out) {
  const uint32_t L = reg2_at<BS>(B, l, swp), lcA = reg2_at<BS + 1>(A, l, swp);
  const uint32_t Ab = reg2_at<BS>(A, l, swp), Bb1 = reg2_at<BS - 1>(B, l, swp);
  const uint32_t lcAt = mmulsub(L, Ab, lcA, Bb1, p, pinv);
  const uint32_t alpha = mmul(L, L, p, pinv);
  const uint32_t beta = p - mmul(L, lcA, p, pinv);  // in [1, p]: mmad3 takes operands up to p
  const uint32_t gamma = p - lcAt;
  constexpr int KE = (BS - 1) / 2;  // last element updated (lane 1 may write R[BS], never read)
  uint32_t bsw[KE + 1];
#pragma unroll
  for (int k = 0; k <= KE; ++k) bsw[k] = swp(B[k]);
#pragma unroll
  for (int k = 0; k <= KE; ++k) {
    // B[j - 1] for j = 2k + l: lane 1 takes the partner's element k, lane 0 its element k - 1
    const uint32_t prev = l ? bsw[k] : (k > 0 ? bsw[k - 1] : 0u);
    A[k] = mmad3(alpha, A[k], beta, prev, gamma, B[k], p, pinv);
  }
  *L_out = L;
  *y_out = alpha;
  return reg2_at<BS - 1>(A, l, swp) != 0u;
}

template <int BS, int N>
struct RegChain2 {
  template <class Swap>
  RSL_HD static void run(uint32_t (&X)[N], uint32_t (&Y)[N], int l, int b0, uint32_t p, uint32_t pinv, Swap swp,
                         uint32_t& num, uint32_t& den, uint32_t& U, bool& slow, int& f_bs, uint32_t& f_L,
                         uint32_t& f_y) {
    if (BS <= b0 && !slow) {
      uint32_t L, y;
      const bool generic = (BS & 1) ? reg2_step<BS>(X, Y, l, p, pinv, swp, &L, &y)
                                    : reg2_step<BS>(Y, X, l, p, pinv, swp, &L, &y);
      if (generic) {
        num = mmul(num, y, p, pinv);
        U = mmul(U, y, p, pinv);
        den = mmul(den, U, p, pinv);
      } else {
        slow = true;
        f_bs = BS;
        f_L = L;
        f_y = y;
      }
    }
    RegChain2<BS - 1, N>::run(X, Y, l, b0, p, pinv, swp, num, den, U, slow, f_bs, f_L, f_y);
  }
};
template <int N>
struct RegChain2<0, N> {
  template <class Swap>
  RSL_HD static void run(uint32_t (&)[N], uint32_t (&)[N], int, int, uint32_t, uint32_t, Swap, uint32_t&, uint32_t&,
                         uint32_t&, bool&, int&, uint32_t&, uint32_t&) {}
};

// The generic chain without per-step branches: every step runs whatever its
// divisor's leading coefficient, and ok collects whether each new remainder
// kept degree deg B - 1 (if not, the value returned is meaningless and the
// caller restarts from the original coefficients with ures2_columns).  All
// branches depend only on the (per-problem) degrees, so the chain runs
// without divergence; num equals U throughout the generic pattern.
template <int BS, int N>
struct RegChain2Gen {
  template <class Swap>
  RSL_HD static void run(uint32_t (&X)[N], uint32_t (&Y)[N], int l, int b0, uint32_t p, uint32_t pinv, Swap swp,
                         uint32_t& den, uint32_t& U, bool& ok) {
    if (BS <= b0) {
      uint32_t L, y;
      const bool generic = (BS & 1) ? reg2_step<BS>(X, Y, l, p, pinv, swp, &L, &y)
                                    : reg2_step<BS>(Y, X, l, p, pinv, swp, &L, &y);
      ok = ok && generic;
      U = mmul(U, y, p, pinv);
      den = mmul(den, U, p, pinv);
    }
    RegChain2Gen<BS - 1, N>::run(X, Y, l, b0, p, pinv, swp, den, U, ok);
  }
};
template <int N>
struct RegChain2Gen<0, N> {
  template <class Swap>
  RSL_HD static void run(uint32_t (&)[N], uint32_t (&)[N], int, int, uint32_t, uint32_t, Swap, uint32_t&, uint32_t&,
                         bool&) {}
};

// Res_{m,n}(A, B) by a lane pair along the generic pattern only (layout as in
// ures_regs2).  *ok is false when the shape is not the register form's, a
// leading coefficient vanishes (*bad), or a remainder drops more than one
// degree; both lanes get the same ok and result.
template <int NMAX, class Swap>
RSL_HD uint32_t ures_regs2_generic(uint32_t (&X)[RegPoly2<NMAX>::kN], uint32_t (&Y)[RegPoly2<NMAX>::kN], int m,
                                   int n, int l, const PrimeConst& pc, bool* ok, bool* bad, Swap swp) {
  constexpr int N = RegPoly2<NMAX>::kN;
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  const uint32_t lcf = reg2_get(X, m, l, swp), lcg = reg2_get(Y, n, l, swp);
  *bad = (lcf == 0u) || (lcg == 0u);
  const bool shape_ok = m >= 1 && n >= 1 && m <= NMAX && n <= NMAX && (m - n <= 1) && (n - m <= 1);
  bool good = shape_ok && !*bad;
  uint32_t neg = 0u, den = one, U = one;
  if (!shape_ok) {
    *ok = false;
    return 0u;
  }
  if (m < n) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const uint32_t t = X[k];
      X[k] = Y[k];
      Y[k] = t;
    }
    neg = static_cast<uint32_t>(m * n) & 1u;
    const int t = m;
    m = n;
    n = t;
  }
  bool a_in_x = true;
  int b0 = n;
  if (m == n) {  // first division, k = 1: R = L A - lc(A) B
    const uint32_t L = reg2_get(Y, n, l, swp), lcA = reg2_get(X, n, l, swp);
#pragma unroll
    for (int k = 0; k < N; ++k) X[k] = (2 * k + l < n) ? mmulsub(L, X[k], lcA, Y[k], p, pinv) : 0u;
    good = good && reg2_get(X, n - 1, l, swp) != 0u;
    neg ^= static_cast<uint32_t>(n * n) & 1u;
    U = L;
    den = L;
    a_in_x = false;
    b0 = n - 1;
  }
  if (b0 >= 1) {
    if (a_in_x != ((b0 & 1) != 0)) {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const uint32_t t = X[k];
        X[k] = Y[k];
        Y[k] = t;
      }
    }
    RegChain2Gen<NMAX - 1, N>::run(X, Y, l, b0, p, pinv, swp, den, U, good);
  }
  *ok = good;
  // the last remainder (degree 0) is in X; num = U
  const uint32_t num = mmul(U, reg2_at<0>(X, l, swp), p, pinv);
  const uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
  return neg ? mneg(r, p) : r;
}

// Res_{m,n}(A, B) from the start by the general column code: the lane pair
// writes its halves of A and B to its two columns, lane 0 runs ures_formal,
// and both lanes return its result.
template <int NMAX, class Col, class Swap, class Sync>
RSL_HD uint32_t ures2_columns(const uint32_t (&X)[RegPoly2<NMAX>::kN], const uint32_t (&Y)[RegPoly2<NMAX>::kN],
                              int m, int n, int l, const PrimeConst& pc, Col CA, Col CB, Swap swp, Sync sync) {
  constexpr int N = RegPoly2<NMAX>::kN;
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (2 * k + l <= NMAX) {
      CA[2 * k + l] = X[k];
      CB[2 * k + l] = Y[k];
    }
  sync();
  uint32_t r = 0u;
  if (l == 0) {
    bool b2 = false;
    r = ures_formal(CA, CB, m, n, pc, &b2);
  }
  const uint32_t ro = swp(r);
  return l == 0 ? r : ro;
}

// Res_{m,n}(A, B) by a lane pair: lane l holds A's coefficients j = 2k + l in
// X[k] and B's in Y[k].  Both lanes return the result.  CA, CB: the pair's two
// shared scratch columns (NMAX + 1 entries); lanes that leave the register
// path write their halves there and lane 0 finishes with the column code
// (sync() orders the two lanes' column writes before lane 0 reads them).
template <int NMAX, class Col, class Swap, class Sync>
RSL_HD uint32_t ures_regs2(uint32_t (&X)[RegPoly2<NMAX>::kN], uint32_t (&Y)[RegPoly2<NMAX>::kN], int m, int n,
                           int l, const PrimeConst& pc, bool* bad, Col CA, Col CB, Swap swp, Sync sync) {
  constexpr int N = RegPoly2<NMAX>::kN;
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  const uint32_t lcf = reg2_get(X, m, l, swp), lcg = reg2_get(Y, n, l, swp);
  *bad = (lcf == 0u) || (lcg == 0u);
  const bool shape_ok = m >= 1 && n >= 1 && m <= NMAX && n <= NMAX && (m - n <= 1) && (n - m <= 1);
  uint32_t neg = 0u, num = one, den = one, U = one;
  bool slow = false;
  int f_a = 0, f_b = 0, f_k = 0;
  uint32_t f_L = 0, f_y = 0;
  bool r_in_x = false;
  bool fresh = !shape_ok || *bad;  // leave at once: the general code from the start
  if (!fresh) {
    if (m < n) {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const uint32_t t = X[k];
        X[k] = Y[k];
        Y[k] = t;
      }
      neg = static_cast<uint32_t>(m * n) & 1u;
      const int t = m;
      m = n;
      n = t;
    }
    bool a_in_x = true;
    int b0;
    if (m == n) {
      const uint32_t L = reg2_get(Y, n, l, swp), lcA = reg2_get(X, n, l, swp);
#pragma unroll
      for (int k = 0; k < N; ++k) X[k] = (2 * k + l < n) ? mmulsub(L, X[k], lcA, Y[k], p, pinv) : 0u;
      if (reg2_get(X, n - 1, l, swp) != 0u) {
        neg ^= static_cast<uint32_t>(n * n) & 1u;
        num = mmul(num, L, p, pinv);
        U = mmul(U, L, p, pinv);
        den = mmul(den, U, p, pinv);
      } else {
        slow = true;
        f_a = n;
        f_b = n;
        f_k = 1;
        f_L = L;
        f_y = L;
        r_in_x = true;
      }
      a_in_x = false;
      b0 = n - 1;
    } else {
      b0 = n;
    }
    if (!slow && b0 >= 1) {
      if (a_in_x != ((b0 & 1) != 0)) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const uint32_t t = X[k];
          X[k] = Y[k];
          Y[k] = t;
        }
      }
      int f_bs = 0;
      RegChain2<NMAX - 1, N>::run(X, Y, l, b0, p, pinv, swp, num, den, U, slow, f_bs, f_L, f_y);
      if (slow) {
        f_a = f_bs + 1;
        f_b = f_bs;
        f_k = 2;
        r_in_x = (f_bs & 1) != 0;
      }
    }
    if (!slow) {
      num = mmul(num, reg2_at<0>(X, l, swp), p, pinv);
      const uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
      return neg ? mneg(r, p) : r;
    }
  }
  // leave the register path: both lanes write their halves of the two columns
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (2 * k + l <= NMAX) {
      if (fresh) {
        CA[2 * k + l] = X[k];
        CB[2 * k + l] = Y[k];
      } else {
        CA[2 * k + l] = r_in_x ? X[k] : Y[k];  // R
        CB[2 * k + l] = r_in_x ? Y[k] : X[k];  // B
      }
    }
  sync();
  uint32_t r = 0u;
  if (l == 0) {
    if (fresh) {
      bool b2 = false;
      r = ures_formal(CA, CB, m, n, pc, &b2);
    } else {
      int c = f_b - 1;
      while (c >= 0 && CA[c] == 0u) --c;
      if (c >= 0) {
        neg ^= static_cast<uint32_t>(f_a * f_b) & 1u;
        const int delta = f_b - c;
        const int enum_ = f_k - 1 + delta;
        num = mmul(num, mpow(f_L, static_cast<uint32_t>(enum_), one, p, pinv), p, pinv);
        U = mmul(U, f_y, p, pinv);
        den = mmul(den, mpow(U, static_cast<uint32_t>(delta), one, p, pinv), p, pinv);
        r = ures_run(CB, CA, UresState{f_b, c, num, den, U, neg}, pc);
      }
    }
  }
  const uint32_t ro = swp(r);
  return l == 0 ? r : ro;
}

}  // namespace rsl

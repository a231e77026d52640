// Per-lane evaluation and univariate resultant over Z_p (host + device).
//
// One lane owns one (prime, point) pair.  Its two polynomials A(y) = f(x_i, y)
// and B(y) = g(x_i, y) live in two columns of a scratch array (LDS on the
// device, a plain array on the host) with a fixed element stride, so that the
// same code runs in the kernel and in the host-side self-test.
//
// What is computed: the determinant of the Sylvester matrix of A and B with
// the FORMAL degrees m = m_y, n = n_y, i.e. the image of R^(y)(x_i) mod p
// (paper Sec. 3.1 and Sec. 4.1: the evaluation homomorphism commutes with the
// determinant).  Leading coefficients that vanish at x_i are handled by the
// formal-degree identities
//   Res_{m,n}(A,B) = (-1)^{n(m-a)} lc(B)^{m-a} Res_{a,n}(A,B)   (deg A = a < m)
//   Res_{m,n}(A,B) = lc(A)^{n-b} Res_{m,b}(A,B)                 (deg B = b < n)
// and the value is 0 when both vanish.
//
// The Euclidean remainder sequence is computed division-free: each division
// step replaces A by the pseudo-remainder L^k A mod B (L = lc(B),
// k = deg A - deg B + 1), formed by k elimination passes
//   A <- L A - lc(A) y^(deg A - deg B) B .
// With R = A mod B of degree c, Res(A,B) = (-1)^{ab} L^{a-c} Res(B,R) and
// Res(B, L^k R) = L^{k b} Res(B, R); the scale factors are kept as a
// numerator and a denominator so that only one inversion is needed at the end.
// The denominator prod_t (L_t^{k_t})^{b_t} is accumulated as
// prod_t U_t^{b_t - b_{t+1}} with U_t = prod_{i<=t} L_i^{k_i}, which costs two
// multiplies per step in the usual case b_{t+1} = b_t - 1.  In the usual case
// deg A = deg B + 1 the two passes are fused into one:
//   R~[j] = L^2 A[j] - L lc(A) B[j-1] - lc(A~) B[j],  lc(A~) = L A[b] - lc(A) B[b-1].
#pragma once
#include "modarith.h"

namespace rsl {

template <int STRIDE>
struct Column {
  uint32_t* base;
  RSL_HD uint32_t& operator[](int j) const { return base[j * STRIDE]; }
};

// Horner evaluation of nrows polynomials in x (Montgomery x~ = x R) whose
// coefficients are stored as c R^2 mod p ("double" Montgomery form), so that
// one REDC per step gives acc <- acc x + c in Montgomery form:
//   REDC(acc~ x~ + c R^2) = (acc x + c) R.
template <class Col>
RSL_HD void eval_rows(Col out, const uint32_t* coeff, int nrows, int rowstride,
                      const int* rdeg, uint32_t xt, uint32_t p, uint32_t pinv) {
  for (int j = 0; j < nrows; ++j) {
    const uint32_t* c = coeff + j * rowstride;
    uint32_t acc = 0;
    for (int i = rdeg[j]; i >= 0; --i)
      acc = redc(static_cast<uint64_t>(acc) * xt + c[i], p, pinv);
    out[j] = acc;
  }
}

// Four fused updates r_i = (al a_i + be q_i + ga b_i) / R mod p with
// (q_0..q_3) = (bp, b0, b1, b2), phases interleaved across the four (see mmad3).
RSL_HD void mmad3x4(uint32_t al, uint32_t be, uint32_t ga, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                    uint32_t bp, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, uint32_t p, uint32_t pinv,
                    uint32_t* r0, uint32_t* r1, uint32_t* r2, uint32_t* r3) {
  uint64_t t0 = static_cast<uint64_t>(al) * a0, t1 = static_cast<uint64_t>(al) * a1;
  uint64_t t2 = static_cast<uint64_t>(al) * a2, t3 = static_cast<uint64_t>(al) * a3;
  t0 += static_cast<uint64_t>(be) * bp;
  t1 += static_cast<uint64_t>(be) * b0;
  t2 += static_cast<uint64_t>(be) * b1;
  t3 += static_cast<uint64_t>(be) * b2;
  t0 += static_cast<uint64_t>(ga) * b0;
  t1 += static_cast<uint64_t>(ga) * b1;
  t2 += static_cast<uint64_t>(ga) * b2;
  t3 += static_cast<uint64_t>(ga) * b3;
  uint32_t h0 = static_cast<uint32_t>(t0 >> 32), h1 = static_cast<uint32_t>(t1 >> 32);
  uint32_t h2 = static_cast<uint32_t>(t2 >> 32), h3 = static_cast<uint32_t>(t3 >> 32);
  h0 = umin32(h0, h0 - p);
  h1 = umin32(h1, h1 - p);
  h2 = umin32(h2, h2 - p);
  h3 = umin32(h3, h3 - p);
  t0 = (static_cast<uint64_t>(h0) << 32) | static_cast<uint32_t>(t0);
  t1 = (static_cast<uint64_t>(h1) << 32) | static_cast<uint32_t>(t1);
  t2 = (static_cast<uint64_t>(h2) << 32) | static_cast<uint32_t>(t2);
  t3 = (static_cast<uint64_t>(h3) << 32) | static_cast<uint32_t>(t3);
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  const uint32_t m2 = static_cast<uint32_t>(t2) * pinv, m3 = static_cast<uint32_t>(t3) * pinv;
  const uint32_t u0 = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  const uint32_t u1 = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
  const uint32_t u2 = static_cast<uint32_t>((t2 + static_cast<uint64_t>(m2) * p) >> 32);
  const uint32_t u3 = static_cast<uint32_t>((t3 + static_cast<uint64_t>(m3) * p) >> 32);
  *r0 = umin32(u0, u0 - p);
  *r1 = umin32(u1, u1 - p);
  *r2 = umin32(u2, u2 - p);
  *r3 = umin32(u3, u3 - p);
}

// Four fused updates r_i = (al a_i + be q_i + ga b_i) / R mod p with independent q_i.
RSL_HD void mmad3x4s(uint32_t al, uint32_t be, uint32_t ga, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                     uint32_t q0, uint32_t q1, uint32_t q2, uint32_t q3, uint32_t b0, uint32_t b1, uint32_t b2,
                     uint32_t b3, uint32_t p, uint32_t pinv, uint32_t* r0, uint32_t* r1, uint32_t* r2, uint32_t* r3) {
  uint64_t t0 = static_cast<uint64_t>(al) * a0, t1 = static_cast<uint64_t>(al) * a1;
  uint64_t t2 = static_cast<uint64_t>(al) * a2, t3 = static_cast<uint64_t>(al) * a3;
  t0 += static_cast<uint64_t>(be) * q0;
  t1 += static_cast<uint64_t>(be) * q1;
  t2 += static_cast<uint64_t>(be) * q2;
  t3 += static_cast<uint64_t>(be) * q3;
  t0 += static_cast<uint64_t>(ga) * b0;
  t1 += static_cast<uint64_t>(ga) * b1;
  t2 += static_cast<uint64_t>(ga) * b2;
  t3 += static_cast<uint64_t>(ga) * b3;
  uint32_t h0 = static_cast<uint32_t>(t0 >> 32), h1 = static_cast<uint32_t>(t1 >> 32);
  uint32_t h2 = static_cast<uint32_t>(t2 >> 32), h3 = static_cast<uint32_t>(t3 >> 32);
  h0 = umin32(h0, h0 - p);
  h1 = umin32(h1, h1 - p);
  h2 = umin32(h2, h2 - p);
  h3 = umin32(h3, h3 - p);
  t0 = (static_cast<uint64_t>(h0) << 32) | static_cast<uint32_t>(t0);
  t1 = (static_cast<uint64_t>(h1) << 32) | static_cast<uint32_t>(t1);
  t2 = (static_cast<uint64_t>(h2) << 32) | static_cast<uint32_t>(t2);
  t3 = (static_cast<uint64_t>(h3) << 32) | static_cast<uint32_t>(t3);
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  const uint32_t m2 = static_cast<uint32_t>(t2) * pinv, m3 = static_cast<uint32_t>(t3) * pinv;
  const uint32_t u0 = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  const uint32_t u1 = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
  const uint32_t u2 = static_cast<uint32_t>((t2 + static_cast<uint64_t>(m2) * p) >> 32);
  const uint32_t u3 = static_cast<uint32_t>((t3 + static_cast<uint64_t>(m3) * p) >> 32);
  *r0 = umin32(u0, u0 - p);
  *r1 = umin32(u1, u1 - p);
  *r2 = umin32(u2, u2 - p);
  *r3 = umin32(u3, u3 - p);
}

// Resultant with formal degrees (m, n) of the polynomials in columns A, B
// (Montgomery form; both columns are overwritten).  Returns the result in
// Montgomery form.  *bad is set when lc_y f(x_i) or lc_y g(x_i) vanishes.
// State of the remainder sequence between divisions: actual degrees a, b of
// the polynomials in A, B, the numerator and denominator of the scale factor,
// the running product U of the L_t^{k_t}, and the sign.
struct UresState {
  int a, b;
  uint32_t num, den, U, neg;
};

template <class Col>
RSL_HD uint32_t ures_run(Col A, Col B, UresState st, const PrimeConst& pc);

template <class Col>
RSL_HD uint32_t ures_formal(Col A, Col B, int m, int n, const PrimeConst& pc, bool* bad) {
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  *bad = (A[m] == 0u) || (B[n] == 0u);
  if (n == 0) return mpow(B[0], static_cast<uint32_t>(m), one, p, pinv);
  if (m == 0) return mpow(A[0], static_cast<uint32_t>(n), one, p, pinv);
  int a = m;
  while (a >= 0 && A[a] == 0u) --a;
  int b = n;
  while (b >= 0 && B[b] == 0u) --b;
  if (a < 0 || b < 0 || (a < m && b < n)) return 0u;
  uint32_t num = one;
  uint32_t neg = 0;
  if (a < m) {
    num = mpow(B[b], static_cast<uint32_t>(m - a), one, p, pinv);
    neg ^= static_cast<uint32_t>(n * (m - a)) & 1u;
  }
  if (b < n) num = mpow(A[a], static_cast<uint32_t>(n - b), one, p, pinv);
  return ures_run(A, B, UresState{a, b, num, one, one, neg}, pc);
}

// The division loop from state st (A, B of actual degrees st.a, st.b).
template <class Col>
RSL_HD uint32_t ures_run(Col A, Col B, UresState st, const PrimeConst& pc) {
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  int a = st.a, b = st.b;
  uint32_t num = st.num, den = st.den, U = st.U, neg = st.neg;

  // In the usual case (deg A = deg B + 1 and every remainder one degree lower)
  // the scalars a division needs -- L = lc(B), lc(A), A[b], B[b-1] -- are
  // carried in registers from the previous division: new A = old B, new B = R~,
  // so lc(A') = L, A'[b'] = B[b-1], L' = R~[b-1], B'[b'-1] = R~[b-2].
  bool carried = false;
  uint32_t cL = 0, clcA = 0, cAb = 0, cBb1 = 0;
  for (;;) {
    if (b == 0) {  // B a nonzero constant: Res(A, B) = B^a
      num = mmul(num, mpow(carried ? cL : B[0], static_cast<uint32_t>(a), one, p, pinv), p, pinv);
      break;
    }
    if (a == 0) {  // A a nonzero constant: Res(A, B) = A^b
      num = mmul(num, mpow(A[0], static_cast<uint32_t>(b), one, p, pinv), p, pinv);
      break;
    }
    if (a < b) {  // Res(A, B) = (-1)^{ab} Res(B, A)
      Col t = A; A = B; B = t;
      int ti = a; a = b; b = ti;
      neg ^= static_cast<uint32_t>(a * b) & 1u;
      carried = false;
      continue;
    }
    const uint32_t L = carried ? cL : B[b];
    const int k = a - b + 1;
    uint32_t y;  // L^k
    int c;       // degree of the remainder
    uint32_t last1 = 0, last2 = 0;  // R~[b-1], R~[b-2]
    uint32_t Bb1 = 0;               // B[b-1]
    if (k == 2) {
      const uint32_t lcA = carried ? clcA : A[a];
      const uint32_t Ab = carried ? cAb : A[b];
      Bb1 = carried ? cBb1 : B[b - 1];
      const uint32_t lcAt = mmulsub(L, Ab, lcA, Bb1, p, pinv);
      const uint32_t alpha = mmul(L, L, p, pinv);
      const uint32_t beta = mneg(mmul(L, lcA, p, pinv), p);
      const uint32_t gamma = mneg(lcAt, p);
      uint32_t prevB = 0u;
      int j = 0;
      if (b >= 4) {
        // software-pipelined: the next four A/B values are loaded before the
        // current four are combined, so LDS latency overlaps the arithmetic
        uint32_t b0 = B[0], b1 = B[1], b2 = B[2], b3 = B[3];
        uint32_t a0 = A[0], a1 = A[1], a2 = A[2], a3 = A[3];
        for (; j + 4 <= b; j += 4) {
          const bool more = j + 8 <= b;
          const uint32_t nb0 = more ? B[j + 4] : 0u, nb1 = more ? B[j + 5] : 0u;
          const uint32_t nb2 = more ? B[j + 6] : 0u, nb3 = more ? B[j + 7] : 0u;
          const uint32_t na0 = more ? A[j + 4] : 0u, na1 = more ? A[j + 5] : 0u;
          const uint32_t na2 = more ? A[j + 6] : 0u, na3 = more ? A[j + 7] : 0u;
          uint32_t r0, r1, r2, r3;
          mmad3x4(alpha, beta, gamma, a0, a1, a2, a3, prevB, b0, b1, b2, b3, p, pinv, &r0, &r1, &r2, &r3);
          A[j] = r0;
          A[j + 1] = r1;
          A[j + 2] = r2;
          A[j + 3] = r3;
          last2 = r2;
          last1 = r3;
          prevB = b3;
          b0 = nb0; b1 = nb1; b2 = nb2; b3 = nb3;
          a0 = na0; a1 = na1; a2 = na2; a3 = na3;
        }
      }
      for (; j < b; ++j) {
        const uint32_t bj = B[j];
        const uint32_t r = mmad3(alpha, A[j], beta, prevB, gamma, bj, p, pinv);
        A[j] = r;
        last2 = last1;
        last1 = r;
        prevB = bj;
      }
      y = alpha;
      if (last1 != 0u) {
        c = b - 1;
      } else {
        c = b - 2;
        while (c >= 0 && A[c] == 0u) --c;
      }
    } else {
      for (int d = a; d >= b; --d) {
        const uint32_t lc = A[d];
        const int sh = d - b;
        for (int j = 0; j < d; ++j) {
          const uint32_t bj = (j >= sh) ? B[j - sh] : 0u;
          A[j] = mmulsub(L, A[j], lc, bj, p, pinv);
        }
      }
      y = mpow(L, static_cast<uint32_t>(k), one, p, pinv);
      c = b - 1;
      while (c >= 0 && A[c] == 0u) --c;
      if (c == b - 1) {  // the next division may still use carried scalars
        Bb1 = B[b - 1];
        last1 = A[b - 1];
        last2 = (b >= 2) ? A[b - 2] : 0u;
      }
    }
    if (c < 0) return 0u;  // zero remainder with deg B >= 1: common factor at x_i
    neg ^= static_cast<uint32_t>(a * b) & 1u;
    const int delta = b - c;
    const int enum_ = k - 1 + delta;  // exponent of L in the numerator
    num = mmul(num, (enum_ == k) ? y : mpow(L, static_cast<uint32_t>(enum_), one, p, pinv), p, pinv);
    U = mmul(U, y, p, pinv);
    den = mmul(den, (delta == 1) ? U : mpow(U, static_cast<uint32_t>(delta), one, p, pinv), p, pinv);
    carried = (delta == 1);
    if (carried) {
      cL = last1;    // lc of the new B (= R~)
      clcA = L;      // lc of the new A (= old B)
      cAb = Bb1;     // new A[new b] = old B[b-1]
      cBb1 = last2;  // new B[new b - 1] = R~[b-2]
    }
    Col t = A; A = B; B = t;  // (A, B) <- (B, R~)
    a = b;
    b = c;
  }
  uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
  return neg ? mneg(r, p) : r;
}

}  // namespace rsl

namespace rsl {

// The same resultant computed by a group of K lanes that share the columns A
// and B (K > 1).  Every lane keeps the same scalar state; the elimination
// passes over the coefficient index j are split cyclically (lane l takes
// j = l, l+K, ...).  Within a pass a lane writes only its own A[j] and reads
// A[j], B[j], B[j-1] and scalars that the pass does not write, so lanes only
// need to agree between passes: sync() is called after every pass (a wave's
// lanes run in lockstep, so on the device sync() only has to stop the compiler
// from moving memory operations across it).  The caller syncs after writing
// the columns.
template <int K, class Col, class Sync>
RSL_HD uint32_t ures_group(Col A, Col B, int m, int n, const PrimeConst& pc, int l, bool* bad, Sync sync) {
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  *bad = (A[m] == 0u) || (B[n] == 0u);
  if (n == 0) return mpow(B[0], static_cast<uint32_t>(m), one, p, pinv);
  if (m == 0) return mpow(A[0], static_cast<uint32_t>(n), one, p, pinv);
  int a = m;
  while (a >= 0 && A[a] == 0u) --a;
  int b = n;
  while (b >= 0 && B[b] == 0u) --b;
  if (a < 0 || b < 0 || (a < m && b < n)) return 0u;
  uint32_t num = one, den = one, U = one;
  uint32_t neg = 0;
  if (a < m) {
    num = mpow(B[b], static_cast<uint32_t>(m - a), one, p, pinv);
    neg ^= static_cast<uint32_t>(n * (m - a)) & 1u;
  }
  if (b < n) num = mpow(A[a], static_cast<uint32_t>(n - b), one, p, pinv);

  // usual case: lc(A') = L and A'[b'] = B[b-1] are known from the previous
  // division (new A = old B); L' and B'[b'-1] are read after the pass
  bool carried = false;
  uint32_t clcA = 0, cAb = 0;
  for (;;) {
    if (b == 0) {
      num = mmul(num, mpow(B[0], static_cast<uint32_t>(a), one, p, pinv), p, pinv);
      break;
    }
    if (a == 0) {
      num = mmul(num, mpow(A[0], static_cast<uint32_t>(b), one, p, pinv), p, pinv);
      break;
    }
    if (a < b) {
      Col t = A; A = B; B = t;
      int ti = a; a = b; b = ti;
      neg ^= static_cast<uint32_t>(a * b) & 1u;
      carried = false;
      continue;
    }
    const uint32_t L = B[b];
    const int k = a - b + 1;
    uint32_t y;
    int c;
    uint32_t Bb1 = 0;
    if (k == 2) {
      const uint32_t lcA = carried ? clcA : A[a];
      const uint32_t Ab = carried ? cAb : A[b];
      Bb1 = B[b - 1];
      const uint32_t lcAt = mmulsub(L, Ab, lcA, Bb1, p, pinv);
      const uint32_t alpha = mmul(L, L, p, pinv);
      const uint32_t beta = mneg(mmul(L, lcA, p, pinv), p);
      const uint32_t gamma = mneg(lcAt, p);
      int j = l;
      for (; j + 3 * K < b; j += 4 * K) {
        const uint32_t bp = (j > 0) ? B[j - 1] : 0u;
        uint32_t r0, r1, r2, r3;
        // q_i = B[j_i - 1], b_i = B[j_i] for j_i = j + iK
        const uint32_t a0 = A[j], a1 = A[j + K], a2 = A[j + 2 * K], a3 = A[j + 3 * K];
        const uint32_t b0 = B[j], b1 = B[j + K], b2 = B[j + 2 * K], b3 = B[j + 3 * K];
        const uint32_t q1 = B[j + K - 1], q2 = B[j + 2 * K - 1], q3 = B[j + 3 * K - 1];
        mmad3x4s(alpha, beta, gamma, a0, a1, a2, a3, bp, q1, q2, q3, b0, b1, b2, b3, p, pinv, &r0, &r1, &r2, &r3);
        A[j] = r0;
        A[j + K] = r1;
        A[j + 2 * K] = r2;
        A[j + 3 * K] = r3;
      }
      for (; j < b; j += K) {
        const uint32_t bp = (j > 0) ? B[j - 1] : 0u;
        A[j] = mmad3(alpha, A[j], beta, bp, gamma, B[j], p, pinv);
      }
      sync();
      y = alpha;
      const uint32_t last1 = A[b - 1];
      if (last1 != 0u) {
        c = b - 1;
      } else {
        c = b - 2;
        while (c >= 0 && A[c] == 0u) --c;
      }
    } else {
      for (int d = a; d >= b; --d) {
        const uint32_t lc = A[d];
        const int sh = d - b;
        for (int j = l; j < d; j += K) {
          const uint32_t bj = (j >= sh) ? B[j - sh] : 0u;
          A[j] = mmulsub(L, A[j], lc, bj, p, pinv);
        }
        sync();
      }
      y = mpow(L, static_cast<uint32_t>(k), one, p, pinv);
      c = b - 1;
      while (c >= 0 && A[c] == 0u) --c;
      Bb1 = B[b - 1];
    }
    if (c < 0) return 0u;
    neg ^= static_cast<uint32_t>(a * b) & 1u;
    const int delta = b - c;
    const int enum_ = k - 1 + delta;
    num = mmul(num, (enum_ == k) ? y : mpow(L, static_cast<uint32_t>(enum_), one, p, pinv), p, pinv);
    U = mmul(U, y, p, pinv);
    den = mmul(den, (delta == 1) ? U : mpow(U, static_cast<uint32_t>(delta), one, p, pinv), p, pinv);
    carried = (delta == 1);
    clcA = L;
    cAb = Bb1;
    Col t = A; A = B; B = t;
    a = b;
    b = c;
  }
  uint32_t r = mmul(num, minv(den, one, p, pinv), p, pinv);
  return neg ? mneg(r, p) : r;
}

}  // namespace rsl

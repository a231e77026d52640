// Arithmetic modulo primes 2^30 < p < 2^32 / 3 in Montgomery form, R = 2^32.
//
// Shared by the device kernels and the host planner (all functions are
// __host__ __device__).  On gfx950 the 32x32->64 multiply (v_mad_u64_u32) and
// v_mul_lo_u32 issue at full VALU rate, so one Montgomery reduction is three
// multiplies and two double-rate adds:
//   m = t_lo * (-1/p) mod 2^32;  u = t + m p;  r = u_hi;  r = min(r, r - p).
// REDC(t) = t / R mod p is exact for t < p R and returns a value in [0, p).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rsl {

#define RSL_HD __host__ __device__ __forceinline__

struct PrimeConst {
  uint32_t p;     // the prime, 2^30 < p < 2^32 / 3
  uint32_t pinv;  // -p^{-1} mod 2^32
  uint32_t r1;    // R mod p        (Montgomery form of 1)
  uint32_t r2;    // R^2 mod p      (to enter Montgomery form)
  uint32_t r3;    // R^3 mod p      (to enter "double" Montgomery form c R^2)
  uint32_t pad[3];
};

RSL_HD uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// t / R mod p for t < p * 2^32
RSL_HD uint32_t redc(uint64_t t, uint32_t p, uint32_t pinv) {
  uint32_t m = static_cast<uint32_t>(t) * pinv;
  uint64_t u = t + static_cast<uint64_t>(m) * p;
  uint32_t r = static_cast<uint32_t>(u >> 32);
  return umin32(r, r - p);
}

// a b / R mod p for a, b < p
RSL_HD uint32_t mmul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  return redc(static_cast<uint64_t>(a) * b, p, pinv);
}

// (a b - c d) / R mod p for a, b, c, d < p  (t < 2 p^2 < p R)
RSL_HD uint32_t mmulsub(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t p, uint32_t pinv) {
  uint64_t t = static_cast<uint64_t>(a) * b + static_cast<uint64_t>(p - c) * d;
  return redc(t, p, pinv);
}

// (a b + c d + e f) / R mod p for all operands <= p: the sum is at most 3 p^2,
// below p R because 3p < 2^32 for every prime of the table, so it goes to REDC
// as it is (three multiply-adds and one reduction).
RSL_HD uint32_t mmad3(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e, uint32_t f,
                      uint32_t p, uint32_t pinv) {
  const uint64_t t = static_cast<uint64_t>(a) * b + static_cast<uint64_t>(c) * d +
                     static_cast<uint64_t>(e) * f;
  return redc(t, p, pinv);
}

RSL_HD uint32_t maddm(uint32_t a, uint32_t b, uint32_t p) {  // (a + b) mod p
  uint32_t s = a + b;
  return umin32(s, s - p);
}
RSL_HD uint32_t msubm(uint32_t a, uint32_t b, uint32_t p) {  // (a - b) mod p
  uint32_t s = a - b;
  return umin32(s, s + p);
}
RSL_HD uint32_t mneg(uint32_t a, uint32_t p) { return a ? p - a : 0u; }

// base^e in Montgomery form (base in Montgomery form, one = R mod p)
RSL_HD uint32_t mpow(uint32_t base, uint32_t e, uint32_t one, uint32_t p, uint32_t pinv) {
  uint32_t r = one;
  while (e) {
    if (e & 1u) r = mmul(r, base, p, pinv);
    e >>= 1;
    if (e) base = mmul(base, base, p, pinv);
  }
  return r;
}

// Inverse by Fermat: a^(p-2); a in Montgomery form, a != 0.
RSL_HD uint32_t minv(uint32_t a, uint32_t one, uint32_t p, uint32_t pinv) {
  return mpow(a, p - 2u, one, p, pinv);
}

// Host-side construction of the constants for one prime.
inline PrimeConst make_prime_const(uint32_t p) {
  PrimeConst c{};
  c.p = p;
  uint32_t inv = 1;  // Newton iteration for p^{-1} mod 2^32 (p odd)
  for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
  c.pinv = 0u - inv;
  uint64_t r1 = (static_cast<uint64_t>(1) << 32) % p;
  c.r1 = static_cast<uint32_t>(r1);
  c.r2 = static_cast<uint32_t>((r1 * r1) % p);
  c.r3 = static_cast<uint32_t>((static_cast<uint64_t>(c.r2) * r1) % p);
  return c;
}

}  // namespace rsl

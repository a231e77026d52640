// Device-side problem and table descriptors shared by the kernels and the
// host pipeline.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "modarith.h"

namespace rsl {

// Constant tables owned by a context (indexed by global prime index g).
struct DevTables {
  const PrimeConst* pc;     // [g]
  const uint32_t* fact;     // [g * kstride + t] = t! R mod p_g          (t <= kcap)
  const uint32_t* ifact;    // [g * kstride + t] = (t!)^{-1} R mod p_g
  const uint32_t* stir;     // [g * sstride + k(k+1)/2 + j] = s(k, j) R mod p_g  (k <= scap)
  int64_t sstride;
  int kstride;
  int kcap;                 // factorials available for t <= kcap
  int scap;                 // Stirling rows available for k <= scap
  int npcap;                // global prime indices < npcap
};

// One resultant problem as laid out in device memory.
struct DevProblem {
  // shape
  int my, ny;        // formal degrees in the eliminated variable
  int rowf, rowg;    // row strides of the f and g coefficient tiles
  int goff, CS;      // offset of the g tile, words per prime tile
  int ncoef, L_in;   // input coefficients (f tile then g tile), limbs each
  int D, E;          // degree bound; points origin..origin+E are evaluated
  int origin, formal;
  int np, L_out;     // primes, CRT output limbs
  int LP, tgs;       // row stride of Plimb and of Tg
  int pad0, pad1;
  // inputs (uploaded)
  const uint32_t* coeff;  // ncoef * L_in two's complement limbs
  const int* rdeg;        // my+1 row degrees of f, then ny+1 of g
  const int* pidx;        // np global prime indices
  const uint32_t* Hm;     // np: (M-1)/2 mod p_i
  const uint32_t* NH;     // L_out: 2^(32 L_out) - (M-1)/2
  const uint32_t* Tg;     // [j * tgs + i]  (prod_{l<j} p_l mod p_i) R
  const uint32_t* invM;   // [i]            (prod_{l<i} p_l)^{-1} R mod p_i
  const uint32_t* Plimb;  // [j * LP + t]   limbs of prod_{l<j} p_l
  // intermediates and output
  uint32_t* resid;        // np * CS     coefficients as c R^2 mod p
  uint32_t* zval;         // np * (E+1)  R(x_i) mod p, normal form
  uint8_t* zbad;          // np * (E+1)  leading coefficient vanished at x_i
  uint32_t* aconv;        // np * (D+1)  Newton coefficients (consecutive points)
  uint32_t* cres;         // np * (D+1)  coefficients of R mod p, normal form
  uint32_t* out;          // (D+1) * L_out two's complement limbs of R
  int* status;            // [0]: error bits, [1 + slot]: 1 if the slot was interpolated on a gapped point set
};

// status[0] error bits
enum : int {
  kErrTooFewGoodPoints = 1,
};

}  // namespace rsl

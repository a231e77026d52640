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
  const uint32_t* stir;     // [g * sstride + stir_rowoff(k) + j] = s(k, j) R mod p_g  (k <= scap)
  int64_t sstride;
  int kstride;
  int kcap;                 // factorials available for t <= kcap
  int scap;                 // Stirling rows available for k <= scap
  int npcap;                // global prime indices < npcap
};

// Row k of the Stirling triangle (k + 1 entries) starts at a multiple of 32
// words, so that 64-column segments of a row are whole 128-byte lines:
//   stir_rowoff(k) = 32 sum_{i<k} ceil((i + 1) / 32) = 32 (a + 1)(16 a + b),  k = 32 a + b.
__host__ __device__ inline int64_t stir_rowoff(int k) {
  const int64_t a = k >> 5, b = k & 31;
  return 32 * (a + 1) * (16 * a + b);
}

// Rows of the transposed residue tiles are padded to a multiple of this
// (Horner evaluates this many rows at once from one LDS broadcast read).
constexpr int kRowGroup = 4;

// One resultant problem as laid out in device memory.
struct DevProblem {
  // shape
  int my, ny;        // formal degrees in the eliminated variable
  int rowf, rowg;    // input row strides (x-degree + 1) of f and g
  int myp, nyp;      // my+1 and ny+1 rounded up to kRowGroup
  int goff, CS;      // offset of the g tile, words per prime tile (transposed tiles)
  int ncoef, L_in;   // input coefficients (f rows then g rows), limbs each
  int D, E;          // degree bound; points origin..origin+E are evaluated
  int origin, formal;
  int np, L_out;     // primes, CRT output limbs
  int LP, tgs;       // row stride of Plimb and of Tg
  int nchunk, kchunk;// Stirling partial sums: k-chunks and rows per chunk
  int ncchunk, cchunk;// convolution partial sums: i-chunks and terms per chunk
  int evk, evpb;     // evaluation: lanes per (prime, point) pair (1, 2, 4), pairs per block (64 / evk)
  int regn;          // evaluation with the polynomials in registers up to this degree (8..32), 0 = no
  int crt_garner;    // 1: CRT by Garner's digits only (test hook), 0: direct form with Garner fallback
  int schur;         // 1: univariate resultants by the Schur algorithm (one wave per pair)
  int wide;          // 1: CRT by the wide path (more primes than the per-lane slots cover)
  int evmf;          // 1: the register form's Horner sums on the matrix cores (from the digit tiles)
  int dRTf, dRTg;    // digit tiles: 16-row tiles of f and of g
  int dfr;           // digit tiles: operand fragments per prime slot, 5 (dRTf + dRTg)
  // the same system eliminated in x (the next problem): the reduction of prime
  // slots < pshared also writes its residue tiles (transposed positions)
  int pshared, pmyp, pnyp, pgoff, pCS;
  uint32_t* presid;
  int pdRTf, pdRTg, pdfr;  // the partner's digit tile shape (0 when it has none)
  uint64_t* pdig;
  int Lw;            // limbs of the rows of Mi and of negM: L_out, or L_out + 1 for the wide path
  // inputs (uploaded)
  const uint32_t* coeff;  // ncoef * L_in two's complement limbs
  const int* gdeg;        // max x-degree per group of kRowGroup rows: f groups then g groups
  const int* pidx;        // np global prime indices
  const uint32_t* Hm;     // np: (M-1)/2 mod p_i
  const uint32_t* NH;     // L_out: 2^(32 L_out) - (M-1)/2
  const uint32_t* Tg;     // [j * tgs + i]  (prod_{l<j} p_l mod p_i) R
  const uint32_t* invM;   // [i]            (prod_{l<i} p_l)^{-1} R mod p_i
  const uint32_t* Plimb;  // [j * LP + t]   limbs of prod_{l<j} p_l
  const uint32_t* Mi;     // [j * Lw + t]   limbs of M / p_j (direct CRT)
  const uint32_t* wdir;   // [i]            (M / p_i)^{-1} R mod p_i
  const uint32_t* rinv;   // [2 i], [2 i + 1] low, high word of floor(2^64 / p_i)
  const uint32_t* negM;   // Lw: 2^(32 Lw) - M
  const uint32_t* Mw;     // Lw limbs of M (wide path)
  const uint32_t* NHM;    // L_out: -(M-1)/2 - M mod 2^(32 L_out) (wide path)
  // intermediates and output
  uint32_t* resid;        // np * CS     transposed tiles, c R^2 mod p
  uint64_t* dig;          // np * dfr * 64  7-bit digits of c mod p in matrix-core operand order (evmf)
  uint32_t* zval;         // np * (E+1)  R(x_i) mod p, normal form
  uint8_t* zbad;          // np * (E+1)  leading coefficient vanished at x_i
  uint64_t* aconv;        // ncchunk * np * (D+1): partial sums, REDC(sum) = Newton coefficient a_k
  uint64_t* cpart;        // nchunk * np * (D+1): partial sums, REDC(sum) = coefficient mod p
  uint32_t* wT;           // wdpad * wnpad  t_{k,i} = u_{k,i} (M / p_i)^{-1} mod p_i, zero padded (wide path)
  uint32_t* wq;           // D+1         quotient estimate floor(sum_i f_{k,i} / 2^32) (wide path)
  uint64_t* wS;           // (D+1) * Lw * 2  column sum of each limb as (low, high) 64-bit words (wide path)
  const int8_t* wMd;      // 5 * wlpad * wnpad  7-bit digit planes of the M_i limbs, [digit][limb][prime]
  int wdpad, wlpad, wnpad;// D+1, Lw and np rounded up (64, 32, 64); wT rows have wnpad entries
  int wide_mfma;          // 1: contraction on the matrix cores
  uint32_t* out;          // (D+1) * L_out two's complement limbs of R
  int* status;            // [0] error bits, [1+slot] 1 if gapped interpolation, [1+np] bad pairs,
                          // [2+np+slot] 1 if a point among 0..D was bad for the prime
};

// A unit of work of a stage kernel: one block processes one item.
struct WorkItem {
  int prob;  // index into the problem array
  int slot;  // prime slot (or -1)
  int blk;   // block index inside the (problem, slot)
  int sub;   // stage-specific (Stirling k-chunk)
};

// Problems of a job that use the same prime share the basis-change table
// reads: a group lists (problem, slot) members of one global prime index.
struct StirMember {
  int prob;
  int slot;
};
struct StirGroup {
  int g;       // global prime index
  int first;   // first member in the member list
  int count;   // members (at most kStirGroupMax)
  int maxD;    // largest degree bound among the members
};
constexpr int kStirGroupMax = 8;
constexpr int kSlotCrtPrimes = 512;  // CRT with the primes in per-lane slots (up to 8 per lane)
constexpr int kMaxPrimes = 4096;     // primes per problem (the wide CRT beyond kSlotCrtPrimes)

// status[0] error bits
enum : int {
  kErrTooFewGoodPoints = 1,
  kErrQueueStall = 2,
};

}  // namespace rsl

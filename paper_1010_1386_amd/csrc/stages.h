// Device code of the pipeline stages.  Each stage_* function processes one
// work item with one thread block; the stage kernels (kernels.hip) and the
// persistent batched kernel call the same functions.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.h"
#include "ures.h"
#include "ures_regs.h"

namespace rsl {

enum : int {
  kStageReduce = 0,
  kStageEval = 1,
  kStageConv = 2,
  kStageStir = 3,
  kStageNewton = 4,
  kStageCrt = 5,
  kNumStages = 6,
};

constexpr int kCrtWaves = 8;          // waves of a CRT block (one coefficient each)
// waves of a CRT block with ns prime slots per lane (more slots: fewer waves,
// two coefficients each, to stay within the LDS of a block)
__host__ __device__ inline int crt_block_waves(int ns) { return ns > 4 ? 4 : kCrtWaves; }
constexpr int kLdsWords = 16384;      // 64 KB of dynamic LDS per block at most

// ------------------------------------------------------------------ helpers

// acc + x y with acc kept below p 2^32 (one conditional subtraction on the high word)
__device__ __forceinline__ uint64_t mac_fold(uint64_t acc, uint32_t x, uint32_t y, uint32_t p) {
  acc += static_cast<uint64_t>(x) * y;
  uint32_t hi = static_cast<uint32_t>(acc >> 32);
  hi = umin32(hi, hi - p);
  return (static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(acc);
}

// a + b for a, b < p 2^32, result < p 2^32
__device__ __forceinline__ uint64_t add_fold(uint64_t a, uint64_t b, uint32_t p) {
  const uint64_t s = a + b;
  uint32_t hi = static_cast<uint32_t>(s >> 32);
  hi = umin32(hi, hi - p);
  return (static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(s);
}

// Lazy Horner steps acc <- REDC(acc x~ + c) with acc kept in [0, 2p): the
// input stays below 2p^2 + p < p 2^32, so REDC's bound holds without the final
// conditional subtraction.  The phases of the independent chains are written
// interleaved so that each dependent instruction has others to hide behind.
__device__ __forceinline__ void horner_step4(uint32_t* a, const uint4 c, uint32_t xt, uint32_t p, uint32_t pinv) {
  const uint64_t t0 = static_cast<uint64_t>(a[0]) * xt + c.x;
  const uint64_t t1 = static_cast<uint64_t>(a[1]) * xt + c.y;
  const uint64_t t2 = static_cast<uint64_t>(a[2]) * xt + c.z;
  const uint64_t t3 = static_cast<uint64_t>(a[3]) * xt + c.w;
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  const uint32_t m2 = static_cast<uint32_t>(t2) * pinv, m3 = static_cast<uint32_t>(t3) * pinv;
  a[0] = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  a[1] = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
  a[2] = static_cast<uint32_t>((t2 + static_cast<uint64_t>(m2) * p) >> 32);
  a[3] = static_cast<uint32_t>((t3 + static_cast<uint64_t>(m3) * p) >> 32);
}

__device__ __forceinline__ void horner_step8(uint32_t* a, uint32_t* b, const uint4 c, const uint4 d, uint32_t xt,
                                             uint32_t p, uint32_t pinv) {
  const uint64_t t0 = static_cast<uint64_t>(a[0]) * xt + c.x;
  const uint64_t t1 = static_cast<uint64_t>(a[1]) * xt + c.y;
  const uint64_t t2 = static_cast<uint64_t>(a[2]) * xt + c.z;
  const uint64_t t3 = static_cast<uint64_t>(a[3]) * xt + c.w;
  const uint64_t t4 = static_cast<uint64_t>(b[0]) * xt + d.x;
  const uint64_t t5 = static_cast<uint64_t>(b[1]) * xt + d.y;
  const uint64_t t6 = static_cast<uint64_t>(b[2]) * xt + d.z;
  const uint64_t t7 = static_cast<uint64_t>(b[3]) * xt + d.w;
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  const uint32_t m2 = static_cast<uint32_t>(t2) * pinv, m3 = static_cast<uint32_t>(t3) * pinv;
  const uint32_t m4 = static_cast<uint32_t>(t4) * pinv, m5 = static_cast<uint32_t>(t5) * pinv;
  const uint32_t m6 = static_cast<uint32_t>(t6) * pinv, m7 = static_cast<uint32_t>(t7) * pinv;
  a[0] = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  a[1] = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
  a[2] = static_cast<uint32_t>((t2 + static_cast<uint64_t>(m2) * p) >> 32);
  a[3] = static_cast<uint32_t>((t3 + static_cast<uint64_t>(m3) * p) >> 32);
  b[0] = static_cast<uint32_t>((t4 + static_cast<uint64_t>(m4) * p) >> 32);
  b[1] = static_cast<uint32_t>((t5 + static_cast<uint64_t>(m5) * p) >> 32);
  b[2] = static_cast<uint32_t>((t6 + static_cast<uint64_t>(m6) * p) >> 32);
  b[3] = static_cast<uint32_t>((t7 + static_cast<uint64_t>(m7) * p) >> 32);
}

// Two and four chains of the same lazy Horner step (lane-pair layout).
__device__ __forceinline__ void horner_step2(uint32_t* a, uint32_t c0, uint32_t c1, uint32_t xt, uint32_t p,
                                             uint32_t pinv) {
  const uint64_t t0 = static_cast<uint64_t>(a[0]) * xt + c0;
  const uint64_t t1 = static_cast<uint64_t>(a[1]) * xt + c1;
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  a[0] = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  a[1] = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
}
__device__ __forceinline__ void horner_step2x2(uint32_t* a, uint32_t* b, uint32_t c0, uint32_t c1, uint32_t d0,
                                               uint32_t d1, uint32_t xt, uint32_t p, uint32_t pinv) {
  const uint64_t t0 = static_cast<uint64_t>(a[0]) * xt + c0;
  const uint64_t t1 = static_cast<uint64_t>(a[1]) * xt + c1;
  const uint64_t t2 = static_cast<uint64_t>(b[0]) * xt + d0;
  const uint64_t t3 = static_cast<uint64_t>(b[1]) * xt + d1;
  const uint32_t m0 = static_cast<uint32_t>(t0) * pinv, m1 = static_cast<uint32_t>(t1) * pinv;
  const uint32_t m2 = static_cast<uint32_t>(t2) * pinv, m3 = static_cast<uint32_t>(t3) * pinv;
  a[0] = static_cast<uint32_t>((t0 + static_cast<uint64_t>(m0) * p) >> 32);
  a[1] = static_cast<uint32_t>((t1 + static_cast<uint64_t>(m1) * p) >> 32);
  b[0] = static_cast<uint32_t>((t2 + static_cast<uint64_t>(m2) * p) >> 32);
  b[1] = static_cast<uint32_t>((t3 + static_cast<uint64_t>(m3) * p) >> 32);
}

// ------------------------------------------------------------------ reduce

// Coefficient t of the prime's transposed tile: f part [i][j] (j padded to
// myp), then g part [i][j] (j padded to nyp).  Stores c R^2 mod p (0 for padding).
// With zero_status, the block of (slot 0, block 0) also clears the problem's
// status words (a launch that runs before every other stage of the problem).
// A two's complement value of L limbs mod p, without divisions: the signed top
// limb plus 2p lies in (0, 4p) since p > 2^30; each lower limb w (< 2^32 < 4p)
// enters as r <- r 2^32 + w, with r 2^32 mod p = mmul(r, R^2).
__device__ inline uint32_t limbs_mod_p(const uint32_t* wd, int L, const PrimeConst& pc) {
  const uint32_t p = pc.p;
  const int32_t top = static_cast<int32_t>(wd[L - 1]);
  uint64_t x = static_cast<uint64_t>(static_cast<int64_t>(top) + 2 * static_cast<int64_t>(p));  // < 4p
  x = (x >= 2ull * p) ? x - 2ull * p : x;
  x = (x >= p) ? x - p : x;
  uint32_t r = static_cast<uint32_t>(x);
  for (int l = L - 2; l >= 0; --l) {
    uint32_t wl = wd[l];
    wl = umin32(wl, wl - p);
    wl = umin32(wl, wl - p);
    wl = umin32(wl, wl - p);
    r = maddm(mmul(r, pc.r2, p, pc.pinv), wl, p);
  }
  return r;
}

// Position in the partner's tiles (the system eliminated in x) of the
// coefficient at tile position t (inside the f or g rectangle): x^i y^j there
// is y'^i x'^j, so [x-power i][row j] becomes [x'-power j][row i].
__device__ inline int partner_pos(const DevProblem& P, int t) {
  if (t < P.goff) {
    const int i = t / P.myp, j = t - i * P.myp;
    return j * P.pmyp + i;
  }
  const int u = t - P.goff;
  const int i = u / P.nyp, j = u - i * P.nyp;
  return P.pgoff + j * P.pnyp + i;
}

// Tile position t -> polynomial gp (0: f, 1: g), x-power i and row j; returns
// the input coefficient's index, -1 for a padding position.
__device__ inline int tile_coord(const DevProblem& P, int t, int* gp, int* i, int* j) {
  if (t < P.goff) {
    *gp = 0;
    *i = t / P.myp;
    *j = t - *i * P.myp;
    return (*j <= P.my) ? *j * P.rowf + *i : -1;
  }
  const int u = t - P.goff;
  *gp = 1;
  *i = u / P.nyp;
  *j = u - *i * P.nyp;
  return (*i < P.rowg && *j <= P.ny) ? (P.my + 1) * P.rowf + *j * P.rowg + *i : -1;
}

// Digit tiles (evaluation on the matrix cores).  The residue c mod p of the
// coefficient at x-power i (< 32; x-power 32, the one beyond the products' K
// range, stays in the residue tile) and row j of f (gp = 0) or g (gp = 1) is
// kept as five 7-bit digits: digit b lies in operand fragment b RT + j / 16 of
// its polynomial (RT = its 16-row tiles; g's fragments follow f's), lane
// (j mod 16) + 16 (i / 8), byte i mod 8 -- the B operand order of
// v_mfma_i32_16x16x32_i8 (lane l: column l mod 16, K slice l / 16), so that a
// wave reads one fragment as one coalesced 8-byte load per lane.  Padding
// positions are never written (the tiles are cleared at upload).
__host__ __device__ inline int dig_rt(int rows) { return (rows + 15) / 16; }
constexpr int kDigits = 5;
__device__ inline void write_digits(uint64_t* dig, int fr, int rtf, int rtg, int slot, int gp, int i, int j,
                                    uint32_t r) {
  if (i >= 32) return;  // x-power 32: added on the vector ALUs from the residue tile
  const int rt = gp ? rtg : rtf;
  uint8_t* base = reinterpret_cast<uint8_t*>(dig + (static_cast<size_t>(slot) * fr + (gp ? kDigits * rtf : 0)) * 64);
  const size_t at = (static_cast<size_t>(j >> 4) * 64 + (j & 15) + 16 * (i >> 3)) * 8 + (i & 7);
#pragma unroll
  for (int b = 0; b < kDigits; ++b)
    base[static_cast<size_t>(b) * rt * 512 + at] = static_cast<uint8_t>((r >> (7 * b)) & 127u);
}

// staged = true (the reduction launched as its own kernel): the residue tiles
// are written only for problems whose staged evaluation reads them (Horner
// forms; of a matrix-core form only x-power 32, which it adds on the vector
// ALUs); the persistent schedule evaluates by Horner and writes them all.
__device__ inline void stage_reduce(const DevProblem& P, const DevTables& T, const WorkItem& w,
                                    bool zero_status = false, bool staged = false) {
  if (zero_status && w.slot == 0 && w.blk == 0)
    for (int i = threadIdx.x; i < 2 * P.np + 2; i += blockDim.x) P.status[i] = 0;
  const int t = w.blk * blockDim.x + threadIdx.x;
  if (t >= P.CS) return;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  int gp, ci, cj;
  const int in = tile_coord(P, t, &gp, &ci, &cj);
  const bool own_tile = !(staged && P.evmf), partner_tile = !(staged && P.pdig);
  uint32_t v = 0;
  if (in >= 0) {
    const uint32_t p = pc.p;
    const uint32_t r = limbs_mod_p(P.coeff + static_cast<size_t>(in) * P.L_in, P.L_in, pc);
    v = mmul(r, pc.r3, p, pc.pinv);
    if (w.slot < P.pshared && (partner_tile || cj == 32))
      P.presid[static_cast<size_t>(w.slot) * P.pCS + partner_pos(P, t)] = v;
    if (P.dig) write_digits(P.dig, P.dfr, P.dRTf, P.dRTg, w.slot, gp, ci, cj, r);
    if (P.pdig && w.slot < P.pshared) write_digits(P.pdig, P.pdfr, P.pdRTf, P.pdRTg, w.slot, gp, cj, ci, r);
  }
  if (own_tile || ci == 32) P.resid[static_cast<size_t>(w.slot) * P.CS + t] = v;
}

// Problems whose evaluation takes its sums from the matrix cores and that
// share no reduction with a partner (inputs of at most two limbs): one thread
// per (row, 8 consecutive x-powers) of a prime slot, which writes each of the
// five digit planes' 8 bytes of that row and K slice as one word (eight
// separate byte stores per plane otherwise); x-power 32, beyond the products'
// K range, goes to the residue tile.  Consecutive threads take consecutive
// rows.  Item (slot, block of 256 words, sub = 2).
__host__ __device__ inline int reduce_words(int my, int ny, int rowf, int rowg) {
  return (my + 1) * ((rowf + 7) / 8) + (ny + 1) * ((rowg + 7) / 8);
}
__device__ inline void stage_reduce_words(const DevProblem& P, const DevTables& T, const WorkItem& w) {
  if (w.slot == 0 && w.blk == 0)
    for (int i = threadIdx.x; i < 2 * P.np + 2; i += blockDim.x) P.status[i] = 0;
  const int t = w.blk * blockDim.x + threadIdx.x;
  const int nwf = (P.my + 1) * ((P.rowf + 7) / 8);
  if (t >= reduce_words(P.my, P.ny, P.rowf, P.rowg)) return;
  const int gp = t >= nwf ? 1 : 0;
  const int u = gp ? t - nwf : t;
  const int rows = gp ? P.ny + 1 : P.my + 1;
  const int k = u / rows, j = u - k * rows;
  const int len = gp ? P.rowg : P.rowf;
  const uint32_t* src =
      P.coeff + (static_cast<size_t>(gp ? (P.my + 1) * P.rowf : 0) + static_cast<size_t>(j) * len) * P.L_in;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  uint32_t r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int i = 8 * k + e;
    r[e] = (i < len) ? limbs_mod_p(src + static_cast<size_t>(i) * P.L_in, P.L_in, pc) : 0u;
  }
  if (k < 4) {
    const int rt = gp ? P.dRTg : P.dRTf;
    uint64_t* base = P.dig + (static_cast<size_t>(w.slot) * P.dfr + (gp ? kDigits * P.dRTf : 0)) * 64 +
                     static_cast<size_t>(j >> 4) * 64 + (j & 15) + 16 * k;
#pragma unroll
    for (int b = 0; b < kDigits; ++b) {
      uint64_t word = 0;
#pragma unroll
      for (int e = 0; e < 8; ++e) word |= static_cast<uint64_t>((r[e] >> (7 * b)) & 127u) << (8 * e);
      base[static_cast<size_t>(b) * rt * 64] = word;
    }
  } else {  // x-power 32 (rowf or rowg = 33): the residue tile, c R^2 mod p
    const int at = (gp ? P.goff + 32 * P.nyp : 32 * P.myp) + j;
    P.resid[static_cast<size_t>(w.slot) * P.CS + at] = mmul(r[0], pc.r3, pc.p, pc.pinv);
  }
}

// Multi-limb inputs: a block takes 64 transposed positions and 32 prime slots
// (item: slot = first slot, blk = position block, sub = 1).  The 64
// coefficients' limbs are staged in LDS 64 limbs at a time (coalesced reads of
// each coefficient's limb run, stored [limb][coefficient] with a padded row);
// thread (c, q) runs the Horner steps of the limbs, top limb first, for slots
// slot + q + 4 r, r < 8: eight independent chains.
constexpr int kReduceMlCoeffs = 64;
constexpr int kReduceMlSlots = 32;
constexpr int kReduceMlLimbs = 64;
__host__ __device__ inline int reduce_ml_lds_words() { return kReduceMlLimbs * (kReduceMlCoeffs + 1); }

__device__ inline void stage_reduce_ml(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds,
                                       bool staged = false) {
  if (w.slot == 0 && w.blk == 0)
    for (int i = threadIdx.x; i < 2 * P.np + 2; i += blockDim.x) P.status[i] = 0;
  constexpr int kPer = kReduceMlSlots / 4;
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int t = w.blk * kReduceMlCoeffs + c;
  auto input_of = [&](int tt) {
    if (tt >= P.CS) return -1;
    if (tt < P.goff) {
      const int i = tt / P.myp, j = tt - i * P.myp;
      return (j <= P.my) ? j * P.rowf + i : -1;
    }
    const int u = tt - P.goff;
    const int i = u / P.nyp, j = u - i * P.nyp;
    return (i < P.rowg && j <= P.ny) ? (P.my + 1) * P.rowf + j * P.rowg + i : -1;
  };
  const int in = input_of(t);
  uint32_t p[kPer], pinv[kPer], r2[kPer], r3[kPer], acc[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int sl = w.slot + q + 4 * r;
    const PrimeConst pc = T.pc[P.pidx[sl < P.np ? sl : 0]];
    p[r] = pc.p;
    pinv[r] = pc.pinv;
    r2[r] = pc.r2;
    r3[r] = pc.r3;
    acc[r] = 0u;
  }
  const int L = P.L_in;
  for (int l1 = L; l1 > 0; l1 -= kReduceMlLimbs) {  // limbs [l0, l1), top chunk first
    const int l0 = l1 > kReduceMlLimbs ? l1 - kReduceMlLimbs : 0, nl = l1 - l0;
    __syncthreads();
    for (int e = threadIdx.x; e < kReduceMlCoeffs * nl; e += blockDim.x) {
      const int cc = e / nl, l = e - cc * nl;
      const int ci = input_of(w.blk * kReduceMlCoeffs + cc);
      lds[l * (kReduceMlCoeffs + 1) + cc] = (ci >= 0) ? P.coeff[static_cast<size_t>(ci) * L + l0 + l] : 0u;
    }
    __syncthreads();
    for (int l = nl - 1; l >= 0; --l) {
      const uint32_t wd = lds[l * (kReduceMlCoeffs + 1) + c];
      if (l0 + l == L - 1) {
        // the signed top limb plus 2p lies in (0, 4p) since p > 2^30
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          uint64_t x = static_cast<uint64_t>(static_cast<int64_t>(static_cast<int32_t>(wd)) + 2 * static_cast<int64_t>(p[r]));
          x = (x >= 2ull * p[r]) ? x - 2ull * p[r] : x;
          x = (x >= p[r]) ? x - p[r] : x;
          acc[r] = static_cast<uint32_t>(x);
        }
      } else {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          uint32_t wl = umin32(wd, wd - p[r]);
          wl = umin32(wl, wl - p[r]);
          wl = umin32(wl, wl - p[r]);
          acc[r] = maddm(mmul(acc[r], r2[r], p[r], pinv[r]), wl, p[r]);
        }
      }
    }
  }
  if (t >= P.CS) return;
  const int tp = (in >= 0 && w.slot < P.pshared) ? partner_pos(P, t) : 0;
  int gp, ci, cj;
  tile_coord(P, t, &gp, &ci, &cj);
  const bool own_tile = !(staged && P.evmf), partner_tile = !(staged && P.pdig);
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int sl = w.slot + q + 4 * r;
    if (sl < P.np) {
      const uint32_t v = (in >= 0) ? mmul(acc[r], r3[r], p[r], pinv[r]) : 0u;
      if (own_tile || ci == 32) P.resid[static_cast<size_t>(sl) * P.CS + t] = v;
      if (in >= 0 && sl < P.pshared && (partner_tile || cj == 32)) P.presid[static_cast<size_t>(sl) * P.pCS + tp] = v;
      if (in >= 0 && P.dig) write_digits(P.dig, P.dfr, P.dRTf, P.dRTg, sl, gp, ci, cj, acc[r]);
      if (in >= 0 && P.pdig && sl < P.pshared)
        write_digits(P.pdig, P.pdfr, P.pdRTf, P.pdRTg, sl, gp, cj, ci, acc[r]);
    }
  }
}

// -------------------------------------------------------------- eval + ures

// Bad-pair bookkeeping of one eval wave: the count, and a per-prime flag set
// when a bad point lies among 0..D (the interpolation then needs the gapped
// point set).
__device__ inline void eval_report_bad(const DevProblem& P, int slot, int pt, bool live, bool bad) {
  const uint64_t nbad = __ballot(live && bad);
  const uint64_t early = __ballot(live && bad && pt <= P.D);
  if ((threadIdx.x & 63) == 0) {
    if (nbad) atomicAdd(P.status + 1 + P.np, static_cast<int>(__popcll(nbad)));
    if (early) atomicOr(P.status + 2 + P.np + slot, 1);
  }
}

// LDS words needed by one eval block (one wave).
__host__ __device__ inline int eval_lds_words(const DevProblem& P) {
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  return P.CS + 2 * nm1 * 64;
}

// One wave: 64 consecutive points of one prime.  The prime's coefficient tile
// is copied to LDS once; Horner then runs on kRowGroup rows of f and of g at a
// time (eight independent chains per lane), each step reading kRowGroup
// coefficients with one broadcast LDS load.  The values f_j(x_i), g_j(x_i) go
// to two LDS columns per lane and the univariate resultant runs there.
__device__ inline void stage_eval_ures(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  const int lane = threadIdx.x;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv;
  uint32_t* tile = lds;
  const uint32_t* src = P.resid + static_cast<size_t>(w.slot) * P.CS;
  for (int t = lane; t < P.CS; t += 64) tile[t] = src[t];
  __syncthreads();

  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  uint32_t* cols = lds + P.CS;
  Column<64> A{cols + lane};
  Column<64> B{cols + nm1 * 64 + lane};
  const int pt = w.blk * 64 + lane;
  const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
  const uint32_t xt = mmul(x, pc.r2, p, pinv);

  const int gf = P.myp / kRowGroup, gg = P.nyp / kRowGroup;
  const int ng = gf > gg ? gf : gg;
  const uint32_t* ftile = tile;
  const uint32_t* gtile = tile + P.goff;
  for (int q = 0; q < ng; ++q) {
    // group degrees are uniform: keep them (and the loop bounds) in SGPRs
    const int df = __builtin_amdgcn_readfirstlane((q < gf) ? P.gdeg[q] : -1);
    const int dg = __builtin_amdgcn_readfirstlane((q < gg) ? P.gdeg[gf + q] : -1);
    const int dboth = df < dg ? df : dg;
    uint32_t a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
    const uint32_t* fq = ftile + kRowGroup * q;
    const uint32_t* gq = gtile + kRowGroup * q;
    int i = df > dg ? df : dg;
    for (; i > dboth; --i) {  // only the higher-degree tile is active
      if (i <= df) horner_step4(a, *reinterpret_cast<const uint4*>(fq + i * P.myp), xt, p, pinv);
      else horner_step4(b, *reinterpret_cast<const uint4*>(gq + i * P.nyp), xt, p, pinv);
    }
    if (i >= 0) {  // both tiles: eight independent chains, next rows prefetched
      uint4 cf = *reinterpret_cast<const uint4*>(fq + i * P.myp);
      uint4 cg = *reinterpret_cast<const uint4*>(gq + i * P.nyp);
      for (; i > 0; --i) {
        const uint4 nf = *reinterpret_cast<const uint4*>(fq + (i - 1) * P.myp);
        const uint4 ng = *reinterpret_cast<const uint4*>(gq + (i - 1) * P.nyp);
        horner_step8(a, b, cf, cg, xt, p, pinv);
        cf = nf;
        cg = ng;
      }
      horner_step8(a, b, cf, cg, xt, p, pinv);
    }
    const int j = kRowGroup * q;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (j + r <= P.my) A[j + r] = umin32(a[r], a[r] - p);  // Horner keeps values below 2p
      if (j + r <= P.ny) B[j + r] = umin32(b[r], b[r] - p);
    }
  }
  bool bad = false;
  const uint32_t r = ures_formal(A, B, P.my, P.ny, pc, &bad);
  const bool live = pt <= P.E;
  if (live) {
    const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
    P.zval[o] = redc(r, p, pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  eval_report_bad(P, w.slot, pt, live, bad);
}

// LDS words of a grouped eval block (K lanes per pair, 64/K pairs).
__host__ __device__ inline int eval_group_lds_words(const DevProblem& P, int K) {
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  return P.CS + 2 * nm1 * (64 / K);
}

// Lanes of one wave meet here: LDS operations of a wave execute in program
// order, so the fences only keep the compiler from moving memory operations
// across this point.
struct WaveSync {
  __device__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// One wave, K lanes per (prime, point) pair: 64/K consecutive points of one
// prime.  Lane l of a pair evaluates rows j = 4q + l + K r (r < 4/K) of every
// row group q, so all lanes walk the same group degrees; the columns hold pair
// q at LDS word q + j (64/K), which makes the K lanes' accesses to one j-slice
// conflict-free.  The K lanes then run ures_group on the shared columns.
template <int K>
__device__ inline void stage_eval_ures_group(const DevProblem& P, const DevTables& T, const WorkItem& w,
                                             uint32_t* lds) {
  constexpr int PB = 64 / K;            // pairs per block
  constexpr int R = kRowGroup / K;      // rows of a group per lane
  constexpr int NG = (R == 1) ? 2 : 1;  // groups per Horner pass (four chains per lane)
  const int lane = threadIdx.x;
  const int l = lane / PB, q = lane % PB;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv;
  uint32_t* tile = lds;
  {
    const uint4* src = reinterpret_cast<const uint4*>(P.resid + static_cast<size_t>(w.slot) * P.CS);
    uint4* dst = reinterpret_cast<uint4*>(tile);
    for (int t = lane; t < P.CS / 4; t += 64) dst[t] = src[t];
  }
  __syncthreads();

  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  uint32_t* cols = lds + P.CS;
  Column<PB> A{cols + q};
  Column<PB> B{cols + nm1 * PB + q};
  const int pt = w.blk * PB + q;
  const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
  const uint32_t xt = mmul(x, pc.r2, p, pinv);

  const int gf = P.myp / kRowGroup, gg = P.nyp / kRowGroup;
  const int ng = gf > gg ? gf : gg;
  for (int q0 = 0; q0 < ng; q0 += NG) {
    // chains: [group][f or g][row]; a missing group reads column l of row 0
    // (in the tile) and is never stored
    int deg[NG][2];
    const uint32_t* base[NG][2];
    int stride[2] = {P.myp, P.nyp};
    int top = -1;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int qq = q0 + gi;
      deg[gi][0] = __builtin_amdgcn_readfirstlane((qq < gf) ? P.gdeg[qq] : -1);
      deg[gi][1] = __builtin_amdgcn_readfirstlane((qq < gg) ? P.gdeg[gf + qq] : -1);
      base[gi][0] = tile + ((qq < gf) ? kRowGroup * qq : 0) + l;
      base[gi][1] = tile + P.goff + ((qq < gg) ? kRowGroup * qq : 0) + l;
      top = deg[gi][0] > top ? deg[gi][0] : top;
      top = deg[gi][1] > top ? deg[gi][1] : top;
    }
    uint32_t acc[NG][2][R];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[gi][s][r] = 0u;
    for (int i = top; i >= 0; --i) {
      uint32_t c[NG][2][R];
#pragma unroll
      for (int gi = 0; gi < NG; ++gi)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const bool on = i <= deg[gi][s];  // uniform; rows above a chain's degree add zeros
          const uint32_t* rowp = base[gi][s] + (on ? i : 0) * stride[s];
#pragma unroll
          for (int r = 0; r < R; ++r) c[gi][s][r] = on ? rowp[K * r] : 0u;
        }
      uint64_t t[NG][2][R];
#pragma unroll
      for (int gi = 0; gi < NG; ++gi)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R; ++r) t[gi][s][r] = static_cast<uint64_t>(acc[gi][s][r]) * xt + c[gi][s][r];
      uint32_t mm[NG][2][R];
#pragma unroll
      for (int gi = 0; gi < NG; ++gi)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R; ++r) mm[gi][s][r] = static_cast<uint32_t>(t[gi][s][r]) * pinv;
#pragma unroll
      for (int gi = 0; gi < NG; ++gi)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < R; ++r)
            acc[gi][s][r] = static_cast<uint32_t>((t[gi][s][r] + static_cast<uint64_t>(mm[gi][s][r]) * p) >> 32);
    }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = kRowGroup * (q0 + gi) + l + K * r;
        const uint32_t va = acc[gi][0][r], vb = acc[gi][1][r];
        if (q0 + gi < gf && j <= P.my) A[j] = umin32(va, va - p);  // Horner keeps values below 2p
        if (q0 + gi < gg && j <= P.ny) B[j] = umin32(vb, vb - p);
      }
  }
  WaveSync sync;
  sync();
  bool bad = false;
  const uint32_t r = ures_group<K>(A, B, P.my, P.ny, pc, l, &bad, sync);
  const bool live = pt <= P.E && l == 0;
  if (live) {
    const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
    P.zval[o] = redc(r, p, pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  eval_report_bad(P, w.slot, pt, live, bad);
}

// LDS words of a register-form eval block: the tile plus two scratch columns
// of NMAX + 1 entries per lane for lanes that leave the register path.
__host__ __device__ inline int eval_regs_lds_words(const DevProblem& P, int nmax) {
  return P.CS + 2 * (nmax + 1) * 64;
}

// One wave, one lane per (prime, point) pair, the two polynomials in registers
// (ures_regs): Horner as in stage_eval_ures, then the unrolled remainder
// sequence; no LDS traffic after the tile except for lanes that fall back.
template <int NMAX>
__device__ inline void stage_eval_ures_regs(const DevProblem& P, const DevTables& T, const WorkItem& w,
                                            uint32_t* lds) {
  constexpr int N = RegPoly<NMAX>::kN;
  const int lane = threadIdx.x;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv;
  uint32_t* tile = lds;
  {
    const uint4* src = reinterpret_cast<const uint4*>(P.resid + static_cast<size_t>(w.slot) * P.CS);
    uint4* dst = reinterpret_cast<uint4*>(tile);
    for (int t = lane; t < P.CS / 4; t += 64) dst[t] = src[t];
  }
  __syncthreads();
  uint32_t* cols = lds + P.CS;
  const int pt = w.blk * 64 + lane;
  const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
  const uint32_t xt = mmul(x, pc.r2, p, pinv);

  uint32_t X[N], Y[N];
  const int gf = P.myp / kRowGroup, gg = P.nyp / kRowGroup;
  const int ng = gf > gg ? gf : gg;
  const uint32_t* ftile = tile;
  const uint32_t* gtile = tile + P.goff;
#pragma unroll
  for (int q = 0; q < N / kRowGroup; ++q) {
    uint32_t a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
    if (q < ng) {
      const int df = __builtin_amdgcn_readfirstlane((q < gf) ? P.gdeg[q] : -1);
      const int dg = __builtin_amdgcn_readfirstlane((q < gg) ? P.gdeg[gf + q] : -1);
      const int dboth = df < dg ? df : dg;
      const uint32_t* fq = ftile + kRowGroup * q;
      const uint32_t* gq = gtile + kRowGroup * q;
      int i = df > dg ? df : dg;
      for (; i > dboth; --i) {
        if (i <= df) horner_step4(a, *reinterpret_cast<const uint4*>(fq + i * P.myp), xt, p, pinv);
        else horner_step4(b, *reinterpret_cast<const uint4*>(gq + i * P.nyp), xt, p, pinv);
      }
      if (i >= 0) {
        uint4 cf = *reinterpret_cast<const uint4*>(fq + i * P.myp);
        uint4 cg = *reinterpret_cast<const uint4*>(gq + i * P.nyp);
        for (; i > 0; --i) {
          const uint4 nf = *reinterpret_cast<const uint4*>(fq + (i - 1) * P.myp);
          const uint4 ngv = *reinterpret_cast<const uint4*>(gq + (i - 1) * P.nyp);
          horner_step8(a, b, cf, cg, xt, p, pinv);
          cf = nf;
          cg = ngv;
        }
        horner_step8(a, b, cf, cg, xt, p, pinv);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = kRowGroup * q + r;
      X[j] = (j <= P.my) ? umin32(a[r], a[r] - p) : 0u;  // Horner keeps values below 2p
      Y[j] = (j <= P.ny) ? umin32(b[r], b[r] - p) : 0u;
    }
  }
  bool bad = false;
  uint32_t r;
  if (P.my - P.ny > 1 || P.ny - P.my > 1) {
    // the long shapes: the values go to the lane's own two columns for the
    // first division (ures_regs_long), the chain then runs in registers
    Column<64> CA{cols + lane}, CB{cols + (NMAX + 1) * 64 + lane};
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j <= NMAX) {
        if (j <= P.my) CA[j] = X[j];
        if (j <= P.ny) CB[j] = Y[j];
      }
    r = ures_regs_long<NMAX>(CA, CB, P.my, P.ny, pc, &bad);
  } else {
    r = ures_regs<NMAX>(X, Y, P.my, P.ny, pc, &bad, Column<64>{cols + lane},
                        Column<64>{cols + (NMAX + 1) * 64 + lane});
  }
  const bool live = pt <= P.E;
  if (live) {
    const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
    P.zval[o] = redc(r, p, pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  eval_report_bad(P, w.slot, pt, live, bad);
}

// LDS words of a two-lanes-per-pair register-form block (32 pairs).
__host__ __device__ inline int eval_regs2_lds_words(const DevProblem& P, int nmax) {
  return P.CS + 2 * (nmax + 1) * 32;
}

// Exchange with the partner lane of a lane pair (lanes 2q and 2q + 1).
struct PairSwap {
  __device__ uint32_t operator()(uint32_t v) const {
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0xB1 /* quad_perm 1,0,3,2 */, 0xF,
                                                          0xF, false));
  }
};

// One wave, two lanes per (prime, point) pair (32 pairs): lane l of pair q
// evaluates rows j = 4 g + 2 r + l of every row group g and keeps row j in
// element j / 2, then the pair runs ures_regs2.
template <int NMAX>
__device__ inline void stage_eval_ures_regs2(const DevProblem& P, const DevTables& T, const WorkItem& w,
                                             uint32_t* lds) {
  constexpr int N2 = RegPoly2<NMAX>::kN;
  const int lane = threadIdx.x;
  const int l = lane & 1, q = lane >> 1;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv;
  uint32_t* tile = lds;
  {
    const uint4* src = reinterpret_cast<const uint4*>(P.resid + static_cast<size_t>(w.slot) * P.CS);
    uint4* dst = reinterpret_cast<uint4*>(tile);
    for (int t = lane; t < P.CS / 4; t += 64) dst[t] = src[t];
  }
  __syncthreads();
  uint32_t* cols = lds + P.CS;
  const int pt = w.blk * 32 + q;
  const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
  const uint32_t xt = mmul(x, pc.r2, p, pinv);

  uint32_t X[N2], Y[N2];
  const int gf = P.myp / kRowGroup, gg = P.nyp / kRowGroup;
  const int ng = gf > gg ? gf : gg;
  const uint32_t* ftile = tile;
  const uint32_t* gtile = tile + P.goff;
  // one row group per pass (rows 4 g + l and 4 g + 2 + l of f and of g: four
  // chains): first the steps where only the higher-degree polynomial's rows
  // are nonzero, then all four chains with the next row's values prefetched
#pragma unroll
  for (int gq = 0; gq < N2 / 2; ++gq) {
    uint32_t a[2] = {0u, 0u}, b[2] = {0u, 0u};
    if (gq < ng) {
      const int df = __builtin_amdgcn_readfirstlane((gq < gf) ? P.gdeg[gq] : -1);
      const int dg = __builtin_amdgcn_readfirstlane((gq < gg) ? P.gdeg[gf + gq] : -1);
      const uint32_t* fq = ftile + kRowGroup * (gq < gf ? gq : 0) + l;
      const uint32_t* gqp = gtile + kRowGroup * (gq < gg ? gq : 0) + l;
      const int dboth = df < dg ? df : dg;
      int i = df > dg ? df : dg;
      for (; i > dboth; --i) {
        if (i <= df) {
          const uint32_t* fr = fq + i * P.myp;
          horner_step2(a, fr[0], fr[2], xt, p, pinv);
        } else {
          const uint32_t* gr = gqp + i * P.nyp;
          horner_step2(b, gr[0], gr[2], xt, p, pinv);
        }
      }
      if (i >= 0) {
        const uint32_t* fr = fq + i * P.myp;
        const uint32_t* gr = gqp + i * P.nyp;
        uint32_t f0 = fr[0], f1 = fr[2], g0 = gr[0], g1 = gr[2];
        for (; i > 0; --i) {
          const uint32_t* fn = fq + (i - 1) * P.myp;
          const uint32_t* gn = gqp + (i - 1) * P.nyp;
          const uint32_t nf0 = fn[0], nf1 = fn[2], ng0 = gn[0], ng1 = gn[2];
          horner_step2x2(a, b, f0, f1, g0, g1, xt, p, pinv);
          f0 = nf0;
          f1 = nf1;
          g0 = ng0;
          g1 = ng1;
        }
        horner_step2x2(a, b, f0, f1, g0, g1, xt, p, pinv);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int k = 2 * gq + r;  // element: row 4 gq + 2 r + l
      const int j = 2 * k + l;
      X[k] = (gq < gf && j <= P.my) ? umin32(a[r], a[r] - p) : 0u;
      Y[k] = (gq < gg && j <= P.ny) ? umin32(b[r], b[r] - p) : 0u;
    }
  }
  bool bad = false;
  const uint32_t r = ures_regs2<NMAX>(X, Y, P.my, P.ny, l, pc, &bad, Column<32>{cols + q},
                                      Column<32>{cols + (NMAX + 1) * 32 + q}, PairSwap(), WaveSync());
  const bool live = pt <= P.E && l == 0;
  if (live) {
    const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
    P.zval[o] = redc(r, p, pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  eval_report_bad(P, w.slot, pt, live, bad);
}

// ------------------------------------- eval on the matrix cores + ures_regs2
// The values f_j(x_k) = sum_i c_ij x_k^i mod p of 32 points and every row j
// form the product of the power matrix V[k][i] = x_k^i mod p with the residue
// matrix C[i][j] (i < 32: the K dimension).  Both split into five 7-bit digits
// (non-negative int8 operands); the digit products V_a C_b accumulate on the
// matrix cores into the nine anti-diagonal sums S_s = sum_{a+b=s} V_a C_b,
// each below 5 * 32 * 127^2 < 2^22, and
//   f_j(x_k) R mod p = REDC(sum_s S_s (2^{7s} R^2 mod p))
// (a sum below 9 * 2^22 * p < p 2^32).  Tiles of 16 points x 16 rows;
// lane l of a 16x16x32 product holds A row l mod 16 (a point) and B column
// l mod 16 (a row) for the K slice 8 (l / 16) .. 8 (l / 16) + 7, and gets the
// outputs [4 (l / 16) + r][l mod 16], r < 4.  The values go through LDS into
// the lane-pair layout of ures_regs2 (the same as stage_eval_ures_regs2).
typedef int ev_v4i __attribute__((ext_vector_type(4)));
// LDS: the values [poly][point][row] (odd row stride), and in the same words
// the two scratch columns per pair of the restart path (read only after the
// values of the restarting pairs are back in registers).
__host__ __device__ inline int eval_mfma_row_stride(const DevProblem& P) {
  return ((P.my > P.ny ? P.my : P.ny) + 1) | 1;
}
__host__ __device__ inline int eval_mfma_lds_words(const DevProblem& P, int nmax, int kl) {
  const int pts = 64 / kl;
  const int vals = 2 * pts * eval_mfma_row_stride(P), cols = 2 * (nmax + 1) * pts;
  return vals > cols ? vals : cols;
}

// KL lanes per (prime, point) pair: 64 / KL points per wave (4 / KL tiles of
// 16), then the register form's remainder sequence -- one lane per pair
// (ures_regs_generic) or a lane pair (ures_regs2_generic) -- without per-step
// branches; a pair that leaves the generic pattern starts over from its values
// in LDS with the general column code.
template <int NMAX, int KL>
__device__ inline void stage_eval_ures_mfma(const DevProblem& P, const DevTables& T, const WorkItem& w,
                                            uint32_t* lds) {
  constexpr int PTS = 64 / KL, H = PTS / 16;
  const int lane = threadIdx.x;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv;
  const int SR = eval_mfma_row_stride(P);
  uint32_t* Fv[2] = {lds, lds + PTS * SR};
  uint32_t* cols = lds;  // restart path only

  // B operands (digit fragments of the residues), one group per 16-row tile
  // of f, then of g; the next group's loads are issued a group ahead
  typedef const __attribute__((address_space(1))) uint64_t* gptr;  // global loads (not flat)
  const gptr dg = (gptr)(P.dig + static_cast<size_t>(w.slot) * P.dfr * 64);
  const int ng = P.dRTf + P.dRTg;
  auto frag = [&](int gi, int b) {
    const int f = gi < P.dRTf ? b * P.dRTf + gi : kDigits * P.dRTf + b * P.dRTg + (gi - P.dRTf);
    return dg[static_cast<size_t>(f) * 64 + lane];
  };
  uint64_t Bn[kDigits];
#pragma unroll
  for (int b = 0; b < kDigits; ++b) Bn[b] = frag(0, b);
  __builtin_amdgcn_sched_barrier(0);  // issue the loads here, not next to their use

  // A operands: digit a of x_k^(8 g + e), e < 8, for the point k = lane mod 16
  // of each 16-point tile h and the K slice g = lane / 16
  uint64_t A[H][kDigits];
  const int g = lane >> 4;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int pt = w.blk * PTS + 16 * h + (lane & 15);
    const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
    const uint32_t xt = mmul(x, pc.r2, p, pinv);
    const uint32_t x2 = mmul(xt, xt, p, pinv), x4 = mmul(x2, x2, p, pinv), x8 = mmul(x4, x4, p, pinv);
    const uint32_t x16 = mmul(x8, x8, p, pinv), x24 = mmul(x16, x8, p, pinv);
    uint32_t pw = g == 0 ? pc.r1 : g == 1 ? x8 : g == 2 ? x16 : x24;
    uint32_t v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v[e] = redc(pw, p, pinv);  // x^(8 g + e) mod p
      if (e < 7) pw = mmul(pw, xt, p, pinv);
    }
#pragma unroll
    for (int a = 0; a < kDigits; ++a) {
      uint32_t lo = 0u, hi = 0u;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        lo |= ((v[e] >> (7 * a)) & 127u) << (8 * e);
        hi |= ((v[e + 4] >> (7 * a)) & 127u) << (8 * e);
      }
      A[h][a] = (static_cast<uint64_t>(hi) << 32) | lo;
    }
  }
  // recombination weights 2^(7 s) R^2 mod p
  uint32_t wsum[2 * kDigits - 1];
  wsum[0] = pc.r2;
  const uint32_t t128 = mmul(128u, pc.r2, p, pinv);
#pragma unroll
  for (int s = 1; s < 2 * kDigits - 1; ++s) wsum[s] = mmul(wsum[s - 1], t128, p, pinv);

  for (int gi = 0; gi < ng; ++gi) {
    uint64_t B[kDigits];
#pragma unroll
    for (int b = 0; b < kDigits; ++b) B[b] = Bn[b];
    if (gi + 1 < ng) {
#pragma unroll
      for (int b = 0; b < kDigits; ++b) Bn[b] = frag(gi + 1, b);
    }
    __builtin_amdgcn_sched_barrier(0);
    const int gp = gi >= P.dRTf ? 1 : 0, rt = gp ? gi - P.dRTf : gi;
    uint32_t* F = Fv[gp];
    const int row = 16 * rt + (lane & 15);
    const bool keep = row <= (gp ? P.ny : P.my);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      ev_v4i S[2 * kDigits - 1];
#pragma unroll
      for (int s = 0; s < 2 * kDigits - 1; ++s) S[s] = ev_v4i{0, 0, 0, 0};
#pragma unroll
      for (int a = 0; a < kDigits; ++a)
#pragma unroll
        for (int b = 0; b < kDigits; ++b)
          S[a + b] = __builtin_amdgcn_mfma_i32_16x16x32_i8(static_cast<long>(A[h][a]), static_cast<long>(B[b]),
                                                           S[a + b], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        uint64_t t = 0;
#pragma unroll
        for (int s = 0; s < 2 * kDigits - 1; ++s) t += static_cast<uint64_t>(static_cast<uint32_t>(S[s][r])) * wsum[s];
        if (keep) F[(16 * h + 4 * g + r) * SR + row] = redc(t, p, pinv);
      }
    }
  }
  WaveSync()();
  // x-degree 32: the products cover x-powers 0..31; f_j(x) R += c_{32,j} x^32 R
  // on the vector ALUs, from the residue tile (c R^2) and x^32 in normal form
  if (P.rowf > 32 || P.rowg > 32) {
    const int ptq = w.blk * PTS + (lane < PTS ? lane : 0);
    const uint32_t xq = static_cast<uint32_t>(P.origin + (ptq < P.E ? ptq : P.E));
    uint32_t x32 = mmul(xq, pc.r2, p, pinv);
#pragma unroll
    for (int s = 0; s < 5; ++s) x32 = mmul(x32, x32, p, pinv);
    x32 = redc(x32, p, pinv);  // x^32 of local point `lane`, normal form
    const uint32_t* rs = P.resid + static_cast<size_t>(w.slot) * P.CS;
    for (int gp = 0; gp < 2; ++gp) {
      if ((gp ? P.rowg : P.rowf) <= 32) continue;
      const int rows = gp ? P.ny + 1 : P.my + 1;
      const uint32_t* top = rs + (gp ? P.goff + 32 * P.nyp : 32 * P.myp);
      const int n = PTS * rows;
      for (int t0 = 0; t0 < n; t0 += 64) {  // every lane takes part in each shuffle
        const int t = t0 + lane;
        const int q = (t < n) ? t / rows : 0;
        const uint32_t xv = static_cast<uint32_t>(__shfl(static_cast<int>(x32), q, 64));
        if (t < n) {
          const int j = t - q * rows;
          uint32_t* v = Fv[gp] + q * SR + j;
          *v = maddm(*v, mmul(top[j], xv, p, pinv), p);
        }
      }
    }
    WaveSync()();
  }

  bool ok, bad;
  uint32_t r;
  int pt;
  bool live;
  if constexpr (KL == 2) {
    constexpr int N2 = RegPoly2<NMAX>::kN;
    const int l = lane & 1, q = lane >> 1;
    pt = w.blk * PTS + q;
    live = pt <= P.E && l == 0;
    uint32_t X[N2], Y[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int j = 2 * k + l;
      X[k] = (j <= P.my) ? Fv[0][q * SR + j] : 0u;
      Y[k] = (j <= P.ny) ? Fv[1][q * SR + j] : 0u;
    }
    r = ures_regs2_generic<NMAX>(X, Y, P.my, P.ny, l, pc, &ok, &bad, PairSwap());
    if (!ok) {
#pragma unroll
      for (int k = 0; k < N2; ++k) {
        const int j = 2 * k + l;
        X[k] = (j <= P.my) ? Fv[0][q * SR + j] : 0u;
        Y[k] = (j <= P.ny) ? Fv[1][q * SR + j] : 0u;
      }
      WaveSync()();  // every restarting pair has its values before the columns overwrite them
      r = ures2_columns<NMAX>(X, Y, P.my, P.ny, l, pc, Column<32>{cols + q},
                              Column<32>{cols + (NMAX + 1) * 32 + q}, PairSwap(), WaveSync());
    }
  } else if (P.my - P.ny > 1 || P.ny - P.my > 1) {
    // the long shapes: first division on the lane's own value rows, then the
    // branch-free chain in registers (ures_regs_long); no other lane's rows are touched
    pt = w.blk * PTS + lane;
    live = pt <= P.E;
    r = ures_regs_long<NMAX>(Column<1>{Fv[0] + lane * SR}, Column<1>{Fv[1] + lane * SR}, P.my, P.ny, pc, &bad);
  } else {
    constexpr int N = RegPoly<NMAX>::kN;
    pt = w.blk * PTS + lane;
    live = pt <= P.E;
    uint32_t X[N], Y[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      X[j] = (j <= P.my) ? Fv[0][lane * SR + j] : 0u;
      Y[j] = (j <= P.ny) ? Fv[1][lane * SR + j] : 0u;
    }
    r = ures_regs_generic<NMAX>(X, Y, P.my, P.ny, pc, &ok, &bad);
    if (!ok) {
      // the restarting lanes read their values before any column is written
      uint32_t va[NMAX + 1], vb[NMAX + 1];
#pragma unroll
      for (int j = 0; j <= NMAX; ++j) {
        va[j] = (j <= P.my) ? Fv[0][lane * SR + j] : 0u;
        vb[j] = (j <= P.ny) ? Fv[1][lane * SR + j] : 0u;
      }
      WaveSync()();
      Column<64> CA{cols + lane}, CB{cols + (NMAX + 1) * 64 + lane};
#pragma unroll
      for (int j = 0; j <= NMAX; ++j) {
        CA[j] = va[j];
        CB[j] = vb[j];
      }
      bool b2 = false;
      r = ures_formal(CA, CB, P.my, P.ny, pc, &b2);
    }
  }
  if (live) {
    const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
    P.zval[o] = redc(r, p, pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  eval_report_bad(P, w.slot, pt, live, bad);
}

// ------------------------------------------------ eval + Schur (Sec. 4.1)
// The univariate resultant as the determinant of the Sylvester matrix S
// (n_y rows of f's coefficients, then m_y rows of g's), triangularised by the
// generalised Schur algorithm on its displacement generators.  With K the
// down-shift inside each of the two row blocks and Z the column shift,
//   S - K S Z^T = G B^T,  G = [e_0, e_n],  B = [row 0 of S, row n of S],
// a rank-2 displacement (a single generator when one block is empty).  Step
// k reads the pivot row (g0, b0) of the current generators, d = g0 . b0, and
// forms the generators of the Schur complement without divisions:
//   G' = [ g0_1 G_0 - g0_0 G_1 ,  (f d e_0 + K' G b0) ],
//   B' = [ b0_1 B_0 - b0_0 B_1 ,  d e_0 + Z' (B g0) ],
// which represent d times the complement of the represented matrix; so the
// pivots of S are d_k / sigma_k with sigma_{k+1} = d_k sigma_k, and
// det S = prod d_k / prod sigma_k (one inversion at the end).  (f = 1 when
// rows k and k+1 lie in the same block; K' shifts inside blocks.)  A zero
// pivot before the last step (a vanishing leading minor) ends the recursion:
// the point then goes through the remainder sequence, as do bad points and
// problems with an empty block.
//
// One wave per (prime, point); lane l holds row l of both generators (degree
// sum m_y + n_y <= 64); the points of a block (kSchurPts) run one after the
// other over the prime's tile, staged once.  Lane j evaluates the
// coefficients a_{m-j} = f_{m-j}(x_i) and b_{n-j} = g_{n-j}(x_i).
constexpr int kSchurPts = 16;
constexpr int kSchurMaxR = 64;
__host__ __device__ inline int eval_schur_lds_words(const DevProblem& P) {
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  return P.CS + 2 * nm1;
}

__device__ inline void stage_eval_schur(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  const int lane = threadIdx.x;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  uint32_t* tile = lds;
  const uint32_t* src = P.resid + static_cast<size_t>(w.slot) * P.CS;
  for (int t = lane; t < P.CS; t += 64) tile[t] = src[t];
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  uint32_t* colA = lds + P.CS;  // columns of the one-lane fallback
  uint32_t* colB = colA + nm1;
  __syncthreads();
  const int m = P.my, n = P.ny, r = m + n;
  const bool two = n > 0 && m > 0;
  const int nxa = P.rowf, nxb = P.rowg;
  const int nx = nxa > nxb ? nxa : nxb;
  const int ra = m - lane, rb = n - lane;  // this lane's rows of f and g
  for (int s = 0; s < kSchurPts; ++s) {
    const int pt = w.blk * kSchurPts + s;
    if (pt > P.E) break;
    const uint32_t x = static_cast<uint32_t>(P.origin + pt);
    const uint32_t xt = mmul(x, pc.r2, p, pinv);
    // Horner in x over every power (zero coefficients beyond a row's degree);
    // values stay below 2p as in horner_step4
    auto hstep = [&](uint32_t acc, uint32_t c) {
      const uint64_t t = static_cast<uint64_t>(acc) * xt + c;
      const uint32_t mq = static_cast<uint32_t>(t) * pinv;
      return static_cast<uint32_t>((t + static_cast<uint64_t>(mq) * p) >> 32);
    };
    uint32_t av = 0u, bv = 0u;
    for (int i = nx - 1; i >= 0; --i) {
      av = hstep(av, (ra >= 0 && i < nxa) ? tile[i * P.myp + ra] : 0u);
      bv = hstep(bv, (rb >= 0 && i < nxb) ? tile[P.goff + i * P.nyp + rb] : 0u);
    }
    av = umin32(av, av - p);
    bv = umin32(bv, bv - p);
    const uint32_t lcf = __builtin_amdgcn_readlane(av, 0), lcg = __builtin_amdgcn_readlane(bv, 0);
    bool bad = (lcf == 0u) || (lcg == 0u);
    uint32_t res = 0u;
    bool done = false;
    if (!bad && two && r <= kSchurMaxR) {
      uint32_t G0 = (lane == 0) ? one : 0u, G1 = (lane == n) ? one : 0u;
      uint32_t B0 = av, B1 = bv;  // S[0][l] = a_{m-l}, S[n][l] = b_{n-l}
      uint32_t num = one, den = one, sigma = one;
      done = true;
      for (int k = 0; k < r; ++k) {
        const uint32_t ga = __builtin_amdgcn_readlane(G0, k), gb = __builtin_amdgcn_readlane(G1, k);
        const uint32_t ba = __builtin_amdgcn_readlane(B0, k), bb = __builtin_amdgcn_readlane(B1, k);
        const uint32_t d = mmulsub(ga, ba, mneg(gb, p), bb, p, pinv);  // ga ba + gb bb
        num = mmul(num, d, p, pinv);
        den = mmul(den, sigma, p, pinv);
        if (k == r - 1) break;
        if (d == 0u) {  // a vanishing leading minor
          done = false;
          break;
        }
        const uint32_t xg = mmulsub(gb, G0, ga, G1, p, pinv);
        const uint32_t yb = mmulsub(bb, B0, ba, B1, p, pinv);
        const uint32_t c = mmulsub(G0, ba, mneg(G1, p), bb, p, pinv);  // G b0
        const uint32_t u = mmulsub(ga, B0, mneg(gb, p), B1, p, pinv);  // B g0
        const uint32_t cprev = static_cast<uint32_t>(__shfl_up(static_cast<int>(c), 1, 64));
        const uint32_t uprev = static_cast<uint32_t>(__shfl_up(static_cast<int>(u), 1, 64));
        if (lane > k) {
          G0 = xg;
          G1 = (lane == n) ? 0u : ((lane == k + 1) ? d : cprev);
          B0 = yb;
          B1 = (lane == k + 1) ? d : uprev;
        }
        sigma = mmul(sigma, d, p, pinv);
      }
      if (done) res = (num == 0u) ? 0u : mmul(num, minv(den, one, p, pinv), p, pinv);
    }
    if (!done) {
      // remainder sequence in lane 0 on the evaluated coefficients
      if (ra >= 0) colA[ra] = av;
      if (rb >= 0) colB[rb] = bv;
      WaveSync()();
      if (lane == 0) res = ures_formal(Column<1>{colA}, Column<1>{colB}, m, n, pc, &bad);
      WaveSync()();
    }
    if (lane == 0) {
      const size_t o = static_cast<size_t>(w.slot) * (P.E + 1) + pt;
      P.zval[o] = redc(res, p, pinv);
      P.zbad[o] = bad ? 1 : 0;
    }
    eval_report_bad(P, w.slot, pt, lane == 0, bad);
  }
}

// LDS words of the evaluation launch for the problem's layout.
__host__ __device__ inline int eval_stage_lds_words(const DevProblem& P) {
  if (P.schur) return eval_schur_lds_words(P);
  if (P.evmf) return eval_mfma_lds_words(P, P.regn, P.evk);
  if (P.evk == 2 && P.regn) return eval_regs2_lds_words(P, P.regn);
  if (P.evk > 1) return eval_group_lds_words(P, P.evk);
  return P.regn ? eval_regs_lds_words(P, P.regn) : eval_lds_words(P);
}

// Evaluation layouts; each has a kernel of its own (own register budget).
enum : int {
  kEvBase = 0,  // one lane per pair, LDS columns
  kEvG2,        // two lanes per pair, LDS columns
  kEvG4,        // four lanes per pair, LDS columns
  kEvR8, kEvR16, kEvR24, kEvR32,  // one lane per pair, registers (degree bound)
  kEvP8, kEvP16, kEvP24, kEvP32,  // two lanes per pair, registers
  kEvSchur,     // one wave per pair, Schur algorithm on the Sylvester generators
  kEvM8, kEvM16, kEvM24, kEvM32,  // two lanes per pair, registers, Horner sums on the matrix cores
  kEvQ8, kEvQ16, kEvQ24, kEvQ32,  // one lane per pair, registers, Horner sums on the matrix cores
  kEvNum
};
__host__ __device__ inline int eval_variant(const DevProblem& P) {
  if (P.schur) return kEvSchur;
  const int r = P.regn == 8 ? 0 : P.regn == 16 ? 1 : P.regn == 24 ? 2 : 3;
  if (P.evmf) return (P.evk == 2 ? kEvM8 : kEvQ8) + r;
  if (P.evk == 2 && P.regn) return kEvP8 + r;
  if (P.evk == 2) return kEvG2;
  if (P.evk == 4) return kEvG4;
  if (P.regn) return kEvR8 + r;
  return kEvBase;
}
template <int V>
__device__ inline void stage_eval_variant(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  if constexpr (V == kEvBase) stage_eval_ures(P, T, w, lds);
  else if constexpr (V == kEvG2) stage_eval_ures_group<2>(P, T, w, lds);
  else if constexpr (V == kEvG4) stage_eval_ures_group<4>(P, T, w, lds);
  else if constexpr (V >= kEvR8 && V <= kEvR32) stage_eval_ures_regs<8 * (V - kEvR8 + 1)>(P, T, w, lds);
  else if constexpr (V == kEvSchur) stage_eval_schur(P, T, w, lds);
  else if constexpr (V >= kEvQ8) stage_eval_ures_mfma<8 * (V - kEvQ8 + 1), 1>(P, T, w, lds);
  else if constexpr (V >= kEvM8) stage_eval_ures_mfma<8 * (V - kEvM8 + 1), 2>(P, T, w, lds);
  else stage_eval_ures_regs2<8 * (V - kEvP8 + 1)>(P, T, w, lds);
}

// Dispatch on the problem's evaluation layout (block-uniform).  With
// use_regs = false the register form is skipped (the LDS-column code computes
// the same values), which keeps the register budget of a kernel that also
// runs the other stages small.
template <bool use_regs = true>
__device__ inline void stage_eval(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  if (use_regs && P.evk == 2) {
    switch (P.regn) {
      case 8: stage_eval_ures_regs2<8>(P, T, w, lds); return;
      case 16: stage_eval_ures_regs2<16>(P, T, w, lds); return;
      case 24: stage_eval_ures_regs2<24>(P, T, w, lds); return;
      case 32: stage_eval_ures_regs2<32>(P, T, w, lds); return;
      default: break;
    }
  }
  switch (P.evk) {
    case 2: stage_eval_ures_group<2>(P, T, w, lds); return;
    case 4: stage_eval_ures_group<4>(P, T, w, lds); return;
    default: break;
  }
  if (!use_regs) {
    stage_eval_ures(P, T, w, lds);
    return;
  }
  switch (P.regn) {
    case 8: stage_eval_ures_regs<8>(P, T, w, lds); return;
    case 16: stage_eval_ures_regs<16>(P, T, w, lds); return;
    case 24: stage_eval_ures_regs<24>(P, T, w, lds); return;
    case 32: stage_eval_ures_regs<32>(P, T, w, lds); return;
    default: stage_eval_ures(P, T, w, lds); return;
  }
}

// ------------------------------------------------------------ interpolation

// The consecutive fast path applies when the D+1 points used are origin ..
// origin + D: always with formal-degree values, otherwise when none of them
// was flagged bad (the evaluation stage sets a per-prime flag).  It
// interpolates in t = x - origin; for a shifted origin the Newton stage takes
// the result back to x.
__device__ inline bool fast_prime(const DevProblem& P, int slot) {
  if (P.newton_all) return false;
  if (P.formal) return true;
  return __builtin_amdgcn_readfirstlane(P.status[2 + P.np + slot]) == 0;
}

// Newton forward differences at 0..D as a convolution, one i-chunk of it:
//   a_k = Delta^k z_0 / k! = sum_{i<=k} (z_i / i!) ((-1)^(k-i) / (k-i)!)
// Each thread owns one k; the chunk's partial sum is stored unreduced
// (below p 2^32; REDC of the sum over chunks is a_k).
__device__ inline void stage_interp_conv(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  if (!fast_prime(P, w.slot)) return;
  const int g = P.pidx[w.slot];
  const PrimeConst pc = T.pc[g];
  const uint32_t p = pc.p, pinv = pc.pinv;
  const uint32_t* ifact = T.ifact + static_cast<size_t>(g) * T.kstride;
  const int nt = blockDim.x;
  const int k0 = w.blk * nt;
  const int kmax = (k0 + nt - 1 < P.D) ? k0 + nt - 1 : P.D;
  const int ib = w.sub * P.cchunk;
  const int ie = (ib + P.cchunk - 1 < kmax) ? ib + P.cchunk - 1 : kmax;  // last i used by this block
  // alpha_i = z_i / i! for i in [ib, ie]; beta_t = (-1)^t / t! R for t in [k0 - ie, kmax - ib]
  const int tb = (k0 - ie > 0) ? k0 - ie : 0;
  const int te = kmax - ib;
  const int na = ie - ib + 1 > 0 ? ie - ib + 1 : 0;
  const int nb = te - tb + 1 > 0 ? te - tb + 1 : 0;
  uint32_t* alpha = lds;
  uint32_t* beta = lds + na;
  const uint32_t* z = P.zval + static_cast<size_t>(w.slot) * (P.E + 1);
  // alpha then beta as one index range, two entries per thread per pass so
  // that their loads are in flight together
  for (int base = threadIdx.x; base < na + nb; base += 2 * nt) {
    uint32_t zv[2], fv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = base + u * nt;
      const int ec = e < na + nb ? e : na + nb - 1;
      const int idx = ec < na ? ib + ec : tb + (ec - na);
      fv[u] = ifact[idx];
      zv[u] = ec < na ? z[idx] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = base + u * nt;
      if (e < na) {
        alpha[e] = mmul(zv[u], fv[u], p, pinv);
      } else if (e < na + nb) {
        const int t = tb + (e - na);
        beta[e - na] = (t & 1) ? mneg(fv[u], p) : fv[u];
      }
    }
  }
  __syncthreads();
  const int k = k0 + threadIdx.x;
  if (k > P.D) return;
  const int iend = (ie < k) ? ie : k;
  uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  int i = ib;
  for (; i + 3 <= iend; i += 4) {
    c0 = mac_fold(c0, alpha[i - ib], beta[k - i - tb], p);
    c1 = mac_fold(c1, alpha[i + 1 - ib], beta[k - i - 1 - tb], p);
    c2 = mac_fold(c2, alpha[i + 2 - ib], beta[k - i - 2 - tb], p);
    c3 = mac_fold(c3, alpha[i + 3 - ib], beta[k - i - 3 - tb], p);
  }
  for (; i <= iend; ++i) c0 = mac_fold(c0, alpha[i - ib], beta[k - i - tb], p);
  const uint64_t acc = add_fold(add_fold(c0, c1, p), add_fold(c2, c3, p), p);
  P.aconv[(static_cast<size_t>(w.sub) * P.np + w.slot) * (P.D + 1) + k] = acc;
}

// Falling-factorial basis -> monomials, one k-chunk of the sum
//   c_j = sum_{k >= j} a_k s(k, j)
// written as partial sums per chunk (REDC of the sum over the chunks that
// reach j is c_j).  The context keeps only every kCkpt-th row of the Stirling
// triangle.  The rows k0 .. k0 + kCkpt - 1 after a checkpoint row k0 follow
// from it by x^(k0 + t) = x^(k0) (x - k0)^(t) (falling factorials), so their
// contribution to c_j is a short convolution with that row:
//   sum_t a_{k0+t} s(k0 + t, j) = sum_{i < kCkpt} h_i s(k0, j - i),
// h = the monomial coefficients of sum_t a_{k0+t} (x - k0)^(t).  A segment's h
// is expanded once by Horner's rule (h <- h (x - k0 - t) + a_{k0+t}, one
// coefficient per lane of a half wave) into `hseg`; the basis change then
// streams only checkpoint rows: one column per thread, the row's window and
// the members' h in LDS.

// a_k = REDC(sum of the convolution chunks that reach k) for k in [kb, ke]
// (0 beyond the problem's degree bound), into dst[k - kb].
__device__ inline void load_newton_coeffs(const DevProblem& P, int slot, const PrimeConst& pc, int kb, int ke,
                                          uint32_t* dst) {
  const uint32_t p = pc.p;
  const uint64_t* ap = P.aconv + static_cast<size_t>(slot) * (P.D + 1);
  const size_t astride = static_cast<size_t>(P.np) * (P.D + 1);
  for (int k = kb + static_cast<int>(threadIdx.x); k <= ke; k += blockDim.x) {
    uint32_t v = 0u;
    if (k <= P.D) {
      const int nch = k / P.cchunk + 1;
      uint64_t q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = ap[(u < nch ? u : nch - 1) * astride + k];
      uint64_t sacc = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nch) sacc = add_fold(sacc, q[u], p);
      for (int ch = 8; ch < nch; ++ch) sacc = add_fold(sacc, ap[ch * astride + k], p);
      v = redc(sacc, p, pc.pinv);
    }
    dst[k - kb] = v;
  }
}

// h of the segment starting at k0 (rows k0 .. min(k0 + kCkpt - 1, ke), a_k at
// a[k - kb]) by one half wave: lane i of the half gets h_i.
__device__ inline uint32_t segment_h(const uint32_t* a, int kb, int k0, int ke, const PrimeConst& pc) {
  const uint32_t p = pc.p, pinv = pc.pinv;
  const int i = threadIdx.x & (kCkpt - 1);
  uint32_t h = 0u;
  uint32_t ct = mmul(static_cast<uint32_t>(k0 + kCkpt - 1), pc.r2, p, pinv);  // (k0 + t) R mod p
  for (int t = kCkpt - 1; t >= 0; --t) {
    const int k = k0 + t;
    const uint32_t av = (k <= ke) ? a[k - kb] : 0u;
    const uint32_t prev = static_cast<uint32_t>(__shfl_up(static_cast<int>(h), 1, kCkpt));
    h = msubm(i > 0 ? prev : 0u, mmul(h, ct, p, pinv), p);
    if (i == 0) h = maddm(h, av, p);
    ct = msubm(ct, pc.r1, p);
  }
  return h;
}

// The segments' h of one problem and prime: item (problem, slot, block of
// kHsegRows rows), one segment per half wave.
constexpr int kHsegRows = 256;
__device__ inline void stage_interp_hseg(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  if (!fast_prime(P, w.slot)) return;
  const PrimeConst pc = T.pc[P.pidx[w.slot]];
  const int kb = w.blk * kHsegRows;
  const int ke = (kb + kHsegRows - 1 < P.D) ? kb + kHsegRows - 1 : P.D;
  load_newton_coeffs(P, w.slot, pc, kb, ke, lds);
  __syncthreads();
  const int k0 = kb + kCkpt * (static_cast<int>(threadIdx.x) / kCkpt);
  if (k0 > ke) return;
  const uint32_t h = segment_h(lds, kb, k0, ke, pc);
  P.hseg[static_cast<size_t>(w.slot) * P.hstride + k0 + (threadIdx.x & (kCkpt - 1))] = h;
}

// Rows [k1, ke] (k1 a multiple of kCkpt) into the partial sums acc[m] of
// column j0 + threadIdx.x for G members; the block's threads are its columns.
// h of member m for the segment at k0: hsrc[m][k0 + i] (HG), or expanded here
// from a_k at lds_a[k - kb] (G = 1).  LDS: lh (G kCkpt words), lw (blockDim + kCkpt - 1).
template <int GM, bool HG>
__device__ inline void basis_block(const uint32_t* S, int j0, int k1, int ke, int kb, int G,
                                   const uint32_t* const* hsrc, const int* hmax, const uint32_t* lds_a,
                                   const PrimeConst& pc, uint32_t* lh, uint32_t* lw, uint64_t (&acc)[GM]) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const uint32_t p = pc.p;
  // the next segment's h (HG: one value per thread, nt >= GM kCkpt) and row
  // window (two values per thread, nt >= kCkpt - 1) are loaded into registers
  // while the current segment is convolved
  uint32_t nh = 0u, nw0 = 0u, nw1 = 0u;
  auto fetch = [&](int k0) {
    if constexpr (HG) {
      const int m = tid / kCkpt, u = tid & (kCkpt - 1);
      nh = 0u;
#pragma unroll
      for (int mm = 0; mm < GM; ++mm)
        if (mm == m && mm < G && k0 <= hmax[mm]) nh = hsrc[mm][k0 + u];  // beyond a member's bound: h = 0
    }
    const uint32_t* row = S + ckpt_rowoff(k0 / kCkpt);
    const int ja = j0 - (kCkpt - 1) + tid, jb = ja + nt;
    nw0 = (ja >= 0 && ja <= k0) ? row[ja] : 0u;
    nw1 = (tid < kCkpt - 1 && jb >= 0 && jb <= k0) ? row[jb] : 0u;
  };
  if (k1 <= ke) fetch(k1);
  for (int k0 = k1; k0 <= ke; k0 += kCkpt) {
    if constexpr (HG) {
      if (tid < GM * kCkpt) lh[tid] = nh;
    } else {
      if (tid < kCkpt) lh[tid] = segment_h(lds_a, kb, k0, ke, pc);
    }
    lw[tid] = nw0;
    if (tid < kCkpt - 1) lw[nt + tid] = nw1;
    __syncthreads();
    if (k0 + kCkpt <= ke) fetch(k0 + kCkpt);
#pragma unroll 8
    for (int i = 0; i < kCkpt; ++i) {
      const uint32_t w = lw[tid + kCkpt - 1 - i];  // s(k0, j - i)
#pragma unroll
      for (int m = 0; m < GM; ++m)
        if (m < G) acc[m] = mac_fold(acc[m], lh[m * kCkpt + i], w, p);
    }
    __syncthreads();  // the next segment overwrites lh and lw
  }
}

// ------------------------------------- interpolation on the matrix cores
// For the problems of one prime the two triangular factors of the
// interpolation are shared matrices, so the columns of all those problems
// (and of the x and y problems alike) form one matrix product each:
//   Newton coefficients  a_k = sum_{i <= k} T(k - i) y_i,   T(d) = (-1)^d / d!,
//                        y_i = z_i / i!   (the forward differences of Sec. 4.1's
//                        consecutive points, a Toeplitz factor),
//   basis change         c_j = sum_{segments k0} sum_{i < kCkpt} s(k0, j - i) h_{k0,i}
//                        (the checkpoint rows of the Stirling triangle and the
//                        segments' polynomials h of stage_interp_hseg).
// Both have a Toeplitz operand A[row][K] = v(row - K + const); the data
// operand B holds the problems' columns as 7-bit digit planes (five digits of
// each residue), and the 16x16x32 int8 products of the five digits of each
// side accumulate the nine anti-diagonal sums S_s over the whole K range
// (each below 5 (kMmMaxD + 32) 127^2 < 2^31), recombined as in the evaluation:
//   out = sum_s S_s (2^{7s} mod p), below 9 * 2^29 p < p 2^32,
// whose REDC is the coefficient in Montgomery form (the operands are
// Montgomery representatives), written as the single chunk of aconv / cpart.

// Digit planes of one problem slot: WHICH 1, y_n = z_n ifact_n; WHICH 2, hseg
// (zero beyond D and, for the basis change, for a prime with bad points).
// Each thread writes eight consecutive entries of every plane (one 64-bit
// store per plane); item (problem, slot, block of 2048 entries).
constexpr int kDigitsPerBlock = 2048;
template <int WHICH>
__device__ inline void stage_interp_digits(const DevProblem& P, const DevTables& T, const WorkItem& w) {
  const int n0 = 8 * (w.blk * blockDim.x + threadIdx.x);
  const int Dp = P.hstride;
  if (n0 >= Dp) return;
  const int g = P.pidx[w.slot];
  uint32_t v[8];
  if constexpr (WHICH == 1) {
    const PrimeConst pc = T.pc[g];
    const uint32_t* z = P.zval + static_cast<size_t>(w.slot) * (P.E + 1);
    const uint32_t* fi = T.ifact + static_cast<size_t>(g) * T.kstride;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (n0 + e <= P.D) ? mmul(z[n0 + e], fi[n0 + e], pc.p, pc.pinv) : 0u;
  } else {
    const bool fast = fast_prime(P, w.slot);
    const uint32_t* h = P.hseg + static_cast<size_t>(w.slot) * P.hstride;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (fast && n0 + e <= P.D) ? h[n0 + e] : 0u;
  }
  uint64_t* dst = reinterpret_cast<uint64_t*>((WHICH == 1 ? P.ydig : P.hdig) +
                                              static_cast<size_t>(w.slot) * kDigits * Dp + n0);
#pragma unroll
  for (int b = 0; b < kDigits; ++b) {
    uint64_t word = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) word |= static_cast<uint64_t>((v[e] >> (7 * b)) & 127u) << (8 * e);
    dst[static_cast<size_t>(b) * (Dp / 8)] = word;
  }
}

// Item (group, 64-row set rs, column tiles ct0 .. ct0 + nct - 1 of 16 members
// each; members sorted by degree bound, largest first).  The block stages
// once, in LDS, the Toeplitz operand of its 64 rows over every K slice its
// tiles reach -- as 7-bit digit planes, reversed so that a lane's eight K
// entries are eight consecutive bytes -- and the tiles' column descriptors.
// Then wave w runs row tile rs0 + 16 w against each column tile in turn with
// no further barrier: B fragments come from the members' digit planes in
// global memory, the next slice's loads issued before the current slice's 25
// products.  Lane l's fragments: row / column l mod 16, K entries 8 (l / 16)
// .. + 7; its outputs are rows 4 (l / 16) .. + 3 of column l mod 16.
constexpr int kMmTilesMax = 16;  // column tiles per item
constexpr int kMmRunSlices = 48; // K slices per item (over its tiles), about
constexpr int kMmMaxD = 2880;    // the basis change stages 640 bytes per slice: LDS below 64 KB
struct MmCol {
  const uint8_t* b;  // the member's digit planes (plane stride Dp bytes)
  uint64_t* out;     // its sums: aconv or cpart of the slot
  int D, Dp;         // degree bound (-1: no member), plane stride
};
constexpr int kMmColBytes = kMmTilesMax * 16 * static_cast<int>(sizeof(MmCol));

// LDS bytes of the Toeplitz operand of an item: rows rs0 .. rs0 + 63, columns
// of degree bound at most tileD.
__host__ __device__ inline int mm_slices_lo(int which, int rs0) {
  return which == 1 ? 0 : (rs0 >= 31 ? (rs0 - 31) / 32 : 0);
}
__host__ __device__ inline int mm_slices_hi(int which, int rs0, int tileD) {
  return which == 1 ? ((rs0 + 63 < tileD) ? rs0 + 63 : tileD) / 32 : tileD / 32;
}
__host__ __device__ inline int mm_operand_bytes(int which, int rs0, int tileD) {
  const int lo = mm_slices_lo(which, rs0), hi = mm_slices_hi(which, rs0, tileD);
  return which == 1 ? kDigits * (32 * hi + 104) : kDigits * 128 * (hi - lo + 1);
}

template <int WHICH>
__device__ inline void stage_interp_mm(const DevProblem* probs, const StirGroup& G, const StirMember* members,
                                       const WorkItem& w, const DevTables& T, uint8_t* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const PrimeConst pc = T.pc[G.g];
  const uint32_t p = pc.p;
  const int rs0 = 64 * w.slot;      // first row of the block
  const int rw0 = rs0 + 16 * wave;  // first row of this wave's tile
  const int ct0 = w.blk, nct = w.sub & 31, tileD0 = w.sub >> 5;  // tileD0: the first tile's largest bound
  const int q = lane >> 4, r = lane & 15;
  MmCol* cols = reinterpret_cast<MmCol*>(lds);
  uint8_t* opnd = lds + kMmColBytes;
  const int s_lo = mm_slices_lo(WHICH, rs0), s_hi = mm_slices_hi(WHICH, rs0, tileD0);

  // column descriptors
  for (int t = tid; t < 16 * nct; t += blockDim.x) {
    const int mi = 16 * ct0 + t;
    MmCol c{nullptr, nullptr, -1, 0};
    if (mi < G.count) {
      const StirMember M = members[G.first + mi];
      const DevProblem& Pm = probs[M.prob];
      c.D = Pm.D;
      c.Dp = Pm.hstride;
      c.b = (WHICH == 1 ? Pm.ydig : Pm.hdig) + static_cast<size_t>(M.slot) * kDigits * Pm.hstride;
      c.out = (WHICH == 1 ? Pm.aconv : Pm.cpart) + static_cast<size_t>(M.slot) * (Pm.D + 1);
    }
    cols[t] = c;
  }
  // the Toeplitz operand: WHICH 1, one reversed vector R[y] = T(rs0 + 63 - y),
  // T(x) = (-1)^x / x! for 0 <= x <= maxD; WHICH 2, per slice s a window
  // W_s[y] = s(32 s, rs0 + 63 - y) for y < 128 (zero outside 0 .. 32 s)
  if constexpr (WHICH == 1) {
    const int Lr = 32 * s_hi + 104;
    const uint32_t* ifact = T.ifact + static_cast<size_t>(G.g) * T.kstride;
    for (int y = tid; y < Lr; y += blockDim.x) {
      const int x = rs0 + 63 - y;
      uint32_t v = 0u;
      if (x >= 0 && x <= G.maxD) {
        const uint32_t f = ifact[x];
        v = (x & 1) ? p - f : f;
      }
#pragma unroll
      for (int b = 0; b < kDigits; ++b) opnd[b * Lr + y] = static_cast<uint8_t>((v >> (7 * b)) & 127u);
    }
  } else {
    const uint32_t* srow = T.stir + static_cast<size_t>(G.g) * T.sstride;
    const int n = (s_hi - s_lo + 1) * 128;
    for (int t = tid; t < n; t += blockDim.x) {
      const int s = s_lo + (t >> 7), y = t & 127, x = rs0 + 63 - y;
      const uint32_t v = (x >= 0 && x <= 32 * s) ? srow[ckpt_rowoff(s) + x] : 0u;
      uint8_t* pl = opnd + (s - s_lo) * kDigits * 128 + y;
#pragma unroll
      for (int b = 0; b < kDigits; ++b) pl[b * 128] = static_cast<uint8_t>((v >> (7 * b)) & 127u);
    }
  }
  uint32_t wgt[2 * kDigits - 1];  // 2^(7 s) mod p
  wgt[0] = 1u;
#pragma unroll
  for (int s = 1; s < 2 * kDigits - 1; ++s) {
    const uint64_t t = static_cast<uint64_t>(wgt[s - 1]) << 7;
    wgt[s] = static_cast<uint32_t>(t % p);
  }
  __syncthreads();

  // lane's first byte of its A fragment in the operand (plus 32 s for WHICH 1)
  const int y0 = 63 - 16 * wave - r + 8 * q;
  const int sh = (y0 & 7) * 8;
  const uint64_t* op64 = reinterpret_cast<const uint64_t*>(opnd);
  const int Lr8 = (32 * s_hi + 104) / 8;  // WHICH 1 plane stride in words
  for (int ct = 0; ct < nct; ++ct) {
    const MmCol C = cols[16 * ct + r];
    const int tileD = __builtin_amdgcn_readfirstlane(cols[16 * ct].D);  // the tile's largest degree bound
    if (rw0 > tileD) break;             // wave-uniform; later tiles have smaller bounds
    int sa, sb;
    if constexpr (WHICH == 1) {
      sa = 0;
      sb = ((rw0 + 15 < tileD) ? rw0 + 15 : tileD) / 32;  // T(k - i) = 0 for i > k
    } else {
      sa = rw0 / 32;  // s(k0, j - i) = 0 for j - i > k0: slices with k0 + 31 >= rw0
      sb = tileD / 32;
    }
    auto load_b = [&](int s, uint64_t (&Bf)[kDigits]) {
      const bool have = 32 * s <= C.D;
      const uint8_t* src = C.b + 32 * s + 8 * q;
#pragma unroll
      for (int b = 0; b < kDigits; ++b)
        Bf[b] = have ? *reinterpret_cast<const uint64_t*>(src + static_cast<size_t>(b) * C.Dp) : 0u;
    };
    ev_v4i S[2 * kDigits - 1];
#pragma unroll
    for (int s = 0; s < 2 * kDigits - 1; ++s) S[s] = ev_v4i{0, 0, 0, 0};
    uint64_t Bn[kDigits];
    load_b(sa, Bn);
    for (int s = sa; s <= sb; ++s) {
      uint64_t B[kDigits];
#pragma unroll
      for (int b = 0; b < kDigits; ++b) B[b] = Bn[b];
      if (s < sb) load_b(s + 1, Bn);
      uint64_t A[kDigits];
#pragma unroll
      for (int b = 0; b < kDigits; ++b) {
        int wi;
        if constexpr (WHICH == 1) wi = b * Lr8 + ((y0 + 32 * s) >> 3);
        else wi = ((s - s_lo) * kDigits + b) * 16 + (y0 >> 3);
        const uint64_t lo = op64[wi], hi = op64[wi + 1];
        A[b] = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
      }
#pragma unroll
      for (int a = 0; a < kDigits; ++a)
#pragma unroll
        for (int b = 0; b < kDigits; ++b)
          S[a + b] = __builtin_amdgcn_mfma_i32_16x16x32_i8(static_cast<long>(A[a]), static_cast<long>(B[b]),
                                                           S[a + b], 0, 0, 0);
    }
    if (rw0 > C.D) continue;
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int row = rw0 + 4 * q + r4;
      uint64_t t = 0;
#pragma unroll
      for (int s = 0; s < 2 * kDigits - 1; ++s) t += static_cast<uint64_t>(static_cast<uint32_t>(S[s][r4])) * wgt[s];
      if (row <= C.D) C.out[row] = t;
    }
  }
}

// LDS words of a basis-change block: members' h, the row window, and (when h
// is expanded in the block) the chunk's a_k.
__host__ __device__ inline int basis_lds_words(int members, int nthreads, int K_or_0) {
  return kCkpt * members + nthreads + kCkpt - 1 + K_or_0;
}

// One problem: item (problem, slot, block of blockDim columns, chunk).  With
// h_global the segments' h come from hseg (staged and plain schedules, after
// stage_interp_hseg); otherwise the block expands them itself (the persistent
// schedule's single-wave tasks).
template <bool h_global>
__device__ inline void stage_interp_stir(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  if (!fast_prime(P, w.slot)) return;
  const int g = P.pidx[w.slot];
  const PrimeConst pc = T.pc[g];
  const int nt = blockDim.x;
  const int kb = w.sub * P.kchunk;
  const int ke = (kb + P.kchunk - 1 < P.D) ? kb + P.kchunk - 1 : P.D;
  const int j0 = w.blk * nt;
  uint32_t* lh = lds;
  uint32_t* lw = lds + kCkpt;
  uint32_t* la = lw + nt + kCkpt - 1;
  if constexpr (!h_global) {
    load_newton_coeffs(P, w.slot, pc, kb, ke, la);
    __syncthreads();
  }
  if (j0 > ke || j0 > P.D) return;  // block-uniform: no row of the chunk reaches these columns
  // rows below j0 contribute nothing to them: start at j0's checkpoint
  const int jc = (j0 / kCkpt) * kCkpt;
  const int k1 = kb > jc ? kb : jc;
  uint64_t acc[1] = {0u};
  const uint32_t* hrow = P.hseg + static_cast<size_t>(w.slot) * P.hstride;
  const int hmax[1] = {P.D};
  basis_block<1, h_global>(T.stir + static_cast<int64_t>(g) * T.sstride, j0, k1, ke, kb, 1, &hrow, hmax, la, pc, lh,
                           lw, acc);
  const int j = j0 + static_cast<int>(threadIdx.x);
  if (j <= P.D) P.cpart[(static_cast<size_t>(w.sub) * P.np + w.slot) * (P.D + 1) + j] = acc[0];
}

// The same basis change for every member of a prime group (problems that use
// one prime): each checkpoint row is read once and convolved into every
// member's partial sums.  Item: (group, -, block of blockDim columns, k-chunk);
// all members share the chunk length (kchunk) and their rows k > D_m have h = 0.
__host__ __device__ inline int stir_group_lds_words(int count, int nthreads) {
  return basis_lds_words(count, nthreads, 0);
}

__device__ inline void stage_interp_stir_group(const DevProblem* probs, const StirGroup* groups,
                                               const StirMember* members, const DevTables& T, const WorkItem& w,
                                               uint32_t* lds) {
  const StirGroup G = groups[w.prob];
  const int nt = blockDim.x;
  const int j0 = w.blk * nt;
  const PrimeConst pc = T.pc[G.g];
  const int K = probs[members[G.first].prob].kchunk;
  const int kb = w.sub * K;
  const int ke = (kb + K - 1 < G.maxD) ? kb + K - 1 : G.maxD;
  if (j0 > ke) return;
  // the active members (degree bound reaching the chunk and the block,
  // consecutive points), compacted
  int na = 0, which[kStirGroupMax];
  for (int m = 0; m < G.count; ++m) {
    const StirMember M = members[G.first + m];
    const DevProblem& P = probs[M.prob];
    if (P.D >= kb && P.D >= j0 && fast_prime(P, M.slot)) which[na++] = m;
  }
  if (na == 0) return;  // block-uniform
  const uint32_t* hsrc[kStirGroupMax];
  int hmax[kStirGroupMax];
#pragma unroll
  for (int q = 0; q < kStirGroupMax; ++q) {
    hsrc[q] = nullptr;
    hmax[q] = -1;
    if (q < na) {
      const StirMember M = members[G.first + which[q]];
      hsrc[q] = probs[M.prob].hseg + static_cast<size_t>(M.slot) * probs[M.prob].hstride;
      hmax[q] = probs[M.prob].D;
    }
  }
  const int jc = (j0 / kCkpt) * kCkpt;
  const int k1 = kb > jc ? kb : jc;
  uint64_t acc[kStirGroupMax];
#pragma unroll
  for (int m = 0; m < kStirGroupMax; ++m) acc[m] = 0u;
  // rows k > D_m of a member are zero in its h (its a_k vanish there), and the
  // h of a member is read only for segments at or below its degree bound
  basis_block<kStirGroupMax, true>(T.stir + static_cast<int64_t>(G.g) * T.sstride, j0, k1, ke, kb, na, hsrc, hmax,
                                   nullptr, pc, lds, lds + kCkpt * kStirGroupMax, acc);
#pragma unroll
  for (int q = 0; q < kStirGroupMax; ++q)
    if (q < na) {
      const StirMember M = members[G.first + which[q]];
      const DevProblem& P = probs[M.prob];
      const int j = j0 + static_cast<int>(threadIdx.x);
      if (j <= P.D) P.cpart[(static_cast<size_t>(w.sub) * P.np + M.slot) * (P.D + 1) + j] = acc[q];
    }
}

// LDS words of the gapped-interpolation block.
__host__ __device__ inline int newton_lds_words(const DevProblem& P, int nthreads) {
  const int e1 = P.E + 1;
  return 3 * e1 + (e1 > nthreads ? e1 : nthreads);
}

// Consecutive points from a shifted origin o: the fast path left the
// coefficients ct_k of R(t + o) in the slot's partial sums; R(x) has
//   c_j = sum_{k >= j} C(k, j) (-o)^(k-j) ct_k,
// a correlation j! c_j = sum_d u_{j+d} v_d with u_k = k! ct_k and
// v_d = (-o)^d / d! (a Taylor shift), one thread per j.  Written as the
// Newton stage writes its result: c_j 2^32 in the first chunk the CRT reads
// for j, zero in the later ones.  LDS: 2 (D+1) words.
__device__ inline void shift_origin(const DevProblem& P, const DevTables& T, int slot, uint32_t* lds) {
  const int tid = threadIdx.x, nt = blockDim.x, D = P.D;
  const int g = P.pidx[slot];
  const PrimeConst pc = T.pc[g];
  const uint32_t p = pc.p, pinv = pc.pinv;
  const uint32_t* fact = T.fact + static_cast<size_t>(g) * T.kstride;
  const uint32_t* ifact = T.ifact + static_cast<size_t>(g) * T.kstride;
  const size_t cstride = static_cast<size_t>(P.np) * (D + 1);
  uint64_t* cp = P.cpart + static_cast<size_t>(slot) * (D + 1);
  uint32_t* u = lds;
  uint32_t* v = lds + (D + 1);
  const uint32_t mo = mmul(p - static_cast<uint32_t>(P.origin), pc.r2, p, pinv);  // -o R (o < 2^24 < p)
  for (int k = tid; k <= D; k += nt) {
    uint64_t cs = 0;
    for (int ch = k / P.kchunk; ch < P.nchunk; ++ch) cs = add_fold(cs, cp[ch * cstride + k], p);
    u[k] = mmul(redc(cs, p, pinv), fact[k], p, pinv);  // k! ct_k
    uint32_t pw = pc.r1, base = mo;                     // (-o)^k R by squaring
    for (int e = k; e; e >>= 1) {
      if (e & 1) pw = mmul(pw, base, p, pinv);
      base = mmul(base, base, p, pinv);
    }
    v[k] = mmul(pw, ifact[k], p, pinv);  // (-o)^k / k! R
  }
  __syncthreads();  // every partial sum is read before any is overwritten
  for (int j = tid; j <= D; j += nt) {
    uint64_t acc = 0;
    for (int d = 0; d <= D - j; ++d) acc = mac_fold(acc, u[j + d], v[d], p);
    const uint32_t c = mmul(redc(acc, p, pinv), ifact[j], p, pinv);
    const int ch0 = j / P.kchunk;
    cp[ch0 * cstride + j] = static_cast<uint64_t>(c) << 32;
    for (int ch = ch0 + 1; ch < P.nchunk; ++ch) cp[ch * cstride + j] = 0;
  }
}

// Gapped point sets (bad points replaced): one block per prime; select the
// first D+1 usable points, Newton divided differences, then the Newton form
// expanded in the monomial basis by Horner.  Slots that took the consecutive
// path need only the shift back from a nonzero origin.
__device__ inline void stage_interp_newton(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int slot = w.slot;
  const bool fast = fast_prime(P, slot);
  if (tid == 0) P.status[1 + slot] = fast ? 0 : 1;
  if (fast) {
    if (P.origin != 0) shift_origin(P, T, slot, lds);
    return;
  }
  const int g = P.pidx[slot];
  const PrimeConst pc = T.pc[g];
  const uint32_t p = pc.p, pinv = pc.pinv;
  const int E = P.E, D = P.D;
  const uint32_t* fact = T.fact + static_cast<size_t>(g) * T.kstride;
  const uint32_t* ifact = T.ifact + static_cast<size_t>(g) * T.kstride;
  const uint32_t* z = P.zval + static_cast<size_t>(slot) * (E + 1);
  const uint8_t* zb = P.zbad + static_cast<size_t>(slot) * (E + 1);

  uint32_t* xs = lds;                 // E+1: selected point indices
  uint32_t* d0 = xs + (E + 1);        // E+1
  uint32_t* invt = d0 + (E + 1);      // E+1: 1/t R mod p
  uint32_t* d1 = invt + (E + 1);      // max(E+1, nt); also the scan buffer
  int* cnt = reinterpret_cast<int*>(d1);

  for (int t = tid + 1; t <= E; t += nt) invt[t] = mmul(ifact[t], fact[t - 1], p, pinv);

  // selection: first D+1 usable points (all points in formal mode)
  const int chunk = (E + 1 + nt - 1) / nt;
  const int lo = tid * chunk;
  const int hi = (lo + chunk < E + 1) ? lo + chunk : E + 1;
  int c = 0;
  for (int i = lo; i < hi; ++i) c += (P.formal || !zb[i]) ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {  // inclusive Hillis-Steele scan
    const int v = (tid >= off) ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int total = cnt[nt - 1];
  int q = cnt[tid] - c;
  __syncthreads();
  if (total < D + 1) {
    if (tid == 0) atomicOr(P.status, kErrTooFewGoodPoints);
    return;  // block-uniform
  }
  for (int i = lo; i < hi && q <= D; ++i)
    if (P.formal || !zb[i]) {
      xs[q] = static_cast<uint32_t>(i);
      d0[q] = z[i];
      ++q;
    }
  __syncthreads();

  // divided differences, level by level (ping-pong buffers)
  uint32_t* cur = d0;
  uint32_t* nxt = d1;
  for (int k = 1; k <= D; ++k) {
    for (int i = tid; i <= D; i += nt) {
      if (i >= k) {
        const uint32_t diff = msubm(cur[i], cur[i - 1], p);
        nxt[i] = mmul(diff, invt[xs[i] - xs[i - k]], p, pinv);
      } else {
        nxt[i] = cur[i];
      }
    }
    __syncthreads();
    uint32_t* t = cur; cur = nxt; nxt = t;
  }
  // Newton form -> monomials: P <- P (x - x_k) + a_k, k = D-1 .. 0
  uint32_t* coef = invt;  // the inverse table is no longer needed
  for (int i = tid; i <= D; i += nt) coef[i] = cur[i];
  __syncthreads();
  uint32_t* pa = nxt;
  uint32_t* pb = cur;
  if (tid == 0) pa[0] = coef[D];
  __syncthreads();
  for (int k = D - 1; k >= 0; --k) {
    const uint32_t xk = static_cast<uint32_t>(P.origin) + xs[k];
    const uint32_t xkt = mmul(xk, pc.r2, p, pinv);
    const int deg = D - k;  // degree after this step
    for (int j = tid; j <= deg; j += nt) {
      const uint32_t left = (j > 0) ? pa[j - 1] : 0u;
      const uint32_t mid = (j < deg) ? pa[j] : 0u;
      uint32_t v = msubm(left, mmul(mid, xkt, p, pinv), p);
      if (j == 0) v = maddm(v, coef[k], p);
      pb[j] = v;
    }
    __syncthreads();
    uint32_t* t = pa; pa = pb; pb = t;
  }
  // the first chunk the CRT reads for coefficient j carries c_j 2^32 (REDC gives
  // c_j); the later chunks are zero
  for (int j = tid; j <= D; j += nt) {
    const int ch0 = j / P.kchunk;
    P.cpart[(static_cast<size_t>(ch0) * P.np + slot) * (D + 1) + j] = static_cast<uint64_t>(pa[j]) << 32;
    for (int ch = ch0 + 1; ch < P.nchunk; ++ch)
      P.cpart[(static_cast<size_t>(ch) * P.np + slot) * (D + 1) + j] = 0;
  }
}

// ----------------------------------------------------------------------- CRT

// Whether the Garner table (np^2 words) and the limb table of the prefix
// products (np L_out words) of a problem are staged in LDS by the CRT kernel,
// and the CRT block's LDS words.
// dst[t] = src(t) for t < n with the block's threads; every thread issues up
// to eight loads (clamped to valid indices) before storing any, so a small
// table costs about one memory latency.
template <class F>
__device__ inline void block_stage(uint32_t* dst, int n, F src) {
  const int nt = blockDim.x;
  for (int base = threadIdx.x; base < n; base += 8 * nt) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * nt;
      v[u] = src(t < n ? t : n - 1);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * nt;
      if (t < n) dst[t] = v[u];
    }
  }
}

// Residues of the block's coefficients (kCrtBlockCoeffs per block) are
// staged in LDS first: [coefficient][prime].
constexpr int kCrtBlockCoeffs = 8;
constexpr int kCrtConsts = 6;  // per prime: p, -p^{-1}, Garner inverse, w, r_lo, r_hi
__host__ __device__ inline int crt_wave_words(int ns) { return 3 * 64 * ns + 4; }
__host__ __device__ inline int crt_base_words(const DevProblem& P, int ns, int nwaves) {
  return nwaves * crt_wave_words(ns) + kCrtBlockCoeffs * P.np + kCrtConsts * P.np;
}
// The table of the M / p_j limbs is staged in LDS when it fits.
__host__ __device__ inline bool crt_stage_mi(const DevProblem& P, int ns, int nwaves) {
  return P.np * P.L_out + crt_base_words(P, ns, nwaves) <= kLdsWords;
}
__host__ __device__ inline int crt_lds_words(const DevProblem& P, int ns, int nwaves) {
  return (crt_stage_mi(P, ns, nwaves) ? P.np * P.L_out : 0) + crt_base_words(P, ns, nwaves);
}

// Sum of a 32-bit value over the 64 lanes of a wave (every lane gets it).
__device__ inline uint32_t wave_sum32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), m, 64));
  return v;
}

// Radix conversion of one coefficient (lanes own output limbs t = lane + 64 r):
//   Z_t = init_t + sum_j v_j tab[j][t]   (96-bit column sums),
// carries resolved with wave ballots; writes Z mod 2^(32 L_out).
// Each v_j < 2^32 comes in 16-bit halves -- the caller leaves lo16(v_j) in
// vbuf[j] and hi16(v_j) in sb[j] (sb is free until the carry phase) -- so that
// the column sums
//   A_t = sum_j lo16(v_j) tab[j][t],  B_t = sum_j hi16(v_j) tab[j][t]
// take one 64-bit multiply-add per term with no carry handling: every term is
// below 2^48 and at most 512 primes come here, so both sums stay below 2^57.
// Then Z_t = init_t + A_t + 2^16 B_t, formed once per limb in 96 bits.
template <int NS>
__device__ inline void crt_radix(const DevProblem& P, int k, bool valid, const uint32_t* vbuf, const uint32_t* tab,
                                 int tstride, const uint64_t* init, uint32_t* sb, uint32_t* sc) {
  const int lane = threadIdx.x & 63;
  const int np = P.np, L = P.L_out;
  // two independent accumulator pairs per limb (short dependency chains)
  uint64_t A0[NS], B0[NS], A1[NS], B1[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) A0[r] = B0[r] = A1[r] = B1[r] = 0u;
  int j = 0;
  for (; j + 4 <= np; j += 4) {
    const uint64_t l0 = vbuf[j], l1 = vbuf[j + 1], l2 = vbuf[j + 2], l3 = vbuf[j + 3];
    const uint64_t h0 = sb[j], h1 = sb[j + 1], h2 = sb[j + 2], h3 = sb[j + 3];
    const uint32_t* p0 = tab + static_cast<size_t>(j) * tstride;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int t = lane + 64 * r;
      if (t < L) {
        const uint64_t w0 = p0[t], w1 = p0[tstride + t], w2 = p0[2 * tstride + t], w3 = p0[3 * tstride + t];
        A0[r] += l0 * w0;
        B0[r] += h0 * w0;
        A1[r] += l1 * w1;
        B1[r] += h1 * w1;
        A0[r] += l2 * w2;
        B0[r] += h2 * w2;
        A1[r] += l3 * w3;
        B1[r] += h3 * w3;
      }
    }
  }
  for (; j < np; ++j) {
    const uint64_t l0 = vbuf[j], h0 = sb[j];
    const uint32_t* p0 = tab + static_cast<size_t>(j) * tstride;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int t = lane + 64 * r;
      if (t < L) {
        const uint64_t w0 = p0[t];
        A0[r] += l0 * w0;
        B0[r] += h0 * w0;
      }
    }
  }
  uint64_t lo[NS];
  uint32_t hc[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const uint64_t A = A0[r] + A1[r], B = B0[r] + B1[r];  // each < 2^58
    uint64_t z = init[r] + A;
    uint32_t h = z < A ? 1u : 0u;
    const uint64_t Bs = B << 16;
    z += Bs;
    h += (z < Bs ? 1u : 0u) + static_cast<uint32_t>(B >> 48);
    lo[r] = z;
    hc[r] = h;
  }
  // limb t receives lo32(S_t) + hi32(S_{t-1}) + top32(S_{t-2})
  WaveSync sync;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    sb[t + 1] = static_cast<uint32_t>(lo[r] >> 32);
    sc[t + 2] = hc[r];
  }
  if (lane == 0) {
    sb[0] = 0;
    sc[0] = 0;
    sc[1] = 0;
  }
  sync();
  uint32_t l1[NS], h1[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    const uint64_t wv = static_cast<uint64_t>(static_cast<uint32_t>(lo[r])) + sb[t] + sc[t];
    l1[r] = static_cast<uint32_t>(wv);
    h1[r] = static_cast<uint32_t>(wv >> 32);  // <= 2
  }
  sync();
#pragma unroll
  for (int r = 0; r < NS; ++r) sb[lane + 64 * r + 1] = h1[r];
  sync();
  uint64_t cin = 0;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    const uint64_t x2 = static_cast<uint64_t>(l1[r]) + sb[t];
    const uint32_t l2 = static_cast<uint32_t>(x2);
    const bool gen = (x2 >> 32) != 0 && t < L;
    const bool prop = (l2 == 0xFFFFFFFFu) && t < L;
    const uint64_t G = __ballot(gen);
    const uint64_t Pm = __ballot(prop);
    const uint64_t X = G | Pm;
    const unsigned __int128 tot = static_cast<unsigned __int128>(X) + G + cin;
    const uint64_t S = static_cast<uint64_t>(tot);
    const uint64_t C = S ^ X ^ G;  // carry into each limb of this group
    cin = static_cast<uint64_t>(tot >> 64);
    const uint32_t limb = l2 + static_cast<uint32_t>((C >> lane) & 1u);
    if (valid && t < L) P.out[static_cast<size_t>(k) * L + t] = limb;
  }
}

// One wave per coefficient k; lanes own primes (slot i = lane + 64 r) with the
// shifted residues u_i = c_k + H mod p_i, H = (M-1)/2, so that Y = c_k + H lies
// in [0, M) and c_k = Y - H is the symmetric residue.
//
// Direct form: with M_i = M / p_i and t_i = u_i (M_i^{-1} mod p_i),
//   Y = sum_i t_i M_i - q M,  q = floor(sum_i t_i / p_i).
// q is found from 32-bit fixed-point parts f_i = floor(t_i floor(2^64/p_i) / 2^32),
// which undershoot t_i 2^32 / p_i by less than 2 each: q = floor(sum f_i / 2^32)
// whenever the fraction of that sum is below 2^32 - 2 np.  Otherwise (rare)
// the wave computes Y by Garner's mixed-radix digits instead: digit v_j is
// formed in lane j and broadcast, every lane i > j adds v_j (prod_{l<j} p_l
// mod p_i), and Y = sum_j v_j prod_{l<j} p_l.
// The output Z = Y - H mod 2^(32 L_out) is formed by crt_radix with
// init = 2^(32 L_out) - H (+ q (2^(32 L_out) - M) in the direct form).
template <int NS>
__device__ inline void crt_one(const DevProblem& P, int k_raw, const uint32_t* mi, int mstride, uint32_t* wb,
                               const uint32_t* ures, const uint32_t* pconst) {
  const int lane = threadIdx.x & 63;
  const bool valid = k_raw <= P.D;
  const int k = valid ? k_raw : P.D;
  const int np = P.np;
  const int L = P.L_out;
  uint32_t* vbuf = wb;
  uint32_t* sb = wb + 64 * NS;
  uint32_t* sc = sb + 64 * NS + 2;
  const uint32_t* cp = pconst;               // p
  const uint32_t* cpinv = pconst + np;       // -p^{-1} mod 2^32
  const uint32_t* cinvm = pconst + 2 * np;   // Garner inverse (Montgomery)
  const uint32_t* cw = pconst + 3 * np;      // (M / p_i)^{-1} mod p_i (Montgomery)
  const uint32_t* crlo = pconst + 4 * np;    // floor(2^64 / p_i), low word
  const uint32_t* crhi = pconst + 5 * np;    //                    high word

  uint32_t u[NS];
  // f_i < 2^32 split as fa + fb 2^16: both halves summed over up to 512 primes
  // stay below 2^25, so the 32-bit wave sums cannot wrap
  uint32_t fa = 0u, fb = 0u;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int i = lane + 64 * r;
    u[r] = 0u;
    if (i < np) {
      u[r] = ures[i];
      const uint32_t p = cp[i];
      const uint32_t t = mmul(u[r], cw[i], p, cpinv[i]);
      vbuf[i] = t & 0xFFFFu;  // the halves crt_radix multiplies with
      sb[i] = t >> 16;
      const uint64_t f = static_cast<uint64_t>(t) * crhi[i] + __umulhi(t, crlo[i]);
      fa += static_cast<uint32_t>(f) & 0xFFFFu;
      fb += static_cast<uint32_t>(f >> 16);
    }
  }
  const uint64_t Sf = static_cast<uint64_t>(wave_sum32(fa)) + (static_cast<uint64_t>(wave_sum32(fb)) << 16);
  const uint32_t q = static_cast<uint32_t>(Sf >> 32);
  const bool direct = static_cast<uint32_t>(Sf) < 0xFFFFFFFFu - 2u * static_cast<uint32_t>(np) && !P.crt_garner;
  uint64_t init[NS];
  if (__builtin_amdgcn_readfirstlane(direct ? 1 : 0)) {
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int t = lane + 64 * r;
      init[r] = (t < L) ? static_cast<uint64_t>(P.NH[t]) + static_cast<uint64_t>(q) * P.negM[t] : 0u;
    }
    WaveSync()();
    crt_radix<NS>(P, k, valid, vbuf, mi, mstride, init, sb, sc);
    return;
  }
  // Garner fallback (tables read from global memory)
  uint32_t acc[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) acc[r] = 0u;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    for (int jj = 0; jj < 64; ++jj) {
      const int j = r * 64 + jj;
      if (j >= np) break;
      const int i0 = lane + 64 * r;
      const uint32_t pr = i0 < np ? cp[i0] : 3u, pir = i0 < np ? cpinv[i0] : 0u;
      const uint32_t im = i0 < np ? cinvm[i0] : 0u;
      const uint32_t vloc = mmul(msubm(u[r], acc[r], pr), im, pr, pir);
      const uint32_t vj = __builtin_amdgcn_readlane(vloc, jj);
      if (lane == 0) {
        vbuf[j] = vj & 0xFFFFu;
        sb[j] = vj >> 16;
      }
#pragma unroll
      for (int rr = r; rr < NS; ++rr) {
        const int i = lane + 64 * rr;
        if (i > j && i < np) {
          const uint32_t tji = P.Tg[static_cast<size_t>(j) * P.tgs + i];
          acc[rr] = maddm(acc[rr], mmul(vj, tji, cp[i], cpinv[i]), cp[i]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    init[r] = (t < L) ? P.NH[t] : 0u;
  }
  WaveSync()();
  crt_radix<NS>(P, k, valid, vbuf, P.Plimb, P.LP, init, sb, sc);
}

// One item: kCrtBlockCoeffs coefficients, `cpw` per wave,
// k = (blk * waves + wave) * cpw + c (waves * cpw = kCrtBlockCoeffs).  With
// `fresh` the per-prime constants and (when it fits) the M / p_j limb table
// are staged in LDS first; a block that takes several items of one problem
// in a row (the staged launch) stages them once.  The residues u_i of the
// item's coefficients are summed from the basis-change partial sums, with the
// block's threads reading kCrtBlockCoeffs consecutive coefficients of one
// prime together.
constexpr int kCrtItemsPerBlock = 4;  // items per block of the staged launch
template <int NS>
__device__ inline void stage_crt(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds,
                                 int cpw = 1, bool fresh = true) {
  const int nw = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int np = P.np;
  const bool staged_mi = crt_stage_mi(P, NS, nw);
  const int L = P.L_out;
  uint32_t* mis = lds;
  uint32_t* wbase = lds + (staged_mi ? np * L : 0);
  uint32_t* wb = wbase + wave * crt_wave_words(NS);
  uint32_t* ures = wbase + nw * crt_wave_words(NS);  // [kCrtBlockCoeffs][np]
  uint32_t* pconst = ures + kCrtBlockCoeffs * np;     // [kCrtConsts][np]
  const size_t cstride = static_cast<size_t>(np) * (P.D + 1);
  const int kbase = w.blk * kCrtBlockCoeffs;
  if (fresh && staged_mi)
    block_stage(mis, np * L, [&](int t) {
      const int j = t / L, l = t - j * L;
      return P.Mi[static_cast<size_t>(j) * L + l];
    });
  {
    for (int t = threadIdx.x; t < np * kCrtBlockCoeffs; t += blockDim.x) {
      const int i = t / kCrtBlockCoeffs, c = t - i * kCrtBlockCoeffs;
      const int k = (kbase + c <= P.D) ? kbase + c : P.D;
      const uint64_t* cpp = P.cpart + static_cast<size_t>(i) * (P.D + 1) + k;
      const int ch0 = k / P.kchunk;
      uint64_t q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ch = ch0 + u < P.nchunk ? ch0 + u : P.nchunk - 1;
        q[u] = cpp[ch * cstride];
      }
      const PrimeConst pc = T.pc[P.pidx[i]];
      const uint32_t hm = P.Hm[i];
      uint64_t cs = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (ch0 + u < P.nchunk) cs = add_fold(cs, q[u], pc.p);
      for (int ch = ch0 + 8; ch < P.nchunk; ++ch) cs = add_fold(cs, cpp[ch * cstride], pc.p);
      ures[c * np + i] = maddm(redc(cs, pc.p, pc.pinv), hm, pc.p);
      if (c == 0 && fresh) {
        pconst[i] = pc.p;
        pconst[np + i] = pc.pinv;
        pconst[2 * np + i] = P.invM[i];
        pconst[3 * np + i] = P.wdir[i];
        pconst[4 * np + i] = P.rinv[2 * i];
        pconst[5 * np + i] = P.rinv[2 * i + 1];
      }
    }
    __syncthreads();
    // two calls rather than one with a selected pointer: with the table in
    // LDS the compiler then reads it with LDS instructions, not flat loads
    for (int c = 0; c < cpw; ++c) {
      const int local = wave * cpw + c;
      if (staged_mi)
        crt_one<NS>(P, kbase + local, mis, L, wb, ures + local * np, pconst);
      else
        crt_one<NS>(P, kbase + local, P.Mi, L, wb, ures + local * np, pconst);
    }
  }
}

// ------------------------------------------------------------------ wide CRT
// Problems with more primes than the per-lane slots cover.  The same direct
// form Y = sum_i t_i M_i - q M (M_i = M / p_i, t_i = u_i M_i^{-1} mod p_i) in
// three passes over device memory:
//   1. per coefficient k: t_{k,i} for every prime, and the quotient estimate
//      q_k = floor(sum_i f_{k,i} / 2^32) from the fixed-point parts, which is
//      the true quotient or one short of it (each f undershoots by < 2);
//   2. the integer contraction S[k][h] = sum_i t_{k,i} m_{i,h} over 16-bit
//      halves m_{i,h} of the M_i limbs (each term < 2^47, so 4096 primes sum
//      below 2^59 without carries), tiled 16 coefficients x 256 limbs;
//   3. one wave per coefficient: Y0 = sum_h S[k][h] 2^(16 h) + q_k (2^(32 Lw) - M)
//      mod 2^(32 Lw), which lies in [0, 2M) (Lw = L_out + 1 limbs hold it),
//      compared with M; the output is Y0 - H (- M when Y0 >= M) mod 2^(32 L_out).
constexpr int kWideTCoeffs = 8;    // coefficients per block of pass 1 (256 threads)
constexpr int kWideKT = 16;        // coefficients per block of pass 2
constexpr int kWideHT = 256;       // limbs per block of pass 2 (one per thread)
constexpr int kWideChunk = 64;     // primes per LDS chunk of pass 2
constexpr int kWideDigits = 5;     // 7-bit digits of t and of the M_i limbs (matrix-core pass 2)

__host__ __device__ inline int wide_t_lds_words() { return 4 * 2 * kWideTCoeffs; }
__host__ __device__ inline int wide_sum_lds_words() { return kWideChunk * kWideKT; }
__host__ __device__ inline int wide_fin_lds_words(const DevProblem& P) { return P.Lw; }

// Carry into this lane when every lane adds its `gen` (carry out of its own
// limb) and passes an incoming carry on when `prop` (limb all ones); `cin` is
// the carry into lane 0 and becomes the carry out of lane 63.
__device__ inline uint32_t wave_carry_in(bool gen, bool prop, uint64_t* cin) {
  const int lane = threadIdx.x & 63;
  const uint64_t G = __ballot(gen);
  const uint64_t X = G | __ballot(prop);
  const unsigned __int128 tot = static_cast<unsigned __int128>(X) + G + *cin;
  const uint64_t C = static_cast<uint64_t>(tot) ^ X ^ G;
  *cin = static_cast<uint64_t>(tot >> 64);
  return static_cast<uint32_t>((C >> lane) & 1u);
}

// Pass 1: block item blk covers coefficients blk*8 .. blk*8+7; thread owns
// coefficient c = tid mod 8 and primes tid/8 + 32 r.
__device__ inline void stage_crt_wide_t(const DevProblem& P, const DevTables& T, const WorkItem& w, uint32_t* lds) {
  const int c = threadIdx.x & (kWideTCoeffs - 1);
  const int k_raw = w.blk * kWideTCoeffs + c;
  const bool valid = k_raw <= P.D;
  const int k = valid ? k_raw : P.D;
  const int np = P.np;
  const size_t cstride = static_cast<size_t>(np) * (P.D + 1);
  uint32_t fa = 0u, fb = 0u;  // 16-bit halves of the f parts, summed
  for (int i = threadIdx.x / kWideTCoeffs; i < np; i += blockDim.x / kWideTCoeffs) {
    const uint64_t* cpp = P.cpart + static_cast<size_t>(i) * (P.D + 1) + k;
    const PrimeConst pc = T.pc[P.pidx[i]];
    uint64_t cs = 0;
    for (int ch = 0; ch < P.nchunk; ++ch) cs = add_fold(cs, cpp[ch * cstride], pc.p);
    const uint32_t u = maddm(redc(cs, pc.p, pc.pinv), P.Hm[i], pc.p);  // c_k + H mod p
    const uint32_t t = mmul(u, P.wdir[i], pc.p, pc.pinv);
    if (valid) P.wT[static_cast<size_t>(k) * P.wnpad + i] = t;
    const uint64_t f = static_cast<uint64_t>(t) * P.rinv[2 * i + 1] + __umulhi(t, P.rinv[2 * i]);
    fa += static_cast<uint32_t>(f) & 0xFFFFu;
    fb += static_cast<uint32_t>(f >> 16);
  }
  // lanes of one coefficient differ in lane bits 3..5
#pragma unroll
  for (int m = kWideTCoeffs; m < 64; m <<= 1) {
    fa += static_cast<uint32_t>(__shfl_xor(static_cast<int>(fa), m, 64));
    fb += static_cast<uint32_t>(__shfl_xor(static_cast<int>(fb), m, 64));
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (lane < kWideTCoeffs) {
    lds[wave * 2 * kWideTCoeffs + lane] = fa;
    lds[wave * 2 * kWideTCoeffs + kWideTCoeffs + lane] = fb;
  }
  __syncthreads();
  if (threadIdx.x < kWideTCoeffs && valid) {
    uint64_t sa = 0, sb = 0;
    for (int v = 0; v < nw; ++v) {
      sa += lds[v * 2 * kWideTCoeffs + c];
      sb += lds[v * 2 * kWideTCoeffs + kWideTCoeffs + c];
    }
    P.wq[k] = static_cast<uint32_t>((sa + (sb << 16)) >> 32);
  }
}

// Pass 2: item (blk = coefficient tile, sub = limb tile); the block's t values
// for 64 primes at a time are staged in LDS as [prime][coefficient] (read
// back as broadcasts); each thread streams one limb column of the M_i table
// and splits it into its two 16-bit halves, so every t value feeds two
// multiply-adds.  Loads go out a group of 8 primes ahead of their use, from
// clamped (always valid) addresses.
__device__ inline void stage_crt_wide_sum(const DevProblem& P, const WorkItem& w, uint32_t* lds) {
  constexpr int G = 8;
  const int np = P.np, Lw = P.Lw, nh = 2 * Lw;
  const int k0 = w.blk * kWideKT;
  const int t = w.sub * kWideHT + static_cast<int>(threadIdx.x);
  const bool tv_ok = t < Lw;
  const uint32_t* Mcol = P.Mi + (tv_ok ? t : Lw - 1);
  uint64_t alo[kWideKT], ahi[kWideKT];
#pragma unroll
  for (int c = 0; c < kWideKT; ++c) alo[c] = ahi[c] = 0u;
  // no masks needed: the staged t values are zero beyond the last prime, and
  // lanes beyond the last limb store nothing
  auto load_group = [&](int ibase, uint32_t* m) {
#pragma unroll
    for (int u = 0; u < G; ++u) m[u] = Mcol[static_cast<size_t>(min(ibase + u, np - 1)) * Lw];
  };
  uint32_t mcur[G], mnext[G];
  load_group(0, mcur);
  for (int i0 = 0; i0 < np; i0 += kWideChunk) {
    __syncthreads();  // the previous chunk is consumed
    for (int e = threadIdx.x; e < kWideChunk * kWideKT; e += blockDim.x) {
      const int c = e / kWideChunk, ii = e - c * kWideChunk;  // coalesced along the primes of one row
      const int i = i0 + ii, k = k0 + c;
      lds[ii * kWideKT + c] = (i < np && k <= P.D) ? P.wT[static_cast<size_t>(k) * P.wnpad + i] : 0u;
    }
    __syncthreads();
    const int n = min(kWideChunk, np - i0);
    for (int ii = 0; ii < n; ii += G) {
      load_group(i0 + ii + G, mnext);  // beyond np: clamped (their t values are zero)
      __builtin_amdgcn_sched_barrier(0);  // issue them before this group's arithmetic
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const uint32_t lo = mcur[u] & 0xFFFFu, hi = mcur[u] >> 16;
        const uint4* tv = reinterpret_cast<const uint4*>(lds + (ii + u) * kWideKT);
#pragma unroll
        for (int q4 = 0; q4 < kWideKT / 4; ++q4) {
          const uint4 t4 = tv[q4];
          alo[4 * q4 + 0] += static_cast<uint64_t>(t4.x) * lo;
          ahi[4 * q4 + 0] += static_cast<uint64_t>(t4.x) * hi;
          alo[4 * q4 + 1] += static_cast<uint64_t>(t4.y) * lo;
          ahi[4 * q4 + 1] += static_cast<uint64_t>(t4.y) * hi;
          alo[4 * q4 + 2] += static_cast<uint64_t>(t4.z) * lo;
          ahi[4 * q4 + 2] += static_cast<uint64_t>(t4.z) * hi;
          alo[4 * q4 + 3] += static_cast<uint64_t>(t4.w) * lo;
          ahi[4 * q4 + 3] += static_cast<uint64_t>(t4.w) * hi;
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) mcur[u] = mnext[u];
    }
  }
  if (tv_ok)
#pragma unroll
    for (int c = 0; c < kWideKT; ++c)
      if (k0 + c <= P.D) {  // column sum of limb t: alo + ahi 2^16 (< 2^76) as (low, high) words
        const unsigned __int128 v = static_cast<unsigned __int128>(alo[c]) + (static_cast<unsigned __int128>(ahi[c]) << 16);
        uint64_t* dst = P.wS + static_cast<size_t>(k0 + c) * nh + 2 * t;
        dst[0] = static_cast<uint64_t>(v);
        dst[1] = static_cast<uint64_t>(v >> 64);
      }
}

// Pass 2 on the matrix cores.  t and the M_i limbs are split into five 7-bit
// digits each (t = sum_a t_a 2^(7a), m = sum_b m_b 2^(7b), 35 bits >= 32), so
// every digit is a non-negative int8; the int8 MFMA (16 x 16 outputs, 64
// primes per step) accumulates sum_i t_a m_b in int32 per anti-diagonal
// s = a + b: at most 5 * 127^2 * 4096 < 2^29 for 4096 primes, exact.  The
// column sum is then sum_s D_s 2^(7s) < 2^85.  The limb digits are planes
// Md[b][t][i] built with the job (a limb's primes contiguous); the block
// stages its 32 limbs x 64 primes x 5 digits in LDS once per step for its
// four waves.  The t values come from wT (rows padded with zeros to wnpad)
// and are split into digits in registers.  Wave w takes coefficients
// k0 + 16 w ... (one 16-row tile) and the block's 32 limbs (two 16-column
// tiles); a lane holds row r of A and column r of B for the 16 primes of its
// quarter kg (any fixed assignment of primes to the K slots serves, as long
// as A and B use the same one).
constexpr int kWideMfmaK = 64;   // primes per MFMA step (planes padded to a multiple)
constexpr int kWideMfmaKT = 64;  // coefficients per block (four waves)
constexpr int kWideMfmaTT = 32;  // limbs per block
__host__ __device__ inline int wide_mfma_lds_words() { return kWideDigits * kWideMfmaTT * kWideMfmaK / 4; }
typedef int wide_v4i __attribute__((ext_vector_type(4)));

__device__ inline void stage_crt_wide_sum_mfma(const DevProblem& P, const WorkItem& w, uint32_t* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int Lw = P.Lw, nh = 2 * Lw;
  const int k0 = w.blk * kWideMfmaKT + 16 * wave;  // this wave's coefficient tile
  const int t0 = w.sub * kWideMfmaTT;
  const int r = lane & 15, kg = lane >> 4;
  const size_t mplane = static_cast<size_t>(P.wlpad) * P.wnpad;
  const uint32_t* trow = P.wT + static_cast<size_t>(k0 + r) * P.wnpad + 16 * kg;
  uint4* bl = reinterpret_cast<uint4*>(lds);  // [digit][limb][prime quarter]
  wide_v4i acc[2][2 * kWideDigits - 1];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int d = 0; d < 2 * kWideDigits - 1; ++d) acc[u][d] = wide_v4i{0, 0, 0, 0};
  for (int i0 = 0; i0 < P.wnpad; i0 += kWideMfmaK) {
    __syncthreads();  // the previous step's tile is consumed
    for (int e = threadIdx.x; e < kWideDigits * kWideMfmaTT * 4; e += blockDim.x) {
      const int d = e / (kWideMfmaTT * 4), rem = e - d * (kWideMfmaTT * 4), tl = rem >> 2, q = rem & 3;
      bl[e] = *reinterpret_cast<const uint4*>(P.wMd + d * mplane + static_cast<size_t>(t0 + tl) * P.wnpad + i0 + 16 * q);
    }
    // the wave's A: 16 t values, split into digit bytes
    uint32_t tv[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(trow + i0 + 4 * q);
      tv[4 * q] = v.x;
      tv[4 * q + 1] = v.y;
      tv[4 * q + 2] = v.z;
      tv[4 * q + 3] = v.w;
    }
    wide_v4i a[kWideDigits];
#pragma unroll
    for (int d = 0; d < kWideDigits; ++d)
#pragma unroll
      for (int wd = 0; wd < 4; ++wd) {
        uint32_t word = 0;
#pragma unroll
        for (int by = 0; by < 4; ++by) word |= ((tv[4 * wd + by] >> (7 * d)) & 127u) << (8 * by);
        a[d][wd] = static_cast<int>(word);
      }
    __syncthreads();
#pragma unroll
    for (int db = 0; db < kWideDigits; ++db) {
      const wide_v4i b0 = *reinterpret_cast<const wide_v4i*>(&bl[(db * kWideMfmaTT + r) * 4 + kg]);
      const wide_v4i b1 = *reinterpret_cast<const wide_v4i*>(&bl[(db * kWideMfmaTT + 16 + r) * 4 + kg]);
#pragma unroll
      for (int da = 0; da < kWideDigits; ++da) {
        acc[0][da + db] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b0, acc[0][da + db], 0, 0, 0);
        acc[1][da + db] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b1, acc[1][da + db], 0, 0, 0);
      }
    }
  }
  // lane holds rows 4 kg + e (coefficients) of column r (limb) of each tile
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = t0 + 16 * u + r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + 4 * kg + e;
      unsigned __int128 v = 0;
#pragma unroll
      for (int d = 0; d < 2 * kWideDigits - 1; ++d)
        v += static_cast<unsigned __int128>(static_cast<uint32_t>(acc[u][d][e])) << (7 * d);
      if (k <= P.D && t < Lw) {
        uint64_t* dst = P.wS + static_cast<size_t>(k) * nh + 2 * t;
        dst[0] = static_cast<uint64_t>(v);
        dst[1] = static_cast<uint64_t>(v >> 64);
      }
    }
  }
}

// Pass 3: one wave (the whole block) per coefficient k = blk.
__device__ inline void stage_crt_wide_fin(const DevProblem& P, const WorkItem& w, uint32_t* lds) {
  const int lane = threadIdx.x & 63;
  const int k = w.blk;
  const int Lw = P.Lw, L = P.L_out;
  const uint64_t* S = P.wS + static_cast<size_t>(k) * 2 * Lw;
  const uint32_t q = P.wq[k];
  uint32_t* y = lds;
  // Y0 limbs, 64 at a time; V_t = (column sum of limb t) + q negM_t < 2^86 is
  // (lo: 64 bits, hi: 32 bits), and limb t is lo32(V_t) + mid32(V_{t-1}) +
  // hi(V_{t-2}) plus carries; the values of lanes 62 and 63 carry over
  uint32_t pm = 0u, ph1 = 0u, ph2 = 0u, pc1 = 0u;
  uint64_t cin = 0u;
  for (int t0 = 0; t0 < Lw; t0 += 64) {
    const int t = t0 + lane;
    uint64_t lo = 0u;
    uint32_t hi = 0u;
    if (t < Lw) {
      lo = S[2 * t];
      hi = static_cast<uint32_t>(S[2 * t + 1]);
      const uint64_t b = static_cast<uint64_t>(q) * P.negM[t];
      lo += b;
      hi += (lo < b) ? 1u : 0u;
    }
    const uint32_t mid = static_cast<uint32_t>(lo >> 32);
    uint32_t mprev = static_cast<uint32_t>(__shfl_up(static_cast<int>(mid), 1, 64));
    uint32_t hprev2 = static_cast<uint32_t>(__shfl_up(static_cast<int>(hi), 2, 64));
    if (lane == 0) {
      mprev = pm;
      hprev2 = ph2;
    }
    if (lane == 1) hprev2 = ph1;
    const uint64_t s = static_cast<uint64_t>(static_cast<uint32_t>(lo)) + mprev + hprev2;
    const uint32_t l1 = static_cast<uint32_t>(s), h1 = static_cast<uint32_t>(s >> 32);  // h1 <= 2
    uint32_t h1prev = static_cast<uint32_t>(__shfl_up(static_cast<int>(h1), 1, 64));
    if (lane == 0) h1prev = pc1;
    const uint64_t x2 = static_cast<uint64_t>(l1) + h1prev;
    const uint32_t l2 = static_cast<uint32_t>(x2);
    const uint32_t cy = wave_carry_in((x2 >> 32) != 0, l2 == 0xFFFFFFFFu, &cin);
    if (t < Lw) y[t] = l2 + cy;
    pm = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(mid), 63));
    ph1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(hi), 63));
    ph2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(hi), 62));
    pc1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(h1), 63));
  }
  WaveSync()();
  // Y0 >= M ?  (top limbs first; equal counts as >=)
  int ge = 1;
  for (int t0 = ((Lw - 1) / 64) * 64; t0 >= 0; t0 -= 64) {
    const int t = t0 + lane;
    const uint32_t yv = (t < Lw) ? y[t] : 0u, mv = (t < Lw) ? P.Mw[t] : 0u;
    const uint64_t gt = __ballot(yv > mv), lt = __ballot(yv < mv);
    const uint64_t d = gt | lt;
    if (d) {
      const int top = 63 - __clzll(static_cast<long long>(d));
      ge = static_cast<int>((gt >> top) & 1u);
      break;
    }
  }
  // output: Y0 - H (- M) mod 2^(32 L_out)
  const uint32_t* A = ge ? P.NHM : P.NH;
  cin = 0u;
  for (int t0 = 0; t0 < L; t0 += 64) {
    const int t = t0 + lane;
    const uint64_t x = (t < L) ? static_cast<uint64_t>(y[t]) + A[t] : 0u;
    const uint32_t l = static_cast<uint32_t>(x);
    const uint32_t cy = wave_carry_in((x >> 32) != 0, l == 0xFFFFFFFFu && t < L, &cin);
    if (t < L) P.out[static_cast<size_t>(k) * L + t] = l + cy;
  }
}

}  // namespace rsl

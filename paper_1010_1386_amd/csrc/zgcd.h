// Modular gcd over Z[x] for the square-free step after the resultant (the
// Project step of the paper's Sec. 3.2 takes a square-free factorisation of
// R by Yun's algorithm, i.e. gcds of R and its derivatives; the outlook of
// Sec. 6 proposes the modular route for it).  Device stages, per prime slot:
//   zreduce  u, v mod p (two's complement limbs, division-free)
//   zgcd     Euclid's algorithm over Z_p in LDS, one wave per prime,
//            division-free steps; the gcd made monic and scaled by
//            ell = gcd(lc u, lc v) mod p
//   zpack    the kept slots' scaled gcds in the CRT input layout
//   zcof     G mod p = scaled gcd / (signed content), then the exact quotients
//            u / G and v / G by long division over Z_p (a nonzero remainder
//            flags a certificate failure)
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "modarith.h"
#include "stages.h"

namespace rsl {

struct ZgcdDesc {
  int nu, nv;           // degrees of u and v (nv = -1: v is zero)
  int Lu, Lv;           // limbs per coefficient
  int np;               // prime slots of the first pass
  int gs;               // row stride of the scaled gcds
  const uint32_t* u;    // (nu + 1) * Lu
  const uint32_t* v;    // (nv + 1) * Lv
  const int* pidx;      // np global prime indices
  const uint32_t* ell;  // np: ell mod p (normal form)
  uint32_t* up;         // np * (nu + 1) residues, normal form
  uint32_t* vp;         // np * (nv + 1)
  uint32_t* gt;         // np * gs: ell * (monic gcd mod p), normal form
  int* gdeg;            // np: degree of the gcd mod p
  // kept slots (least gcd degree)
  int nk, dg;           // kept slots, degree of G
  const int* kept;      // nk slot indices
  const uint32_t* sinv; // nk: (signed content of the scaled gcd)^{-1} mod p, normal form
  uint64_t* c0;         // nk * (dg + 1): scaled gcd, CRT input layout (Montgomery form)
  uint64_t* cg;         // nk * (dg + 1): G mod p
  uint64_t* ca;         // nk * (nu - dg + 1): u / G mod p
  uint64_t* cb;         // nk * (nv - dg + 1): v / G mod p (nv >= dg)
  int* rem;             // [0] set when a division leaves a remainder
};

constexpr int kZThreads = 256;  // reduce and pack; Euclid and the divisions run one wave per slot

// residues of u (sub 0) or v (sub 1): item slot, block of 256 coefficients
__device__ inline void stage_zreduce(const ZgcdDesc& Z, const DevTables& T, const WorkItem& w) {
  const int n = w.sub ? Z.nv : Z.nu, L = w.sub ? Z.Lv : Z.Lu;
  const int t = w.blk * kZThreads + static_cast<int>(threadIdx.x);
  if (t > n) return;
  const PrimeConst pc = T.pc[Z.pidx[w.slot]];
  const uint32_t* src = (w.sub ? Z.v : Z.u) + static_cast<size_t>(t) * L;
  uint32_t* dst = w.sub ? Z.vp : Z.up;
  dst[static_cast<size_t>(w.slot) * (n + 1) + t] = limbs_mod_p(src, L, pc);
}

__host__ __device__ inline int zgcd_lds_words(const ZgcdDesc& Z) { return (Z.nu + 1) + (Z.nv + 2); }

// Degree of a[0..d-1] (its entries below d): the highest nonzero, found 64
// entries at a time by a wave ballot (-1 when all are zero).  Wave-uniform.
__device__ inline int zdeg_below(const uint32_t* a, int d) {
  const int lane = threadIdx.x & 63;
  for (int top = d; top > 0; top -= 64) {
    const int j = top - 64 + lane;
    const uint64_t nz = __ballot(j >= 0 && a[j] != 0u);
    if (nz) return top - 64 + (63 - __clzll(static_cast<long long>(nz)));
  }
  return -1;
}

// One wave per prime slot.  Pseudo-remainder steps without divisions,
//   A <- lc(B) A - lc(A) x^(deg A - deg B) B,
// keep A a nonzero multiple of the remainder sequence's members, so the last
// nonzero one is a multiple of the gcd; one inversion at the end makes it monic.
__device__ inline void stage_zgcd(const ZgcdDesc& Z, const DevTables& T, int slot, uint32_t* lds) {
  const int lane = threadIdx.x;
  const PrimeConst pc = T.pc[Z.pidx[slot]];
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  uint32_t* X = lds;                 // nu + 1 words
  uint32_t* Y = lds + (Z.nu + 1);    // nv + 1 words
  for (int k = lane; k <= Z.nu; k += 64) X[k] = mmul(Z.up[static_cast<size_t>(slot) * (Z.nu + 1) + k], pc.r2, p, pinv);
  for (int k = lane; k <= Z.nv; k += 64) Y[k] = mmul(Z.vp[static_cast<size_t>(slot) * (Z.nv + 1) + k], pc.r2, p, pinv);
  WaveSync()();
  uint32_t* A = X;
  uint32_t* B = Y;
  int da = zdeg_below(X, Z.nu + 1), db = (Z.nv >= 0) ? zdeg_below(Y, Z.nv + 1) : -1;
  if (da < db) {
    uint32_t* t = A; A = B; B = t;
    const int d = da; da = db; db = d;
  }
  while (db >= 0) {
    while (da >= db) {
      const uint32_t la = A[da], lb = B[db];
      const int s = da - db;
      for (int j = lane; j < da; j += 64)
        A[j] = (j >= s) ? mmulsub(lb, A[j], la, B[j - s], p, pinv) : mmul(lb, A[j], p, pinv);
      WaveSync()();
      da = zdeg_below(A, da);
    }
    uint32_t* t = A; A = B; B = t;
    const int d = da; da = db; db = d;
  }
  const uint32_t inv = (da >= 0) ? minv(A[da], one, p, pinv) : 0u;
  for (int k = lane; k <= da; k += 64)
    Z.gt[static_cast<size_t>(slot) * Z.gs + k] = mmul(mmul(A[k], inv, p, pinv), Z.ell[slot], p, pinv);
  if (lane == 0) Z.gdeg[slot] = da;
}

// kept slot i: the scaled gcd in the CRT input layout (Montgomery form: the
// CRT reduces each entry once)
__device__ inline void stage_zpack(const ZgcdDesc& Z, const DevTables& T, int i) {
  const int slot = Z.kept[i];
  const PrimeConst pc = T.pc[Z.pidx[slot]];
  for (int k = threadIdx.x; k <= Z.dg; k += blockDim.x)
    Z.c0[static_cast<size_t>(i) * (Z.dg + 1) + k] =
        mmul(Z.gt[static_cast<size_t>(slot) * Z.gs + k], pc.r2, pc.p, pc.pinv);
}

__host__ __device__ inline int zcof_lds_words(const ZgcdDesc& Z) {
  const int n = Z.nu > Z.nv ? Z.nu : Z.nv;
  return (n + 1) + (Z.dg + 1);
}

// Long division of W (degree n, Montgomery) by G (degree dg, Montgomery,
// inverse leading coefficient ginv): quotient coefficients to q[0..n-dg]
// (Montgomery form, the CRT input layout), remainder check.
__device__ inline void zdivide(uint32_t* W, int n, const uint32_t* G, int dg, uint32_t ginv, uint64_t* q,
                               int* rem, const PrimeConst& pc) {
  const uint32_t p = pc.p, pinv = pc.pinv;
  const int lane = threadIdx.x;
  for (int k = n - dg; k >= 0; --k) {
    const uint32_t qk = mmul(W[k + dg], ginv, p, pinv);
    if (lane == 0) q[k] = qk;
    for (int j = lane; j < dg; j += 64) W[k + j] = msubm(W[k + j], mmul(qk, G[j], p, pinv), p);
    WaveSync()();
  }
  if (zdeg_below(W, dg) >= 0 && lane == 0) rem[0] = 1;
}

// kept slot i: G mod p, then u / G and v / G
__device__ inline void stage_zcof(const ZgcdDesc& Z, const DevTables& T, int i, uint32_t* lds) {
  const int tid = threadIdx.x;
  const int slot = Z.kept[i];
  const PrimeConst pc = T.pc[Z.pidx[slot]];
  const uint32_t p = pc.p, pinv = pc.pinv, one = pc.r1;
  const int n = Z.nu > Z.nv ? Z.nu : Z.nv;
  uint32_t* W = lds;              // n + 1 words
  uint32_t* G = lds + (n + 1);    // dg + 1 words
  const uint32_t sM = mmul(Z.sinv[i], pc.r2, p, pinv);
  for (int k = tid; k <= Z.dg; k += 64) {
    const uint32_t g = mmul(mmul(Z.gt[static_cast<size_t>(slot) * Z.gs + k], pc.r2, p, pinv), sM, p, pinv);
    G[k] = g;
    Z.cg[static_cast<size_t>(i) * (Z.dg + 1) + k] = g;
  }
  for (int k = tid; k <= Z.nu; k += 64) W[k] = mmul(Z.up[static_cast<size_t>(slot) * (Z.nu + 1) + k], pc.r2, p, pinv);
  WaveSync()();
  const uint32_t ginv = minv(G[Z.dg], one, p, pinv);
  zdivide(W, Z.nu, G, Z.dg, ginv, Z.ca + static_cast<size_t>(i) * (Z.nu - Z.dg + 1), Z.rem, pc);
  if (Z.nv < Z.dg) return;  // v = 0 (no cofactor)
  for (int k = tid; k <= Z.nv; k += 64) W[k] = mmul(Z.vp[static_cast<size_t>(slot) * (Z.nv + 1) + k], pc.r2, p, pinv);
  WaveSync()();
  zdivide(W, Z.nv, G, Z.dg, ginv, Z.cb + static_cast<size_t>(i) * (Z.nv - Z.dg + 1), Z.rem, pc);
}

}  // namespace rsl

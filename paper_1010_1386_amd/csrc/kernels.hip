// HIP kernels of the modular resultant pipeline for gfx950 (wave64).
//
//   k_reduce        coefficients (multi-limb) -> residues c R^2 mod p      (paper Sec. 4.1, step 1)
//   k_eval_ures     one lane per (prime, point): Horner evaluation at x_i and
//                   the univariate resultant over Z_p                      (Sec. 4.1, steps 1-2)
//   k_interp_conv   Newton forward differences on consecutive points      (Sec. 4.1, step 3)
//   k_interp_stir   Newton (falling-factorial) basis -> monomial basis
//   k_interp_newton divided differences on a gapped point set (bad points skipped)
//   k_crt           Garner mixed-radix digits + radix conversion to limbs (Sec. 4.1, step 3)
//   k_stirling_build  per-prime table of Stirling numbers of the first kind
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.h"
#include "kernels.h"
#include "ures.h"

namespace rsl {

// ---------------------------------------------------------------- reduce

__global__ __launch_bounds__(256) void k_reduce(DevProblem P, DevTables T) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int ps = blockIdx.y;
  if (t >= P.ncoef) return;
  const PrimeConst pc = T.pc[P.pidx[ps]];
  const uint32_t* w = P.coeff + static_cast<size_t>(t) * P.L_in;
  // two's complement value mod p, top limb signed; -2^31 + 2p > 0 since p > 2^30
  const int32_t top = static_cast<int32_t>(w[P.L_in - 1]);
  uint64_t r = static_cast<uint64_t>(static_cast<int64_t>(top) + 2 * static_cast<int64_t>(pc.p)) % pc.p;
  for (int l = P.L_in - 2; l >= 0; --l) r = ((r << 32) | w[l]) % pc.p;
  P.resid[static_cast<size_t>(ps) * P.CS + t] = mmul(static_cast<uint32_t>(r), pc.r3, pc.p, pc.pinv);
}

// ---------------------------------------------------------- eval + ures

// One wave per (prime, 64 consecutive points); each lane keeps A = f(x_i, y)
// and B = g(x_i, y) in two LDS columns (stride 64 words: conflict-free when
// all lanes touch the same coefficient index).
__global__ __launch_bounds__(64) void k_eval_ures(DevProblem P, DevTables T) {
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x;
  const int ps = blockIdx.y;
  const int pt = blockIdx.x * 64 + lane;
  const PrimeConst pc = T.pc[P.pidx[ps]];
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  Column<64> A{lds + lane};
  Column<64> B{lds + nm1 * 64 + lane};
  const uint32_t x = static_cast<uint32_t>(P.origin + (pt < P.E ? pt : P.E));
  const uint32_t xt = mmul(x, pc.r2, pc.p, pc.pinv);
  const uint32_t* tile = P.resid + static_cast<size_t>(ps) * P.CS;
  eval_rows(A, tile, P.my + 1, P.rowf, P.rdeg, xt, pc.p, pc.pinv);
  eval_rows(B, tile + P.goff, P.ny + 1, P.rowg, P.rdeg + P.my + 1, xt, pc.p, pc.pinv);
  bool bad = false;
  const uint32_t r = ures_formal(A, B, P.my, P.ny, pc, &bad);
  const bool live = pt <= P.E;
  if (live) {
    const size_t o = static_cast<size_t>(ps) * (P.E + 1) + pt;
    P.zval[o] = redc(r, pc.p, pc.pinv);
    P.zbad[o] = bad ? 1 : 0;
  }
  const uint64_t nbad = __ballot(live && bad);
  if (lane == 0 && nbad) atomicAdd(P.status + 1 + P.np, __popcll(nbad));
}

// ---------------------------------------------------------- interpolation

// The consecutive fast path applies when the D+1 points used are origin 0..D:
// always with formal-degree values at origin 0, otherwise when none of the
// points 0..D was flagged bad.  Block-uniform result.
__device__ bool fast_prime(const DevProblem& P, int ps) {
  if (P.origin != 0) return false;
  if (P.formal) return true;
  const uint8_t* zb = P.zbad + static_cast<size_t>(ps) * (P.E + 1);
  int any = 0;
  for (int i = threadIdx.x; i <= P.D; i += blockDim.x) any |= zb[i];
  return __syncthreads_or(any) == 0;
}

// a -> a + x y with a kept below p 2^32 (fold of the high word)
__device__ __forceinline__ uint64_t mac_fold(uint64_t acc, uint32_t x, uint32_t y, uint32_t p) {
  acc += static_cast<uint64_t>(x) * y;
  uint32_t hi = static_cast<uint32_t>(acc >> 32);
  hi = umin32(hi, hi - p);
  return (static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(acc);
}

// Newton forward differences at 0..D as a convolution:
//   a_k = Delta^k z_0 / k! = sum_{i<=k} (z_i / i!) ((-1)^(k-i) / (k-i)!)
__global__ __launch_bounds__(256) void k_interp_conv(DevProblem P, DevTables T) {
  extern __shared__ uint32_t sm[];
  const int ps = blockIdx.y;
  if (!fast_prime(P, ps)) return;
  const int g = P.pidx[ps];
  const PrimeConst pc = T.pc[g];
  const uint32_t* ifact = T.ifact + static_cast<size_t>(g) * T.kstride;
  const int k0 = blockIdx.x * 256;
  const int kmax = (k0 + 255 < P.D) ? k0 + 255 : P.D;
  uint32_t* alpha = sm;
  uint32_t* beta = sm + (kmax + 1);
  const uint32_t* z = P.zval + static_cast<size_t>(ps) * (P.E + 1);
  for (int i = threadIdx.x; i <= kmax; i += 256) {
    const uint32_t f = ifact[i];
    alpha[i] = mmul(z[i], f, pc.p, pc.pinv);       // z_i / i!          (normal)
    beta[i] = (i & 1) ? mneg(f, pc.p) : f;         // (-1)^i / i! R     (Montgomery)
  }
  __syncthreads();
  const int k = k0 + threadIdx.x;
  if (k > P.D) return;
  uint64_t acc = 0;
  for (int i = 0; i <= k; ++i) acc = mac_fold(acc, alpha[i], beta[k - i], pc.p);
  P.aconv[static_cast<size_t>(ps) * (P.D + 1) + k] = redc(acc, pc.p, pc.pinv);
}

// Falling-factorial basis -> monomials: c_j = sum_{k>=j} a_k s(k, j).
__global__ __launch_bounds__(256) void k_interp_stir(DevProblem P, DevTables T) {
  extern __shared__ uint32_t sm[];
  const int ps = blockIdx.y;
  if (!fast_prime(P, ps)) return;
  const int g = P.pidx[ps];
  const PrimeConst pc = T.pc[g];
  const int j0 = blockIdx.x * 256;
  const uint32_t* a = P.aconv + static_cast<size_t>(ps) * (P.D + 1);
  for (int k = j0 + threadIdx.x; k <= P.D; k += 256) sm[k - j0] = a[k];
  __syncthreads();
  const int j = j0 + threadIdx.x;
  const uint32_t* S = T.stir + static_cast<int64_t>(g) * T.sstride;
  uint64_t acc = 0;
  for (int k = j0; k <= P.D; ++k) {
    const uint32_t* row = S + static_cast<int64_t>(k) * (k + 1) / 2;
    if (j <= k) acc = mac_fold(acc, sm[k - j0], row[j], pc.p);
  }
  if (j <= P.D) P.cres[static_cast<size_t>(ps) * (P.D + 1) + j] = redc(acc, pc.p, pc.pinv);
}

// Gapped point sets (bad points replaced, or a shifted origin): one block per
// prime; select the first D+1 usable points, Newton divided differences, then
// the Newton form expanded by Horner in the monomial basis.
__global__ __launch_bounds__(1024) void k_interp_newton(DevProblem P, DevTables T) {
  extern __shared__ uint32_t sm[];
  const int ps = blockIdx.x;
  const int tid = threadIdx.x;
  const bool fast = fast_prime(P, ps);
  if (tid == 0) P.status[1 + ps] = fast ? 0 : 1;
  if (fast) return;
  const int g = P.pidx[ps];
  const PrimeConst pc = T.pc[g];
  const uint32_t p = pc.p, pinv = pc.pinv;
  const int E = P.E, D = P.D;
  const uint32_t* fact = T.fact + static_cast<size_t>(g) * T.kstride;
  const uint32_t* ifact = T.ifact + static_cast<size_t>(g) * T.kstride;
  const uint32_t* z = P.zval + static_cast<size_t>(ps) * (E + 1);
  const uint8_t* zb = P.zbad + static_cast<size_t>(ps) * (E + 1);

  uint32_t* xs = sm;              // E+1: selected point indices
  uint32_t* d0 = xs + (E + 1);    // E+1
  uint32_t* d1 = d0 + (E + 1);    // E+1
  uint32_t* invt = d1 + (E + 1);  // E+1: 1/t R mod p
  __shared__ int cnt[1024];

  for (int t = tid + 1; t <= E; t += 1024) invt[t] = mmul(ifact[t], fact[t - 1], p, pinv);

  // selection: first D+1 usable points (all points in formal mode)
  const int chunk = (E + 1 + 1023) / 1024;
  const int lo = tid * chunk;
  const int hi = (lo + chunk < E + 1) ? lo + chunk : E + 1;
  int c = 0;
  for (int i = lo; i < hi; ++i) c += (P.formal || !zb[i]) ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    int v = (tid >= off) ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  if (cnt[1023] < D + 1) {
    if (tid == 0) atomicOr(P.status, kErrTooFewGoodPoints);
    return;  // block-uniform
  }
  int q = cnt[tid] - c;
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
    for (int i = tid; i <= D; i += 1024) {
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
  // cur[] holds a_0..a_D; build the polynomial in nxt/d-buffers.
  uint32_t* coef = invt;  // reuse: invt no longer needed after the differences
  __syncthreads();
  uint32_t* poly = nxt;
  for (int i = tid; i <= D; i += 1024) {
    coef[i] = cur[i];
    poly[i] = 0;
  }
  __syncthreads();
  if (tid == 0) poly[0] = coef[D];
  __syncthreads();
  uint32_t* pa = poly;
  uint32_t* pb = cur;
  for (int k = D - 1; k >= 0; --k) {
    const uint32_t xk = static_cast<uint32_t>(P.origin) + xs[k];
    const uint32_t xkt = mmul(xk, pc.r2, p, pinv);
    const int deg = D - k;  // degree after this step
    for (int j = tid; j <= deg; j += 1024) {
      const uint32_t left = (j > 0) ? pa[j - 1] : 0u;
      const uint32_t mid = (j < deg) ? pa[j] : 0u;
      uint32_t v = msubm(left, mmul(mid, xkt, p, pinv), p);
      if (j == 0) v = maddm(v, coef[k], p);
      pb[j] = v;
    }
    __syncthreads();
    uint32_t* t = pa; pa = pb; pb = t;
  }
  for (int j = tid; j <= D; j += 1024) P.cres[static_cast<size_t>(ps) * (D + 1) + j] = pa[j];
}

// ---------------------------------------------------------------- CRT

// One wave per coefficient k.  Garner: lanes own primes (slot i = lane + 64 r);
// digit v_j is formed in lane j and broadcast, then every lane i > j adds
// v_j * (prod_{l<j} p_l mod p_i).  Radix conversion: lanes own output limbs,
// S_t = NH_t + sum_j v_j * limb_t(prod_{l<j} p_l) in 96 bits, then carries are
// resolved with wave ballots.  The result is (Y - H) mod 2^(32 L_out) with
// Y = sum_j v_j prod_{l<j} p_l in [0, M) and H = (M-1)/2: the symmetric residue.
template <int NS>
__global__ __launch_bounds__(256) void k_crt(DevProblem P, DevTables T) {
  __shared__ uint32_t vbuf[4][64 * NS];
  __shared__ uint32_t sb[4][64 * NS + 2];
  __shared__ uint32_t sc[4][64 * NS + 2];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int k_raw = blockIdx.x * 4 + wave;
  const bool valid = k_raw <= P.D;
  const int k = valid ? k_raw : P.D;
  const int np = P.np;

  uint32_t u[NS], acc[NS], pp[NS], pinv[NS], invm[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int i = lane + 64 * r;
    acc[r] = 0;
    if (i < np) {
      const PrimeConst pc = T.pc[P.pidx[i]];
      pp[r] = pc.p;
      pinv[r] = pc.pinv;
      u[r] = maddm(P.cres[static_cast<size_t>(i) * (P.D + 1) + k], P.Hm[i], pc.p);
      invm[r] = P.invM[i];
    } else {
      pp[r] = 3u; pinv[r] = 0u; u[r] = 0u; invm[r] = 0u;
    }
  }
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    for (int jj = 0; jj < 64; ++jj) {
      const int j = r * 64 + jj;
      if (j >= np) break;
      const uint32_t vloc = mmul(msubm(u[r], acc[r], pp[r]), invm[r], pp[r], pinv[r]);
      const uint32_t vj = __builtin_amdgcn_readlane(vloc, jj);
      if (lane == 0) vbuf[wave][j] = vj;
      const uint32_t* trow = P.Tg + static_cast<size_t>(j) * P.tgs;
#pragma unroll
      for (int rr = r; rr < NS; ++rr) {
        const int i = lane + 64 * rr;
        if (i > j && i < np)
          acc[rr] = maddm(acc[rr], mmul(vj, trow[i], pp[rr], pinv[rr]), pp[rr]);
      }
    }
  }
  __syncthreads();

  // radix conversion: 96-bit column sums per output limb
  const int L = P.L_out;
  uint64_t lo[NS];
  uint32_t hc[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    lo[r] = (t < L) ? P.NH[t] : 0u;
    hc[r] = 0u;
  }
  for (int j = 0; j < np; ++j) {
    const uint32_t vj = vbuf[wave][j];
    const uint32_t* pl = P.Plimb + static_cast<size_t>(j) * P.LP;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int t = lane + 64 * r;
      if (t < L) {
        const uint64_t prod = static_cast<uint64_t>(vj) * pl[t];
        lo[r] += prod;
        hc[r] += (lo[r] < prod) ? 1u : 0u;
      }
    }
  }
  // limb t receives lo32(S_t) + hi32(S_{t-1}) + top32(S_{t-2})
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    sb[wave][t + 1] = static_cast<uint32_t>(lo[r] >> 32);
    sc[wave][t + 2] = hc[r];
  }
  if (lane == 0) { sb[wave][0] = 0; sc[wave][0] = 0; sc[wave][1] = 0; }
  __syncthreads();
  uint32_t l1[NS], h1[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    const uint64_t w = static_cast<uint64_t>(static_cast<uint32_t>(lo[r])) + sb[wave][t] + sc[wave][t];
    l1[r] = static_cast<uint32_t>(w);
    h1[r] = static_cast<uint32_t>(w >> 32);  // <= 2
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NS; ++r) sb[wave][lane + 64 * r + 1] = h1[r];
  __syncthreads();
  uint64_t cin = 0;
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int t = lane + 64 * r;
    const uint64_t x2 = static_cast<uint64_t>(l1[r]) + sb[wave][t];
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

// ------------------------------------------------------------- Stirling table

// s(k+1, j) = s(k, j-1) - k s(k, j); one block per prime, rows in LDS.
__global__ __launch_bounds__(1024) void k_stirling_build(uint32_t* stir, int64_t sstride,
                                                         const PrimeConst* pcs, int g0, int scap) {
  extern __shared__ uint32_t sm[];
  const int g = g0 + blockIdx.x;
  const PrimeConst pc = pcs[g];
  uint32_t* cur = sm;
  uint32_t* nxt = sm + (scap + 2);
  uint32_t* S = stir + static_cast<int64_t>(g) * sstride;
  if (threadIdx.x == 0) { cur[0] = pc.r1; S[0] = pc.r1; }
  __syncthreads();
  for (int k = 0; k < scap; ++k) {
    const uint32_t kt = mmul(static_cast<uint32_t>(k), pc.r2, pc.p, pc.pinv);
    uint32_t* row = S + static_cast<int64_t>(k + 1) * (k + 2) / 2;
    for (int j = threadIdx.x; j <= k + 1; j += 1024) {
      const uint32_t left = (j > 0) ? cur[j - 1] : 0u;
      const uint32_t mid = (j <= k) ? cur[j] : 0u;
      const uint32_t v = msubm(left, mmul(mid, kt, pc.p, pc.pinv), pc.p);
      nxt[j] = v;
      row[j] = v;
    }
    __syncthreads();
    uint32_t* t = cur; cur = nxt; nxt = t;
  }
}

// ------------------------------------------------------------ launchers

static inline int blocks_of(int n, int b) { return (n + b - 1) / b; }

hipError_t launch_pipeline(const DevProblem& P, const DevTables& T, hipStream_t st) {
  const int ncoef = P.ncoef;
  hipLaunchKernelGGL(k_reduce, dim3(blocks_of(ncoef, 256), P.np), dim3(256), 0, st, P, T);
  const int nm1 = (P.my > P.ny ? P.my : P.ny) + 1;
  hipLaunchKernelGGL(k_eval_ures, dim3(blocks_of(P.E + 1, 64), P.np), dim3(64),
                     static_cast<size_t>(2) * nm1 * 64 * sizeof(uint32_t), st, P, T);
  const int nb = blocks_of(P.D + 1, 256);
  hipLaunchKernelGGL(k_interp_conv, dim3(nb, P.np), dim3(256),
                     static_cast<size_t>(2) * (P.D + 1) * sizeof(uint32_t), st, P, T);
  hipLaunchKernelGGL(k_interp_stir, dim3(nb, P.np), dim3(256),
                     static_cast<size_t>(P.D + 1) * sizeof(uint32_t), st, P, T);
  hipLaunchKernelGGL(k_interp_newton, dim3(P.np), dim3(1024),
                     static_cast<size_t>(4) * (P.E + 1) * sizeof(uint32_t), st, P, T);
  const int ns = (P.np + 63) / 64;
  const dim3 gc(blocks_of(P.D + 1, 4));
  switch (ns) {
    case 1: hipLaunchKernelGGL(k_crt<1>, gc, dim3(256), 0, st, P, T); break;
    case 2: hipLaunchKernelGGL(k_crt<2>, gc, dim3(256), 0, st, P, T); break;
    case 3: hipLaunchKernelGGL(k_crt<3>, gc, dim3(256), 0, st, P, T); break;
    case 4: hipLaunchKernelGGL(k_crt<4>, gc, dim3(256), 0, st, P, T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stirling_build(uint32_t* stir, int64_t sstride, const PrimeConst* pcs, int g0,
                                 int count, int scap, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stirling_build, dim3(count), dim3(1024),
                     static_cast<size_t>(2) * (scap + 2) * sizeof(uint32_t), st, stir, sstride, pcs,
                     g0, scap);
  return hipGetLastError();
}

}  // namespace rsl

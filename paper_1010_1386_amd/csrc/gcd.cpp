// gcd over Z[x] and the square-free part by the modular route (include/rsl.h:
// rsl_gcd, rsl_sqfree_part; device stages in zgcd.h).
//
//   1. primes (not dividing lc u or lc v) until their product passes twice the
//      certificate bound below, plus a few spare;
//   2. per prime on the device: u, v mod p, Euclid over Z_p, the gcd made monic
//      and scaled by ell = gcd(lc u, lc v) (lc G divides ell);
//   3. the primes of least gcd degree are kept (the others are unlucky);
//      Chinese remaindering gives G~ = (ell / lc G) G, whose content s is
//      removed modularly: G mod p = G~ mod p / (sign s), then u / G and v / G
//      mod p by exact long division, and Chinese remaindering of all three;
//   4. certificate: with Mignotte's bounds B_G, B_u, B_v on factors of u and v,
//      the kept product exceeds 2 (deg u + deg v + 2) B_G max(B_u, B_v); every
//      reconstructed coefficient is checked against its bound and every
//      division left no remainder, so G (u/G) = u and G (v/G) = v hold over Z;
//      G divides u and v and has the least modular degree, hence is the gcd.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"
#include "kernels.h"
#include "plan.h"

namespace rsl {
namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int blocks_of(int n, int b) { return (n + b - 1) / b; }

struct UPoly {  // trimmed univariate polynomial, two's complement limbs
  int deg = -1, L = 1;
  std::vector<uint32_t> c;  // (deg + 1) * L
  const uint32_t* at(int k) const { return c.data() + static_cast<size_t>(k) * L; }
};

int read_upoly(const rsl_upoly* in, UPoly* out, std::string* err) {
  if (!in || in->deg < -1 || in->deg > (1 << 20) || in->limbs < 1 || in->limbs > 4096 ||
      (in->deg >= 0 && !in->coeff)) {
    *err = "invalid univariate polynomial descriptor";
    return RSL_EINVAL;
  }
  const int L = in->limbs;
  int d = in->deg;
  auto nonzero = [&](int k) {
    for (int l = 0; l < L; ++l)
      if (in->coeff[static_cast<size_t>(k) * L + l]) return true;
    return false;
  };
  while (d >= 0 && !nonzero(d)) --d;
  out->L = L;
  out->deg = d;
  out->c.assign(in->coeff, in->coeff + static_cast<size_t>(d + 1) * L);
  return RSL_OK;
}

// u': coefficient k is (k + 1) u_{k+1}, one limb wider (two's complement
// product by a small positive factor, exact in the wider width)
UPoly derivative(const UPoly& u) {
  UPoly r;
  r.L = u.L + 1;
  r.deg = u.deg - 1;
  if (r.deg < 0) {
    r.deg = -1;
    return r;
  }
  r.c.assign(static_cast<size_t>(r.deg + 1) * r.L, 0u);
  for (int k = 0; k <= r.deg; ++k) {
    const uint32_t* s = u.at(k + 1);
    const uint64_t ext = (s[u.L - 1] >> 31) ? 0xFFFFFFFFull : 0ull;
    uint64_t carry = 0;
    for (int l = 0; l < r.L; ++l) {
      carry += ((l < u.L) ? s[l] : ext) * static_cast<uint64_t>(k + 1);
      r.c[static_cast<size_t>(k) * r.L + l] = static_cast<uint32_t>(carry);
      carry >>= 32;
    }
  }
  return r;
}

BigU abs_coeff(const UPoly& u, int k, bool* neg) { return abs_limbs(u.at(k), u.L, neg); }

// ||u||_2 < 2^bits
int norm2_bits(const UPoly& u) {
  BigU s;
  for (int k = 0; k <= u.deg; ++k) {
    bool n;
    const BigU a = abs_coeff(u, k, &n);
    s = BigU::add(s, BigU::mul(a, a));
  }
  return (s.bitlen() + 2) / 2;
}

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = r * a % m;
    a = a * a % m;
    e >>= 1;
  }
  return r;
}

int bitlen_i(int64_t v) {
  int b = 0;
  while (v > 0) {
    ++b;
    v >>= 1;
  }
  return b;
}

// Bump allocator over the context workspace (null, and bad, past its end).
// Uploads of a phase are gathered on the host and sent by flush() as one copy
// from pinned memory.
struct Dev {
  uint8_t* base;
  size_t cap, used = 0;
  bool bad = false;
  std::vector<uint8_t> host;  // staged bytes of [lo, hi)
  size_t lo = 0, hi = 0;
  template <class T>
  T* take(size_t count) {
    const size_t at = align_up(used, 256), bytes = sizeof(T) * std::max<size_t>(count, 1);
    if (bad || at + bytes > cap) {
      bad = true;
      return nullptr;
    }
    used = at + bytes;
    return reinterpret_cast<T*>(base + at);
  }
  void put(void* dst, const void* src, size_t bytes) {
    if (!bytes || !dst) return;
    const size_t off = static_cast<uint8_t*>(dst) - base;
    if (hi == lo) lo = hi = off;
    if (off < lo) {  // allocations only grow: not expected, but keep it correct
      host.insert(host.begin(), lo - off, 0u);
      lo = off;
    }
    if (off + bytes > hi) {
      host.resize(off + bytes - lo, 0u);
      hi = off + bytes;
    }
    std::memcpy(host.data() + (off - lo), src, bytes);
  }
};

int flush(rsl_ctx* ctx, Dev* D) {
  if (D->bad) return fail(ctx, RSL_ENOMEM, "workspace smaller than the gcd footprint");
  if (D->hi == D->lo) return RSL_OK;
  const size_t n = D->hi - D->lo;
  // the pinned buffer may still feed an earlier copy of this call
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  if (!rc) rc = ensure_staging(ctx, n, 0);
  if (rc) return rc;
  std::memcpy(ctx->h_up, D->host.data(), n);
  rc = hip_check(ctx, hipMemcpyAsync(D->base + D->lo, ctx->h_up, n, hipMemcpyHostToDevice, ctx->stream), "upload");
  D->host.clear();
  D->lo = D->hi = 0;
  return rc;
}

// Device copies of a prime list's CRT tables.
struct CrtDev {
  Plan P;
  int* pidx = nullptr;
  uint32_t *Hm = nullptr, *NH = nullptr, *Mi = nullptr, *wdir = nullptr, *rinv = nullptr, *negM = nullptr;
  uint32_t *Mw = nullptr, *NHM = nullptr, *Tg = nullptr, *invM = nullptr, *Plimb = nullptr;
};

template <class T>
int upload_vec(rsl_ctx* ctx, Dev* D, const std::vector<T>& v, T** out) {
  *out = D->take<T>(v.size());
  if (!*out) return fail(ctx, RSL_ENOMEM, "workspace smaller than the gcd footprint");
  D->put(*out, v.data(), v.size() * sizeof(T));
  return RSL_OK;
}

int crt_setup(rsl_ctx* ctx, Dev* D, const std::vector<int>& pidx, CrtDev* C) {
  C->P = Plan();
  C->P.pidx = pidx;
  plan_crt(&C->P);
  const Plan& P = C->P;
  int rc;
  if ((rc = upload_vec(ctx, D, P.pidx, &C->pidx)) || (rc = upload_vec(ctx, D, P.crt->Hm, &C->Hm)) ||
      (rc = upload_vec(ctx, D, P.crt->NH, &C->NH)) || (rc = upload_vec(ctx, D, P.crt->Mi, &C->Mi)) ||
      (rc = upload_vec(ctx, D, P.crt->wdir, &C->wdir)) || (rc = upload_vec(ctx, D, P.crt->rinv, &C->rinv)) ||
      (rc = upload_vec(ctx, D, P.crt->negM, &C->negM)))
    return rc;
  if (P.wide && ((rc = upload_vec(ctx, D, P.crt->Mw, &C->Mw)) || (rc = upload_vec(ctx, D, P.crt->NHM, &C->NHM)))) return rc;
  if (!P.canonical && !P.wide &&
      ((rc = upload_vec(ctx, D, P.crt->Tg, &C->Tg)) || (rc = upload_vec(ctx, D, P.crt->invM, &C->invM)) ||
       (rc = upload_vec(ctx, D, P.crt->Plimb, &C->Plimb))))
    return rc;
  return RSL_OK;
}

// A CRT problem over the residues cpart[i][k] (k <= Dg, Montgomery form) into out.
DevProblem crt_problem(const rsl_ctx* ctx, Dev* D, const CrtDev& C, int Dg, uint64_t* cpart, uint32_t* out) {
  const Plan& P = C.P;
  DevProblem d{};
  d.D = Dg;
  d.np = P.np;
  d.L_out = P.L_out;
  d.Lw = P.Lw;
  d.wide = P.wide ? 1 : 0;
  d.kchunk = Dg + 1;
  d.nchunk = 1;
  d.crt_garner = ctx->crt_garner ? 1 : 0;
  d.cpart = cpart;
  d.out = out;
  d.pidx = C.pidx;
  d.Hm = C.Hm;
  d.NH = C.NH;
  d.Mi = C.Mi;
  d.wdir = C.wdir;
  d.rinv = C.rinv;
  d.negM = C.negM;
  d.Mw = C.Mw;
  d.NHM = C.NHM;
  if (P.canonical) {
    d.Tg = ctx->d_Tg;
    d.tgs = ctx->garner_np;
    d.invM = ctx->d_invM;
    d.Plimb = ctx->d_Plimb;
    d.LP = ctx->LPg;
  } else {
    d.Tg = C.Tg;
    d.tgs = P.np;
    d.invM = C.invM;
    d.Plimb = C.Plimb;
    d.LP = P.L_out;
  }
  if (P.wide) {  // the vector-ALU contraction (rows of wT padded to a multiple of 64 primes)
    d.wnpad = (P.np + 63) / 64 * 64;
    d.wdpad = (Dg + 1 + 63) / 64 * 64;
    d.wT = D->take<uint32_t>(static_cast<size_t>(d.wdpad) * d.wnpad);
    d.wq = D->take<uint32_t>(Dg + 1);
    d.wS = D->take<uint64_t>(static_cast<size_t>(Dg + 1) * 2 * P.Lw);
  }
  return d;
}

// Chinese remaindering of several problems (same prime list) in one launch per pass.
int run_crt(rsl_ctx* ctx, Dev* D, const std::vector<DevProblem>& probs) {
  if (probs.empty()) return RSL_OK;
  const bool wide = probs[0].wide != 0;
  const int np = probs[0].np;
  DevProblem* dprobs = nullptr;
  int rc = upload_vec(ctx, D, probs, &dprobs);
  if (rc) return rc;
  const DevTables T = tables_of(ctx);
  if (!wide) {
    int ns = (np + 63) / 64;
    if (ns == 5 || ns == 7) ++ns;
    std::vector<WorkItem> items;
    size_t lds = 0;
    for (size_t q = 0; q < probs.size(); ++q) {
      for (int b = 0; b < blocks_of(probs[q].D + 1, kCrtWaves); ++b) items.push_back({static_cast<int>(q), -1, b, 0});
      lds = std::max(lds, static_cast<size_t>(crt_lds_words(probs[q], ns, crt_block_waves(ns))) * 4);
    }
    WorkItem* ditems = nullptr;
    if ((rc = upload_vec(ctx, D, items, &ditems)) || (rc = flush(ctx, D))) return rc;
    return hip_check(ctx, launch_stage(kStageCrt, dprobs, ditems, static_cast<int>(items.size()), lds, ns, T, ctx->stream),
                     "gcd CRT");
  }
  std::vector<WorkItem> items[3];
  size_t lds[3] = {static_cast<size_t>(wide_t_lds_words()) * 4, static_cast<size_t>(wide_sum_lds_words()) * 4, 0};
  for (size_t q = 0; q < probs.size(); ++q) {
    const DevProblem& d = probs[q];
    const int qi = static_cast<int>(q);
    for (int b = 0; b < blocks_of(d.D + 1, kWideTCoeffs); ++b) items[0].push_back({qi, -1, b, 0});
    for (int ht = 0; ht < blocks_of(d.Lw, kWideHT); ++ht)
      for (int kt = 0; kt < blocks_of(d.D + 1, kWideKT); ++kt) items[1].push_back({qi, -1, kt, ht});
    for (int k = 0; k <= d.D; ++k) items[2].push_back({qi, -1, k, 0});
    lds[2] = std::max(lds[2], static_cast<size_t>(wide_fin_lds_words(d)) * 4);
  }
  WorkItem* ditems[3];
  for (int pass = 0; pass < 3; ++pass)
    if ((rc = upload_vec(ctx, D, items[pass], &ditems[pass]))) return rc;
  if ((rc = flush(ctx, D))) return rc;
  for (int pass = 0; pass < 3; ++pass)
    if ((rc = hip_check(ctx, launch_crt_wide(pass, dprobs, ditems[pass], static_cast<int>(items[pass].size()), lds[pass],
                                             T, ctx->stream),
                        "gcd CRT")))
      return rc;
  return RSL_OK;
}

int download(rsl_ctx* ctx, void* dst, const void* src, size_t bytes) {
  int rc = hip_check(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream), "download");
  if (rc) return rc;
  return hip_check(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
}

// bit length of the largest |coefficient| of a CRT output ((D+1) x L limbs)
int max_bits(const std::vector<uint32_t>& limbs, int D, int L) {
  int b = 0;
  for (int k = 0; k <= D; ++k) {
    bool n;
    b = std::max(b, abs_limbs(limbs.data() + static_cast<size_t>(k) * L, L, &n).bitlen());
  }
  return b;
}

void put_zero(rsl_result* r) {
  if (r) {
    r->deg = -1;
    r->needed_limbs = 1;
  }
}

// CRT output limbs ((D + 1) x L) as a trimmed polynomial
UPoly as_upoly(const std::vector<uint32_t>& limbs, int D, int L) {
  UPoly r;
  r.L = L;
  r.deg = D;
  auto nonzero = [&](int k) {
    for (int l = 0; l < L; ++l)
      if (limbs[static_cast<size_t>(k) * L + l]) return true;
    return false;
  };
  while (r.deg >= 0 && !nonzero(r.deg)) --r.deg;
  r.c.assign(limbs.begin(), limbs.begin() + static_cast<size_t>(r.deg + 1) * L);
  return r;
}

int write_result(const UPoly& u, rsl_result* r) {
  if (!r) return RSL_OK;
  if (u.deg < 0) {
    put_zero(r);
    return RSL_OK;
  }
  Plan shape;
  shape.L_out = u.L;
  shape.D = u.deg;
  return decode_result(shape, u.c.data(), r);
}

// x - y, one limb wider than the wider operand
UPoly sub_upoly(const UPoly& x, const UPoly& y) {
  UPoly r;
  r.L = std::max(x.L, y.L) + 1;
  const int n = std::max(x.deg, y.deg);
  r.c.assign(static_cast<size_t>(n + 1) * r.L, 0u);
  auto limb = [](const UPoly& u, int k, int l) -> uint32_t {
    if (k > u.deg) return 0u;
    const uint32_t* c = u.at(k);
    return (l < u.L) ? c[l] : ((c[u.L - 1] >> 31) ? 0xFFFFFFFFu : 0u);
  };
  for (int k = 0; k <= n; ++k) {
    int64_t borrow = 0;
    for (int l = 0; l < r.L; ++l) {
      const int64_t v = static_cast<int64_t>(limb(x, k, l)) - limb(y, k, l) - borrow;
      borrow = v < 0 ? 1 : 0;
      r.c[static_cast<size_t>(k) * r.L + l] = static_cast<uint32_t>(v + (borrow << 32));
    }
  }
  r.deg = n;
  std::vector<uint32_t> tmp = r.c;
  return as_upoly(tmp, n, r.L);
}

// G = gcd(pp(u), pp(v)), A = u / G, B = v / G (see the file comment)
int gcd_core(rsl_ctx* ctx, const UPoly& u, const UPoly& v, UPoly* gout, UPoly* uout, UPoly* vout) {
  if (u.deg < 0 && v.deg < 0) {
    *gout = *uout = *vout = UPoly();
    return RSL_OK;
  }
  if (u.deg < 0) return gcd_core(ctx, v, u, gout, vout, uout);
  const int nu = u.deg, nv = v.deg;  // nv = -1: v is zero
  if (nv < 0) {
    // gcd(u, 0) = pp(u), u / G = sign(lc u) content(u): a one-limb content (the
    // usual case) is found and divided out on the host, with no modular work;
    // a larger one takes the modular route below
    BigU s;
    for (int k = nu; k >= 0; --k) {
      bool n;
      const BigU c = abs_coeff(u, k, &n);
      if (c.is_zero()) continue;
      s = (s.d.size() == 1) ? BigU::gcd(s, BigU(c.mod_small(s.d[0]))) : BigU::gcd(s, c);
      if (s.d.size() == 1 && s.d[0] == 1u) break;
    }
    if (s.d.size() == 1) {
      const uint32_t sv = s.d[0];
      auto put_signed = [](const BigU& mag, bool negative, uint32_t* out, int L) {
        for (int l = 0; l < L; ++l) out[l] = l < static_cast<int>(mag.d.size()) ? mag.d[l] : 0u;
        if (negative) {
          uint64_t carry = 1;
          for (int l = 0; l < L; ++l) {
            const uint64_t t = static_cast<uint64_t>(~out[l]) + carry;
            out[l] = static_cast<uint32_t>(t);
            carry = t >> 32;
          }
        }
      };
      bool lneg;
      (void)abs_coeff(u, nu, &lneg);
      UPoly G;
      G.deg = nu;
      G.L = u.L + 1;  // |u_k| / s with the sign of u_k / lc(u) always fits
      G.c.assign(static_cast<size_t>(nu + 1) * G.L, 0u);
      for (int k = 0; k <= nu; ++k) {
        bool n;
        BigU c = abs_coeff(u, k, &n);
        if (sv != 1u) c = c.div_small(sv);
        put_signed(c, n != lneg, G.c.data() + static_cast<size_t>(k) * G.L, G.L);
      }
      UPoly A;
      A.deg = 0;
      A.L = 2;
      A.c.assign(2, 0u);
      put_signed(BigU(sv), lneg, A.c.data(), 2);
      *gout = G;
      *uout = A;
      *vout = UPoly();
      return RSL_OK;
    }
  }
  bool neg;
  const BigU lcu = abs_coeff(u, nu, &neg);
  const BigU lcv = (nv >= 0) ? abs_coeff(v, nv, &neg) : BigU();
  const BigU ell = BigU::gcd(lcu, lcv);
  const int bu = norm2_bits(u), bv = (nv >= 0) ? norm2_bits(v) : 0;
  const int bG = (nv >= 0) ? std::min(nu, nv) + std::min(bu, bv) : nu + bu;
  const int bA = nu + bu, bB = (nv >= 0) ? nv + bv : 0;
  const int need = 2 + bitlen_i(nu + std::max(nv, 0) + 2) + bG + std::max(bA, bB);

  for (int spare = 3; spare <= 48; spare *= 2) {
    // primes: skip those dividing a leading coefficient
    std::vector<int> pidx;
    std::vector<uint32_t> ellp;
    {
      int bits = 0;
      for (size_t k = 0; static_cast<int>(pidx.size()) < kMaxPrimes * 4; ++k) {
        size_t have = 0;
        const uint32_t* tab = prime_table(k + 1, &have);
        if (k >= have) return fail(ctx, RSL_EPRIMES, "prime table exhausted");
        const uint32_t p = tab[k];
        if (lcu.mod_small(p) == 0 || (nv >= 0 && lcv.mod_small(p) == 0)) continue;
        pidx.push_back(static_cast<int>(k));
        ellp.push_back(ell.mod_small(p));
        bits += 30;  // every table prime exceeds 2^30
        if (bits > need + 31 * spare) break;
      }
    }
    const int np = static_cast<int>(pidx.size());
    if (np > kMaxPrimes) return fail(ctx, RSL_EINVAL, "gcd needs more than 4096 primes (inputs too large)");
    if (ctx->server) return workspace_taken(ctx);
    int rc = ensure_tables(ctx, pidx.back() + 1, std::max(ctx->kcap, 0), std::max(ctx->scap, 0));
    if (rc) return rc;
    const DevTables T = tables_of(ctx);

    Dev D{ctx->ws, ctx->ws_bytes};
    ZgcdDesc Z{};
    Z.nu = nu;
    Z.nv = nv;
    Z.Lu = u.L;
    Z.Lv = v.L;
    Z.np = np;
    Z.gs = (nv >= 0 ? std::min(nu, nv) : nu) + 1;
    std::vector<WorkItem> items;
    for (int s = 0; s < np; ++s) {
      for (int b = 0; b < blocks_of(nu + 1, kZThreads); ++b) items.push_back({0, s, b, 0});
      for (int b = 0; b < blocks_of(nv + 1, kZThreads); ++b) items.push_back({0, s, b, 1});
    }
    uint32_t *du = D.take<uint32_t>(u.c.size()), *dv = D.take<uint32_t>(v.c.size());
    int* dp = D.take<int>(np);
    uint32_t* dell = D.take<uint32_t>(np);
    WorkItem* ditems = D.take<WorkItem>(items.size());
    Z.up = D.take<uint32_t>(static_cast<size_t>(np) * (nu + 1));
    Z.vp = D.take<uint32_t>(static_cast<size_t>(np) * (nv + 1));
    Z.gt = D.take<uint32_t>(static_cast<size_t>(np) * Z.gs);
    Z.gdeg = D.take<int>(np);
    if (D.bad) return fail(ctx, RSL_ENOMEM, "workspace smaller than the gcd footprint");
    Z.u = du;
    Z.v = dv;
    Z.pidx = dp;
    Z.ell = dell;
    D.put(du, u.c.data(), u.c.size() * 4);
    D.put(dv, v.c.data(), v.c.size() * 4);
    D.put(dp, pidx.data(), np * 4);
    D.put(dell, ellp.data(), np * 4);
    D.put(ditems, items.data(), items.size() * sizeof(WorkItem));
    if ((rc = flush(ctx, &D)) ||
        (rc = hip_check(ctx, launch_zgcd_pass(0, Z, ditems, static_cast<int>(items.size()), T, ctx->stream), "zreduce")) ||
        (rc = hip_check(ctx, launch_zgcd_pass(1, Z, nullptr, 0, T, ctx->stream), "zgcd")))
      return rc;
    std::vector<int> gdeg(np);
    if ((rc = download(ctx, gdeg.data(), Z.gdeg, np * 4))) return rc;

    // the least gcd degree; primes above it were unlucky
    const int dg = *std::min_element(gdeg.begin(), gdeg.end());
    std::vector<int> kept, kpidx;
    BigU M(1);
    const uint32_t* tab = prime_table(0);
    for (int s = 0; s < np; ++s)
      if (gdeg[s] == dg) {
        kept.push_back(s);
        kpidx.push_back(pidx[s]);
        M = BigU::mul_small(M, tab[pidx[s]]);
      }
    if (M.bitlen() <= need + 1) continue;  // too many unlucky primes: more spare
    const int nk = static_cast<int>(kept.size());
    Z.nk = nk;
    Z.dg = dg;
    int* dkept = nullptr;
    if ((rc = upload_vec(ctx, &D, kept, &dkept))) return rc;
    Z.kept = dkept;
    Z.c0 = D.take<uint64_t>(static_cast<size_t>(nk) * (dg + 1));
    CrtDev C;
    if ((rc = crt_setup(ctx, &D, kpidx, &C))) return rc;
    const int L = C.P.L_out;
    uint32_t* out0 = D.take<uint32_t>(static_cast<size_t>(dg + 1) * L);
    std::vector<DevProblem> p0{crt_problem(ctx, &D, C, dg, Z.c0, out0)};
    if (D.bad) return fail(ctx, RSL_ENOMEM, "workspace smaller than the gcd footprint");
    if ((rc = flush(ctx, &D)) || (rc = hip_check(ctx, launch_zgcd_pass(2, Z, nullptr, 0, T, ctx->stream), "zpack")) ||
        (rc = run_crt(ctx, &D, p0)))
      return rc;
    std::vector<uint32_t> gt(static_cast<size_t>(dg + 1) * L);
    if ((rc = download(ctx, gt.data(), out0, gt.size() * 4))) return rc;

    // content s of G~ and the sign of its leading coefficient: G = G~ / (sign s)
    BigU s;
    for (int k = dg; k >= 0; --k) {  // leading coefficient first (nonzero)
      bool n;
      const BigU c = abs_limbs(gt.data() + static_cast<size_t>(k) * L, L, &n);
      if (s.d.size() == 1 && !c.is_zero()) {  // a one-limb content: reduce c first
        const uint32_t r = c.mod_small(s.d[0]);
        s = BigU::gcd(s, BigU(r));
      } else {
        s = BigU::gcd(s, c);
      }
      if (s.d.size() == 1 && s.d[0] == 1u) break;  // content 1
    }
    bool lneg;
    (void)abs_limbs(gt.data() + static_cast<size_t>(dg) * L, L, &lneg);
    if (s.is_zero()) return fail(ctx, RSL_EDEVICE, "modular gcd: zero scaled gcd");
    std::vector<uint32_t> sinv(nk);
    for (int i = 0; i < nk; ++i) {
      const uint32_t p = tab[kpidx[i]];
      uint64_t sm = s.mod_small(p);
      if (lneg) sm = (p - sm) % p;
      if (sm == 0) return fail(ctx, RSL_EDEVICE, "modular gcd: content divisible by a kept prime");
      sinv[i] = static_cast<uint32_t>(powmod(sm, p - 2, p));
    }
    uint32_t* dsinv = nullptr;
    if ((rc = upload_vec(ctx, &D, sinv, &dsinv))) return rc;
    Z.sinv = dsinv;
    Z.cg = D.take<uint64_t>(static_cast<size_t>(nk) * (dg + 1));
    Z.ca = D.take<uint64_t>(static_cast<size_t>(nk) * (nu - dg + 1));
    Z.cb = D.take<uint64_t>(static_cast<size_t>(nk) * std::max(nv - dg + 1, 1));
    Z.rem = D.take<int>(1);
    const int na = nu - dg, nb = nv - dg;
    uint32_t* outg = D.take<uint32_t>(static_cast<size_t>(dg + 1) * L);
    uint32_t* outa = D.take<uint32_t>(static_cast<size_t>(na + 1) * L);
    uint32_t* outb = D.take<uint32_t>(static_cast<size_t>(std::max(nb, 0) + 1) * L);
    std::vector<DevProblem> p1{crt_problem(ctx, &D, C, dg, Z.cg, outg), crt_problem(ctx, &D, C, na, Z.ca, outa)};
    if (nv >= 0) p1.push_back(crt_problem(ctx, &D, C, nb, Z.cb, outb));
    if (D.bad) return fail(ctx, RSL_ENOMEM, "workspace smaller than the gcd footprint");
    const int zero = 0;
    D.put(Z.rem, &zero, 4);
    if ((rc = flush(ctx, &D)) || (rc = hip_check(ctx, launch_zgcd_pass(3, Z, nullptr, 0, T, ctx->stream), "zcof")) ||
        (rc = run_crt(ctx, &D, p1)))
      return rc;
    std::vector<uint32_t> g(static_cast<size_t>(dg + 1) * L), a(static_cast<size_t>(na + 1) * L), b;
    int remv = 0;
    if ((rc = download(ctx, g.data(), outg, g.size() * 4)) || (rc = download(ctx, a.data(), outa, a.size() * 4)) ||
        (rc = download(ctx, &remv, Z.rem, 4)))
      return rc;
    if (nv >= 0) {
      b.resize(static_cast<size_t>(nb + 1) * L);
      if ((rc = download(ctx, b.data(), outb, b.size() * 4))) return rc;
    }
    // certificate
    if (remv || max_bits(g, dg, L) > bG || max_bits(a, na, L) > bA || (nv >= 0 && max_bits(b, nb, L) > bB))
      continue;  // all kept primes unlucky (vanishingly rare): more primes
    *gout = as_upoly(g, dg, L);
    *uout = as_upoly(a, na, L);
    *vout = (nv >= 0) ? as_upoly(b, nb, L) : UPoly();
    return RSL_OK;
  }
  return fail(ctx, RSL_EPRIMES, "modular gcd: no consistent set of primes found");
}

}  // namespace
}  // namespace rsl

using namespace rsl;

extern "C" {

int rsl_gcd(rsl_ctx* ctx, const rsl_upoly* u, const rsl_upoly* v, rsl_result* g, rsl_result* ug, rsl_result* vg) {
  if (!ctx || !u || !v) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  UPoly U, V;
  std::string err;
  int rc = read_upoly(u, &U, &err);
  if (!rc) rc = read_upoly(v, &V, &err);
  if (rc) return fail(ctx, rc, err);
  UPoly G, A, B;
  if ((rc = gcd_core(ctx, U, V, &G, &A, &B))) return rc;
  int r1 = write_result(G, g), r2 = write_result(A, ug), r3 = write_result(B, vg);
  return r1 ? r1 : (r2 ? r2 : r3);
}

int rsl_sqfree_part(rsl_ctx* ctx, const rsl_upoly* r, rsl_result* q, rsl_result* g) {
  if (!ctx || !r) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  UPoly R;
  std::string err;
  int rc = read_upoly(r, &R, &err);
  if (rc) return fail(ctx, rc, err);
  if (R.deg < 0) {  // zero: q = 0, G = 0
    put_zero(q);
    put_zero(g);
    return RSL_OK;
  }
  UPoly G, Q, C;
  if ((rc = gcd_core(ctx, R, derivative(R), &G, &Q, &C))) return rc;
  const int r1 = write_result(Q, q), r2 = write_result(G, g);
  return r1 ? r1 : r2;
}

int rsl_sqfree_factor(rsl_ctx* ctx, const rsl_upoly* r, int max_factors, rsl_result* factors, int* nfactors) {
  if (!ctx || !r || !nfactors || max_factors < 0 || (max_factors > 0 && !factors)) return RSL_EINVAL;
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  if (ctx->poisoned) return RSL_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, RSL_EDEVICE, "hipSetDevice");
  ctx->err.clear();
  UPoly R;
  std::string err;
  int rc = read_upoly(r, &R, &err);
  if (rc) return fail(ctx, rc, err);
  // Yun: a = gcd(f, f'), b = f / a, c = f' / a, d = c - b'; then
  // r_i = gcd(b, d), b <- b / r_i, c <- d / r_i, d <- c - b' while deg b > 0
  std::vector<UPoly> out;
  if (R.deg > 0) {
    UPoly G, B, C;
    if ((rc = gcd_core(ctx, R, derivative(R), &G, &B, &C))) return rc;
    UPoly D = sub_upoly(C, derivative(B));
    while (B.deg > 0) {
      UPoly Ri, B2, C2;
      if ((rc = gcd_core(ctx, B, D, &Ri, &B2, &C2))) return rc;
      out.push_back(Ri);
      B = B2;
      D = sub_upoly(C2, derivative(B));
    }
    auto is_one = [](const UPoly& u) {
      if (u.deg != 0) return false;
      for (int l = 0; l < u.L; ++l)
        if (u.c[l] != (l == 0 ? 1u : 0u)) return false;
      return true;
    };
    while (!out.empty() && is_one(out.back())) out.pop_back();
  }
  *nfactors = static_cast<int>(out.size());
  if (static_cast<int>(out.size()) > max_factors) return fail(ctx, RSL_ERANGE, "more square-free factors than buffers");
  int first = RSL_OK;
  for (size_t i = 0; i < out.size(); ++i) {
    const int ri = write_result(out[i], &factors[i]);
    if (ri && !first) first = ri;
  }
  return first;
}

}  // extern "C"

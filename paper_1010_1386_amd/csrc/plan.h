// Host-side planning of one resultant problem: trimmed view in the
// eliminated variable, degree bound, Hadamard bound, prime selection with
// the bad-prime screen, evaluation points, CRT constants and the device
// footprint.
#pragma once
#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rsl.h"
#include "bigint.h"
#include "device.h"
#include "modarith.h"

namespace rsl {

// Descending primes below 2^32 / 3 (index 0 = largest; all above 2^30); grows on demand.
// The table of primes p with 2^30 < p < 2^32 / 3 (descending), extended to at least
// `at_least` entries (capped at its maximum; *avail = entries present).  The
// pointer stays valid for the life of the process; entries below *avail, or
// below an index a previous call reported, may be read without a lock.
const uint32_t* prime_table(size_t at_least, size_t* avail = nullptr);
bool is_prime_u32(uint32_t n);

// One input polynomial viewed in the eliminated variable ("y"): rows j are the
// coefficients of y^j, each a polynomial in the other variable ("x").
struct View {
  int dy = -1;              // actual degree in y (-1: zero polynomial)
  int dx = -1;              // max actual degree in x over all rows
  int tdeg = -1;            // total degree
  int L = 1;                // limbs per coefficient
  std::vector<int> rdeg;    // per-row x-degree, -1 for a zero row
  std::vector<uint32_t> c;  // rows 0..dy, cols 0..dx, L limbs each (two's complement)
  std::vector<BigU> row_l1; // per row j: ||f_j||_1, the sum of |coefficient| (planning only)
  std::vector<BigU> lc_abs; // |coefficient| of the leading row (bad-prime screen)
  std::vector<uint8_t> lc_neg;  // its signs
};

// CRT constants of one ordered prime list with product M (Sec. 4.1: the
// integer result is lifted from its images modulo the primes).  Shared by
// every plan with that list: canonical lists (primes 0..np-1 of the table)
// come from a process-wide cache.
struct CrtConst {
  int np = 0;
  int L_out = 1;            // CRT output limbs (two's complement)
  bool wide = false;        // CRT by the wide path (more than kSlotCrtPrimes primes)
  int Lw = 1;               // limbs of the Mi rows and of negM: L_out, or L_out + 1 when wide
  std::vector<uint32_t> Hm; // (M-1)/2 mod p_i
  std::vector<uint32_t> NH; // 2^(32 L_out) - (M-1)/2, L_out limbs
  // Garner tables (only for a non-canonical list on the slot path)
  std::vector<uint32_t> Tg, invM, Plimb;
  // direct CRT tables: limbs of M / p_j ([np][Lw]), (M / p_i)^{-1} R mod p_i,
  // floor(2^64 / p_i) as (low, high) words, 2^(32 Lw) - M
  std::vector<uint32_t> Mi, wdir, rinv, negM;
  // wide path: M in Lw limbs, -(M-1)/2 - M mod 2^(32 L_out)
  std::vector<uint32_t> Mw, NHM;
};

int make_view(const rsl_poly* f, int var, View* v, std::string* err);

struct Plan {
  View f, g;
  bool zero = false;        // R = 0 by convention (a zero input)
  int my = 0, ny = 0;       // formal degrees used on the device
  int D = 0;                // degree bound
  int s = 0;                // spare points: deg lc_y f + deg lc_y g
  int E = 0;                // points 0..E are evaluated (E = D + s + extra)
  int origin = 0;           // first evaluation point (chosen when the option is 0)
  int formal = 0;           // RSL_POINTS_FORMAL
  int np = 0;               // primes used
  std::vector<int> pidx;    // indices into prime_table()
  bool canonical = true;    // pidx == 0..np-1 (global CRT tables apply)
  int bad_primes = 0;
  int bound_bits = 0;
  int L_out = 1;            // CRT output limbs (copied from crt)
  bool wide = false;        // CRT by the wide path (copied from crt)
  int Lw = 1;               // copied from crt
  std::shared_ptr<const CrtConst> crt;
  // device layout
  int rowf = 0, rowg = 0;   // row strides (dx + 1) of the residue tiles
  int CS = 0;               // residue words per prime (f tile + g tile, padded)
  int goff = 0;             // offset of the g tile inside a prime's residues
  size_t footprint = 0;
};

int make_plan(const rsl_poly* f, const rsl_poly* g, int var, const rsl_opts* opts, Plan* P,
              std::string* err);

// CRT constants of P->pidx (prime product M): np, canonical, L_out, H mod p_i,
// 2^(32 L_out) - H, the wide-path choice, Garner tables (non-canonical slot
// path only) and the direct-CRT tables.  Canonical lists are computed once
// per process and shared.
void plan_crt(Plan* P);

// Shape of a problem from its inputs alone (one pass over the coefficients, no
// big integers): the degrees the plan will have, and estimates of the prime
// count (from the Hadamard bound in double precision) and of the device work.
struct ShapeEst {
  bool zero = true;         // an input is the zero polynomial (no device work)
  bool bad = false;         // invalid descriptor
  int my = 0, ny = 0, D = 0, E = 0;
  int L = 1;                // most limbs of the inputs
  int np_est = 0;           // primes for the bound (bad primes not counted)
  double cost = 0.0;        // evaluation, resultant and interpolation products
};
ShapeEst estimate_shape(const rsl_poly* f, const rsl_poly* g, int var);

// Run fn(i) for i in [0, n) on up to `threads` host threads (0: the default,
// at most 16); blocks of `grain` consecutive indices per task.
void parallel_for(int n, int grain, const std::function<void(int)>& fn, int threads = 0);

// CRT tables for an ordered prime list (Garner constants and prefix products).
//   Tg[j*np + i] = (prod_{l<j} p_l mod p_i) R mod p_i          (j < i)
//   invM[i]      = (prod_{l<i} p_l)^{-1} R mod p_i
//   Plimb[j*LP + t] = limb t of prod_{l<j} p_l
void crt_tables(const std::vector<uint32_t>& primes, int LP, std::vector<uint32_t>* Tg,
                std::vector<uint32_t>* invM, std::vector<uint32_t>* Plimb);

// Direct-CRT tables for an ordered prime list with product M (see Plan).
void direct_crt_tables(const std::vector<uint32_t>& primes, const BigU& M, int L, std::vector<uint32_t>* Mi,
                       std::vector<uint32_t>* wdir, std::vector<uint32_t>* rinv, std::vector<uint32_t>* negM);

}  // namespace rsl

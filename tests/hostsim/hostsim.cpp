// Host build of the kernels' per-lane arithmetic, for CPU tests of its logic
// against the oracle (test infrastructure only; not part of the library).
#include <cstdint>
#include <vector>
#include "../../paper_1010_1386_amd/csrc/modarith.h"
#include "../../paper_1010_1386_amd/csrc/ures.h"

using namespace rsl;

extern "C" {

// Resultant over Z_p with formal degrees (m, n) of A (m+1 coefficients) and B
// (n+1 coefficients), given and returned in normal form.
int hs_ures(uint32_t p, int m, int n, const uint32_t* A, const uint32_t* B, uint32_t* out, int* bad) {
  PrimeConst pc = make_prime_const(p);
  int nm = (m > n ? m : n) + 1;
  std::vector<uint32_t> a(nm, 0), b(nm, 0);
  for (int j = 0; j <= m; ++j) a[j] = mmul(A[j] % p, pc.r2, p, pc.pinv);
  for (int j = 0; j <= n; ++j) b[j] = mmul(B[j] % p, pc.r2, p, pc.pinv);
  bool bd = false;
  uint32_t r = ures_formal(Column<1>{a.data()}, Column<1>{b.data()}, m, n, pc, &bd);
  *out = redc(r, p, pc.pinv);
  *bad = bd;
  return 0;
}

// Horner evaluation of rows of coefficients (normal form) at x, result normal form.
int hs_eval(uint32_t p, int nrows, int rowstride, const uint32_t* coeff, const int* rdeg, uint32_t x,
            uint32_t* out) {
  PrimeConst pc = make_prime_const(p);
  std::vector<uint32_t> c(static_cast<size_t>(nrows) * rowstride);
  for (size_t i = 0; i < c.size(); ++i) c[i] = mmul(coeff[i] % p, pc.r3, p, pc.pinv);
  uint32_t xt = mmul(x % p, pc.r2, p, pc.pinv);
  std::vector<uint32_t> o(nrows);
  eval_rows(Column<1>{o.data()}, c.data(), nrows, rowstride, rdeg, xt, p, pc.pinv);
  for (int j = 0; j < nrows; ++j) out[j] = redc(o[j], p, pc.pinv);
  return 0;
}

}

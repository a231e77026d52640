"""CPU oracle for bivariate resultants over Z[x] -- TEST INFRASTRUCTURE ONLY.

Nothing in the product path (the HIP library and its Python binding) may
import, call or link anything under this package.  Only the test-suite, the
``smoke()`` check of the graft entry point and the ``cpu_baseline`` leg of the
benchmark use it.

What it computes, and where the paper defines it:

* ``res(f, g, var)`` -- the resultant R^(y) = res(f, g, y) as the determinant
  of the (m_y + n_y) x (m_y + n_y) Sylvester matrix over Z[x] (paper, Sec. 3.1,
  the displayed matrix S^(y)(f, g)); R^(x) is the same with the roles of x and
  y exchanged (same section).  The determinant is taken by fraction-free
  Gaussian elimination (Bareiss) over Z[x]; the paper itself notes that the
  resultant reduces to the triangular factorisation of the Sylvester matrix
  (Sec. 4.1).  No primes, no evaluation points, no interpolation.
* ``leibniz_det`` -- the permutation expansion of a determinant, used as the
  brute-force pin on tiny inputs.
* ``det_mod`` / ``res_at_point_mod`` -- Gaussian elimination over Z_q, used for
  randomised checks of large results (Schwartz-Zippel).
* ``res_at_int_point`` -- exact integer Bareiss determinant of the Sylvester
  matrix specialised at an integer x0 (formal degrees), used for exact point
  checks where the full oracle is too slow.
* ``zx_gcd`` / ``sqfree_part`` / ``yun`` -- gcd, square-free part and the
  square-free factorisation (Yun's algorithm) over Z[x] for the Project step
  (Sec. 3.2), by the primitive Euclidean algorithm with exact integers.

Parity status of each function is documented in its docstring; all of them
are pinned by tests in ``tests/test_oracle_*.py``.
"""

from .poly import (padd, psub, pmul, pdivexact, ptrim, peval, pcompose_y,
                   bivar_trim, bivar_transpose, bivar_mul, bivar_eval_x)
from .resultant import (sylvester, bareiss_det, res, res_y, res_x, leibniz_det,
                        degree_bound, hadamard_bound_sq)
from .modular import (det_mod, res_at_point_mod, res_at_int_point, poly_eval_mod,
                      is_probable_prime, next_check_primes)
from .sqfree import (zx_gcd, zx_pp, zx_content, zx_deriv, zx_divexact, sqfree_part, yun)

__all__ = [
    "padd", "psub", "pmul", "pdivexact", "ptrim", "peval", "pcompose_y",
    "bivar_trim", "bivar_transpose", "bivar_mul", "bivar_eval_x",
    "sylvester", "bareiss_det", "res", "res_y", "res_x", "leibniz_det",
    "degree_bound", "hadamard_bound_sq",
    "det_mod", "res_at_point_mod", "res_at_int_point", "poly_eval_mod",
    "is_probable_prime", "next_check_primes",
    "zx_gcd", "zx_pp", "zx_content", "zx_deriv", "zx_divexact", "sqfree_part", "yun",
]

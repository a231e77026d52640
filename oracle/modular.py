"""Point checks of a resultant: exact at an integer point, or modulo a check prime.

Test infrastructure only (see the package docstring).

Evaluation commutes with the determinant: for any ring homomorphism phi,
phi(det S) = det phi(S).  Taking phi = "evaluate x at x0" (and optionally
"reduce mod q") of the Sylvester matrix built with the actual degrees m_y, n_y
over Z[x] therefore gives R(x0) (mod q) -- the paper uses exactly this
commutation for its evaluation homomorphism (Sec. 4.1).  These checks compute
the specialised determinant by their own elimination, independent of the
Bareiss-over-Z[x] routine, and serve as exact or Schwartz-Zippel pins where
the full oracle is too slow.  Parity status: pinned (tests compare them with
``res`` evaluated at the same point on small inputs, and with brute force).
"""

from __future__ import annotations

from .poly import bivar_transpose, bivar_trim, peval


def poly_eval_mod(a, x, q):
    acc = 0
    for c in reversed(a):
        acc = (acc * x + c) % q
    return acc


def det_mod(M, q):
    """Determinant of an integer matrix modulo a prime q by Gaussian elimination."""
    r = len(M)
    A = [[v % q for v in row] for row in M]
    det = 1
    for k in range(r):
        piv = next((i for i in range(k, r) if A[i][k]), None)
        if piv is None:
            return 0
        if piv != k:
            A[k], A[piv] = A[piv], A[k]
            det = -det
        akk = A[k][k]
        det = det * akk % q
        inv = pow(akk, q - 2, q)
        for i in range(k + 1, r):
            if A[i][k]:
                f = A[i][k] * inv % q
                rowi, rowk = A[i], A[k]
                for j in range(k + 1, r):
                    rowi[j] = (rowi[j] - f * rowk[j]) % q
    return det % q


def _int_det(M):
    """Exact determinant of an integer matrix (integer Bareiss with pivoting)."""
    r = len(M)
    if r == 0:
        return 1
    A = [list(row) for row in M]
    sign = 1
    prev = 1
    for k in range(r - 1):
        if A[k][k] == 0:
            piv = next((i for i in range(k + 1, r) if A[i][k]), None)
            if piv is None:
                return 0
            A[k], A[piv] = A[piv], A[k]
            sign = -sign
        akk = A[k][k]
        for i in range(k + 1, r):
            aik = A[i][k]
            rowi, rowk = A[i], A[k]
            for j in range(k + 1, r):
                n = akk * rowi[j] - aik * rowk[j]
                qq, rr = divmod(n, prev)
                if rr:
                    raise ArithmeticError("integer Bareiss: inexact division")
                rowi[j] = qq
        prev = akk
    return sign * A[r - 1][r - 1]


def _specialised_sylvester(F, G, var, point_fn):
    if var == "x":
        F, G = bivar_transpose(F), bivar_transpose(G)
    F, G = bivar_trim(F), bivar_trim(G)
    if not F or not G:
        return None
    fy = [point_fn(r) for r in F]  # formal degree m_y kept even if the top value vanishes
    gy = [point_fn(r) for r in G]
    my, ny = len(fy) - 1, len(gy) - 1
    r = my + ny
    S = [[0] * r for _ in range(r)]
    for i in range(ny):
        for t in range(my + 1):
            S[i][i + t] = fy[my - t]
    for l in range(my):
        for t in range(ny + 1):
            S[ny + l][l + t] = gy[ny - t]
    return S


def res_at_point_mod(F, G, t, q, var="y"):
    """R(t) mod q, as det of the Sylvester matrix specialised at t, over Z_q."""
    S = _specialised_sylvester(F, G, var, lambda row: poly_eval_mod(row, t, q))
    if S is None:
        return 0
    return det_mod(S, q) if S else 1 % q


def res_at_int_point(F, G, x0, var="y"):
    """R(x0) exactly, as det of the Sylvester matrix specialised at the integer x0."""
    S = _specialised_sylvester(F, G, var, lambda row: peval(row, x0))
    if S is None:
        return 0
    return _int_det(S)


def is_probable_prime(n):
    """Miller-Rabin with the first 12 prime bases: deterministic for n < 3.3e24."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_check_primes(count, below=1 << 61):
    """The ``count`` largest primes below ``below`` (61-bit check primes by default)."""
    out = []
    n = below - 1
    while len(out) < count:
        if is_probable_prime(n):
            out.append(n)
        n -= 2 if n % 2 else 1
    return out

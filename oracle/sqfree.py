"""Univariate gcd, square-free part and square-free factorisation over Z[x]
-- TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Project step (Sec. 3.2) needs, besides R, a square-free
factorisation R = prod_i r_i^i with square-free, pairwise coprime r_i, built
by Yun's algorithm from gcds of R and its derivatives; the outlook (Sec. 6)
proposes the modular route for it.  This module computes the same objects by
their plain definitions, with exact integer arithmetic and no primes:

* ``zx_gcd(u, v)`` -- the primitive Euclidean algorithm: pseudo-remainders,
  each replaced by its primitive part; the result is the primitive gcd of
  pp(u) and pp(v) with positive leading coefficient;
* ``sqfree_part(r)`` -- pp(r) / gcd(pp(r), pp(r)'), leading coefficient
  positive;
* ``yun(r)`` -- Yun's iteration on pp(r): a = gcd(f, f'), b = f / a,
  c = f' / a, d = c - b'; then repeatedly r_i = gcd(b, d), b <- b / r_i,
  c <- d / r_i, d <- c - b'.

Polynomials are lists of Python ints, lowest power first; [] is zero.
Parity status: pinned by closed forms (products of known factors with known
multiplicities), divisibility, coprimality of the cofactors through the
resultant oracle (a different algorithm), and pp(r) = prod r_i^i in
``tests/test_oracle_sqfree.py``.
"""

from math import gcd

from .poly import ptrim, pmul


def zx_content(a):
    c = 0
    for v in a:
        c = gcd(c, v)
    return c


def zx_pp(a):
    """Primitive part with positive leading coefficient ([] for zero)."""
    a = ptrim(list(a))
    if not a:
        return []
    c = zx_content(a)
    if a[-1] < 0:
        c = -c
    return [v // c for v in a]


def zx_deriv(a):
    return ptrim([k * a[k] for k in range(1, len(a))])


def zx_sub(a, b):
    n = max(len(a), len(b))
    return ptrim([(a[i] if i < len(a) else 0) - (b[i] if i < len(b) else 0) for i in range(n)])


def zx_divmod_exact(a, b):
    """Quotient of a by b in Z[x]; raises if the division is not exact."""
    a = ptrim(list(a))
    b = ptrim(list(b))
    if not b:
        raise ZeroDivisionError("division by the zero polynomial")
    q = [0] * max(len(a) - len(b) + 1, 0)
    lb = b[-1]
    for k in range(len(a) - len(b), -1, -1):
        c = a[k + len(b) - 1]
        if c % lb:
            raise ArithmeticError("inexact division")
        t = c // lb
        q[k] = t
        for j, bj in enumerate(b):
            a[k + j] -= t * bj
    if any(a):
        raise ArithmeticError("inexact division")
    return ptrim(q)


def zx_divexact(a, b):
    return zx_divmod_exact(a, b)


def _prem(a, b):
    """Pseudo-remainder of a by b: lc(b)^(deg a - deg b + 1) a mod b."""
    a = list(a)
    lb = b[-1]
    while len(a) >= len(b) and a:
        c = a[-1]
        s = len(a) - len(b)
        a = [lb * v for v in a]
        for j, bj in enumerate(b):
            a[s + j] -= c * bj
        a = ptrim(a)
    return a


def zx_gcd(u, v):
    """Primitive gcd of pp(u) and pp(v), positive leading coefficient (gcd(0, 0) = [])."""
    a, b = zx_pp(u), zx_pp(v)
    if not a:
        return b
    if not b:
        return a
    if len(a) < len(b):
        a, b = b, a
    while b:
        r = _prem(a, b)
        a, b = b, zx_pp(r)
    return zx_pp(a)


def sqfree_part(r):
    """pp(r) / gcd(pp(r), pp(r)') with positive leading coefficient."""
    f = zx_pp(r)
    if len(f) <= 1:
        return f
    return zx_pp(zx_divexact(f, zx_gcd(f, zx_deriv(f))))


def yun(r):
    """Square-free factorisation of pp(r): [r_1, r_2, ...] with pp(r) = prod r_i^i,
    each r_i primitive with positive leading coefficient (trailing ones dropped)."""
    f = zx_pp(r)
    if len(f) <= 1:
        return []
    fp = zx_deriv(f)
    a = zx_gcd(f, fp)
    b = zx_divexact(f, a)
    c = zx_divexact(fp, a)
    d = zx_sub(c, zx_deriv(b))
    out = []
    while len(b) > 1:
        ri = zx_gcd(b, d)
        b = zx_divexact(b, ri)
        c = zx_divexact(d, ri)
        d = zx_sub(c, zx_deriv(b))
        out.append(ri)
    while out and out[-1] == [1]:
        out.pop()
    return out


def zx_pow(a, e):
    r = [1]
    for _ in range(e):
        r = pmul(r, a)
    return r

"""Exact polynomial arithmetic over Z[x] for the oracle (test infrastructure only).

A univariate polynomial is a Python list of ints, index = power of x, with no
trailing zeros; the zero polynomial is ``[]``.  A bivariate polynomial is a
list of rows ``F[j][i]`` = coefficient of x^i y^j (the layout of the paper's
Eq. (2.1) written as a sum over powers of y, Sec. 2).

Products use Kronecker substitution (evaluate at 2^B, multiply the two
integers, read the coefficients back from B-bit slots), exact quotients use a
2-adic inverse of the divisor's Kronecker image.  Both are plain library-level
primitives of "multiply two polynomials" and "divide exactly"; every exact
quotient is re-multiplied and compared with the dividend before it is
returned, so a wrong slot width cannot go unnoticed.
"""

from __future__ import annotations


def ptrim(a):
    """Drop trailing zero coefficients (returns a new list)."""
    n = len(a)
    while n and a[n - 1] == 0:
        n -= 1
    return list(a[:n])


def padd(a, b):
    if len(a) < len(b):
        a, b = b, a
    out = list(a)
    for i, c in enumerate(b):
        out[i] += c
    return ptrim(out)


def psub(a, b):
    out = list(a) + [0] * max(0, len(b) - len(a))
    for i, c in enumerate(b):
        out[i] -= c
    return ptrim(out)


def _maxbits(a):
    m = 0
    for c in a:
        b = abs(c).bit_length()
        if b > m:
            m = b
    return m


def _slot(bits):
    """Slot width in bits (multiple of 8) holding signed values of ``bits`` magnitude bits."""
    b = bits + 2
    return (b + 7) // 8 * 8


def _bias(n, B):
    """Sum_{i<n} 2^(B-1) * 2^(iB): the offset that makes every slot non-negative."""
    nb = B // 8
    one = (1 << (B - 1)).to_bytes(nb, "little")
    return int.from_bytes(one * n, "little")


def _pack(a, B):
    """Kronecker image sum_i a_i 2^(iB) of a signed coefficient list."""
    if not a:
        return 0
    nb = B // 8
    half = 1 << (B - 1)
    buf = b"".join((c + half).to_bytes(nb, "little") for c in a)
    return int.from_bytes(buf, "little") - _bias(len(a), B)


def _unpack(v, B, n):
    """Inverse of _pack for n slots; requires every coefficient < 2^(B-1) in magnitude."""
    if n <= 0:
        return []
    nb = B // 8
    half = 1 << (B - 1)
    u = v + _bias(n, B)
    if u < 0 or u.bit_length() > n * B:
        raise ArithmeticError("Kronecker unpack: value outside the slot range")
    buf = u.to_bytes(n * nb, "little")
    return ptrim([int.from_bytes(buf[i * nb:(i + 1) * nb], "little") - half for i in range(n)])


def pmul(a, b):
    """Product of two polynomials in Z[x]."""
    if not a or not b:
        return []
    if len(a) == 1:
        return ptrim([a[0] * c for c in b])
    if len(b) == 1:
        return ptrim([b[0] * c for c in a])
    bits = _maxbits(a) + _maxbits(b) + min(len(a), len(b)).bit_length()
    B = _slot(bits)
    return _unpack(_pack(a, B) * _pack(b, B), B, len(a) + len(b) - 1)


def pmulsub(a, b, c, d):
    """a*b - c*d in Z[x], with one shared Kronecker slot."""
    if not a or not b:
        return psub([], pmul(c, d))
    if not c or not d:
        return pmul(a, b)
    bits = max(_maxbits(a) + _maxbits(b) + min(len(a), len(b)).bit_length(),
               _maxbits(c) + _maxbits(d) + min(len(c), len(d)).bit_length()) + 1
    B = _slot(bits)
    n = max(len(a) + len(b), len(c) + len(d)) - 1
    return _unpack(_pack(a, B) * _pack(b, B) - _pack(c, B) * _pack(d, B), B, n)


def _inv_2adic(a, K):
    """Inverse of the odd integer a modulo 2^K by Newton (Hensel) iteration."""
    x = 1
    prec = 1
    while prec < K:
        prec = min(2 * prec, K)
        mask = (1 << prec) - 1
        x = (x * (2 - (a & mask) * x)) & mask
    return x


class ExactDivisor:
    """Exact division by a fixed nonzero polynomial d in Z[x].

    ``div(n, qbits)`` returns q with n = q*d, given that such q exists and
    that its coefficients have at most ``qbits`` magnitude bits (if the hint
    is too small the verification fails and the slot width is doubled).
    Raises ArithmeticError if d does not divide n.
    """

    def __init__(self, d):
        d = ptrim(d)
        if not d:
            raise ZeroDivisionError("division by the zero polynomial")
        self.d = d
        self._cache = {}  # slot width B -> (shift v, odd part, inverse, precision K)

    def div(self, n, qbits=None):
        n = ptrim(n)
        d = self.d
        if not n:
            return []
        if len(n) < len(d):
            raise ArithmeticError("inexact division: degree of dividend below divisor")
        if len(d) == 1:
            d0 = d[0]
            q = []
            for c in n:
                qq, rr = divmod(c, d0)
                if rr:
                    raise ArithmeticError("inexact division by a constant")
                q.append(qq)
            return q
        qlen = len(n) - len(d) + 1
        if qbits is None:
            qbits = 0
        # The slot must hold the dividend's and the quotient's coefficients; it
        # is rounded to 256 bits so that one cached inverse serves many calls.
        B = (_slot(max(qbits, _maxbits(n))) + 255) // 256 * 256
        for _ in range(8):
            q = self._div_slot(n, qlen, B)
            if q is not None and pmul(q, d) == n:
                return q
            B *= 2
        raise ArithmeticError("inexact division in Z[x]")

    def _div_slot(self, n, qlen, B):
        K = B * qlen
        ent = self._cache.get(B)
        if ent is None or ent[3] < K:
            dv = _pack(self.d, B)
            v = (dv & -dv).bit_length() - 1
            odd = dv >> v
            ent = (v, odd, _inv_2adic(odd, K), K)
            self._cache[B] = ent
        v, odd, inv, _ = ent
        nv = _pack(n, B)
        if nv & ((1 << v) - 1):
            return None
        mask = (1 << K) - 1
        qv = ((nv >> v) * (inv & mask)) & mask
        if qv >> (K - 1):
            qv -= 1 << K
        try:
            return _unpack(qv, B, qlen)
        except ArithmeticError:
            return None


def pdivexact(n, d, qbits=None):
    """Exact quotient n / d in Z[x] (raises ArithmeticError when d does not divide n)."""
    return ExactDivisor(d).div(n, qbits)


def peval(a, x):
    """a(x) for an integer (or any ring element supporting * and +) x, by Horner."""
    acc = 0
    for c in reversed(a):
        acc = acc * x + c
    return acc


# ---------------------------------------------------------------- bivariate


def bivar_trim(F):
    """Trim a bivariate coefficient array F[j][i]: drop zero top rows and trailing zeros."""
    rows = [ptrim(r) for r in F]
    while rows and not rows[-1]:
        rows.pop()
    return rows


def bivar_transpose(F):
    """Exchange the roles of x and y: G[i][j] = F[j][i]."""
    F = bivar_trim(F)
    if not F:
        return []
    nx = max(len(r) for r in F)
    return bivar_trim([[F[j][i] if i < len(F[j]) else 0 for j in range(len(F))] for i in range(nx)])


def bivar_mul(F, G):
    """Product of two bivariate polynomials (rows are y-powers, entries polynomials in x)."""
    F, G = bivar_trim(F), bivar_trim(G)
    if not F or not G:
        return []
    out = [[] for _ in range(len(F) + len(G) - 1)]
    for j, fj in enumerate(F):
        if not fj:
            continue
        for l, gl in enumerate(G):
            if gl:
                out[j + l] = padd(out[j + l], pmul(fj, gl))
    return bivar_trim(out)


def bivar_eval_x(F, x0):
    """F(x0, y) as a list of y-coefficients (not trimmed: formal y-degree kept)."""
    return [peval(r, x0) for r in F]


def pcompose_y(G, a):
    """G(x, a(x)) in Z[x] for a bivariate G and a univariate a, by Horner in y."""
    G = bivar_trim(G)
    acc = []
    for row in reversed(G):
        acc = padd(pmul(acc, a), row)
    return acc

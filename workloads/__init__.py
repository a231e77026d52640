"""Seeded synthetic inputs for the resultant workloads (shared by tests, bench and smoke).

This module only draws and shapes random integer coefficient arrays; it holds
none of the resultant method's arithmetic.  Inputs are bivariate polynomials
given as ``F[j][i]`` = coefficient of x^i y^j (Python ints), dense arrays of
shape (dy+1) x (dx+1) with zeros where a term is absent.

The paper's own inputs (its special curves, Tables 1/4, and the random curves
of Table 3) are not available; these generators stand in for them at the
paper's scale: y-degrees 8..48 (its Table 2/5 instances run from 8 to 42) and
coefficient sizes from 8 to 64 bits.

Every draw uses ``numpy.random.default_rng(SeedSequence(BASE_SEED,
spawn_key=(config, problem, part)))`` so that any single problem can be
regenerated on its own.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 10101386


def rng_for(config, problem=0, part=0):
    return np.random.default_rng(np.random.SeedSequence(BASE_SEED, spawn_key=(config, problem, part)))


def _uniform_signed(rng, bits, size):
    """Uniform integers on [-2^(bits-1), 2^(bits-1) - 1] as Python ints."""
    if bits <= 63:
        lo, hi = -(1 << (bits - 1)), (1 << (bits - 1)) - 1
        return [int(v) for v in rng.integers(lo, hi, size=size, endpoint=True, dtype=np.int64)]
    if bits == 64:
        return [int(v) for v in rng.integers(-(1 << 63), (1 << 63) - 1, size=size, endpoint=True,
                                             dtype=np.int64)]
    # wider than 64 bits: assemble from 32-bit words
    words = (bits + 31) // 32
    raw = rng.integers(0, 1 << 32, size=(size, words), dtype=np.uint64)
    out = []
    for row in raw:
        v = 0
        for w in reversed(row):
            v = (v << 32) | int(w)
        v &= (1 << bits) - 1
        out.append(v - (1 << (bits - 1)))
    return out


def dense_total(rng, d, bits, force_top=True):
    """Dense polynomial of total degree d: every coefficient with i + j <= d drawn.

    With ``force_top`` the y^d coefficient is redrawn until nonzero, so that
    the y-degree (and the total degree) is exactly d.
    """
    n = (d + 1) * (d + 2) // 2
    vals = _uniform_signed(rng, bits, n)
    F = [[0] * (d + 1) for _ in range(d + 1)]
    t = 0
    for j in range(d + 1):
        for i in range(d + 1 - j):
            F[j][i] = vals[t]
            t += 1
    while force_top and F[d][0] == 0:
        F[d][0] = _uniform_signed(rng, bits, 1)[0]
    return F


def sparse_total(rng, d, bits, zero_prob=0.3):
    """Total degree d, each coefficient zeroed independently with probability ``zero_prob``.

    Redrawn until the total degree is exactly d; the leading y-coefficient is
    not forced nonzero, so the y-degree may fall below d.
    """
    while True:
        F = dense_total(rng, d, bits, force_top=False)
        mask = rng.random(((d + 1), (d + 1))) < zero_prob
        for j in range(d + 1):
            for i in range(d + 1 - j):
                if mask[j][i]:
                    F[j][i] = 0
        if any(F[j][d - j] for j in range(d + 1)):
            return F


def _bmul(F, G):
    """Product of two coefficient arrays (input construction only)."""
    dyf, dxf = len(F), max(len(r) for r in F)
    dyg, dxg = len(G), max(len(r) for r in G)
    out = [[0] * (dxf + dxg - 1) for _ in range(dyf + dyg - 1)]
    for j, fr in enumerate(F):
        for i, a in enumerate(fr):
            if a:
                for l, gr in enumerate(G):
                    orow = out[j + l]
                    for k, b in enumerate(gr):
                        if b:
                            orow[i + k] += a * b
    return out


def _dy(F):
    """Partial derivative in y of a coefficient array (input construction only)."""
    return [[j * c for c in F[j]] for j in range(1, len(F))] or [[0]]


# ---------------------------------------------------------------------- configs


def config1():
    """Single pair, dense total degree 8, signed 10-bit coefficients; res_y."""
    return dense_total(rng_for(1, 0, 0), 8, 10), dense_total(rng_for(1, 0, 1), 8, 10)


def config2():
    """Single pair, dense total degree 24, uniform signed 32-bit; res_y and res_x."""
    return dense_total(rng_for(2, 0, 0), 24, 32), dense_total(rng_for(2, 0, 1), 24, 32)


def config3(variant="a", a_point=None):
    """Curve analysis: f = F * (y^2 - h(x)), g = f_y; res_y(f, f_y) is a discriminant.

    F: dense total degree 40, signed 16-bit; h: degree 6, signed 8-bit, nonzero
    leading coefficient.  Variant 'b' drops F's y^40 term and plants
    lc_y F = c (x - a), so that x = a is a bad point for every prime; variant
    'c' plants h = (x - a) h1, so that R(a) = 0.  Returns (f, g, F, h).
    """
    rng = rng_for(3, 0, 0)
    F = dense_total(rng, 40, 16)
    h = _uniform_signed(rng, 8, 7)
    while h[6] == 0:
        h[6] = _uniform_signed(rng, 8, 1)[0]
    if a_point is None:
        a_point = int(rng.integers(1, 200))
    if variant == "b":
        F = [list(r) for r in F[:40]]
        c = 0
        while c == 0:
            c = _uniform_signed(rng, 16, 1)[0]
        F[39] = [0] * len(F[39])
        F[39][0], F[39][1] = -c * a_point, c
    elif variant == "c":
        h1 = _uniform_signed(rng, 8, 6)
        while h1[5] == 0:
            h1[5] = _uniform_signed(rng, 8, 1)[0]
        h = [0] * 7
        for k, v in enumerate(h1):
            h[k + 1] += v
            h[k] -= a_point * v
    elif variant != "a":
        raise ValueError("variant must be 'a', 'b' or 'c'")
    Q = [[-v for v in h], [0] * 7, [1] + [0] * 6]  # y^2 - h(x)
    f = _bmul(F, Q)
    g = _dy(f)
    return f, g, F, h


def config4(count=512):
    """Batch of independent pairs: total degrees U{6..32}, coefficient bits U{8..64}.

    Pairs 0..255 dense, 256..511 with each coefficient zeroed with probability 0.3.
    """
    out = []
    for k in range(count):
        pair = []
        for part in (0, 1):
            rng = rng_for(4, k, part)
            d = int(rng.integers(6, 32, endpoint=True))
            b = int(rng.integers(8, 64, endpoint=True))
            pair.append(dense_total(rng, d, b, force_top=False) if k < 256 else sparse_total(rng, d, b))
        out.append(tuple(pair))
    return out


def config5(count=1000):
    """Serving stream: per request var in {y, x} w.p. 1/2, d ~ U{8..48}, bits ~ U{8..48}, dense.

    Returns a list of (f, g, var); arrival times are drawn by the caller for a
    chosen rate (``poisson_arrivals``).
    """
    out = []
    for k in range(count):
        rng = rng_for(5, k, 0)
        var = "y" if rng.random() < 0.5 else "x"
        polys = []
        for part in (1, 2):
            r2 = rng_for(5, k, part)
            d = int(r2.integers(8, 48, endpoint=True))
            b = int(r2.integers(8, 48, endpoint=True))
            polys.append(dense_total(r2, d, b))
        out.append((polys[0], polys[1], var))
    return out


def table3_curves(degree, shift, sparse=False, count=5, bits=8):
    """Random-curve instances of the large-coefficient experiment (paper Table 3):
    ``count`` curves of total degree ``degree`` (dense, or with each coefficient
    zeroed with probability 0.3), signed ``bits``-bit base coefficients (the
    paper leaves the base distribution open), each multiplied by 2^shift with
    the constant coefficient then increased by one.  The instance set is all
    pairs of the curves."""
    rng = rng_for(6, 1000 * degree + (1 if sparse else 0), shift)
    curves = []
    for _ in range(count):
        F = sparse_total(rng, degree, bits) if sparse else dense_total(rng, degree, bits)
        F = [[c << shift for c in row] for row in F]
        F[0][0] += 1
        curves.append(F)
    return [(curves[a], curves[b]) for a in range(count) for b in range(a + 1, count)]


def poisson_arrivals(count, rate, seed_part=0):
    """Arrival times (seconds) of a Poisson stream with the given rate (requests/s)."""
    rng = rng_for(5, 1 << 20, seed_part)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def small_random(rng, dy, dx, bits, density=1.0):
    """Arbitrary-shape random array (for tests): shape (dy+1) x (dx+1)."""
    vals = _uniform_signed(rng, bits, (dy + 1) * (dx + 1))
    F = [vals[j * (dx + 1):(j + 1) * (dx + 1)] for j in range(dy + 1)]
    if density < 1.0:
        mask = rng.random((dy + 1, dx + 1)) >= density
        for j in range(dy + 1):
            for i in range(dx + 1):
                if mask[j][i]:
                    F[j][i] = 0
    return F

"""Pins of the CPU oracle against facts fixed outside the oracle itself.

The paper prints no resultant values and no worked example, so every pin
here comes from the definition (the Sylvester determinant of Sec. 3.1,
expanded by brute force), closed forms, textbook resultant identities, a
third-party implementation (sympy), the degree bound of Sec. 3.1 and the
commutation of evaluation with the determinant (Sec. 4.1).
"""

import itertools
import random

import numpy as np
import pytest
import sympy

import oracle
from oracle import (bivar_mul, bivar_transpose, bivar_trim, degree_bound, hadamard_bound_sq,
                    leibniz_det, pcompose_y, peval, pmul, psub, res, res_at_int_point,
                    res_at_point_mod, sylvester)
from oracle.poly import ExactDivisor, pmulsub
from workloads import rng_for, small_random

X, Y = sympy.symbols("x y")


def rnd(rng, dy, dx, b, density=1.0):
    return small_random(rng, dy, dx, max(2, b), density)


def naive_mul(a, b):
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] += u * v
    while out and out[-1] == 0:
        out.pop()
    return out


# ------------------------------------------------------------------ primitives


def test_kronecker_product_matches_schoolbook():
    r = random.Random(5)
    for _ in range(300):
        a = [r.randint(-(1 << r.randint(1, 300)), 1 << r.randint(1, 300)) for _ in range(r.randint(0, 30))]
        b = [r.randint(-(1 << r.randint(1, 300)), 1 << r.randint(1, 300)) for _ in range(r.randint(0, 30))]
        while a and a[-1] == 0:
            a.pop()
        while b and b[-1] == 0:
            b.pop()
        assert pmul(a, b) == naive_mul(a, b)
        c = [r.randint(-99, 99) for _ in range(r.randint(0, 9))]
        d = [r.randint(-99, 99) for _ in range(r.randint(0, 9))]
        while c and c[-1] == 0:
            c.pop()
        while d and d[-1] == 0:
            d.pop()
        assert pmulsub(a, b, c, d) == psub(naive_mul(a, b), naive_mul(c, d))


def test_exact_division_recovers_quotient_and_rejects_inexact():
    r = random.Random(6)
    for _ in range(200):
        q = [r.randint(-(1 << 200), 1 << 200) for _ in range(r.randint(1, 25))]
        d = [r.randint(-(1 << 90), 1 << 90) for _ in range(r.randint(1, 12))]
        if q[-1] == 0:
            q[-1] = 3
        if d[-1] == 0:
            d[-1] = -5
        n = naive_mul(q, d)
        assert ExactDivisor(d).div(n) == q
    with pytest.raises(ArithmeticError):
        ExactDivisor([1, 2]).div([1, 0, 1])  # (x^2 + 1) / (2x + 1) is not exact
    with pytest.raises(ArithmeticError):
        ExactDivisor([3]).div([1, 3])


# -------------------------------------------------------- definition / brute


@pytest.mark.parametrize("seed", range(40))
def test_bareiss_equals_leibniz_expansion(seed):
    rng = rng_for(900, seed)
    F = rnd(rng, int(rng.integers(0, 4)), int(rng.integers(0, 3)), 6, 0.8)
    G = rnd(rng, int(rng.integers(0, 4)), int(rng.integers(0, 3)), 6, 0.8)
    for var in "yx":
        A, B = (F, G) if var == "y" else (bivar_transpose(F), bivar_transpose(G))
        A, B = bivar_trim(A), bivar_trim(B)
        if not A or not B:
            assert res(F, G, var) == []
            continue
        assert res(F, G, var) == leibniz_det(sylvester(A, B))


def _closed_tiny(F, G):
    """Closed forms for y-degrees <= 1 (the only cases in the exhaustive space)."""
    F, G = bivar_trim(F), bivar_trim(G)
    if not F or not G:
        return []
    my, ny = len(F) - 1, len(G) - 1
    if my == 0 and ny == 0:
        return [1]
    if my == 0:  # R = f_0^{n_y}
        return F[0]
    if ny == 0:  # R = g_0^{m_y}
        return G[0]
    return psub(pmul(F[1], G[0]), pmul(F[0], G[1]))  # det [[f1, f0], [g1, g0]]


def test_exhaustive_tiny_space():
    """All 3^4 x 3^4 pairs with y-degree <= 1, x-degree <= 1, coefficients in {-1, 0, 1}."""
    cells = list(itertools.product((-1, 0, 1), repeat=4))
    arrs = [[[c[0], c[1]], [c[2], c[3]]] for c in cells]
    for F in arrs:
        for G in arrs:
            assert res(F, G) == _closed_tiny(F, G), (F, G)


# ---------------------------------------------------------------- sympy (3rd party)


def _sym(F):
    return sum(c * X ** i * Y ** j for j, row in enumerate(F) for i, c in enumerate(row))


@pytest.mark.parametrize("seed", range(25))
def test_against_sympy_resultant(seed):
    """sympy.resultant agrees with det S^(y) when deg_y f >= deg_y g.

    (For deg_y f < deg_y g with m_y n_y odd, sympy 1.14 was observed to return
    res(g, f) instead; that order is covered by the antisymmetry pin.)
    """
    rng = rng_for(901, seed)
    ny = int(rng.integers(1, 4))
    my = ny + int(rng.integers(0, 3))
    F = rnd(rng, my, int(rng.integers(1, 4)), 12)
    G = rnd(rng, ny, int(rng.integers(1, 4)), 12)
    F[my][0] = F[my][0] or 7
    G[ny][0] = G[ny][0] or -3
    ref = sympy.Poly(sympy.resultant(_sym(F), _sym(G), Y), X)
    refl = [int(c) for c in reversed(ref.all_coeffs())] if not ref.is_zero else []
    while refl and refl[-1] == 0:
        refl.pop()
    assert res(F, G) == refl


# --------------------------------------------------------------- closed forms


@pytest.mark.parametrize("seed", range(10))
def test_linear_substitution_closed_form(seed):
    """res_y(y - a(x), g) = g(x, a(x))."""
    rng = rng_for(902, seed)
    a = [int(v) for v in rng.integers(-20, 20, size=int(rng.integers(1, 4)))]
    while a and a[-1] == 0:
        a.pop()
    f = [[-c for c in a] or [0], [1]]
    G = rnd(rng, int(rng.integers(1, 5)), int(rng.integers(0, 4)), 10)
    assert res(f, G) == pcompose_y(G, a)


def test_constant_and_zero_conventions():
    g = [[1, 2], [3], [0, 5]]  # y-degree 2
    assert res([[7]], g) == [49]  # f = 7, n_y = 2 -> 7^2
    assert res(g, [[-2]]) == [4]  # g first: m_y = 2 -> (-2)^2
    assert res([[3]], [[5, 1]]) == [1]  # both constant in y
    assert res([[0]], g) == [] and res(g, [[0, 0], [0]]) == []
    assert res([[0, 0, 0], [1, 0]], g) == res([[0], [1]], g)  # zero padding is trimmed


# ------------------------------------------------------------------ identities


@pytest.mark.parametrize("seed", range(12))
def test_antisymmetry_scaling_multiplicativity(seed):
    rng = rng_for(903, seed)
    F1 = rnd(rng, 2, 2, 8)
    F2 = rnd(rng, 1, 2, 8)
    G = rnd(rng, 2, 2, 8)
    F1[2][0] = F1[2][0] or 1
    F2[1][0] = F2[1][0] or 1
    G[2][0] = G[2][0] or 1
    my, ny = 2, 2
    R12 = res(F1, G)
    assert res(G, F1) == (R12 if (my * ny) % 2 == 0 else psub([], R12))
    R21 = res(F2, G)
    assert res(G, F2) == (R21 if (1 * ny) % 2 == 0 else psub([], R21))
    c = int(rng.integers(2, 9))
    assert res([[c * v for v in r] for r in F1], G) == pmul([c ** ny], R12)
    assert res(bivar_mul(F1, F2), G) == pmul(R12, R21)


@pytest.mark.parametrize("seed", range(8))
def test_row_operation_invariance(seed):
    """res(f, g + q f) = res(f, g) when deg_y q < n_y - m_y."""
    rng = rng_for(904, seed)
    F = rnd(rng, 1, 2, 8)
    G = rnd(rng, 3, 2, 8)
    F[1][0] = F[1][0] or 1
    G[3][0] = G[3][0] or 1
    Q = rnd(rng, 1, 1, 5)  # deg_y q = 1 < 3 - 1
    G2 = bivar_trim(G)
    QF = bivar_mul(Q, F)
    H = [list(r) for r in G2]
    for j, row in enumerate(QF):
        while len(H) <= j:
            H.append([])
        H[j] = psub(H[j], psub([], row))
    assert res(F, H) == res(F, G)


@pytest.mark.parametrize("seed", range(8))
def test_common_root_divides_resultant(seed):
    """(x - x0) | R when f(x0, y0) = g(x0, y0) = 0 (paper Thm 1)."""
    rng = rng_for(905, seed)
    x0, y0 = int(rng.integers(-4, 5)), int(rng.integers(-4, 5))
    F = rnd(rng, 2, 2, 6)
    G = rnd(rng, 2, 2, 6)
    for A in (F, G):
        A[2][0] = A[2][0] or 1
        A[0][0] -= peval([peval(r, x0) for r in A], y0)
    R = res(F, G)
    assert peval(R, x0) == 0


@pytest.mark.parametrize("seed", range(10))
def test_degree_and_coefficient_bounds(seed):
    rng = rng_for(906, seed)
    d1, d2 = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    from workloads import dense_total, sparse_total
    F = dense_total(rng, d1, 12) if seed % 2 else sparse_total(rng, d1, 12)
    G = dense_total(rng, d2, 12) if seed % 2 else sparse_total(rng, d2, 12)
    for var in "yx":
        R = res(F, G, var)
        assert len(R) - 1 <= degree_bound(F, G, var)
        B2 = hadamard_bound_sq(F, G, var)
        assert all(c * c <= B2 for c in R)
        if seed % 2 and var == "y":
            assert len(R) - 1 == d1 * d2  # generic dense case: deg R = m n


# --------------------------------------------------------- evaluation commutes


@pytest.mark.parametrize("seed", range(10))
def test_point_checks_agree_with_full_oracle(seed):
    rng = rng_for(907, seed)
    F = rnd(rng, int(rng.integers(1, 4)), 3, 10, 0.7)
    G = rnd(rng, int(rng.integers(1, 4)), 3, 10, 0.7)
    q = oracle.next_check_primes(1)[0]
    for var in "yx":
        R = res(F, G, var)
        for x0 in (0, 1, -2, 5, 11):
            assert res_at_int_point(F, G, x0, var) == peval(R, x0)
            assert res_at_point_mod(F, G, x0 % q, q, var) == peval(R, x0) % q


def test_check_primes_are_prime_and_61_bit():
    ps = oracle.next_check_primes(4)
    assert all(p.bit_length() == 61 for p in ps)
    assert all(sympy.isprime(p) for p in ps)
    assert oracle.is_probable_prime(2147483647) and not oracle.is_probable_prime(2147483649)


# ------------------------------------------------------- planted oracle mistakes


def _pins_pass():
    """A fast subset of the pins above, used to show that planted mistakes are caught."""
    ok = res([[1], [1]], [[2], [0], [1]]) == [3]  # res(y + 1, y^2 + 2) = g(x, -1)
    F, G = [[1, 2], [3, 1]], [[0, 1], [2, 1]]  # y-degrees 1 and 1
    ok &= res(F, G) == _closed_tiny(F, G)
    ok &= res(G, F) == psub([], res(F, G))  # antisymmetry, m_y n_y odd
    A, B = [[1, 1], [0, 2], [1]], [[3], [1, 1]]
    ok &= res(A, B) == leibniz_det(sylvester(bivar_trim(A), bivar_trim(B)))
    return ok


def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong sign, swapped row blocks, a dropped or shifted term in the oracle fails a pin."""
    import oracle.resultant as R

    assert _pins_pass()
    orig_syl, orig_det = R.sylvester, R.bareiss_det

    def swapped_blocks(fy, gy):
        S = orig_syl(fy, gy)
        ny = len(gy) - 1
        return S[ny:] + S[:ny]

    def dropped_term(fy, gy):
        S = orig_syl(fy, gy)
        S[0][len(fy) - 1] = []
        return S

    def reversed_row(fy, gy):  # lowest y-power first in the f rows
        S = orig_syl(fy, gy)
        ny = len(gy) - 1
        for i in range(ny):
            seg = S[i][i:i + len(fy)]
            S[i][i:i + len(fy)] = seg[::-1]
        return S

    mutants = [("sylvester", swapped_blocks), ("sylvester", dropped_term),
               ("sylvester", reversed_row),
               ("bareiss_det", lambda M: psub([], orig_det(M)))]
    for name, fn in mutants:
        monkeypatch.setattr(R, name, fn)
        assert not _pins_pass(), name
        monkeypatch.undo()
    assert _pins_pass()

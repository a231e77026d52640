"""CPU pins of the oracle's gcd, square-free part and Yun factorisation over
Z[x]: closed forms built from known factors and multiplicities, exact
divisibility, coprimality of the cofactors by the resultant oracle (Sylvester
determinant: a different algorithm from the Euclidean one), and the product
identity pp(r) = prod r_i^i."""

import random

import pytest

import oracle
from oracle.poly import pmul, ptrim
from oracle.sqfree import (sqfree_part, yun, zx_content, zx_deriv, zx_divexact, zx_gcd, zx_pow, zx_pp)


def lin(a, b=1):
    """b x - a"""
    return [-a, b]


def prod(polys):
    r = [1]
    for p in polys:
        r = pmul(r, p)
    return r


def res_int(u, v):
    """Resultant of two integer polynomials by the oracle's Sylvester determinant."""
    fy = [[c] for c in u]
    gy = [[c] for c in v]
    R = oracle.res(fy, gy, "y")
    return R[0] if R else 0


def test_closed_form_multiplicities():
    # r = 6 (x-1)^3 (x+2)^2 (x^2+1) (2x-3)
    f1, f2, f3, f4 = lin(1), lin(-2), [1, 0, 1], lin(3, 2)
    r = [6 * c for c in prod([zx_pow(f1, 3), zx_pow(f2, 2), f3, f4])]
    assert zx_gcd(r, zx_deriv(r)) == zx_pp(prod([zx_pow(f1, 2), f2]))
    assert sqfree_part(r) == zx_pp(prod([f1, f2, f3, f4]))
    assert yun(r) == [zx_pp(pmul(f3, f4)), f2, f1]
    assert yun([-4 * c for c in r]) == yun(r)


def test_gcd_closed_forms_and_degenerate_inputs():
    a, b, c = lin(2), [1, 1, 1], lin(-5, 3)
    u = prod([a, a, b, [7]])
    v = prod([a, c, [-14]])
    assert zx_gcd(u, v) == a
    assert zx_gcd(u, []) == zx_pp(u)
    assert zx_gcd([], v) == zx_pp(v)
    assert zx_gcd([5], v) == [1]
    assert zx_gcd([], []) == []
    assert zx_gcd([-3, 6], [4, -8]) == [-1, 2]  # primitive, positive leading coefficient


@pytest.mark.parametrize("seed", range(6))
def test_random_products_divisibility_and_coprime_cofactors(seed):
    rnd = random.Random(seed)
    facs = [ptrim([rnd.randint(-9, 9) for _ in range(rnd.randint(2, 4))] + [rnd.choice([1, 2, 3])])
            for _ in range(4)]
    common = prod(facs[:2])
    u = prod([common, facs[2], [rnd.randint(1, 5)]])
    v = prod([common, facs[3]])
    g = zx_gcd(u, v)
    qu, qv = zx_divexact(u, g), zx_divexact(v, g)  # raises if not exact
    assert res_int(qu, qv) != 0                    # cofactors coprime
    assert len(g) >= len(zx_pp(common))            # the planted common factor divides g
    zx_divexact(g, zx_pp(common))


@pytest.mark.parametrize("seed", range(6))
def test_yun_product_identity(seed):
    rnd = random.Random(100 + seed)
    parts = []
    for i in range(1, 4):
        for _ in range(rnd.randint(0, 2)):
            parts.append((ptrim([rnd.randint(-5, 5), rnd.randint(-5, 5), rnd.randint(1, 3)]), i))
    if not parts:
        parts = [(lin(1), 2)]
    r = prod([zx_pow(p, e) for p, e in parts] + [[rnd.choice([-6, 1, 10])]])
    fac = yun(r)
    back = prod([zx_pow(fi, i + 1) for i, fi in enumerate(fac)])
    assert back == zx_pp(r)
    for i, fi in enumerate(fac):  # each factor square-free, factors pairwise coprime
        if len(fi) > 1:
            assert len(zx_gcd(fi, zx_deriv(fi))) == 1
        for fj in fac[i + 1:]:
            if len(fi) > 1 and len(fj) > 1:
                assert res_int(fi, fj) != 0


def test_content_and_primitive_part():
    assert zx_content([6, -9, 12]) == 3
    assert zx_pp([6, -9, -12]) == [-2, 3, 4]
    assert sqfree_part([0, 0, 5]) == [0, 1]  # 5 x^2 -> x

"""GPU: gcd in Z[x] and the square-free part by the modular route (per-prime
Euclid, degree vote, Chinese remaindering, certified cofactors) against the
oracle's primitive Euclidean algorithm: closed forms, random products with a
planted common factor, degenerate inputs, multi-limb coefficients, a case
past 512 primes (the wide CRT), and resultants with a repeated factor."""

import random

import pytest

import oracle
from oracle.poly import pmul, ptrim
from oracle.sqfree import sqfree_part, zx_deriv, zx_divexact, zx_gcd, zx_pow, zx_pp
from workloads import dense_total, rng_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1010_1386_amd as rsl
    c = rsl.Context(device=0, workspace_bytes=1 << 30)
    yield c
    c.close()


def prod(polys):
    r = [1]
    for p in polys:
        r = pmul(r, p)
    return r


def check_gcd(ctx, u, v):
    g, a, b = ctx.gcd(u, v)
    want = zx_gcd(u, v)
    assert g == want
    if want:
        assert a == zx_divexact(u, want) and b == zx_divexact(v, want)
    return g


def test_closed_form_square_free_part(ctx):
    f1, f2, f3, f4 = [-1, 1], [2, 1], [1, 0, 1], [-3, 2]
    r = [6 * c for c in prod([zx_pow(f1, 3), zx_pow(f2, 2), f3, f4])]
    q, g = ctx.sqfree_part(r)
    assert g == zx_pp(prod([zx_pow(f1, 2), f2]))
    assert zx_pp(q) == sqfree_part(r) == zx_pp(prod([f1, f2, f3, f4]))
    assert q == zx_divexact(r, g)


@pytest.mark.parametrize("seed", range(5))
def test_random_products(ctx, seed):
    rnd = random.Random(seed)
    facs = [ptrim([rnd.randint(-99, 99) for _ in range(rnd.randint(2, 6))] + [rnd.choice([1, -2, 3, 7])])
            for _ in range(5)]
    common = prod(facs[:2])
    u = prod([common, facs[2], [rnd.randint(1, 50)]])
    v = prod([common, zx_pow(facs[3], 2), facs[4], [-rnd.randint(1, 50)]])
    check_gcd(ctx, u, v)
    check_gcd(ctx, v, u)
    r = prod([zx_pow(facs[0], 3), facs[1], zx_pow(facs[2], 2)])
    q, g = ctx.sqfree_part(r)
    assert zx_pp(q) == sqfree_part(r) and g == zx_gcd(r, zx_deriv(r))


def test_degenerate_inputs(ctx):
    u = prod([[1, 1], [-2, 3]])
    assert ctx.gcd(u, []) == (zx_pp(u), [1], [])
    g, a, b = ctx.gcd([], [4, -8])
    assert g == [-1, 2] and a == [] and b == [-4]
    assert ctx.gcd([], []) == ([], [], [])
    assert ctx.gcd([6], [9, 3]) == ([1], [6], [9, 3])
    assert ctx.gcd(u, u) == (zx_pp(u), [1], [1])
    check_gcd(ctx, [3, 0, -1], [0, 5, 7])          # coprime: G = 1
    check_gcd(ctx, [-4, 0, -4], [2, 0, 2])          # negative leading coefficient, contents
    assert ctx.sqfree_part([]) == ([], [])
    assert ctx.sqfree_part([-7]) == ([-7], [1])
    assert ctx.sqfree_part([0, 0, 0, 5]) == ([0, 5], [0, 0, 1])  # 5 x^3 = 5x * x^2


def test_multi_limb_coefficients(ctx):
    rnd = random.Random(7)
    big = lambda bits: rnd.getrandbits(bits) * rnd.choice([-1, 1]) | 1
    common = [big(300), big(200), big(250)]
    u = prod([common, [big(400), big(100)], [big(64)]])
    v = prod([common, [big(90), big(500), big(30)]])
    check_gcd(ctx, u, v)
    r = prod([zx_pow([big(120), big(80)], 3), [big(200), 0, big(150)]])
    q, g = ctx.sqfree_part(r)
    assert zx_pp(q) == sqfree_part(r)


def test_wide_crt_past_512_primes(ctx):
    """Degree 41 with ~8700-bit coefficients: more than 512 primes for the
    certificate; checked by the exact identities and, independently, by the
    cofactors' gcd being 1."""
    rnd = random.Random(11)
    big = lambda bits: rnd.getrandbits(bits) * rnd.choice([-1, 1]) | 1
    common = [big(4200) for _ in range(12)] + [big(64)]
    u = prod([common, [big(4500) for _ in range(30)]])
    v = prod([common, [big(4200) for _ in range(29)]])
    g, a, b = ctx.gcd(u, v)
    assert pmul(g, a) == u and pmul(g, b) == v
    assert g[-1] > 0 and len(g) >= len(common)
    assert ctx.gcd(a, b)[0] == [1]


def test_square_free_part_of_resultants(ctx):
    """R = res_y(f, f_y) with f = F (y^2 - h) contains res_y(F, y^2 - h)
    squared (a repeated factor); R from the device pipeline, then its
    square-free part from the device gcd, equal to the oracle's."""
    rng = rng_for(721, 0)
    for k in range(3):
        F = dense_total(rng, 3, 6)
        h = [int(v) for v in rng.integers(-9, 10, size=3)]
        h[-1] = h[-1] or 1
        f = oracle.bivar_mul(F, [[-c for c in h], [0], [1]])
        fy = [[(j + 1) * c for c in f[j + 1]] for j in range(len(f) - 1)]
        R = ctx.res(f, fy, "y")
        assert R == oracle.res(f, fy, "y")
        q, g = ctx.sqfree_part(R)
        assert zx_pp(q) == sqfree_part(R)
        assert len(g) > 1  # a repeated factor exists


def test_yun_factorisation_matches_oracle(ctx):
    """Yun's loop on the device gcd: closed form, products with planted
    multiplicities, a resultant with a repeated factor, degenerate inputs."""
    from oracle.sqfree import yun
    f1, f2, f3, f4 = [-1, 1], [2, 1], [1, 0, 1], [-3, 2]
    r = [6 * c for c in prod([zx_pow(f1, 3), zx_pow(f2, 2), f3, f4])]
    assert ctx.sqfree_factor(r) == yun(r) == [zx_pp(pmul(f3, f4)), f2, f1]
    rnd = random.Random(31)
    for _ in range(4):
        parts = [(ptrim([rnd.randint(-20, 20), rnd.randint(-20, 20), rnd.choice([1, 2, 5])]), e)
                 for e in (1, 2, 2, 4) if rnd.random() < 0.8]
        r = prod([zx_pow(p, e) for p, e in parts] + [[rnd.choice([-3, 1, 12])]])
        assert ctx.sqfree_factor(r) == yun(r)
    assert ctx.sqfree_factor([]) == [] and ctx.sqfree_factor([7]) == []
    assert ctx.sqfree_factor([0, 0, 0, 5]) == yun([0, 0, 0, 5]) == [[1], [1], [0, 1]]
    rng = rng_for(723, 0)
    F = dense_total(rng, 4, 6)
    f = oracle.bivar_mul(F, [[-2, 1, 3], [0], [1]])
    fy = [[(j + 1) * c for c in f[j + 1]] for j in range(len(f) - 1)]
    R = ctx.res(f, fy, "y")
    fac = ctx.sqfree_factor(R)
    assert fac == yun(R) and len(fac) >= 2

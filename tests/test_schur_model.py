"""CPU: the generator recursion of the Schur evaluation (paper Sec. 4.1: the
Sylvester matrix has displacement rank two, and the generalised Schur
algorithm triangularises it from its generators), written here in plain
Python with the kernel's steps and conventions, against determinants:
Leibniz expansion on tiny matrices, the oracle's modular elimination on
larger ones.  Breakdowns (a vanishing leading minor) must be reported, never
turned into a wrong value; the kernel sends those points to the remainder
sequence.

Recursion (division-free): S - K S Z^T = G B^T with K the down-shift inside
the two row blocks (n rows of f, then m rows of g) and Z the column shift;
G = [e_0, e_n], B = [row 0, row n].  Step k: d = g0 . b0 with (g0, b0) the
pivot rows;
  G' = [g0_1 G_0 - g0_0 G_1,  f d e_0 + K' (G b0)],
  B' = [b0_1 B_0 - b0_0 B_1,  d e_0 + Z' (B g0)],
which represent d times the Schur complement; det S = prod d_k / prod sigma_k
with sigma_{k+1} = sigma_k d_k."""

import itertools
import random

import pytest

import oracle
from oracle.modular import det_mod

P31 = 2147483647


def sylvester_rows(a, b):
    """Sylvester matrix of a (degree m) and b (degree n), coefficients highest first:
    n rows of a, then m rows of b (the layout of the paper's S^(y))."""
    m, n = len(a) - 1, len(b) - 1
    r = m + n
    S = [[0] * r for _ in range(r)]
    for i in range(n):
        for t, c in enumerate(a):
            S[i][i + t] = c
    for j in range(m):
        for t, c in enumerate(b):
            S[n + j][j + t] = c
    return S


def schur_det(a, b, p):
    """det of the Sylvester matrix mod p by the recursion above, or None on a breakdown."""
    m, n = len(a) - 1, len(b) - 1
    r = m + n
    if r == 0:
        return 1
    S = sylvester_rows(a, b)
    two = 0 < n < r
    G = [[1 if l == 0 else 0, 1 if (two and l == n) else 0] for l in range(r)]
    B = [[S[0][l] % p, (S[n][l] % p) if two else 0] for l in range(r)]
    num, den, sigma = 1, 1, 1
    for k in range(r):
        (ga, gb), (ba, bb) = G[k], B[k]
        d = (ga * ba + gb * bb) % p
        num, den = num * d % p, den * sigma % p
        if k == r - 1:
            break
        if d == 0:
            return None
        c = [(G[l][0] * ba + G[l][1] * bb) % p for l in range(r)]
        u = [(ga * B[l][0] + gb * B[l][1]) % p for l in range(r)]
        for l in range(k + 1, r):
            x = (gb * G[l][0] - ga * G[l][1]) % p
            y = (bb * B[l][0] - ba * B[l][1]) % p
            g1 = 0 if l == n else (d if l == k + 1 else c[l - 1])
            b1 = d if l == k + 1 else u[l - 1]
            G[l], B[l] = [x, g1], [y, b1]
        sigma = sigma * d % p
    return num * pow(den, p - 2, p) % p


def leibniz(M):
    r = len(M)
    tot = 0
    for perm in itertools.permutations(range(r)):
        inv = sum(1 for i in range(r) for j in range(i + 1, r) if perm[i] > perm[j])
        prod = 1
        for i in range(r):
            prod *= M[i][perm[i]]
        tot += -prod if inv & 1 else prod
    return tot


def test_tiny_exhaustive_against_leibniz():
    """Every a, b with degrees <= 2 and coefficients in {-1, 0, 1} (nonzero leading
    coefficients), mod a 31-bit prime and mod 3: equal to the Leibniz determinant
    whenever no breakdown is reported."""
    vals = (-1, 0, 1)
    checked = broke = 0
    for m in range(3):
        for n in range(3):
            for a in itertools.product(vals, repeat=m + 1):
                if a[0] == 0:
                    continue
                for b in itertools.product(vals, repeat=n + 1):
                    if b[0] == 0:
                        continue
                    want = leibniz(sylvester_rows(list(a), list(b))) if m + n else 1
                    for p in (P31, 3):
                        got = schur_det(list(a), list(b), p)
                        if got is None:
                            broke += 1
                            continue
                        assert got == want % p, (a, b, p)
                        checked += 1
    assert checked > 300 and broke > 0


@pytest.mark.parametrize("seed", range(4))
def test_random_against_modular_elimination(seed):
    rnd = random.Random(seed)
    for _ in range(150):
        m, n = rnd.randint(0, 12), rnd.randint(0, 12)
        p = P31 if rnd.random() < 0.7 else rnd.choice([5, 7, 11])
        a = [rnd.randrange(1, p)] + [rnd.randrange(p) for _ in range(m)]
        b = [rnd.randrange(1, p)] + [rnd.randrange(p) for _ in range(n)]
        got = schur_det(a, b, p)
        want = det_mod(sylvester_rows(a, b), p) if m + n else 1
        if got is not None:
            assert got == want, (m, n, p)


def test_planted_breakdown_is_reported():
    """a = y^3 + 2 y^2 + ..., b = 3 y + 6: the leading 2x2 minor of rows (a, b)
    below the n = 1 row of a vanishes (1 * 6 - 2 * 3), so step 1 has d = 0."""
    a, b = [1, 2, 5, 7], [3, 6]
    assert schur_det(a, b, P31) is None
    assert det_mod(sylvester_rows(a, b), P31) != 0


def test_matches_oracle_resultant_at_points():
    """Bivariate inputs specialised at x = t: the recursion mod q equals the oracle's
    resultant mod q of the specialised pair (where no breakdown occurs)."""
    from workloads import dense_total, rng_for
    rng = rng_for(718, 0)
    qs = oracle.next_check_primes(2)
    for k in range(6):
        F = dense_total(rng, 3 + k % 3, 20)
        G = dense_total(rng, 2 + k % 2, 20)
        for q in qs:
            t = (k * 7919 + 13) % q
            fy = [oracle.poly_eval_mod(row, t, q) for row in F]
            gy = [oracle.poly_eval_mod(row, t, q) for row in G]
            while fy and fy[-1] == 0:
                fy.pop()
            while gy and gy[-1] == 0:
                gy.pop()
            got = schur_det(fy[::-1], gy[::-1], q)
            if got is not None:
                assert got == oracle.res_at_point_mod(F, G, t, q, "y")

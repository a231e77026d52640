"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and its
host-side planner (rsl_query: no device work) agrees with the oracle's bounds."""

import ctypes
import math
import os
import re

import pytest

import oracle
from workloads import dense_total, rng_for, small_random, sparse_total

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsl.h")


@pytest.fixture(scope="module")
def rsl():
    import paper_1010_1386_amd as m
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(rsl):
    lib = ctypes.CDLL(rsl.library_path())
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_strerror(rsl):
    assert "gfx950" in rsl.version()
    assert rsl._lib.rsl_strerror(rsl.RSL_EPRIMES) == b"prime table exhausted"
    assert rsl._lib.rsl_strerror(0) == b"ok"


def _table_primes(n):
    # the library's table: the primes below 2^32 / 3, descending
    return oracle.next_check_primes(n, below=(1 << 32) // 3 + 1)


@pytest.mark.parametrize("seed", range(12))
def test_query_matches_oracle_bounds(rsl, seed):
    """D, the Hadamard bound and a minimal prime count Pi p > 2B (readings 5 and 7)."""
    rng = rng_for(800, seed)
    F = dense_total(rng, int(rng.integers(1, 9)), int(rng.integers(4, 60))) if seed % 3 else \
        sparse_total(rng, int(rng.integers(2, 9)), int(rng.integers(4, 60)))
    G = dense_total(rng, int(rng.integers(1, 9)), int(rng.integers(4, 60)))
    for var in "yx":
        q = rsl.query(F, G, var)
        assert q["D"] == oracle.degree_bound(F, G, var)
        B2 = oracle.hadamard_bound_sq(F, G, var)
        assert abs(q["bound_bits"] - (B2.bit_length() + 1) // 2) <= 1
        ps = _table_primes(q["n_primes"])  # no bad primes for these inputs
        M = math.prod(ps)
        assert M * M > 4 * B2
        assert (M // ps[-1]) ** 2 <= 4 * B2
        assert q["out_limbs"] == (M.bit_length() + 31) // 32


def test_query_degrees_and_points(rsl):
    # lc_y f = x (x - 3): two spare points
    F = [[1, 2, 3], [4, 5], [0, -3, 1]]
    G = [[2, -1], [0, 1, 1], [7, 0, 0, 1]]
    q = rsl.query(F, G, "y")
    assert (q["my"], q["ny"]) == (2, 2)
    assert q["n_points"] == q["D"] + 1 + 2 + 3  # s = deg lc_y f + deg lc_y g = 2 + 3
    assert q["origin"] == 1  # lc_y f (0) = 0: every prime's point 0 is bad; lc_y f (1) = -2
    z = rsl.query([[0]], G, "y")
    assert z["D"] == -1


def test_query_rejects_bad_arguments(rsl):
    with pytest.raises(ValueError):
        rsl.query([[1]], [[1]], "z")
    p = rsl.Poly([[1, 2]])
    p.c.limbs = 0
    info = rsl.rsl_info()
    rc = rsl._lib.rsl_query(ctypes.byref(p.c), ctypes.byref(rsl.Poly([[1]]).c), 0, ctypes.byref(info))
    assert rc == rsl.RSL_EINVAL
    rc = rsl._lib.rsl_query(ctypes.byref(rsl.Poly([[1]]).c), ctypes.byref(rsl.Poly([[1]]).c), 7, ctypes.byref(info))
    assert rc == rsl.RSL_EINVAL


def test_bad_prime_detected_by_planner(rsl):
    p0 = 1431655751  # the first prime of the table
    F = [[1, 2, 3], [5, 0, 1], [p0 * 3, p0 * 2]]
    G = [[2, 1], [1, 1, 1], [3]]
    assert rsl.query(F, G, "y")["bad_primes"] == 1
    assert rsl.query(F, G, "x")["bad_primes"] == 0  # lc_x f does not vanish mod p0


def test_multi_limb_inputs_are_planned(rsl):
    rng = rng_for(801, 0)
    F = [[int(v) << 200 for v in row] for row in small_random(rng, 3, 3, 30)]
    G = small_random(rng, 2, 4, 30)
    q = rsl.query(F, G, "y")
    B2 = oracle.hadamard_bound_sq(F, G, "y")
    assert abs(q["bound_bits"] - (B2.bit_length() + 1) // 2) <= 1


def test_factorisation_identity_for_curve_workload():
    """res_y(F Q, (F Q)_y) = (-1)^{d(d-1)/2 + e(e-1)/2} 4 h res_y(F, F_y) res_y(F, Q)^2,
    Q = y^2 - h(x), d = e + 2, with res_y(F, Q) = E(x,h)^2 - h O(x,h)^2 for
    F = E(x, y^2) + y O(x, y^2): the closed form used to pin the curve workload."""
    from oracle import bivar_mul, pmul, psub, res

    for seed in range(4):
        rng = rng_for(802, seed)
        e = 2 + seed % 3
        F = dense_total(rng, e, 6)
        h = [int(v) for v in rng.integers(-9, 10, size=3)]
        h[-1] = h[-1] or 2
        Q = [[-c for c in h], [0], [1]]
        f = bivar_mul(F, Q)
        g = [[j * c for c in f[j]] for j in range(1, len(f))]
        Fy = [[j * c for c in F[j]] for j in range(1, len(F))]
        R = res(f, g)
        d = e + 2
        sign = -1 if (d * (d - 1) // 2 + e * (e - 1) // 2) % 2 else 1
        E, O = [], []
        hp = [1]
        for j, row in enumerate(F):  # F = sum_j F_j y^j
            term = pmul(row, hp) if j % 2 == 0 else None
            if j % 2 == 0:
                E = psub(E, psub([], term))
            else:
                O = psub(O, psub([], pmul(row, hp)))
            if j % 2 == 1:
                hp = pmul(hp, h)
        rFQ = psub(pmul(E, E), pmul(h, pmul(O, O)))
        assert rFQ == res(F, Q)
        rhs = pmul([4 * sign], pmul(h, pmul(res(F, Fy), pmul(rFQ, rFQ))))
        assert R == rhs


@pytest.mark.parametrize("lc, origin", [([1, 1], 0), ([0, 1], 1), ([0, -1, 1], 2), ([0, 0, 1], 1),
                                        ([0, 2, -3, 1], 3), ([7], 0), ([0, 1 << 40], 1)])
def test_automatic_origin(rsl, lc, origin):
    """Default options: origin 0 unless a leading coefficient vanishes at 0 over Z,
    then the first x0 >= 1 where neither does (here lc_y f = the given row)."""
    F = [[3, 1, -2], [1, 4], lc]
    G = [[5, -1], [2, 2, 1], [1, 0, 2]]
    assert rsl.query(F, G, "y")["origin"] == origin
    assert rsl.query(G, F, "y")["origin"] == origin  # either polynomial's coefficient


def test_automatic_origin_needs_a_root_shared_by_every_prime(rsl):
    # constant leading coefficients: no bad point anywhere, origin 0
    F = [[1, 2], [3], [5]]
    G = [[2], [1, 1], [4]]
    assert rsl.query(F, G, "y")["origin"] == 0

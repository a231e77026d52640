"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, bit for bit."""

import json
import os

import pytest

import oracle
import workloads
from workloads import rng_for, small_random, dense_total, sparse_total

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_1010_1386_amd as rsl
    c = rsl.Context(device=0, workspace_bytes=512 << 20)
    yield c
    c.close()


def _golden(cfg):
    with open(os.path.join(GOLDEN, f"cfg{cfg}.json")) as fh:
        return {r["name"]: r for r in json.load(fh)["records"]}


def test_config1_res_y_and_res_x_match_golden(ctx):
    f, g = workloads.config1()
    gold = _golden(1)
    for var in "yx":
        got = ctx.res(f, g, var)
        want = [int(c) for c in gold[f"cfg1_{var}"]["coeffs"]]
        assert got == want, var


@pytest.mark.parametrize("seed", range(16))
def test_small_random_vs_oracle(ctx, seed):
    rng = rng_for(700, seed)
    F = small_random(rng, int(rng.integers(0, 6)), int(rng.integers(0, 6)), int(rng.integers(2, 40)),
                     density=float(rng.choice([1.0, 0.6])))
    G = small_random(rng, int(rng.integers(0, 6)), int(rng.integers(0, 6)), int(rng.integers(2, 40)),
                     density=float(rng.choice([1.0, 0.6])))
    for var in "yx":
        assert ctx.res(F, G, var) == oracle.res(F, G, var), (seed, var)


@pytest.mark.parametrize("seed", range(6))
def test_total_degree_dense_and_sparse(ctx, seed):
    rng = rng_for(701, seed)
    d1, d2 = int(rng.integers(3, 9)), int(rng.integers(3, 9))
    b = int(rng.integers(8, 64))
    F = dense_total(rng, d1, b, force_top=False) if seed % 2 else sparse_total(rng, d1, b)
    G = dense_total(rng, d2, b, force_top=False) if seed % 2 else sparse_total(rng, d2, b)
    for var in "yx":
        assert ctx.res(F, G, var) == oracle.res(F, G, var), (seed, var)


def test_degenerate_inputs(ctx):
    g = [[1, 2], [3], [0, 5]]
    assert ctx.res([[0]], g) == []
    assert ctx.res([[7]], g) == [49]
    assert ctx.res(g, [[-2]]) == [4]
    assert ctx.res([[3]], [[5, 1]]) == [1]
    # common factor (y - x): R = 0
    f = [[0, -1], [1]]                        # y - x
    h = [[0, 0, -2], [1, 2], [0, 1]]          # arbitrary
    fh = oracle.bivar_mul(f, h)
    gh = oracle.bivar_mul(f, [[1, 1], [1]])
    assert ctx.res(fh, gh) == []
    # leading y-coefficient vanishing at integer points: x (x - 3) y^2 + ...
    F = [[1, 2, 3], [4, 5], [0, -3, 1]]
    G = [[2, -1], [0, 1, 1], [7, 0, 0, 1]]
    for var in "yx":
        assert ctx.res(F, G, var) == oracle.res(F, G, var)


def test_planted_bad_point_every_prime(ctx):
    """lc_y f = (x - a): point a is bad for every prime and must be replaced
    (origin 0 kept, so that a = 0 takes the gapped path too)."""
    for a in (0, 1, 5):
        F = [[3, 1, -2], [1, 4], [-a, 1]]
        G = [[5, -1], [2, 2, 1], [1]]
        R = oracle.res(F, G)
        assert ctx.res(F, G) == R
        assert ctx.res(F, G, points="formal") == R
        assert ctx.res(F, G, point_origin=-1) == R
        c = ctx.counters()
        assert c["bad_pairs"] >= 1


def test_automatic_origin_when_zero_is_bad_everywhere(ctx):
    """Leading coefficients vanishing at x = 0 over Z move the default origin:
    x (x - 1) (x - 3) to 2 (point 3 still bad: the gapped path from there),
    x^2 (x - 1) to 2 and 5 x to 1 (no bad point: the consecutive path and the
    shift back).  Every result agrees with the oracle and with origin 0."""
    import paper_1010_1386_amd as rsl
    rng = rng_for(706, 0)
    G = dense_total(rng, 5, 20)
    for lc, origin, bad in (([0, 3, -4, 1], 2, True), ([0, 0, -1, 1], 2, False), ([0, 5], 1, False)):
        F = dense_total(rng, 4, 20)
        F.append(lc)
        for var in "yx":
            R = oracle.res(F, G, var)
            q = rsl.query(F, G, var)
            assert ctx.res(F, G, var) == R
            if var == "y":
                assert q["origin"] == origin
                assert (ctx.counters()["bad_pairs"] > 0) == bad
            assert ctx.res(F, G, var, point_origin=-1) == R


def test_linear_substitution_closed_form(ctx):
    rng = rng_for(702, 0)
    a = [3, -2, 1]
    f = [[-c for c in a], [1]]
    G = small_random(rng, 4, 3, 20)
    assert ctx.res(f, G) == oracle.pcompose_y(G, a)


def test_self_consistency_primes_and_points(ctx):
    """The final R must not depend on which primes or points were used."""
    rng = rng_for(703, 0)
    F = dense_total(rng, 7, 30)
    G = dense_total(rng, 6, 30)
    base = ctx.res(F, G)
    assert base == oracle.res(F, G)
    assert ctx.res(F, G, prime_start=5) == base
    assert ctx.res(F, G, extra_primes=3) == base
    assert ctx.res(F, G, point_origin=1000) == base
    assert ctx.res(F, G, extra_points=17) == base
    assert ctx.res(F, G, points="formal") == base


def test_bad_prime_is_skipped(ctx):
    """lc_y f = p_0 * c: the largest prime divides the leading coefficient."""
    import paper_1010_1386_amd as rsl
    p0 = 1431655751  # largest prime below 2^32 / 3, first in the table
    F = [[1, 2, 3], [5, 0, 1], [p0 * 3, p0 * 2]]
    G = [[2, 1], [1, 1, 1], [3]]
    info = rsl.query(F, G, "y")
    assert info["bad_primes"] >= 1
    assert ctx.res(F, G) == oracle.res(F, G)


def test_prime_table_exhaustion_is_reported(ctx):
    import paper_1010_1386_amd as rsl
    F = dense_total(rng_for(704, 0), 5, 20)
    G = dense_total(rng_for(704, 1), 5, 20)
    with pytest.raises(rsl.RSLError) as ei:
        ctx.res(F, G, prime_limit=2)
    assert ei.value.code == rsl.RSL_EPRIMES


def _digest(coeffs):
    import hashlib
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


@pytest.mark.parametrize("var", ["y", "x"])
def test_config2_matches_golden_digest(ctx, var):
    """Dense total degree 24, signed 32-bit: res_y and res_x bit-exact (SHA-256 of all coefficients)."""
    f, g = workloads.config2()
    rec = _golden(2)[f"cfg2_{var}"]
    got = ctx.res(f, g, var)
    assert len(got) - 1 == rec["degree"]
    for i, v in rec["samples"].items():
        assert got[int(i)] == int(v)
    assert _digest(got) == rec["sha256"]


def test_vandermonde_solve_for_every_prime(ctx):
    """interp_newton: every prime through the divided-difference solve (the
    triangular factors of the Vandermonde matrix, Sec. 4.1) gives the same
    result as the consecutive-point products, for single problems (with and
    without bad points, shifted origin) and a job in both schedules."""
    import paper_1010_1386_amd as rsl
    rng = rng_for(707, 0)
    probs = []
    for k in range(6):
        F = dense_total(rng, 3 + k, 20)
        G = dense_total(rng, 2 + k, 20)
        if k % 3 == 1:
            F.append([0, -2, 1])  # lc_y f = x (x - 2): shifted origin, point 2 bad
        probs.append((F, G, "yx"[k % 2]))
    for F, G, var in probs[:4]:
        want = oracle.res(F, G, var)
        assert ctx.res(F, G, var, interp_newton=True) == want
        assert ctx.res(F, G, var, interp_newton=True, points="formal") == want
    base = ctx.job(probs)
    base.run("staged")
    want = base.results()
    base.close()
    job = ctx.job(probs, interp_newton=True)
    for mode in ("staged", "plain"):
        job.run(mode)
        assert job.results() == want
    job.close()

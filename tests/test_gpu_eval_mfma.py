"""GPU: the register-form evaluation (one lane or a lane pair per (prime,
point)) with its Horner sums on the matrix cores
(7-bit digit tiles written by the reduction, int8 products of the point
powers with the residues, nine anti-diagonal sums recombined modulo p) gives
the same bits as Horner's rule on the vector ALUs and as the oracle: shapes
across the register bounds (y-degrees 8..32, |m - n| <= 1), x-degrees at the
32-power limit and past it (Horner then), joint y/x projections (the x
system's digit tiles written by the y system's reduction), multi-limb inputs,
points where the leading coefficient vanishes, and the dense degree-24 pair
against the oracle's stored digests."""

import hashlib
import json
import os
import random

import pytest

import oracle
import workloads
from workloads import dense_total, rng_for, small_random

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rsl():
    import paper_1010_1386_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(rsl):
    c = rsl.Context(device=0, workspace_bytes=1 << 30)
    yield c
    c.close()


@pytest.fixture(scope="module")
def horner(rsl):
    """A context whose register-form evaluation uses Horner's rule only."""
    os.environ["RSL_EVAL_HORNER"] = "1"
    try:
        c = rsl.Context(device=0, workspace_bytes=1 << 30)
    finally:
        del os.environ["RSL_EVAL_HORNER"]
    yield c
    c.close()


def digest(coeffs):
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


def run(c, probs, modes=("staged", "plain"), lanes=2):
    """Results of one job in each mode (all equal), and its info."""
    job = c.job(probs, eval_lanes=lanes)
    info = job.info()
    out = {}
    for mode in modes:
        job.run(mode)
        out[mode] = job.results()
    job.close()
    first = out[modes[0]]
    for mode in modes[1:]:
        assert out[mode] == first, mode
    return first, info


def modq(probs, res, seed, n=2):
    rnd = random.Random(seed)
    for (f, g, v), R in zip(probs, res):
        for q in oracle.next_check_primes(n):
            t = rnd.randrange(q)
            assert oracle.peval(R, t) % q == oracle.res_at_point_mod(f, g, t, q, v), (q, t)


@pytest.mark.parametrize("lanes", [1, 2])
def test_degree24_pair_matches_oracle_digests(ctx, lanes):
    f, g = workloads.config2()
    res, info = run(ctx, [(f, g, "y"), (f, g, "x")], lanes=lanes)
    assert info["eval_mfma"] == 2 and info["eval_lanes"] == lanes
    with open(os.path.join(HERE, "golden", "cfg2.json")) as fh:
        gold = {r["name"]: r["sha256"] for r in json.load(fh)["records"]}
    assert digest(res[0]) == gold["cfg2_y"] and digest(res[1]) == gold["cfg2_x"]


@pytest.mark.parametrize("lanes", [1, 2])
def test_small_shapes_match_oracle(ctx, lanes):
    """Degrees 8..10 (the smallest with two lanes per pair), both projections
    of each system (shared reduction), a vanishing leading coefficient; one
    lane per pair also at degrees 1..3."""
    rng = rng_for(730, 0)
    probs = []
    for d, bits in [(8, 12), (9, 20), (10, 8)]:
        f, g = dense_total(rng, d, bits), dense_total(rng, d - (d % 2), bits)
        probs += [(f, g, "y"), (f, g, "x")]
    F = dense_total(rng, 10, 10)
    F[10] = [0, -5, 1]  # lc_y = x (x - 5): points 0 and 5 are bad for every prime
    probs.append((F, dense_total(rng, 9, 10), "y"))
    if lanes == 1:
        for d in (1, 2, 3):
            f, g = dense_total(rng, d, 16), dense_total(rng, d, 16)
            probs += [(f, g, "y"), (f, g, "x")]
    res, info = run(ctx, probs, modes=("staged", "plain", "batched"), lanes=lanes)
    assert info["eval_mfma"] == len(probs)
    assert res == [oracle.res(f, g, v) for f, g, v in probs]


@pytest.mark.parametrize("lanes", [1, 2])
def test_register_bounds_equal_horner(ctx, horner, lanes):
    """Degrees up to the 32 bound and x-degrees up to 32 (x-powers 0..31 on the
    matrix cores, x-power 32 added on the vector ALUs) give the same bits as
    Horner's rule; an x-degree past 32 keeps Horner."""
    rng = rng_for(731, 0)
    probs = []
    for dy, dyg, dx in [(16, 16, 16), (17, 16, 12), (24, 24, 24), (25, 24, 20), (31, 32, 6), (32, 32, 8),
                        (8, 9, 31), (12, 12, 31)]:
        probs.append((small_random(rng, dy, dx, 16), small_random(rng, dyg, max(dx - 3, 1), 16), "y"))
    # 33 x-powers in f, in g, in both (the last with y-degrees 32)
    probs.append((small_random(rng, 9, 32, 16), small_random(rng, 9, 5, 16), "y"))
    probs.append((small_random(rng, 12, 7, 16), small_random(rng, 11, 32, 16), "y"))
    probs.append((small_random(rng, 32, 32, 12), small_random(rng, 31, 32, 12), "y"))
    past = (small_random(rng, 9, 33, 16), small_random(rng, 9, 5, 16), "y")  # 34 x-powers: Horner
    probs.append(past)
    got, info = run(ctx, probs, lanes=lanes)
    assert info["eval_mfma"] == len(probs) - 1
    ref, rinfo = run(horner, probs, lanes=3 - lanes)
    assert rinfo["eval_mfma"] == 0
    assert got == ref
    modq(probs, got, 731)


@pytest.mark.parametrize("lanes", [1, 2])
def test_multi_limb_joint_projections(ctx, horner, lanes):
    """160-bit coefficients (the limb-staged reduction writes the digit tiles
    of both projections)."""
    rng = rng_for(732, 0)
    f, g = dense_total(rng, 9, 160), dense_total(rng, 9, 160)
    probs = [(f, g, "y"), (f, g, "x")]
    got, info = run(ctx, probs, lanes=lanes)
    assert info["eval_mfma"] == 2
    assert got == [oracle.res(f, g, v) for f, g, v in probs]
    big = [(dense_total(rng, 20, 100), dense_total(rng, 19, 100), v) for v in "y"]
    big.append((big[0][0], big[0][1], "x"))
    got, info = run(ctx, big, lanes=lanes)
    assert info["eval_mfma"] == 2
    assert got == run(horner, big, lanes=3 - lanes)[0]
    modq(big, got, 732)
    # total degree 32: x-power 32 in both projections, the y problem writing the
    # x problem's x-power-32 residues (its row 32) with its digit tiles
    f32, g32 = dense_total(rng, 32, 8), dense_total(rng, 31, 8)
    pair = [(f32, g32, "y"), (f32, g32, "x")]
    got, info = run(ctx, pair, lanes=lanes)
    assert info["eval_mfma"] == 2
    assert got == run(horner, pair, lanes=3 - lanes)[0]
    modq(pair, got, 733)


def test_repeated_runs_and_relayout(ctx):
    """The digit tiles are rewritten by every run and cleared at upload: runs
    of one job and a fresh job of the same problems agree."""
    rng = rng_for(733, 0)
    probs = [(dense_total(rng, 12, 24), dense_total(rng, 11, 24), v) for v in "yx"]
    job = ctx.job(probs, eval_lanes=2)
    outs = []
    for _ in range(3):
        job.run("staged")
        outs.append(job.results())
    job.close()
    assert outs[0] == outs[1] == outs[2] == run(ctx, probs)[0]
    modq(probs, outs[0], 733)

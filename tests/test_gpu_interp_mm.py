"""GPU: the interpolation on the matrix cores (the columns of all problems that
share a prime as two products with the triangular factors of the Vandermonde
system) gives the same results, bit for bit, as the vector path and the oracle:
single problems, both projections of a system (two columns per prime), a batch
of problems of different degree bounds sharing primes, bad points (the gapped
slots' fix-up after the products), multi-limb inputs, plain runs of the same
layout, and the autotuner's candidate."""

import pytest

import oracle
import workloads
from _golden import check_full, load
from workloads import dense_total, rng_for, small_random

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    import paper_1010_1386_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(rsl):
    c = rsl.Context(device=0, workspace_bytes=1 << 30)
    yield c
    c.close()


def test_single_problems_match_vector_path_and_oracle(rsl, ctx):
    rng = rng_for(740, 0)
    for k in range(8):
        F = dense_total(rng, int(rng.integers(2, 9)), int(rng.integers(8, 64)))
        G = dense_total(rng, int(rng.integers(2, 9)), int(rng.integers(8, 64)))
        for v in "yx":
            want = ctx.res(F, G, v)
            assert ctx.res(F, G, v, interp_mm=True) == want, (k, v)
            if k < 3:
                assert want == oracle.res(F, G, v)


def test_pair_golden_digests(rsl, ctx):
    """The dense degree-24 pair, both projections in one call (two columns per prime)."""
    gold = load(2)
    f, g = workloads.config2()
    Ry, Rx = ctx.res_xy(f, g, interp_mm=True)
    check_full(Ry, gold["cfg2_y"])
    check_full(Rx, gold["cfg2_x"])


def test_bad_points_and_multi_limb(rsl, ctx):
    rng = rng_for(741, 0)
    F = small_random(rng, 4, 5, 40)
    F[4] = [0, -2, 1, 0, 0, 0]  # lc_y = x (x - 2): points 0 and 2 are bad for every prime
    G = small_random(rng, 3, 4, 40)
    want = oracle.res(F, G, "y")
    assert ctx.res(F, G, "y", interp_mm=True) == want
    assert ctx.res(F, G, "y", interp_mm=True, points="formal") == ctx.res(F, G, "y", points="formal")
    big = [[int(v) << 180 for v in row] for row in small_random(rng, 5, 5, 30)]
    G2 = small_random(rng, 4, 4, 30)
    assert ctx.res(big, G2, "y", interp_mm=True) == ctx.res(big, G2, "y")


def test_batch_sharing_primes(rsl, ctx):
    """Problems of different degree bounds (and a few with bad points) in one
    job: every prime's group has columns of different lengths."""
    rng = rng_for(742, 0)
    probs = []
    for k in range(40):
        F = dense_total(rng, int(rng.integers(2, 14)), int(rng.integers(8, 48)))
        G = dense_total(rng, int(rng.integers(2, 14)), int(rng.integers(8, 48)))
        if k % 7 == 3:
            F[-1] = [0, -3, 1]  # a non-constant leading coefficient: bad points
        probs.append((F, G, "yx"[k % 2]))
    base = ctx.job(probs)
    base.run("staged")
    want = base.results()
    base.close()
    job = ctx.job(probs, interp_mm=True)
    for mode in ("staged", "plain", "staged"):
        job.run(mode)
        assert job.results() == want, mode
    job.close()
    for k in (0, 3, 10):
        f, g, v = probs[k]
        assert want[k] == oracle.res(f, g, v)


def test_batch_of_512_subset_against_goldens(rsl, ctx):
    gold = load(4)
    pairs = workloads.config4()
    idx = [k for k in range(len(pairs)) if f"cfg4_{k}_y" in gold][:96]
    probs = [(pairs[k][0], pairs[k][1], "y") for k in idx]
    job = ctx.job(probs, interp_mm=True)
    job.run("staged")
    got = job.results()
    job.close()
    for k, R in zip(idx, got):
        check_full(R, gold[f"cfg4_{k}_y"])


def test_tuner_offers_the_matrix_core_interpolation(rsl, ctx):
    rng = rng_for(743, 0)
    probs = [(dense_total(rng, 8, 32), dense_total(rng, 8, 32), "y") for _ in range(16)]
    job = ctx.job(probs)
    job.run("staged")
    want = job.results()
    t = job.tune(reps=1)  # every candidate, this one included, must give the same bytes
    assert "interp_mm" in t
    job.run("auto")
    assert job.results() == want
    job.close()

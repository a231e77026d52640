"""GPU: the large-coefficient random curves of the paper's Table 3 (curves of
degree 9 and 15, multiplied by 2^k with the constant coefficient increased by
one): hundreds to thousands of primes per problem (CRT with up to eight prime
slots per lane, the wide CRT beyond 512 primes), multi-limb inputs, stored
oracle digests and modulo-q checks."""

import hashlib
import json
import os
import random

import pytest

import oracle
import workloads
from workloads import dense_total, rng_for, small_random, sparse_total

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rsl():
    import paper_1010_1386_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(rsl):
    c = rsl.Context(device=0, workspace_bytes=2 << 30)
    yield c
    c.close()


def digest(coeffs):
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


def modq(f, g, R, var, n, seed):
    rnd = random.Random(seed)
    for q in oracle.next_check_primes(n):
        t = rnd.randrange(q)
        assert oracle.peval(R, t) % q == oracle.res_at_point_mod(f, g, t, q, var), (q, t)


@pytest.fixture(scope="module")
def gold():
    with open(os.path.join(HERE, "golden", "cfg6.json")) as fh:
        return {r["name"]: r for r in json.load(fh)["records"]}


@pytest.mark.parametrize("deg,k,sparse", [(9, 128, False), (9, 512, False), (9, 512, True), (15, 128, False)])
def test_first_pair_matches_oracle_digest(rsl, ctx, gold, deg, k, sparse):
    f, g = workloads.table3_curves(deg, k, sparse)[0]
    R = ctx.res(f, g, "y")
    rec = gold[f"t3_{deg}_{k}_{'sparse' if sparse else 'dense'}_y"]
    assert len(R) - 1 == rec["degree"] and digest(R) == rec["sha256"]


@pytest.mark.parametrize("deg,k", [(9, 512), (15, 512)])
def test_all_pairs_batched_equals_plain_and_modq(rsl, ctx, deg, k):
    """All ten pairs of a set in one job: staged = plain, both variables, modulo-q
    checks; (15, 512) needs 507 primes (eight slots per lane in the CRT)."""
    pairs = workloads.table3_curves(deg, k)
    probs = [(f, g, "yx"[i % 2]) for i, (f, g) in enumerate(pairs)]
    assert max(rsl.query(f, g, v)["n_primes"] for f, g, v in probs) > 256
    got = ctx.batch(probs, mode="staged")
    assert got == ctx.batch(probs, mode="plain")
    for i in (0, 3, 7):
        f, g, v = probs[i]
        modq(f, g, got[i], v, 2, i)


def test_multi_limb_reduction_paths_agree(rsl, ctx):
    """Inputs of 5 limbs: the staged and plain schedules reduce them with staged
    limbs and eight primes per thread, the persistent schedule one chain per
    thread; all ten pairs give the same bits."""
    pairs = workloads.table3_curves(9, 128)
    probs = [(f, g, "yx"[i % 2]) for i, (f, g) in enumerate(pairs)]
    got = ctx.batch(probs, mode="staged")
    assert got == ctx.batch(probs, mode="batched") == ctx.batch(probs, mode="plain")


def test_long_limb_chains_match_oracle(rsl, ctx):
    """Small problems with coefficients of about 2200 bits (70 limbs: two limb
    chunks in the reduction) and of 100 bits, mixed: exact oracle results."""
    rng = rng_for(717, 0)
    probs = []
    for k in range(6):
        bits = 2200 if k % 2 == 0 else 100
        F = small_random(rng, int(rng.integers(1, 4)), int(rng.integers(0, 3)), bits)
        G = small_random(rng, int(rng.integers(1, 3)), int(rng.integers(0, 3)), bits)
        probs.append((F, G, "yx"[k % 2]))
    want = [oracle.res(f, g, v) for f, g, v in probs]
    for mode in ("staged", "plain"):
        assert ctx.batch(probs, mode=mode) == want, mode


def test_persistent_schedule_refuses_many_primes(rsl, ctx):
    f, g = workloads.table3_curves(9, 512)[0]
    with pytest.raises(rsl.RSLError) as ei:
        ctx.batch([(f, g, "y")], mode="batched")
    assert ei.value.code == rsl.RSL_EINVAL
    assert ctx.batch([(f, g, "y")], mode="auto") == ctx.batch([(f, g, "y")], mode="staged")


@pytest.mark.parametrize("extra", [520, 1100])
def test_wide_crt_small_problems_match_oracle(rsl, ctx, extra):
    """Primes beyond the bound (more than 512 in all) send small problems through
    the wide CRT: exact oracle results in both schedules, bad points included."""
    rng = rng_for(716, extra)
    probs = []
    for k in range(8):
        F = dense_total(rng, int(rng.integers(2, 7)), int(rng.integers(8, 64)))
        G = sparse_total(rng, int(rng.integers(3, 7)), int(rng.integers(8, 40)))
        probs.append((F, G, "yx"[k % 2]))
    F = small_random(rng, 3, 4, 20)
    F[3] = [0, -2, 1, 0, 0]  # lc_y = x (x - 2): points 0 and 2 are bad for every prime
    probs.append((F, small_random(rng, 2, 3, 20), "y"))
    want = [oracle.res(f, g, v) for f, g, v in probs]
    job = ctx.job(probs, extra_primes=extra)
    for mode in ("staged", "plain"):
        job.run(mode)
        assert job.results() == want, mode
    with pytest.raises(rsl.RSLError) as ei:
        job.run("batched")
    assert ei.value.code == rsl.RSL_EINVAL
    job.close()


def test_wide_crt_equals_slot_crt(rsl, ctx, gold):
    """The (9, 2^512) pair with 304 primes (slot CRT) and with 564 (wide CRT):
    the same bits, equal to the stored oracle digest."""
    f, g = workloads.table3_curves(9, 512)[0]
    rec = gold["t3_9_512_dense_y"]
    for extra in (0, 260):
        R = ctx.res(f, g, "y", extra_primes=extra)
        assert len(R) - 1 == rec["degree"] and digest(R) == rec["sha256"], extra


@pytest.mark.parametrize("deg", [9, 15])
def test_2048_bit_scale_all_pairs(rsl, ctx, deg):
    """Coefficients times 2^2048 (1196 and 1993 primes): all ten pairs staged =
    plain, both variables, modulo-q checks."""
    pairs = workloads.table3_curves(deg, 2048)
    probs = [(f, g, "yx"[i % 2]) for i, (f, g) in enumerate(pairs)]
    assert min(rsl.query(f, g, v)["n_primes"] for f, g, v in probs) > 512
    got = ctx.batch(probs, mode="staged")
    assert got == ctx.batch(probs, mode="plain")
    for i in (0, 5, 9):
        f, g, v = probs[i]
        modq(f, g, got[i], v, 2, 100 + i)


def test_beyond_4096_primes_is_refused(rsl, ctx):
    f, g = workloads.table3_curves(9, 8192)[0]
    with pytest.raises(rsl.RSLError) as ei:
        ctx.res(f, g, "y")
    assert ei.value.code == rsl.RSL_EINVAL


def test_joint_projections_share_the_reduction(rsl, ctx):
    """res_y and res_x of one system in one job: the y problem's reduction also
    fills the x problem's residue tiles for their common primes.  Equal to the
    separate calls in every schedule, with 5-limb (dense and sparse) and
    one-limb inputs, and with the x problem needing more or fewer primes."""
    rng = rng_for(720, 0)
    systems = [workloads.table3_curves(9, 128)[0], workloads.table3_curves(9, 128, sparse=True)[1],
               (dense_total(rng, 6, 20), dense_total(rng, 4, 30)),
               (small_random(rng, 2, 7, 40), small_random(rng, 5, 1, 12))]
    for F, G in systems:
        sep = [ctx.res(F, G, "y"), ctx.res(F, G, "x")]
        assert list(ctx.res_xy(F, G)) == sep
        for mode in ("staged", "plain", "batched"):
            assert ctx.batch([(F, G, "y"), (F, G, "x")], mode=mode) == sep, mode
    F, G = systems[3]
    assert rsl.query(F, G, "y")["n_primes"] != rsl.query(F, G, "x")["n_primes"]


def test_wide_contraction_matrix_cores_equal_valu(rsl, ctx, monkeypatch):
    """The wide CRT's contraction on the matrix cores (7-bit digit planes, int8
    MFMA, anti-diagonal int32 sums) and on the vector ALUs (16-bit half limbs)
    give the same bits, on the 2^2048 sets and on small problems pushed past
    512 primes."""
    monkeypatch.setenv("RSL_WIDE_VALU", "1")
    cv = rsl.Context(device=0, workspace_bytes=2 << 30)
    monkeypatch.delenv("RSL_WIDE_VALU")
    for deg in (9, 15):
        probs = [(f, g, "y") for f, g in workloads.table3_curves(deg, 2048)[:4]]
        assert ctx.batch(probs, mode="staged") == cv.batch(probs, mode="staged"), deg
    rng = rng_for(724, 0)
    small = [(dense_total(rng, 4, 30), dense_total(rng, 3, 30), "yx"[k % 2]) for k in range(4)]
    ja, jb = ctx.job(small, extra_primes=700), cv.job(small, extra_primes=700)
    for mode in ("staged", "plain"):
        ja.run(mode)
        jb.run(mode)
        assert ja.results() == jb.results() == [oracle.res(f, g, v) for f, g, v in small], mode
    ja.close()
    jb.close()
    cv.close()

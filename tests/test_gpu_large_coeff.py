"""GPU: the large-coefficient random curves of the paper's Table 3 (curves of
degree 9 and 15, multiplied by 2^k with the constant coefficient increased by
one): hundreds of primes per problem (CRT with up to eight prime slots per
lane), multi-limb inputs, stored oracle digests and modulo-q checks."""

import hashlib
import json
import os
import random

import pytest

import oracle
import workloads

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


def test_persistent_schedule_refuses_many_primes(rsl, ctx):
    f, g = workloads.table3_curves(9, 512)[0]
    with pytest.raises(rsl.RSLError) as ei:
        ctx.batch([(f, g, "y")], mode="batched")
    assert ei.value.code == rsl.RSL_EINVAL
    assert ctx.batch([(f, g, "y")], mode="auto") == ctx.batch([(f, g, "y")], mode="staged")


def test_beyond_512_primes_is_refused(rsl, ctx):
    f, g = workloads.table3_curves(9, 2048)[0]
    with pytest.raises(rsl.RSLError) as ei:
        ctx.res(f, g, "y")
    assert ei.value.code == rsl.RSL_EINVAL

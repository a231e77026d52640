"""GPU: the three execution modes (one pipeline per problem, one launch per stage,
one persistent launch with a device task queue) give the same bits, equal to the
oracle, on mixed batches (both variables, bad points, bad primes, zero inputs,
more than 64 primes)."""

import pytest

import oracle
from workloads import dense_total, rng_for, small_random, sparse_total

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1010_1386_amd as rsl
    c = rsl.Context(device=0, workspace_bytes=1 << 30)
    yield c
    c.close()


def mixed_batch(n, seed):
    rng = rng_for(710, seed)
    probs = []
    for k in range(n):
        kind = k % 5
        if kind == 0:
            F = dense_total(rng, int(rng.integers(2, 8)), int(rng.integers(8, 64)))
            G = dense_total(rng, int(rng.integers(2, 8)), int(rng.integers(8, 64)))
        elif kind == 1:
            F = sparse_total(rng, int(rng.integers(3, 8)), int(rng.integers(8, 40)))
            G = sparse_total(rng, int(rng.integers(3, 8)), int(rng.integers(8, 40)))
        elif kind == 2:  # leading y-coefficient x (x - 2): bad points 0 and 2 for every prime
            F = small_random(rng, 3, 4, 20)
            F[3] = [0, -2, 1, 0, 0]
            G = small_random(rng, 2, 3, 20)
        elif kind == 3:
            F = small_random(rng, int(rng.integers(0, 4)), int(rng.integers(0, 4)), 12, 0.5)
            G = small_random(rng, int(rng.integers(0, 4)), int(rng.integers(0, 4)), 12, 0.5)
        else:
            F = dense_total(rng, 4, 10)
            G = [[0]]  # zero polynomial
        probs.append((F, G, "yx"[k % 2]))
    return probs


@pytest.mark.parametrize("seed", range(3))
def test_modes_agree_with_oracle(ctx, seed):
    probs = mixed_batch(25, seed)
    want = [oracle.res(f, g, v) for f, g, v in probs]
    for mode in ("batched", "staged", "plain"):
        assert ctx.batch(probs, mode=mode) == want, mode


def test_persistent_launch_with_many_primes_and_large_degree(ctx):
    """More than 64 primes per problem (two prime slots per lane in CRT) and D > 256."""
    rng = rng_for(711, 0)
    F = dense_total(rng, 10, 64)
    G = dense_total(rng, 10, 64)
    H = dense_total(rng, 6, 120)
    probs = [(F, G, "y"), (G, F, "x"), (H, F, "y")]
    got = ctx.batch(probs, mode="batched")
    assert got == ctx.batch(probs, mode="staged")
    for (f, g, v), r in zip(probs, got):
        assert r == oracle.res(f, g, v)


def test_resident_job_all_modes(ctx):
    probs = mixed_batch(30, 7)
    job = ctx.job(probs)
    outs = []
    for mode in ("batched", "staged", "plain", "batched"):
        job.run(mode)
        outs.append(job.results())
    job.close()
    assert all(o == outs[0] for o in outs)
    assert outs[0] == [oracle.res(f, g, v) for f, g, v in probs]


def test_autotuner_keeps_bits_and_caches_choice(ctx, tmp_path):
    probs = mixed_batch(20, 11)
    want = [oracle.res(f, g, v) for f, g, v in probs]
    job = ctx.job(probs)
    best = job.tune(reps=2)
    assert best["mode"] in ("staged", "batched") and best["candidates"] >= 2
    assert 0 < best["ms"] <= best["ms_worst"]
    job.run("auto")
    assert job.results() == want
    job.close()
    # the choice is cached for the shape bucket: rsl_batch in auto mode uses it
    assert ctx.batch(probs, mode="auto") == want
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    lines = path.read_text().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    key, mode, target, gm, evk, cw, sch, imm, ms = lines[0].split()
    assert int(mode) in (1, 2) and int(target) >= 64 and int(gm) >= 1 and int(evk) in (1, 2, 4)
    assert int(sch) in (0, 1) and int(imm) in (0, 1)
    import paper_1010_1386_amd as rsl
    c2 = rsl.Context(device=0, workspace_bytes=256 << 20)
    c2.tune_load(str(path))
    j2 = c2.job(probs)
    j2.run("auto")
    assert j2.results() == want
    j2.close()
    bad = tmp_path / "bad.txt"
    bad.write_text(key + " 7 4096 1 1 0 0 0 1.0\n")
    with pytest.raises(rsl.RSLError):
        c2.tune_load(str(bad))
    bad.write_text(key + " 1 4096 1 1 0 0 1 1.0\n")  # matrix-core interpolation: staged schedule only
    with pytest.raises(rsl.RSLError):
        c2.tune_load(str(bad))
    c2.close()


def test_queue_wait_bound_ends_the_launch(monkeypatch):
    """A zero wait bound (set from the host) makes the first idle wave give up: the
    persistent launch ends, the run reports a device error, and the context stays
    usable for the other modes."""
    import paper_1010_1386_amd as rsl
    monkeypatch.setenv("RSL_QUEUE_WAIT_MS", "0")
    c = rsl.Context(device=0, workspace_bytes=256 << 20)
    monkeypatch.delenv("RSL_QUEUE_WAIT_MS")
    probs = mixed_batch(10, 12)
    with pytest.raises(rsl.RSLError) as ei:
        c.batch(probs, mode="batched")
    assert ei.value.code == rsl.RSL_EDEVICE
    assert c.batch(probs, mode="staged") == [oracle.res(f, g, v) for f, g, v in probs]
    c.close()


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_eval_lanes_per_pair(ctx, lanes):
    """Evaluation with 1, 2 or 4 lanes per (prime, point) pair gives the same bits in
    every schedule: oracle on the small mixed problems, agreement across lane counts
    and modulo-q checks on problems of degree 16..30 (where 4 lanes apply)."""
    small = mixed_batch(15, 20)
    rng = rng_for(712, 0)
    big = [(dense_total(rng, d, b), dense_total(rng, d - 1, b), "yx"[i % 2])
           for i, (d, b) in enumerate([(16, 12), (22, 30), (30, 8)])]
    # a bad point for every prime at degree 20: leading y-coefficient x (x - 5)
    F = dense_total(rng, 20, 10)
    F[20] = [0, -5, 1]
    big.append((F, dense_total(rng, 18, 10), "y"))
    probs = small + big
    job = ctx.job(probs, eval_lanes=lanes)
    got = {}
    for mode in ("staged", "batched", "plain"):
        job.run(mode)
        got[mode] = job.results()
    job.close()
    assert got["staged"] == got["batched"] == got["plain"]
    res = got["staged"]
    assert res[:len(small)] == [oracle.res(f, g, v) for f, g, v in small]
    ref = ctx.job(probs, eval_lanes=1)
    ref.run("staged")
    assert ref.results() == res
    ref.close()
    rnd = __import__("random").Random(lanes)
    qs = oracle.next_check_primes(2)
    for (f, g, v), R in zip(big, res[len(small):]):
        for q in qs:
            t = rnd.randrange(q)
            assert oracle.peval(R, t) % q == oracle.res_at_point_mod(f, g, t, q, v)


@pytest.mark.parametrize("mode", ["staged", "batched", "plain"])
def test_graph_replays_match_eager(ctx, mode):
    """Captured runs replayed several times, with other eager work and
    synchronisations in between, give the eager bits every time."""
    probs = mixed_batch(20, 13)
    job = ctx.job(probs)
    job.run(mode)
    eager = job.results()
    assert eager == [oracle.res(f, g, v) for f, g, v in probs]
    other = ctx.job(mixed_batch(6, 14))
    for rep in range(4):
        job.run(mode, graph=True)
        assert job.results() == eager, rep
        other.run("staged")  # unrelated eager work on the same stream
        other.results()
        job.run(mode, graph=True)
        job.run(mode, graph=True)
        assert job.results() == eager, rep
    other.close()
    job.close()


def test_register_form_matches_lds_columns(ctx):
    """Pairs kept in registers (degrees <= 32 differing by at most one) give the same
    bits as the LDS-column code, including planted bad points, equal and adjacent
    degrees in both orders, and the oracle on the small ones."""
    rng = rng_for(713, 0)
    probs = []
    for k, (d1, d2) in enumerate([(3, 3), (5, 4), (4, 5), (8, 8), (12, 11), (16, 16), (23, 24), (31, 30), (32, 32)]):
        f = dense_total(rng, d1, 16 if d1 > 8 else 40)
        g = dense_total(rng, d2, 16 if d2 > 8 else 40)
        probs.append((f, g, "yx"[k % 2]))
    F = dense_total(rng, 10, 12)
    F[10] = [0, -3, 1]  # lc_y = x (x - 3): bad points 0 and 3 for every prime
    probs.append((F, dense_total(rng, 10, 12), "y"))
    a = ctx.job(probs)
    b = ctx.job(probs, eval_regs=False)
    for mode in ("staged", "plain"):
        a.run(mode)
        b.run(mode)
        ra, rb = a.results(), b.results()
        assert ra == rb, mode
    a.close()
    b.close()
    for (f, g, v), r in zip(probs[:4], ra[:4]):
        assert r == oracle.res(f, g, v)


def test_crt_direct_form_equals_garner(ctx, monkeypatch):
    """The direct CRT (quotient from fixed-point parts) and Garner's digits give the
    same bits, on mixed problems including more than 64 primes."""
    import paper_1010_1386_amd as rsl
    monkeypatch.setenv("RSL_CRT_GARNER", "1")
    cg = rsl.Context(device=0, workspace_bytes=256 << 20)
    monkeypatch.delenv("RSL_CRT_GARNER")
    rng = rng_for(714, 0)
    probs = mixed_batch(12, 15) + [(dense_total(rng, 10, 64), dense_total(rng, 10, 64), "y")]
    for mode in ("staged", "batched"):
        assert cg.batch(probs, mode=mode) == ctx.batch(probs, mode=mode), mode
    cg.close()


def test_both_projections_in_one_call(ctx):
    """res_xy gives R^(y) and R^(x) of one system, equal to the separate calls
    and to the oracle."""
    rng = rng_for(715, 0)
    for k in range(4):
        f = dense_total(rng, 3 + k, 20)
        g = sparse_total(rng, 4 + k, 16) if k % 2 else dense_total(rng, 2 + k, 30)
        ry, rx = ctx.res_xy(f, g)
        assert ry == ctx.res(f, g, "y") and rx == ctx.res(f, g, "x")
        assert ry == oracle.res(f, g, "y") and rx == oracle.res(f, g, "x")


def test_schur_evaluation_matches_remainder_sequence(ctx):
    """The Schur evaluation (generators of the Sylvester matrix, one wave per pair)
    gives the bits of the remainder sequence: mixed problems (zero inputs, bad
    points, constant degrees), degrees up to 24 + 24, a pair whose leading minor
    vanishes at every point (every point takes the fallback), formal points,
    extra points and a shifted origin; the oracle on the small problems."""
    import paper_1010_1386_amd as rsl
    rng = rng_for(719, 0)
    small = mixed_batch(15, 21)
    a = dense_total(rng, 3, 8)[0]
    h, c, k = dense_total(rng, 2, 8)[0], dense_total(rng, 2, 8)[0], dense_total(rng, 1, 8)[0]
    a = a or [1]
    # f = a y^3 + 2a y^2 + h y + c, g = k (3 y + 6): a 6k - 2a 3k = 0 at every x
    F = [c, h, [2 * v for v in a], a]
    G = [[6 * v for v in k], [3 * v for v in k]]
    small.append((F, G, "y"))
    big = [(dense_total(rng, 24, 32), dense_total(rng, 24, 32), "y"),
           (dense_total(rng, 12, 16), sparse_total(rng, 10, 16), "x")]
    probs = small + big
    want = [oracle.res(f, g, v) for f, g, v in small]
    for opts in ({}, {"points": "formal"}, {"extra_points": 3}, {"point_origin": 1000}):
        js = ctx.job(probs, eval_schur=True, **opts)
        jr = ctx.job(probs, **opts)
        for mode in ("staged", "plain"):
            js.run(mode)
            jr.run(mode)
            got = js.results()
            assert got == jr.results(), (opts, mode)
            assert got[:len(small)] == want, (opts, mode)
        with pytest.raises(rsl.RSLError) as ei:
            js.run("batched")
        assert ei.value.code == rsl.RSL_EINVAL
        js.close()
        jr.close()


def test_context_close_closes_its_jobs_first():
    """A context closed while jobs on it are still open closes them first (their
    destruction waits on the context's stream), so nothing later touches the
    destroyed context; closing them again is a no-op."""
    import paper_1010_1386_amd as rsl
    c = rsl.Context(device=0, workspace_bytes=64 << 20)
    probs = mixed_batch(4, 3)
    jobs = [c.job(probs), c.job(probs, eval_lanes=1)]
    for j in jobs:
        j.run("staged")
    want = [oracle.res(f, g, v) for f, g, v in probs]
    assert jobs[0].results() == jobs[1].results() == want
    c.close()
    assert all(j.h is None for j in jobs)
    for j in jobs:
        j.close()
    del jobs


def test_tune_starts_from_the_jobs_own_layout(tmp_path):
    """A job laid out with a cached choice whose footprint is small (sums taken
    whole, matrix-core interpolation) and bound to exactly that size: the
    default layouts do not fit it, the tuner still times the job's own layout
    (it fits by construction) and the results stay exact."""
    import paper_1010_1386_amd as rsl
    rng = rng_for(760, 0)
    probs = [(dense_total(rng, 16, 40), dense_total(rng, 15, 40), "y") for _ in range(8)]
    ctx = rsl.Context(device=0, workspace_bytes=256 << 20)
    job = ctx.job(probs)
    job.run("staged")
    want = job.results()
    job.tune(reps=1)
    job.close()
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    key = path.read_text().split()[0]
    path.write_text(key + " 2 4096 1 1 1 0 1 1.0\n")
    c2 = rsl.Context(device=0, workspace_bytes=256 << 20)
    c2.tune_load(str(path))
    j2 = c2.job(probs, headroom=0.0)
    t = j2.tune(reps=1)
    assert t["candidates"] >= 1
    j2.run("auto")
    assert j2.results() == want
    j2.close()
    c2.close()
    ctx.close()


def test_stage_profile_times_only_the_stages_that_launch(ctx):
    """Per-stage device times: a stage that launches nothing for a job reads
    zero (its boundary markers go to the stage before), the others are timed."""
    rng = rng_for(733, 0)
    F, G = dense_total(rng, 6, 20), dense_total(rng, 5, 20)
    H = small_random(rng, 3, 4, 20)
    H[3] = [0, -2, 1, 0, 0]  # leading coefficient x (x - 2): the points start at x = 1
    K = small_random(rng, 2, 3, 20)
    for probs, newton in (([(F, G, "y")], False), ([(H, K, "y")], True)):
        job = ctx.job(probs)
        job.run("staged")
        want = job.results()
        ctx.profile_enable(True)
        for _ in range(3):
            job.run("staged")
        stages, runs = ctx.profile_take()
        ctx.profile_enable(False)
        assert job.results() == want
        assert runs == 3
        for k in ("reduce", "eval_ures", "interp_conv", "interp_stir", "crt"):
            assert stages[k] > 0.0, (k, stages)
        assert (stages["interp_newton"] > 0.0) == newton, stages
        job.close()

"""GPU: every device byte the library touches is the caller's -- the constant
tables live in a caller-owned region (or the top of the workspace), resident
jobs run in caller-owned buffers, and a server owns its context's workspace."""

import pytest

from workloads import dense_total, rng_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    import paper_1010_1386_amd as m
    return m


def _pair(seed, d=12, bits=40):
    rng = rng_for(731, seed)
    return dense_total(rng, d, bits), dense_total(rng, d, bits)


def test_table_region_sized_by_query(rsl):
    f, g = _pair(30, d=14, bits=200)  # more than 64 primes: a larger table than small problems
    q = rsl.query(f, g, "y")
    small = dense_total(rng_for(731, 9), 3, 8), dense_total(rng_for(731, 10), 3, 8)
    assert 0 < rsl.query(*small, "y")["table_bytes"] < q["table_bytes"] - 4096
    ref = rsl.Context(device=0, workspace_bytes=64 << 20)
    want = ref.res(f, g, "y")
    ref.close()
    # a region of exactly the reported size is enough
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20, table_bytes=q["table_bytes"])
    assert ctx.res(f, g, "y") == want
    ctx.close()
    # one smaller is refused, with the sizes in the message, and the context stays usable
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20, table_bytes=q["table_bytes"] - 4096)
    with pytest.raises(rsl.RSLError) as ei:
        ctx.res(f, g, "y")
    assert ei.value.code == rsl.RSL_ENOMEM and "table region" in str(ei.value)
    assert ctx.res(*small, "y") == rsl.Context(device=0, workspace_bytes=16 << 20).res(*small, "y")
    ctx.close()


def test_tables_at_the_top_of_the_workspace(rsl):
    f, g = _pair(31, d=14, bits=200)
    ref = rsl.Context(device=0, workspace_bytes=64 << 20)
    want = [ref.res(f, g, v) for v in "yx"]
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20, table_bytes=8 << 20, tables_in_workspace=True)
    # growth in place: first a small problem, then one that needs more primes and rows
    small = dense_total(rng_for(731, 2), 3, 8), dense_total(rng_for(731, 3), 3, 8)
    assert ctx.res(*small, "y") == ref.res(*small, "y")
    assert [ctx.res(f, g, v) for v in "yx"] == want
    assert ctx.batch([(f, g, "y"), (f, g, "x")]) == want
    ctx.close()
    ref.close()


def test_job_in_caller_memory(rsl):
    probs = [(*_pair(4 + k), "yx"[k % 2]) for k in range(6)]
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20)
    want = ctx.batch(probs)
    job = rsl.Job(ctx, probs)
    need = job.info()["device_bytes"]
    assert job.mem.numel() >= need
    job.run("staged")
    assert job.results() == want
    # too little memory: refused, and the job keeps needing a successful bind
    with pytest.raises(rsl.RSLError) as ei:
        job.bind(need - 256)
    assert ei.value.code == rsl.RSL_ENOMEM
    job.bind(need)  # exactly the layout's size
    job.run("staged")
    assert job.results() == want
    t = job.tune(reps=1)  # candidates that do not fit the bound bytes are skipped
    assert t["candidates"] >= 1
    job.run("auto")
    assert job.results() == want
    job.close()
    ctx.close()


def test_server_owns_the_workspace(rsl):
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20)
    f, g = _pair(20, d=6, bits=16)
    want = ctx.res(f, g, "y")
    srv = rsl.Server(ctx, budget_bytes=32 << 20, max_slots=8)
    with pytest.raises(rsl.RSLError) as ei:
        ctx.res(f, g, "y")  # would overwrite the server's arena
    assert ei.value.code == rsl.RSL_EINVAL and "server" in str(ei.value)
    with pytest.raises(rsl.RSLError):
        rsl.Server(ctx, budget_bytes=16 << 20, max_slots=8)  # one server per context
    assert srv.wait(srv.submit(f, g, "y")) == want
    # the allocation-free entry point does not use the workspace
    assert ctx.res_static(f, g, "y") == want
    srv.close()
    assert ctx.res(f, g, "y") == want  # the workspace is the context's again
    ctx.close()


def test_server_refuses_requests_beyond_the_table_region(rsl):
    f, g = _pair(30, d=14, bits=200)
    q = rsl.query(f, g, "y")
    small = dense_total(rng_for(731, 31), 3, 8), dense_total(rng_for(731, 32), 3, 8)
    qs = rsl.query(*small, "y")
    assert qs["table_bytes"] < q["table_bytes"]
    ctx = rsl.Context(device=0, workspace_bytes=64 << 20, table_bytes=qs["table_bytes"])
    srv = rsl.Server(ctx, budget_bytes=32 << 20, max_slots=8)
    with pytest.raises(rsl.RSLError) as ei:
        srv.submit(f, g, "y")
    assert ei.value.code == rsl.RSL_ENOMEM
    got = srv.wait(srv.submit(*small, "y"))
    srv.close()
    assert got == ctx.res(*small, "y")
    ctx.close()

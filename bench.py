"""Throughput of the modular resultant path on one MI355X; prints one JSON line.

A step is one batch of 512 independent resultant problems (the batched
workload: pairs f, g with total degrees uniform in 6..32, signed 8..64-bit
coefficients, half dense and half with 30% of the coefficients zeroed;
res_y of each), computed by one ``rsl_batch`` call from host limbs to host
limbs: planning (degree and Hadamard bounds, primes, points), upload, the
device pipeline (reduction mod p, evaluation and univariate resultants over
Z_p, interpolation, CRT), download and decoding all sit inside the timed
region.  ``value`` is bivariate resultants per second of the autotuned batched
schedule; the plain path (one pipeline per problem) is timed the same way.
The results of the timed calls are checked against the oracle's stored values
(digests of every problem with Sylvester order <= 32, two checks modulo 61-bit
primes of every problem).  Device-only rates of a resident job, the per-stage
split and the dense degree-24 pair with steps in flight are reported beside.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bivariate resultants/s + mod-p univariate resultants/s, batched vs plain, bit-exact"
# Montgomery multiply on gfx950: 3 full-rate 32-bit multiplies (16 lanes/clk/SIMD) and
# 2 double-rate adds (32 lanes/clk/SIMD) per lane -> 0.25 SIMD-clocks per lane-mulmod.
CUS, SIMDS, CLOCK_GHZ = 256, 4, 2.4
PEAK_TMULMOD = CUS * SIMDS * CLOCK_GHZ * 4 / 1000.0  # 9.83 T mulmod/s
PEAK_HBM_GBS = 8000.0


def digest(coeffs):
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_cores():
    """Cores this process may run on (the box's share), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _oracle_res(args):
    """Oracle work unit: the exact resultant by Bareiss elimination over Z[x]."""
    import oracle
    f, g, var = args
    t0 = time.perf_counter()
    R = oracle.res(f, g, var)
    return len(R), time.perf_counter() - t0


def cpu_baseline(problems, r_max=24):
    """The oracle (Bareiss over Z[x], oracle.res) on a bounded sample of the batch: every
    problem whose Sylvester matrix has order at most r_max, over the host's cores."""
    from concurrent.futures import ProcessPoolExecutor
    sample = []
    for f, g, var in problems:
        ff = f if var == "y" else [list(c) for c in zip(*f)]
        gg = g if var == "y" else [list(c) for c in zip(*g)]
        r = (max((j for j, row in enumerate(ff) if any(row)), default=0)
             + max((j for j, row in enumerate(gg) if any(row)), default=0))
        if r <= r_max:
            sample.append((f, g, var))
    cores = host_cores()
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        done = list(ex.map(_oracle_res, sample))
    dt = time.perf_counter() - t0
    cpu_s = sum(t for _, t in done)
    return {
        "value": len(done) / dt,
        "unit": "bivariate resultants/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"the {len(done)} problems of the batch whose Sylvester matrix has order <= {r_max} "
                   f"(of {len(problems)}), each by oracle.res (Bareiss over Z[x]), {dt:.1f} s wall on {cores} "
                   f"processes of '{cpu_model()}' ({cpu_s:.1f} s of CPU, {cpu_s / max(len(done), 1):.2f} s "
                   f"per problem); the larger problems of the batch (order up to 64) cost far more each, so "
                   f"this rate bounds the oracle's rate on the whole batch from above"),
        "cpu_seconds": cpu_s,
    }


def serve_bench(n):
    """Serving workload: requests with degrees U{8..48}, bits U{8..48}, res_y or res_x.

    Saturated throughput T of the server (all requests submitted at once), then
    Poisson arrivals at 0.5 T, 0.8 T and 1.0 T with p50/p99 latency, against the
    serial plain path (one rsl_res call after the other).  Both sides go from
    the callers' prepared inputs to result limbs (the conversion to Python ints
    is left out of both), and every server result is compared with the plain
    path's, limb for limb."""
    import ctypes
    import threading
    import numpy as np
    import paper_1010_1386_amd as rsl
    import workloads

    reqs = workloads.config5(n)
    polys = [(rsl.Poly(f), rsl.Poly(g), rsl._var_code(v)) for f, g, v in reqs]
    outs = []
    for f, g, v in polys:
        info = rsl.rsl_info()
        rsl._lib.rsl_query(ctypes.byref(f.c), ctypes.byref(g.c), v, ctypes.byref(info))
        outs.append(rsl._Result(max(info.D, 0), info.out_limbs))
    ctx = rsl.Context(0, workspace_bytes=1 << 30)
    opts = rsl.rsl_opts()

    def plain_pass():
        lat = []
        t0 = time.perf_counter()
        for (f, g, v), o in zip(polys, outs):
            t1 = time.perf_counter()
            rc = rsl._lib.rsl_res(ctx.h, ctypes.byref(f.c), ctypes.byref(g.c), v, ctypes.byref(opts),
                                  ctypes.byref(o.c))
            if rc:
                raise rsl.RSLError(rc, "rsl_res")
            lat.append((time.perf_counter() - t1) * 1e3)
        return n / (time.perf_counter() - t0), lat

    plain_pass()  # warms the constant tables for the largest shapes
    plain_rate, lat_plain = plain_pass()
    want = [o.raw() for o in outs]

    def run(rate, budget=64 << 20):
        srv = rsl.Server(ctx, budget_bytes=budget, max_slots=256, max_queue=1 << 20)
        arrivals = None if rate is None else workloads.poisson_arrivals(n, rate)
        tickets = [None] * n
        t_start = time.perf_counter()

        def producer():
            for k, (f, g, v) in enumerate(polys):
                if arrivals is not None:
                    dt = arrivals[k] - (time.perf_counter() - t_start)
                    if dt > 0:
                        time.sleep(dt)
                tickets[k] = srv.submit(f, g, v)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        got = [srv.wait(t, raw=True) for t in tickets]
        wall = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        if [o.raw() for o in got] != want:
            print("bench: a served result differs from the plain path", file=sys.stderr)
            sys.exit(1)
        return {"offered_rps": rate, "completed": st["completed"], "resultants_per_s": n / wall,
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                "device_iterations": st["launches"], "max_batch": st["max_batch"],
                "admitted_bytes_peak": st["admitted_bytes_peak"], "budget_bytes": budget,
                "verified_vs_plain": True}

    sat = run(None)
    T = sat["resultants_per_s"]
    loads = [run(f * T) for f in (0.5, 0.8, 1.0)]
    ctx.close()
    return {"metric": "serving: resultants/s and latency, continuous batching vs serial plain path",
            "requests": n, "workload": "degrees U{8..48}, signed U{8..48}-bit, dense, res_y/res_x w.p. 1/2",
            "boundary": "prepared inputs to result limbs on both sides",
            "saturated": sat, "poisson": loads, "saturated_vs_serial": T / plain_rate,
            "serial_plain": {"resultants_per_s": plain_rate, "p50_ms": float(np.percentile(lat_plain, 50)),
                             "p99_ms": float(np.percentile(lat_plain, 99))}}


def batch_bench(steps, warmup):
    """512 independent pairs (total degrees 6..32, 8..64-bit coefficients, half
    30%-sparse), res_y of all: the autotuned batched schedule against one
    pipeline per problem, both on resident inputs, results compared bit for bit."""
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    pairs = workloads.config4()
    probs = [(f, g, "y") for f, g in pairs]
    ctx = rsl.Context(0, workspace_bytes=1 << 30)
    job = ctx.job(probs)
    tune = job.tune(reps=2)
    job.run("auto")
    got = job.results()
    job.run("plain")
    if job.results() != got:
        print("bench: batched and plain results differ", file=sys.stderr)
        sys.exit(1)
    steps = max(1, min(steps, 20))

    def timed(mode):
        for _ in range(max(1, warmup // 10)):
            job.run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            job.run(mode)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tb = timed("auto")
    tp = timed("plain")
    info = job.info()
    job.close()
    ctx.close()
    return {"workload": "batch of 512 pairs, total degrees 6..32, 8..64-bit coefficients, half 30% sparse; res_y",
            "problems": len(probs), "mod_p_pairs": info["pairs"], "steps": steps,
            "batched_resultants_per_s": len(probs) / tb, "batched_ms": tb * 1e3,
            "plain_resultants_per_s": len(probs) / tp, "plain_ms": tp * 1e3, "batched_vs_plain": tp / tb,
            "modp_univariate_resultants_per_s": info["pairs"] / tb, "tune": tune, "verified_batched_eq_plain": True}


def table3_bench(steps, warmup, only=None):
    """The large-coefficient random curves of the paper's Table 3: for each set
    (total degree 9 or 15, dense or 30% sparse, coefficients times 2^k for
    k = 128, 512) the 10 pairs' res_y in one job, autotuned schedule against one
    pipeline per problem, results compared bit for bit; k = 2048 needs more
    primes than the CRT covers and is reported as refused."""
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    ctx = rsl.Context(0, workspace_bytes=2 << 30)
    steps = max(1, min(steps, 20))
    rows = []
    for deg in (9, 15):
        for k in (128, 512, 2048):
            for sparse in (False, True):
                if only and f"{deg}:{k}" not in only:
                    continue
                probs = [(f, g, "y") for f, g in workloads.table3_curves(deg, k, sparse)]
                name = f"degree {deg}, 2^{k}, {'sparse' if sparse else 'dense'}"
                np_max = max(rsl.query(f, g, v)["n_primes"] for f, g, v in probs)
                try:
                    job = ctx.job(probs)
                except rsl.RSLError as e:
                    rows.append({"set": name, "primes": np_max, "refused": str(e)})
                    continue
                # sizes beyond the library's limits are reported per problem
                # when the results are read
                try:
                    job.run("staged")
                    job.results()
                except rsl.RSLError as e:
                    job.close()
                    rows.append({"set": name, "primes": np_max, "refused": str(e)})
                    continue
                tune = job.tune(reps=2)
                job.run("auto")
                got = job.results()
                job.run("plain")
                if job.results() != got:
                    print(f"bench: batched and plain results differ on {name}", file=sys.stderr)
                    sys.exit(1)

                def timed(mode):
                    for _ in range(max(1, warmup // 10)):
                        job.run(mode)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        job.run(mode)
                    torch.cuda.synchronize()
                    return (time.perf_counter() - t0) / steps

                tb, tp = timed("auto"), timed("plain")
                info = job.info()
                job.close()
                rows.append({"set": name, "primes": np_max, "degree_bound": max(len(r) - 1 for r in got),
                             "max_coeff_bits": max(max(abs(c).bit_length() for c in r) for r in got),
                             "batched_ms": tb * 1e3, "plain_ms": tp * 1e3,
                             "ms_per_resultant": tb * 1e3 / len(probs), "mod_p_pairs": info["pairs"],
                             "schedule": tune["mode"]})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    ctx.close()
    return {"workload": "large-coefficient random curves (Table 3): 10 pairs of 5 curves per set, res_y",
            "steps": steps, "sets": rows, "verified_batched_eq_plain": True}


def sqfree_bench(steps, with_cpu_baseline=True):
    """The square-free part of resultants by the modular gcd: R = res_y of the
    dense degree-24 pair (square-free: Euclid runs to a constant gcd), and
    R = res_y(f, f_y) with f = F (y^2 - h), which has a repeated factor.
    Each call is host to host (planning, prime selection, two device passes,
    Chinese remaindering, certificate checks)."""
    import paper_1010_1386_amd as rsl
    import workloads

    ctx = rsl.Context(0, workspace_bytes=1 << 30)
    f, g = workloads.config2()
    cases = [("R = res_y of the dense degree-24 pair", ctx.res(f, g, "y"))]
    rng = workloads.rng_for(722, 0)
    for d in (6, 8):
        F = workloads.dense_total(rng, d, 8)
        h = [int(v) for v in rng.integers(-9, 10, size=3)]
        h[-1] = h[-1] or 1
        fb = [[0] * len(F[0]) for _ in range(len(F) + 2)]
        for j, row in enumerate(F):  # F (y^2 - h): rows are y-powers
            for i, c in enumerate(row):
                fb[j + 2][i] += c
                for t, hc in enumerate(h):
                    if i + t >= len(fb[j]):
                        fb[j].extend([0] * (i + t + 1 - len(fb[j])))
                    fb[j][i + t] -= c * hc
        fy = [[(j + 1) * c for c in fb[j + 1]] for j in range(len(fb) - 1)]
        cases.append((f"R = res_y(f, f_y), f = F (y^2 - h), F dense of total degree {d}", ctx.res(fb, fy, "y")))
    rows = []
    steps = max(1, min(steps, 20))
    for name, R in cases:
        q, gg = ctx.sqfree_part(R)
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.sqfree_part(R)
        dt = (time.perf_counter() - t0) / steps
        fac = ctx.sqfree_factor(R)
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.sqfree_factor(R)
        dty = (time.perf_counter() - t0) / steps
        row = {"case": name, "deg_R": len(R) - 1, "max_coeff_bits": max(abs(c).bit_length() for c in R),
               "deg_gcd": len(gg) - 1, "deg_sqfree_part": len(q) - 1, "ms_per_call": dt * 1e3,
               "yun_factor_degrees": [len(r) - 1 for r in fac], "yun_ms_per_call": dty * 1e3}
        if with_cpu_baseline and len(R) <= 100:
            import oracle
            t0 = time.perf_counter()
            want = oracle.sqfree_part(R)
            row["cpu_baseline"] = {"kind": "oracle", "ms": (time.perf_counter() - t0) * 1e3, "cores": 1,
                                   "matches": oracle.zx_pp(q) == want}
            t0 = time.perf_counter()
            wfac = oracle.yun(R)
            row["cpu_baseline_yun"] = {"kind": "oracle", "ms": (time.perf_counter() - t0) * 1e3, "cores": 1,
                                       "matches": wfac == fac}
        rows.append(row)
    ctx.close()
    return {"workload": "square-free part of resultants (modular gcd of R and R')", "steps": steps, "cases": rows}


def pair_bench(a):
    """The dense total-degree-24 pair with uniform signed 32-bit coefficients: a step is
    res_y and res_x of the pair (57 primes x 577 points each) as one resident job, inputs
    on the device; several steps in flight on their own contexts.  Device-only rates."""
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    f, g = workloads.config2()
    problems = [(f, g, "y"), (f, g, "x")]
    ctx = rsl.Context(0, workspace_bytes=256 << 20)
    # contexts (stream + workspace) of the further steps in flight, made up front
    extra_ctx = [rsl.Context(0, workspace_bytes=256 << 20) for _ in range(max(a.inflight, 1) - 1)]
    job = ctx.job(problems, eval_schur=a.eval_schur, eval_lanes=a.eval_lanes)
    info = job.info()
    # schedule: the autotuner times every candidate layout (staged launches /
    # one persistent launch x interpolation chunking) and keeps the fastest
    if a.schedule == "auto":
        tune = job.tune(reps=max(3, a.pair_warmup // 4))
    else:
        tune = {"mode": a.schedule, "chunk_target": 4096, "grid_mult": 1, "lanes_per_pair": None,
                "candidates": 0, "ms": None, "ms_worst": None}
    mode = tune["mode"]
    info = job.info()  # the layout actually used
    tune["lanes_per_pair"] = info["eval_lanes"]

    # correctness gate: bit-exact against the oracle's stored digests
    job.run(mode)
    res = job.results()
    counts = ctx.counters()  # of that results call: pairs, bad pairs, bad primes
    gold_path = os.path.join(ROOT, "tests", "golden", "cfg2.json")
    verified = None
    if os.path.exists(gold_path):
        with open(gold_path) as fh:
            gold = {r["name"]: r["sha256"] for r in json.load(fh)["records"]}
        verified = digest(res[0]) == gold["cfg2_y"] and digest(res[1]) == gold["cfg2_x"]
        if not verified:
            print("bench: result differs from the oracle digest", file=sys.stderr)
            sys.exit(1)

    # steps in flight: further resident jobs of the same pair, each on a
    # context (stream and workspace) of its own, laid out with the tuned
    # choice; step s runs on job s mod N, so one step's latency-bound stages
    # overlap the next step's evaluation.  Every step is a whole pass.
    extra = []
    if extra_ctx:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            tpath = os.path.join(td, "tune.txt")
            ctx.tune_save(tpath)
            for c in extra_ctx:
                c.tune_load(tpath)
                j = c.job(problems, eval_schur=a.eval_schur, eval_lanes=a.eval_lanes)
                j.run(mode)
                if j.results() != res:
                    print("bench: a further resident job differs from the first", file=sys.stderr)
                    sys.exit(1)
                extra.append((c, j))
    all_jobs = [job] + [j for _, j in extra]
    # the steps in flight may also take the other register-form layout: one
    # lane per (prime, point) pair issues fewer instructions per pair (which
    # counts when steps overlap), a lane pair gives the shorter single launch
    # (which the autotuner times); both sets are timed and the faster kept
    inflight_sets = [(info["eval_lanes"], all_jobs)]
    if extra and mode == "staged" and info.get("eval_mfma", 0) > 0 and not a.eval_schur and not a.eval_lanes:
        alt = 1 if info["eval_lanes"] == 2 else 2
        alt_jobs = []
        for c in [ctx] + extra_ctx:
            j = c.job(problems, eval_lanes=alt)
            j.run(mode)
            if j.results() != res:
                print("bench: a resident job of the other layout differs from the first", file=sys.stderr)
                sys.exit(1)
            alt_jobs.append(j)
        inflight_sets.append((alt, alt_jobs))
    # the autotuner times one launch at a time; when it kept a layout other than
    # the default interpolation form (whole convolution sums, matrix-core
    # products, other chunking), the default layout is timed in flight too, on
    # contexts of its own (no cached choice), in each lane layout
    dctx = []
    if extra and mode == "staged" and not a.eval_schur and any(
            tune.get(k, d) != d for k, d in (("conv_whole", 0), ("interp_mm", 0), ("chunk_target", 4096))):
        dctx = [rsl.Context(0, workspace_bytes=256 << 20) for _ in all_jobs]
        for lanes in sorted({s[0] for s in inflight_sets}):
            djobs = []
            for c in dctx:
                j = c.job(problems, eval_lanes=lanes)
                j.run(mode)
                if j.results() != res:
                    print("bench: a resident job of the default layout differs from the first", file=sys.stderr)
                    sys.exit(1)
                djobs.append(j)
            inflight_sets.append((f"{lanes}, default interpolation layout", djobs))

    def timed(mode, steps, warmup, graph=False):
        for _ in range(warmup):
            job.run(mode, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            job.run(mode, graph=graph)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # launch path: eager launches or one captured graph per step (checked first)
    job.run(mode, graph=True)
    if job.results() != res:
        print("bench: graph replay differs from the eager run", file=sys.stderr)
        sys.exit(1)
    use_graph = timed(mode, a.plain_steps, 5, graph=True) < timed(mode, a.plain_steps, 5)

    def stage_profile(m, steps):
        """Per-stage device ms per step from HIP events on the library's stream
        (a persistent launch is one kernel: its whole duration is reported under
        the first stage)."""
        ctx.profile_enable(True)
        for _ in range(2):  # first pass creates the event sets, second is measured
            ctx.profile_take()
            for _ in range(steps):
                job.run(m)
        stages, runs = ctx.profile_take()
        ctx.profile_enable(False)
        return {k: v / max(runs, 1) for k, v in stages.items()}

    dt1 = timed(mode, a.pair_steps, a.pair_warmup, graph=use_graph)
    serial_value = 2 * a.pair_steps / dt1


    def timed_inflight(jobs, steps, warmup, graph):
        for s in range(warmup):
            jobs[s % len(jobs)].run(mode, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            jobs[s % len(jobs)].run(mode, graph=graph)
        t_issue = time.perf_counter() - t0  # host time to enqueue every step
        torch.cuda.synchronize()
        return time.perf_counter() - t0, t_issue

    inflight_lanes = None
    inflight_ms = {}
    if extra:
        best = None
        for lanes, jobs in inflight_sets:
            for j in jobs:
                j.run(mode, graph=True)
                if j.results() != res:
                    print("bench: graph replay differs from the eager run", file=sys.stderr)
                    sys.exit(1)
            for graph in (True, False):
                t, t_issue = timed_inflight(jobs, a.pair_steps, a.pair_warmup, graph)
                inflight_ms[f"lanes {lanes}, {'graph' if graph else 'eager'}"] = t / a.pair_steps * 1e3
                inflight_ms[f"lanes {lanes}, {'graph' if graph else 'eager'}, host enqueue"] = \
                    t_issue / a.pair_steps * 1e3
                if best is None or t < best[0]:
                    best = (t, graph, lanes)
        dt, use_graph, inflight_lanes = best
    else:
        dt = dt1
    ms_step = dt / a.pair_steps * 1e3
    value = 2 * a.pair_steps / dt
    stages = stage_profile(mode, a.pair_steps)
    other = "staged" if mode == "batched" else "batched"
    try:
        dto = timed(other, a.plain_steps, max(1, a.pair_warmup // 4))
    except rsl.RSLError:  # a layout the persistent schedule does not run (Schur evaluation)
        dto = None
    dtp = timed("plain", a.plain_steps, max(1, a.pair_warmup // 4))
    plain_value = 2 * a.plain_steps / dtp
    schedules = {mode: dt1 / a.pair_steps * 1e3, other: None if dto is None else dto / a.plain_steps * 1e3,
                 "plain": dtp / a.plain_steps * 1e3}
    if extra:
        schedules[f"{mode}, {len(all_jobs)} steps in flight"] = ms_step
    if mode == "batched":
        # the staged launches give the per-stage split of the same work
        staged_split = stage_profile("staged", a.plain_steps)
    else:
        staged_split = stages

    # host-to-host rate through the synchronous C-ABI call, as the batch
    # headline measures it: the caller's prepared inputs (limbs) to result
    # limbs -- planning, layout, copies, kernels and decoding inside the timed
    # region, the conversions from and to Python ints outside; results checked
    import ctypes
    pf, pg = rsl.Poly(f), rsl.Poly(g)
    outs, want = {}, {}
    for var in "yx":
        q = rsl.query(f, g, var)
        outs[var] = rsl._Result(max(q["D"], 0), q["out_limbs"])
        want[var] = ctx.res(f, g, var)
    copts = rsl.rsl_opts()

    def h2h_call(var):
        rc = rsl._lib.rsl_res(ctx.h, ctypes.byref(pf.c), ctypes.byref(pg.c), rsl._var_code(var), ctypes.byref(copts),
                              ctypes.byref(outs[var].c))
        if rc:
            raise rsl.RSLError(rc, "rsl_res")

    for var in "yx":
        h2h_call(var)
    n_h2h = 40
    t0 = time.perf_counter()
    for i in range(n_h2h):
        h2h_call("yx"[i % 2])
    h2h = n_h2h / (time.perf_counter() - t0)
    for var in "yx":
        if outs[var].value() != want[var]:
            print("bench: host-to-host result differs", file=sys.stderr)
            sys.exit(1)

    pairs = info["pairs"]
    mulmods = info["mulmods"]
    if mode == "batched":
        # one kernel runs every stage: price the evaluation + resultant work
        # against the whole launch
        kernel, launch_ms = "persistent (all stages)", sum(stages.values())
    else:
        kernel, launch_ms = "eval_ures", stages["eval_ures"]
    ures_ms = staged_split["eval_ures"]
    dominant = max(staged_split, key=staged_split.get)
    # HBM bytes per launch of the dominant kernel, from the committed counter
    # summary of the same kernel sources and layout (None when either changed)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_eval_ures_cfg2_pair.json")
    if mode != "batched" and os.path.exists(tpath):
        from paper_1010_1386_amd.traffic import traffic_bytes
        with open(tpath) as fh:
            trec = json.load(fh)
        if trec.get("lanes_per_pair") == tune.get("lanes_per_pair"):
            traffic = traffic_bytes(trec)
    # VALU instructions per launch of the same kernel (committed SQ counter
    # summary, same validity rule): lane operations issued per second against
    # the chip's VALU issue peak
    valu = None
    ipath = os.path.join(ROOT, "profiles", "insts_eval_ures_cfg2_pair.json")
    if mode != "batched" and os.path.exists(ipath):
        from paper_1010_1386_amd.traffic import valu_issue
        with open(ipath) as fh:
            irec = json.load(fh)
        if irec.get("lanes_per_pair") == tune.get("lanes_per_pair"):
            vi = valu_issue(irec, launch_ms * 1e-3)
            if vi is not None:
                valu = {"lane_ops_per_launch": vi[0], "frac_of_issue_peak": vi[1],
                        "mfma_insts_per_launch": irec["mfma_insts"]}
    roofline = {
        "bound": "alu",
        "kernel": kernel,
        "achieved": mulmods / (launch_ms * 1e-3) / 1e12,
        "peak": PEAK_TMULMOD,
        "unit": "Tmulmod/s",
        "frac": mulmods / (launch_ms * 1e-3) / 1e12 / PEAK_TMULMOD,
        "traffic": traffic,
        "traffic_unit": "bytes per launch",
        # the same bytes as a rate, against the 8 TB/s HBM peak
        "traffic_gbs": None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9,
        "traffic_frac_of_hbm_peak": None if traffic is None else traffic / (launch_ms * 1e-3) / 8e12,
        "mulmods_per_launch": mulmods,
        "launch_ms": launch_ms,
        "valu_issue": valu,
    }
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bivariate resultants/s",
        "n_gpus": 1,
        "steps": a.pair_steps,
        "warmup": a.pair_warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "dense total-degree-24 pair, uniform signed 32-bit coefficients; "
                               "res_y and res_x per step (57 primes x 577 points each)",
                   "problems_per_step": 2, "primes": 57, "points": 577,
                   "schedule": {"batched": "persistent", "staged": "staged"}[mode] + (" (graph)" if use_graph else ""),
                   "steps_in_flight": len(all_jobs),
                   "lanes_per_pair": tune["lanes_per_pair"],
                   "lanes_per_pair_in_flight": inflight_lanes,
                   "ures": "schur" if (a.eval_schur or tune.get("schur")) else "remainder sequence",
                   "chunk_target": tune["chunk_target"], "grid_mult": tune["grid_mult"]},
        "verified_bit_exact": verified,
        "modp_univariate_resultants_per_s": pairs / (ures_ms * 1e-3),
        "modp_pairs": counts.get("pairs"), "bad_pairs": counts.get("bad_pairs"),
        "bad_primes": counts.get("bad_primes"),
        "serial_value": serial_value,
        "serial_ms_per_step": dt1 / a.pair_steps * 1e3,
        "plain_value": plain_value,
        "batched_vs_plain": value / plain_value,
        "serial_batched_vs_plain": serial_value / plain_value,
        "host_to_host_resultants_per_s": h2h,
        "schedule_ms_per_step": schedules,
        "in_flight_ms_per_step": inflight_ms,
        "tune": tune,
        "stage_ms_per_step": staged_split,
        "dominant_stage": dominant,
        "roofline": roofline,
    }
    for _, jobs in inflight_sets[1:]:
        for j in jobs:
            j.close()
    for c, j in extra:
        j.close()
        c.close()
    for c in dctx:
        c.close()
    job.close()
    ctx.close()
    return out




GOLDEN = os.path.join(ROOT, "tests", "golden")
MFMA_INT8_PEAK_TOPS = 5000.0  # dense int8 matrix-core multiply-adds x 2, TOP/s (MI355X)


def _load_golden(cfg):
    path = os.path.join(GOLDEN, f"cfg{cfg}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return {r["name"]: r for r in json.load(fh)["records"]}


def _eval_mod(R, t, q):
    """R(t) mod q by Horner's rule (checks a result against a stored modular value)."""
    acc = 0
    for c in reversed(R):
        acc = (acc * t + c) % q
    return acc


def verify_batch(results, prefix="cfg4", full_cfg=4, modq_cfg=40, var="y"):
    """Compare results with the oracle's stored values: the digest of every problem the
    full oracle covers, and R(t) mod q for the two stored checks of every problem."""
    full, modq = _load_golden(full_cfg), _load_golden(modq_cfg)
    if not modq:
        return None
    n_full = n_modq = 0
    for k, R in enumerate(results):
        name = f"{prefix}_{k}_{var}"
        rec = modq.get(name)
        if rec is None:
            return False
        for c in rec["checks"]:
            if _eval_mod(R, int(c["t"]), int(c["q"])) != int(c["value"]):
                return False
            n_modq += 1
        if name in full:
            if digest(R) != full[name]["sha256"]:
                return False
            n_full += 1
    return {"full_oracle_digests": n_full, "modq_checks": n_modq}


def profile_batch(a):
    """Only the device pipeline of the 512-pair batch, resident, a.profile_batch
    runs of the layout a saved tuning choice picks: the launches a kernel trace or
    counter run of this command sees are exactly those runs (plus the uploads)."""
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    probs = [(f, g, "y") for f, g in workloads.config4()]
    ctx = rsl.Context(0, workspace_bytes=1 << 30)
    if a.tune_load:
        ctx.tune_load(a.tune_load)
    job = ctx.job(probs)
    info = job.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.profile_batch):
        job.run("auto")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    job.close()
    ctx.close()
    return {"profile_batch_runs": a.profile_batch, "ms_per_run": dt / a.profile_batch * 1e3,
            "layout_mode": info["layout_mode"], "eval_lanes": info["eval_lanes"],
            "chunk_target": info["chunk_target"]}


def profile_h2h(a):
    """Only host-to-host batch calls of the 512-pair batch (a.profile_h2h of them,
    after one warm-up call), laid out with a saved tuning choice: the timeline of
    a kernel and copy trace of this command shows how host work and device work
    of the chunk pipeline overlap."""
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    probs = [(f, g, "y") for f, g in workloads.config4()]
    pb = rsl.PreparedBatch(probs)
    ctx = rsl.Context(0, workspace_bytes=1 << 30)
    if a.tune_load:
        ctx.tune_load(a.tune_load)
    pb.run(ctx, "auto")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    splits = []
    for _ in range(a.profile_h2h):
        pb.run(ctx, "auto")
        splits.append(ctx.counters())
    dt = time.perf_counter() - t0
    ctx.close()
    keys = ("ms_total", "ms_build", "ms_bind", "ms_device", "ms_decode")
    return {"profile_h2h_calls": a.profile_h2h, "ms_per_call": dt / a.profile_h2h * 1e3,
            "split_ms": {k: sum(c[k] for c in splits) / len(splits) for k in keys}}


def tune_line(t):
    """The autotuner's choice as it is saved (mode, chunking, grid, lanes, convolution, Schur,
    matrix-core interpolation)."""
    names = {"staged": 2, "batched": 1}
    return [names.get(t["mode"], t["mode"]), t["chunk_target"], t["grid_mult"], t["lanes_per_pair"],
            t["conv_whole"], t["schur"], t.get("interp_mm", 0)]


def batch_headline(a):
    import numpy as np
    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    # the dense pair's figures first: measured after the batch in the same
    # process, its four resident jobs in flight have taken 44-48 us per step
    # instead of 32-35 us (the serial step and the host's enqueue time per
    # step unchanged)
    pair = None
    if not a.no_pair:
        pa = argparse.Namespace(**vars(a))
        pa.no_cpu_baseline = True
        pair = pair_bench(pa)

    pairs = workloads.config4()
    probs = [(f, g, "y") for f, g in pairs]
    pb = rsl.PreparedBatch(probs)  # the caller's data: limbs in, sized result buffers out
    ctx = rsl.Context(0, workspace_bytes=1 << 30)

    # autotune on a resident job of the batch: the winner is cached for its shape
    # bucket and used by every RSL_AUTO call of this context
    job = ctx.job(probs)
    tune = job.tune(reps=2)
    info = job.info()
    if a.tune_save:  # the choice, for a profiled run of the same layout (--profile-batch)
        ctx.tune_save(a.tune_save)

    def counters_sum(acc, c):
        for k in ("ms_total", "ms_build", "ms_bind", "ms_transfer", "ms_device", "ms_decode"):
            acc[k] = acc.get(k, 0.0) + c[k]

    def timed_batch(mode, steps, warmup):
        for _ in range(warmup):
            pb.run(ctx, mode)
        torch.cuda.synchronize()
        acc = {}
        t0 = time.perf_counter()
        for _ in range(steps):
            pb.run(ctx, mode)
            counters_sum(acc, ctx.counters())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, {k: v / steps for k, v in acc.items()}

    steps = max(1, a.steps)
    dt, split = timed_batch("auto", steps, a.warmup)
    counts = ctx.counters()
    res = pb.results()  # the last timed call's output
    verified = verify_batch(res)
    if verified is False:
        print("bench: a batch result differs from the oracle's stored values", file=sys.stderr)
        sys.exit(1)
    value = len(probs) * steps / dt

    plain_steps = max(1, min(steps, 5))
    dtp, split_p = timed_batch("plain", plain_steps, 1)
    if pb.results() != res:
        print("bench: plain and batched results differ", file=sys.stderr)
        sys.exit(1)
    plain_value = len(probs) * plain_steps / dtp

    # device-only: the same batch resident in device memory
    def timed_job(mode, n):
        job.run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            job.run(mode)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    job.run("auto")
    if job.results() != res:
        print("bench: resident job results differ from the batch call", file=sys.stderr)
        sys.exit(1)
    dev_ms = timed_job("auto", steps) * 1e3
    dev_plain_ms = timed_job("plain", plain_steps) * 1e3
    try:
        dev_persist_ms = timed_job("batched", 2) * 1e3
    except rsl.RSLError:
        dev_persist_ms = None

    # per-stage device time from HIP events on the context's stream (each stage
    # is one launch, the evaluation one launch per layout variant)
    ctx.profile_enable(True)
    for _ in range(2):  # the first pass makes the event sets, the second is measured
        ctx.profile_take()
        for _ in range(steps):
            job.run(tune["mode"])
    stages, runs = ctx.profile_take()
    ctx.profile_enable(False)
    stages = {k: v / max(runs, 1) for k, v in stages.items()}
    eval_ms = stages["eval_ures"]
    job.close()
    ctx.close()

    nps = np.array([i.n_primes for i in pb.infos])
    Ds = np.array([i.D for i in pb.infos])

    def hist(v):
        return {"min": int(v.min()), "p50": int(np.percentile(v, 50)), "p90": int(np.percentile(v, 90)),
                "max": int(v.max()), "sum": int(v.sum())}

    valu_mm, mfma_mm, macs = info["mulmods_valu"], info["mulmods_sums_mfma"], info["mfma_int8_macs"]
    t_eval = eval_ms * 1e-3
    roofline = {
        "bound": "alu",
        "kernel": "eval_ures (the evaluation stage: one launch per layout variant)",
        "achieved": valu_mm / t_eval / 1e12,
        "peak": PEAK_TMULMOD,
        "unit": "Tmulmod/s",
        "frac": valu_mm / t_eval / 1e12 / PEAK_TMULMOD,
        "traffic": None,
        "per_launch": {"valu_mulmods": valu_mm, "launch_ms": eval_ms,
                       "note": "VALU part: remainder-sequence products m_y n_y per (prime, point) pair plus the "
                               "Horner sums of problems whose sums are not on the matrix cores"},
        "mfma": {"achieved": 2.0 * macs / t_eval / 1e12, "peak": MFMA_INT8_PEAK_TOPS, "unit": "TOP/s int8",
                 "frac": 2.0 * macs / t_eval / 1e12 / MFMA_INT8_PEAK_TOPS, "int8_macs_per_launch": macs,
                 "sums_mulmods": mfma_mm,
                 "note": "evaluation sums on the matrix cores: 25 int8 digit products per residue product, "
                         "padded 16x16x32 tiles"},
        "all_products_frac": info["mulmods"] / t_eval / 1e12 / PEAK_TMULMOD,
    }
    # the same launches against the measured issue rates of the units
    # (paper_1010_1386_amd.peak: eight chains per lane, 4 or 8 waves per SIMD)
    try:
        from paper_1010_1386_amd import peak as peakmod
        rates = peakmod.measure()
        mont = rates["montgomery_mul"] / 1e12
        roofline["measured_peak"] = {
            "montgomery_tmulmod_s": mont, "fused_update_t_s": rates["fused_update_3_products"] / 1e12,
            "mfma_int8_top_s": 2.0 * rates["mfma_i32_16x16x32_i8_macs"] / 1e12,
            "valu_frac_of_measured": valu_mm / t_eval / 1e12 / mont,
            "mfma_frac_of_measured": macs / t_eval / rates["mfma_i32_16x16x32_i8_macs"],
            "rates": rates, "source": "paper_1010_1386_amd/peak.py (csrc/peak.hip)"}
    except Exception as e:  # measurement is auxiliary: report, never fail the line
        roofline["measured_peak"] = {"error": str(e)}
    # HBM bytes and VALU instructions of the evaluation stage per run, from the
    # committed counter summaries of the same kernel sources and layout choice
    for key, fname in (("traffic", "traffic_eval_ures_cfg4_batch.json"), ("insts", "insts_eval_ures_cfg4_batch.json")):
        path = os.path.join(ROOT, "profiles", fname)
        if not os.path.exists(path):
            continue
        from paper_1010_1386_amd import traffic as tr
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("tune_line") != tune_line(tune):
            continue
        if key == "traffic":
            b = tr.traffic_bytes(rec)
            if b is not None:
                roofline["traffic"] = b
                roofline["traffic_gbs"] = b / t_eval / 1e9
        else:
            vi = tr.valu_issue(rec, t_eval)
            if vi is not None:
                roofline["valu_issue"] = {"lane_ops_per_run": vi[0], "frac_of_issue_peak": vi[1],
                                          "mfma_insts_per_run": rec["mfma_insts"]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "bivariate resultants/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batch of 512 independent pairs: total degrees U{6..32}, signed U{8..64}-bit "
                               "coefficients, pairs 0-255 dense, 256-511 with 30% of the coefficients zeroed; "
                               "res_y of each, one rsl_batch call per step, host limbs to host limbs",
                   "problems_per_step": len(probs), "schedule": tune["mode"], "tune": tune,
                   "n_primes": hist(nps), "degree_bound_D": hist(Ds)},
        "verified": verified,
        "host_to_host": True,
        "step_split_ms": split,
        "plain_value": plain_value,
        "plain_ms_per_step": dtp / plain_steps * 1e3,
        "plain_step_split_ms": split_p,
        "batched_vs_plain": value / plain_value,
        "device_only": {"resultants_per_s": len(probs) / (dev_ms * 1e-3), "ms_per_batch": dev_ms,
                        "plain_ms_per_batch": dev_plain_ms, "persistent_ms_per_batch": dev_persist_ms,
                        "batched_vs_plain": dev_plain_ms / dev_ms},
        "modp_univariate_resultants_per_s": info["pairs"] / t_eval,
        "modp_pairs": counts["pairs"], "bad_pairs": counts["bad_pairs"], "bad_primes": counts["bad_primes"],
        "stage_ms_per_step": stages,
        "dominant_stage": max(stages, key=stages.get),
        "roofline": roofline,
    }
    if pair is not None:
        pr = pair
        out["pair"] = {k: pr[k] for k in ("value", "ms_per_step", "serial_value", "plain_value", "config",
                                          "tune", "in_flight_ms_per_step", "verified_bit_exact", "roofline")}
        out["pair"]["unit"] = "bivariate resultants/s, device only (inputs resident), steps in flight"
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batches (each is one rsl_batch of 512 problems)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pair", action="store_true",
                    help="only the dense degree-24 pair benchmark (device-only, steps in flight)")
    ap.add_argument("--no-pair", action="store_true", help="leave the pair figures out of the default line")
    ap.add_argument("--pair-steps", type=int, default=400)
    ap.add_argument("--pair-warmup", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=100, help="pair benchmark: steps of the comparison schedules")
    ap.add_argument("--schedule", choices=["auto", "staged", "batched"], default="auto",
                    help="auto: autotune the job first; otherwise that schedule with the default layout")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="serving benchmark instead: N Poisson-arriving requests of the serving workload")
    ap.add_argument("--batch512", action="store_true",
                    help="batch benchmark instead: 512 pairs (res_y), autotuned schedule vs one pipeline per problem")
    ap.add_argument("--table3", action="store_true",
                    help="large-coefficient benchmark instead: the random-curve sets of Table 3, res_y of all pairs")
    ap.add_argument("--inflight", type=int, default=4,
                    help="steps in flight: resident jobs of the pair on their own streams, run in turn")
    ap.add_argument("--eval-lanes", type=int, default=0, choices=[0, 1, 2, 4],
                    help="lanes per (prime, point) pair of the evaluation (0: the layout heuristics / autotuner)")
    ap.add_argument("--eval-schur", action="store_true",
                    help="univariate resultants by the Schur algorithm (comparison runs; use with --schedule staged)")
    ap.add_argument("--sqfree", action="store_true",
                    help="square-free part of resultants by the modular gcd instead")
    ap.add_argument("--table3-only", default="", metavar="DEG:K[,DEG:K]",
                    help="with --table3: only these sets (e.g. 15:2048)")
    ap.add_argument("--tune-save", default="", metavar="FILE",
                    help="batch headline: save the autotuner's choice (rsl_tune_save) to FILE")
    ap.add_argument("--tune-load", default="", metavar="FILE",
                    help="--profile-batch: lay the batch out with the choice saved in FILE")
    ap.add_argument("--profile-batch", type=int, default=0, metavar="K",
                    help="only K device runs of the resident 512-pair batch (for kernel traces and counters)")
    ap.add_argument("--profile-h2h", type=int, default=0, metavar="K",
                    help="only K host-to-host batch calls of the 512-pair batch (for timeline traces)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 5 times (HBM counter calibration)")
    a = ap.parse_args()
    if a.copy_calibration:
        import torch
        src = torch.empty(a.copy_calibration, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.copy_calibration, "copies": 5}))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1010_1386_amd as rsl
    import workloads

    if a.serve:
        print(json.dumps(serve_bench(a.serve)))
        return
    if a.batch512:
        print(json.dumps(batch_bench(a.steps, a.warmup)))
        return
    if a.sqfree:
        print(json.dumps(sqfree_bench(a.steps, not a.no_cpu_baseline)))
        return
    if a.table3:
        only = [x for x in a.table3_only.split(",") if x]
        print(json.dumps(table3_bench(a.steps, a.warmup, only)))
        return

    if a.pair:
        print(json.dumps(pair_bench(a)))
        return
    if a.profile_batch:
        print(json.dumps(profile_batch(a)))
        return
    if a.profile_h2h:
        print(json.dumps(profile_h2h(a)))
        return
    out = batch_headline(a)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

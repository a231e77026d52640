"""GPU: the serving stream -- res_y / res_x requests with degrees U{8..48} and signed
U{8..48}-bit dense coefficients arriving as a Poisson process -- served by the
continuous-batching server.  Every result is checked against the oracle: two modular
checks per request (tests/golden/cfg50.json: R(t) mod q against the determinant of the
Sylvester matrix specialised at t over Z_q, q a 61-bit prime), the full oracle digest on
every request whose Sylvester matrix has order at most 32 (cfg5.json), and every request
replayed alone through the synchronous call must give the same bits as in the mix.
"""

import threading
import time

import pytest

import _golden
import oracle
import workloads

pytestmark = pytest.mark.gpu

N_REQ = 1000        # the whole stream
RATE = 4000.0       # requests/s offered: arrivals overlap work already on the device


@pytest.fixture(scope="module")
def stream():
    return workloads.config5(N_REQ)


def test_serving_stream_is_exact_in_the_mix_and_alone(stream):
    import paper_1010_1386_amd as rsl
    t_start = time.perf_counter()
    polys = [(rsl.Poly(f), rsl.Poly(g), v) for f, g, v in stream]
    ctx = rsl.Context(device=0, workspace_bytes=1 << 30)
    srv = rsl.Server(ctx, budget_bytes=64 << 20, max_slots=256, max_queue=1 << 20)
    arrivals = workloads.poisson_arrivals(N_REQ, RATE)
    tickets = [None] * N_REQ
    t0 = time.perf_counter()

    def producer():
        for k, (f, g, v) in enumerate(polys):
            dt = arrivals[k] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[k] = srv.submit(f, g, v)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    served = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"served {N_REQ} requests in {time.perf_counter() - t0:.2f} s: {st['launches']} device iterations, "
          f"max batch {st['max_batch']}, p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms", flush=True)
    assert st["completed"] == N_REQ and st["in_flight"] == 0
    assert st["max_batch"] >= 2 and st["launches"] < N_REQ  # requests shared device iterations
    assert st["admitted_bytes_peak"] <= 64 << 20

    full = _golden.load(5)
    modq = _golden.load(50)
    assert len(modq) == N_REQ and len(full) >= 80
    n_full = 0
    for k, (f, g, v) in enumerate(stream):
        name = f"cfg5_{k}_{v}"
        _golden.check_modq(served[k], modq[name])
        if name in full:
            _golden.check_full(served[k], full[name])
            n_full += 1
        assert len(served[k]) - 1 <= oracle.degree_bound(f, g, v), name
    assert n_full == len(full)

    # every request alone (synchronous call on a context of its own): the same bits
    alone_ctx = rsl.Context(device=0, workspace_bytes=1 << 30)
    for k, (f, g, v) in enumerate(polys):
        assert alone_ctx.res(f, g, v) == served[k], (k, v)
    alone_ctx.close()
    ctx.close()
    print(f"stream test {time.perf_counter() - t_start:.1f} s", flush=True)

"""Host logic of the serving scheduler, with a simulated backend whose
requests take a known time on their lane."""

import numpy as np
import pytest

from paper_1712_05834_amd.serve import Request, Server, latency_stats, poisson_arrivals


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class SimBackend:
    """Each request runs for req.mesh seconds (the test puts a duration
    there) once submitted; time advances only when the server is idle."""

    def __init__(self, lanes, clock):
        self.lanes = lanes
        self.clock = clock
        self.ends = {}
        self.log = []

    def footprint(self, req):
        return req.npart

    def submit(self, lane, req):
        assert lane not in self.ends, "lane reused while busy"
        self.ends[lane] = self.clock() + req.mesh
        self.log.append(("submit", req.rid, lane, self.clock()))

    def done(self, lane):
        return self.clock() >= self.ends[lane] - 1e-12

    def fetch(self, lane, req):
        return {"rid": req.rid}

    def release(self, lane):
        del self.ends[lane]


def make_server(lanes, budget):
    clock = FakeClock()
    be = SimBackend(lanes, clock)

    def idle():
        # jump to the next event: an arrival or a completion
        clock.t += 1e-3

    return Server(be, budget, clock=clock, idle=idle), be, clock


def req(rid, arrival, duration, size):
    return Request(rid, arrival, duration, None, None, size)


def test_fifo_admission_and_latency_accounting():
    srv, be, _ = make_server(lanes=2, budget=100)
    rs = [req(0, 0.0, 0.010, 10), req(1, 0.0, 0.010, 10), req(2, 0.0, 0.005, 10)]
    out = srv.run(rs)
    by = {r.rid: r for r in out}
    # two lanes: 0 and 1 start at once, 2 waits for the first free lane
    assert by[0].admitted == pytest.approx(0.0) and by[1].admitted == pytest.approx(0.0)
    assert by[2].admitted == pytest.approx(0.010, abs=1.5e-3)
    assert by[2].finished == pytest.approx(0.015, abs=2.5e-3)
    assert all(r.result == {"rid": r.rid} for r in out)
    assert by[2].latency > by[0].latency


def test_budget_blocks_and_no_overtaking():
    srv, be, _ = make_server(lanes=4, budget=100)
    rs = [req(0, 0.0, 0.020, 70), req(1, 0.001, 0.005, 60), req(2, 0.002, 0.001, 10)]
    out = srv.run(rs)
    by = {r.rid: r for r in out}
    # 1 does not fit beside 0; 2 would fit but must not overtake 1
    assert by[1].admitted >= by[0].finished - 1e-9
    assert by[2].admitted >= by[1].admitted
    order = [rid for kind, rid, _, _ in be.log]
    assert order == [0, 1, 2]


def test_request_larger_than_budget_is_rejected():
    srv, _, _ = make_server(lanes=1, budget=5)
    with pytest.raises(ValueError):
        srv.run([req(0, 0.0, 0.001, 6)])


def test_poisson_arrivals_and_stats():
    rng = np.random.default_rng(5)
    t = poisson_arrivals(4000, qps=50.0, rng=rng)
    gaps = np.diff([0.0] + t)
    assert np.all(gaps > 0)
    assert np.mean(gaps) == pytest.approx(1 / 50.0, rel=0.05)
    srv, _, _ = make_server(lanes=3, budget=10 ** 9)
    rs = [req(i, a, 0.004, 1) for i, a in enumerate(t[:300])]
    st = latency_stats(srv.run(rs))
    assert st["requests"] == 300
    assert 4.0 <= st["p50_ms"] <= st["p99_ms"]
    assert st["throughput_rps"] == pytest.approx(50.0, rel=0.2)

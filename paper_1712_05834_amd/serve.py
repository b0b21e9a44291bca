"""Serving FFTPower requests on one GPU with continuous batching.

Requests (a device-resident catalog plus a mesh and a binning) arrive over
time; the server admits each one as soon as a lane is free and its device
footprint fits the memory budget, runs it on that lane concurrently with the
others (``pk_fftpower_async``), and finalises its result on the host as soon
as the lane reports completion.  Latency = result on the host - arrival.

The paper motivates the use case (Sec. 6): estimators evaluated over and over
(MCMC-style repetition, many mocks), where time to solution per request and
throughput both matter.

The scheduling loop is plain host logic over a small backend interface
(``submit`` / ``done`` / ``fetch`` / ``release``), so it is tested on the CPU
with a simulated backend; ``LibpkBackend`` is the real one.  Admission is
first come, first served: a request that does not fit waits, and nothing
behind it overtakes it (no starvation of large requests).
"""

import collections
import math
import time


class Request:
    """One FFTPower request: ``mesh`` / ``bins`` are the C descriptors
    (``_lib.mesh_desc`` / ``_lib.bin_desc``), ``pos`` / ``weight`` device
    tensors, ``arrival`` seconds after the start of the run."""

    __slots__ = ("rid", "arrival", "mesh", "bins", "pos", "weight", "npart", "footprint",
                 "admitted", "finished", "result", "lane")

    def __init__(self, rid, arrival, mesh, bins, pos, npart, weight=None, footprint=0):
        self.rid = rid
        self.arrival = float(arrival)
        self.mesh = mesh
        self.bins = bins
        self.pos = pos
        self.weight = weight
        self.npart = int(npart)
        self.footprint = int(footprint)
        self.admitted = None
        self.finished = None
        self.result = None
        self.lane = None

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class LibpkBackend:
    """Runs requests on the lanes of a libpk context.  The device footprint
    of a request is its workspace plus its result (the catalog is resident
    before it arrives)."""

    def __init__(self, ctx, lanes, device="cuda:0"):
        import torch

        from . import _lib

        self._lib = _lib
        self.torch = torch
        self.ctx = ctx
        self.device = device
        ctx.pk_ctx_set_lanes(lanes)
        self.lanes = lanes
        self._bufs = {}

    def footprint(self, req):
        return (self._lib.workspace_bytes(req.mesh, req.bins, req.npart)
                + 8 * self._lib.result_doubles(req.bins))

    def submit(self, lane, req):
        torch = self.torch
        ws = torch.empty(self._lib.workspace_bytes(req.mesh, req.bins, req.npart),
                         dtype=torch.uint8, device=self.device)
        res = torch.empty(self._lib.result_doubles(req.bins), dtype=torch.float64,
                          device=self.device)
        self._bufs[lane] = (ws, res)
        self.ctx.pk_fftpower_async(lane, req.mesh, req.bins, req.pos, req.weight, req.npart,
                                   ws, res)

    def done(self, lane):
        return self.ctx.pk_lane_query(lane)

    def fetch(self, lane, req):
        _, res = self._bufs[lane]
        return self.ctx.pk_result_to_host(req.mesh, req.bins, res)

    def release(self, lane):
        # the workspace returns to torch's caching allocator: a later request
        # of the same size reuses it without a new device allocation
        self._bufs.pop(lane, None)


class Server:
    """Continuous-batching scheduler over a backend's lanes.

    ``budget`` bounds the sum of the footprints of the requests in flight
    (bytes).  ``clock`` returns seconds (monotonic); ``idle`` is called when
    nothing can progress (default: a 50 us sleep)."""

    def __init__(self, backend, budget, clock=time.perf_counter, idle=None):
        self.backend = backend
        self.budget = int(budget)
        self.clock = clock
        self.idle = idle or (lambda: time.sleep(5e-5))

    def run(self, requests):
        """Serves the requests (arrival times relative to the call) and returns
        them with admitted / finished / result / lane filled in."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if not r.footprint:
                r.footprint = self.backend.footprint(r)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, more than the "
                                 f"budget of {self.budget}")
        pending = collections.deque(reqs)
        queue = collections.deque()
        busy = {}  # lane -> request
        free = list(range(self.backend.lanes))[::-1]
        in_use = 0
        t0 = self.clock()
        while pending or queue or busy:
            now = self.clock() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            for lane in list(busy):
                if self.backend.done(lane):
                    r = busy.pop(lane)
                    r.result = self.backend.fetch(lane, r)
                    r.finished = self.clock() - t0
                    self.backend.release(lane)
                    in_use -= r.footprint
                    free.append(lane)
                    progressed = True
            while queue and free and in_use + queue[0].footprint <= self.budget:
                r = queue.popleft()
                lane = free.pop()
                r.lane = lane
                r.admitted = self.clock() - t0
                self.backend.submit(lane, r)
                busy[lane] = r
                in_use += r.footprint
                progressed = True
            if not progressed:
                self.idle()
        return reqs


def poisson_arrivals(count, qps, rng):
    """count arrival times (s) of a Poisson process of rate qps."""
    t, out = 0.0, []
    for _ in range(count):
        t += rng.exponential(1.0 / qps)
        out.append(t)
    return out


def latency_stats(reqs):
    """p50 / p99 / mean latency (ms) and throughput (requests/s) of a served run."""
    lat = sorted(r.latency for r in reqs)
    n = len(lat)

    def pct(p):
        # nearest-rank percentile
        return lat[max(0, min(n - 1, math.ceil(p / 100.0 * n) - 1))]

    span = max(r.finished for r in reqs) - min(r.arrival for r in reqs)
    return {
        "requests": n,
        "p50_ms": 1e3 * pct(50),
        "p99_ms": 1e3 * pct(99),
        "mean_ms": 1e3 * sum(lat) / n,
        "throughput_rps": n / span if span > 0 else float("inf"),
    }

"""Scheduling logic of the render server on the CPU, with a simulated clock and executor:
FIFO admission, the slot limit, the memory budget, overlap of requests in flight, and the
latency/throughput arithmetic."""
from types import SimpleNamespace

import numpy as np

from paper_2506_13348_amd.serve import Request, Server, _Plan, latency_report


class SimServer(Server):
    """Server whose device work takes `cost(req)` simulated seconds per request."""

    def __init__(self, cost, **kw):
        self.t = 0.0
        self.cost = cost
        super().__init__([SimpleNamespace(n=1000)] * 3, **kw)

    def _make_streams(self, n):
        return list(range(n))

    def _capacity(self, s, W, H):
        return 1000

    def _make_plan(self, s, W, H, cam):
        p = _Plan((s, W, H), None, None, None, nbytes=W * H * 16)
        self.plans[(s, W, H)].append(p)
        self.stats["plans"] += 1
        return p

    def _estimate_bytes(self, req):
        return req.width * req.height * 16

    def _launch(self, req, p, slot):
        req.slot = slot
        req.start = self.t
        return self.t + self.cost(req)

    def _is_done(self, handle):
        return self.t >= handle

    def _overflowed(self, p):
        return False

    def _clock(self):
        return self.t

    def _sync(self):
        pass

    def _idle(self):
        self.t += 1e-4


def _reqs(arrivals, res=(64, 64), scene=0):
    return [Request(i, t, scene, res[0], res[1], {}) for i, t in enumerate(arrivals)]


def test_fifo_single_slot_serialises():
    srv = SimServer(lambda r: 0.01, slots=1)
    reqs = srv.serve(_reqs([0.0, 0.001, 0.002, 0.003]))
    starts = [r.start for r in reqs]
    assert starts == sorted(starts)
    assert all(b.start >= a.done - 1e-9 for a, b in zip(reqs, reqs[1:]))
    assert srv.stats["max_inflight"] == 1


def test_requests_overlap_up_to_the_slot_count():
    srv = SimServer(lambda r: 0.05, slots=4)
    reqs = srv.serve(_reqs([0.0] * 10))
    assert srv.stats["max_inflight"] == 4
    # admitted as slots free up: the 5th starts when the first finishes
    assert abs(sorted(r.start for r in reqs)[4] - 0.05) < 2e-4
    assert len({r.slot for r in reqs}) == 4


def test_memory_budget_limits_admission():
    # each 64x64 plan is 64 KiB; a 150 KiB budget admits two at a time although 4 slots exist
    srv = SimServer(lambda r: 0.02, slots=4, mem_budget=150 * 1024)
    srv.serve(_reqs([0.0] * 6))
    assert srv.stats["max_inflight"] == 2
    assert srv.mem_in_use == 0


def test_no_starvation_of_a_large_request():
    srv = SimServer(lambda r: 0.001 * r.width / 64, slots=2, mem_budget=10 << 20)
    reqs = _reqs([0.0, 0.0005, 0.001, 0.0015])
    reqs[1].width, reqs[1].height = 512, 512
    out = srv.serve(reqs)
    assert all(r.done > 0 for r in out)
    assert out[1].start <= out[2].start   # FIFO: later small requests do not overtake it


def test_latency_report_arithmetic():
    reqs = _reqs([0.0, 0.1, 0.2, 0.3])
    for r, lat in zip(reqs, [0.010, 0.020, 0.030, 0.040]):
        r.done = r.arrival + lat
    rep = latency_report(reqs)
    assert rep["p50_ms"] == np.percentile([10, 20, 30, 40], 50)
    assert abs(rep["p99_ms"] - np.percentile([10, 20, 30, 40], 99)) < 1e-9
    assert abs(rep["mpix_per_s"] - 4 * 64 * 64 / 0.34 / 1e6) < 0.01

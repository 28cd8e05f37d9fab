"""Scheduling logic of the render server on the CPU, with a simulated clock and executor:
FIFO admission, the slot limit, the memory budget over resident plans with least-recently-used
eviction, overlap of requests in flight, continuous batching (requests arriving while a batch
renders join the next one; batch size and depth limits), and the latency/throughput
arithmetic."""
from types import SimpleNamespace

import numpy as np

from paper_2506_13348_amd.serve import Request, Server, _Plan, latency_report


class SimServer(Server):
    """Server whose device work takes simulated time: `cost(req)` seconds per request in mode
    "request"; in mode "batch" the front part is free and a batch takes batch_cost(reqs)
    seconds on one raster stream (batches run one after another)."""

    def __init__(self, cost, batch_cost=None, **kw):
        self.t = 0.0
        self.cost = cost
        self.batch_cost = batch_cost or (lambda reqs: sum(cost(r) for r in reqs))
        self.raster_free = 0.0
        self.made = []
        super().__init__([SimpleNamespace(n=1000)] * 3, **kw)

    def _make_streams(self, n):
        return list(range(n))

    def _setup_batching(self):
        if self.mode == "batch":
            self.free_batch_slots = list(range(self.batch_depth))

    def _capacity(self, s, W, H):
        return 1000

    def _plan_size(self, s, W, H):
        return W * H * 16

    def _make_plan(self, s, W, H, cam):
        p = _Plan((s, W, H), None, None, None, nbytes=W * H * 16)
        self._add_plan(p)
        self.made.append((s, W, H))
        return p

    def _launch(self, req, p, slot):
        req.slot = slot
        req.start = self.t
        return self.t + self.cost(req)

    def _enqueue_front(self, req, p, slot):
        req.admitted = self.t

    def _launch_batch(self, bslot, items):
        start = max(self.t, self.raster_free)
        reqs = [r for r, _ in items]
        for r in reqs:
            r.start = start
        self.raster_free = start + self.batch_cost(reqs)
        return self.raster_free

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
    srv = SimServer(lambda r: 0.01, slots=1, mode="request")
    reqs = srv.serve(_reqs([0.0, 0.001, 0.002, 0.003]))
    starts = [r.start for r in reqs]
    assert starts == sorted(starts)
    assert all(b.start >= a.done - 1e-9 for a, b in zip(reqs, reqs[1:]))
    assert srv.stats["max_inflight"] == 1


def test_requests_overlap_up_to_the_slot_count():
    srv = SimServer(lambda r: 0.05, slots=4, mode="request")
    reqs = srv.serve(_reqs([0.0] * 10))
    assert srv.stats["max_inflight"] == 4
    # admitted as slots free up: the 5th starts when the first finishes
    assert abs(sorted(r.start for r in reqs)[4] - 0.05) < 2e-4
    assert len({r.slot for r in reqs}) == 4


def test_memory_budget_limits_admission():
    # each 64x64 plan is 64 KiB; a 150 KiB budget holds two plans, so two requests run at a
    # time although 4 slots exist, and the two plans are reused
    srv = SimServer(lambda r: 0.02, slots=4, mem_budget=150 * 1024, mode="request")
    srv.serve(_reqs([0.0] * 6))
    assert srv.stats["max_inflight"] == 2
    assert srv.stats["plans"] == 2 and srv.stats["evictions"] == 0
    assert srv.n_busy == 0 and srv.resident == 2 * 64 * 1024
    assert srv.stats["max_resident"] <= 150 * 1024


def test_idle_plans_are_evicted_least_recently_used_first():
    # two plans fit; requests for three keys one after another
    srv = SimServer(lambda r: 0.01, slots=1, mem_budget=150 * 1024, mode="request")
    arr = [0.0, 0.02, 0.04, 0.06, 0.08]
    scenes = [0, 1, 0, 2, 1]
    reqs = [Request(i, t, s, 64, 64, {}) for i, (t, s) in enumerate(zip(arr, scenes))]
    srv.serve(reqs)
    # key 2 evicts key 1 (used before key 0's second request), then key 1 evicts key 0
    assert srv.made == [(0, 64, 64), (1, 64, 64), (2, 64, 64), (1, 64, 64)]
    assert srv.stats["evictions"] == 2
    assert srv.stats["max_resident"] <= 150 * 1024
    assert sorted(k for k, ps in srv.plans.items() if ps) == [(1, 64, 64), (2, 64, 64)]


def test_a_key_with_busy_plans_waits_instead_of_evicting():
    # two plans fit; key 1's plan is idle when two key-0 requests overlap: the second waits for
    # the first's plan rather than evicting key 1's
    srv = SimServer(lambda r: 0.01, slots=2, mem_budget=150 * 1024, mode="request")
    reqs = [Request(0, 0.0, 1, 64, 64, {}), Request(1, 0.02, 0, 64, 64, {}),
            Request(2, 0.021, 0, 64, 64, {})]
    srv.serve(reqs)
    assert srv.made == [(1, 64, 64), (0, 64, 64)] and srv.stats["evictions"] == 0
    assert abs(reqs[2].start - reqs[1].done) < 2e-4


def test_a_request_alone_is_admitted_above_the_budget():
    srv = SimServer(lambda r: 0.01, slots=2, mem_budget=1024, mode="batch")
    reqs = srv.serve(_reqs([0.0, 0.0]))
    assert all(r.done > 0 for r in reqs)
    assert srv.stats["max_inflight"] == 1        # the second waited for the first


def test_no_starvation_of_a_large_request():
    srv = SimServer(lambda r: 0.001 * r.width / 64, slots=2, mem_budget=10 << 20,
                    mode="request")
    reqs = _reqs([0.0, 0.0005, 0.001, 0.0015])
    reqs[1].width, reqs[1].height = 512, 512
    out = srv.serve(reqs)
    assert all(r.done > 0 for r in out)
    assert out[1].start <= out[2].start   # FIFO: later small requests do not overtake it


def test_requests_arriving_during_a_batch_join_the_next_batch():
    srv = SimServer(lambda r: 0.01, mode="batch", batch_depth=1, max_inflight=64,
                    batch_cost=lambda reqs: 0.01 + 0.001 * len(reqs))
    reqs = srv.serve(_reqs([0.0, 0.002, 0.004, 0.006, 0.02]))
    assert [r.batch for r in reqs] == [0, 1, 1, 1, 2]
    assert srv.stats["batches"] == 3 and srv.stats["max_batch_size"] == 3
    # batch 1 starts when batch 0 ends and carries all three
    assert abs(reqs[1].start - 0.011) < 2e-4 and reqs[1].start == reqs[3].start
    assert all(abs(r.done - (0.011 + 0.013)) < 2e-4 for r in reqs[1:4])


def test_batch_depth_and_size_limits():
    srv = SimServer(lambda r: 0.01, mode="batch", batch_depth=2, max_batch=4, max_inflight=64,
                    batch_cost=lambda reqs: 0.005 * len(reqs))
    reqs = srv.serve(_reqs([0.0] * 10))
    sizes = np.bincount([r.batch for r in reqs])
    assert sizes.max() <= 4 and sizes.sum() == 10
    # two batches were launched at once (the second queued behind the first)
    assert reqs[0].batch == 0 and reqs[4].batch == 1 and reqs[4].start == 0.02
    assert srv.n_busy == 0 and not srv.batches


def test_latency_report_arithmetic():
    reqs = _reqs([0.0, 0.1, 0.2, 0.3])
    for r, lat in zip(reqs, [0.010, 0.020, 0.030, 0.040]):
        r.done = r.arrival + lat
    rep = latency_report(reqs)
    assert rep["p50_ms"] == np.percentile([10, 20, 30, 40], 50)
    assert abs(rep["p99_ms"] - np.percentile([10, 20, 30, 40], 99)) < 1e-9
    assert abs(rep["mpix_per_s"] - 4 * 64 * 64 / 0.34 / 1e6) < 0.01
    # warm-up exclusion: only requests arriving at or after 0.15 s
    rep2 = latency_report(reqs, warmup=0.15)
    assert rep2["requests"] == 2 and rep2["p50_ms"] == np.percentile([30, 40], 50)

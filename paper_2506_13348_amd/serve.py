"""Continuous-batching render server over resident textured scenes.

Test-time rendering of optimised scenes is the use the paper builds its texture atlases for
(Sec. 3.4, Supp. Sec. 1). Here several scenes stay resident on one GPU and a stream of render
requests (scene, camera, resolution) is served:

* admission: a request waits in FIFO order until a stream slot is free and the bytes of its
  render plan fit the memory budget next to the plans of the requests in flight;
* plans: one preallocated plan per (scene, resolution) instance, its whole path (preprocess ->
  depth sort and tile lists -> raster with fused shading) captured once as a HIP graph; a
  request copies its camera into the plan and replays the graph on its slot's stream, so
  requests admitted while others run overlap on the device;
* completion is detected from events; latency = completion - arrival;
* pair-list overflow (a camera producing more tile entries than the captured capacity) is
  detected from the plan's status word and the request is rendered again with a larger plan.

`serve_sequential` renders the same stream one request at a time without graphs (the plain
renderer) for comparison. Python here only schedules; all rendering runs in the HIP kernels."""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .render import RenderPlan, cameras_tensor


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the stream
    scene: int
    width: int
    height: int
    cam: dict
    done: float = -1.0
    output: torch.Tensor | None = None
    retried: bool = False


@dataclass
class _Plan:
    key: tuple
    plan: RenderPlan
    graph: torch.cuda.CUDAGraph | None
    cam_host: torch.Tensor
    nbytes: int
    busy: bool = False


def _plan_bytes(plan: RenderPlan) -> int:
    ts = [plan.rec, plan.rect, plan.depth_key, plan.ws, plan.sorted_ids, plan.tile_ranges,
          plan.pair_ids, plan.rgba]
    return int(sum(t.numel() * t.element_size() for t in ts if t is not None))


def estimate_capacity(scene, width, height, samples, margin=1.5):
    """Pair capacity for a (scene, resolution): the largest count over sample cameras."""
    best = 0
    for cam in samples:
        probe = RenderPlan(scene, [cam], width, height, pair_capacity=None)
        best = max(best, probe.cap)
        del probe
    return int(best * margin) + 65536


class Server:
    def __init__(self, scenes, slots=4, mem_budget=16 << 30, use_graphs=True,
                 capacity_samples=None, keep_outputs=False):
        self.scenes = scenes
        self.slots = self._make_streams(slots)
        self.free_slots = list(range(slots))
        self.mem_budget = int(mem_budget)
        self.mem_in_use = 0
        self.use_graphs = use_graphs
        self.plans = collections.defaultdict(list)     # (scene, W, H) -> [_Plan]
        self.capacity = {}
        self.capacity_samples = capacity_samples or {}
        self.keep_outputs = keep_outputs
        self.inflight = []        # (req, slot, plan, event)
        self.stats = {"graph_replays": 0, "plans": 0, "overflow_retries": 0, "max_inflight": 0}

    # -- plans ---------------------------------------------------------------------------
    def _capacity(self, s, W, H):
        key = (s, W, H)
        if key not in self.capacity:
            samples = self.capacity_samples.get(key)
            if not samples:
                raise KeyError(f"no capacity samples for {key}")
            self.capacity[key] = estimate_capacity(self.scenes[s], W, H, samples)
        return self.capacity[key]

    def _make_plan(self, s, W, H, cam):
        key = (s, W, H)
        cap = self._capacity(s, W, H)
        plan = RenderPlan(self.scenes[s], [cam], W, H, pair_capacity=cap)
        cam_host = torch.empty(16, dtype=torch.float32).pin_memory()
        graph = None
        if self.use_graphs:
            stream = torch.cuda.Stream()
            stream.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(stream):
                plan.run()          # warm up outside the capture
            stream.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                plan.run()
            stream.synchronize()
        p = _Plan(key, plan, graph, cam_host, _plan_bytes(plan))
        self.plans[key].append(p)
        self.stats["plans"] += 1
        return p

    def prepare(self, keys_and_cams, per_key=2):
        """Create plans (and capture graphs) before serving, per_key instances each."""
        for (s, W, H), cam in keys_and_cams:
            while len(self.plans[(s, W, H)]) < per_key:
                self._make_plan(s, W, H, cam)
        torch.cuda.synchronize()

    def _idle_plan(self, req):
        key = (req.scene, req.width, req.height)
        for p in self.plans[key]:
            if not p.busy:
                return p
        return None

    # -- request life cycle ----------------------------------------------------------------
    def _try_admit(self, req):
        if not self.free_slots:
            return False
        p = self._idle_plan(req)
        if p is None:
            # a new plan instance is allocated only if it fits next to the plans in flight
            # (a request alone on the device is always admitted, or it could never run)
            est = self._estimate_bytes(req)
            if self.mem_in_use + est > self.mem_budget and self.inflight:
                return False
            p = self._make_plan(req.scene, req.width, req.height, req.cam)
        if self.mem_in_use + p.nbytes > self.mem_budget and self.inflight:
            return False
        slot = self.free_slots.pop(0)
        p.busy = True
        self.mem_in_use += p.nbytes
        handle = self._launch(req, p, slot)
        self.inflight.append((req, slot, p, handle))
        self.stats["max_inflight"] = max(self.stats["max_inflight"], len(self.inflight))
        return True

    def _launch(self, req, p, slot):
        """Copy the camera into the plan and replay its graph on the slot's stream."""
        stream = self.slots[slot]
        cam = cameras_tensor([req.cam], "cpu")[0]
        p.cam_host.copy_(cam)
        with torch.cuda.stream(stream):
            p.plan.cams.view(-1).copy_(p.cam_host, non_blocking=True)
            if p.graph is not None:
                p.graph.replay()
                self.stats["graph_replays"] += 1
            else:
                p.plan.run()
            if self.keep_outputs:
                req.output = p.plan.rgba.view(req.height, req.width, 4).clone()
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def _is_done(self, handle):
        return handle.query()

    def _overflowed(self, p):
        return int(p.plan.status.item()) != 0

    def _estimate_bytes(self, req):
        sc = self.scenes[req.scene]
        cap = self._capacity(req.scene, req.width, req.height)
        return int(sc.n * (28 + 4 + 1 + 1 + 3) * 4 + cap * 4 + req.width * req.height * 16)

    def _poll(self, now_fn):
        still = []
        done = []
        for item in self.inflight:
            req, slot, p, handle = item
            if self._is_done(handle):
                if self._overflowed(p):
                    self._rerender(req, p)
                req.done = now_fn()
                p.busy = False
                self.mem_in_use -= p.nbytes
                self.free_slots.append(slot)
                done.append(req)
            else:
                still.append(item)
        self.inflight = still
        return done

    def _rerender(self, req, p):
        """Pair-list overflow: render again with capacity from the reported need."""
        self.stats["overflow_retries"] += 1
        req.retried = True
        need = int(p.plan.n_pairs.item())
        key = p.key
        self.capacity[key] = int(need * 1.5) + 65536
        plan = RenderPlan(self.scenes[req.scene], [req.cam], req.width, req.height,
                          pair_capacity=self.capacity[key])
        plan.run()
        plan.check()
        if self.keep_outputs:
            req.output = plan.rgba.view(req.height, req.width, 4).clone()
        # the stale plan (and graph) is replaced by one with the new capacity
        self.plans[key].remove(p)
        self._make_plan(req.scene, req.width, req.height, req.cam)

    def serve(self, requests, realtime=True):
        """Serve requests (sorted by arrival). Returns the list with completion times."""
        pending = collections.deque()
        reqs = sorted(requests, key=lambda r: r.arrival)
        i, n_done = 0, 0
        self._sync()
        t0 = self._clock()
        now = lambda: self._clock() - t0
        while n_done < len(reqs):
            t = now() if realtime else float("inf")
            while i < len(reqs) and reqs[i].arrival <= t:
                pending.append(reqs[i])
                i += 1
            progressed = False
            while pending and self._try_admit(pending[0]):
                pending.popleft()
                progressed = True
            done = self._poll(now)
            n_done += len(done)
            if not progressed and not done:
                self._idle()
        return reqs

    # device and clock hooks (a test substitutes a simulated clock and executor)
    def _make_streams(self, n):
        return [torch.cuda.Stream() for _ in range(n)]

    def _clock(self):
        return time.perf_counter()

    def _sync(self):
        torch.cuda.synchronize()

    def _idle(self):
        time.sleep(20e-6)


def serve_sequential(scenes, requests, capacity):
    """The plain renderer: requests in arrival order, one at a time, each fully synchronised."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(20e-6)
        plan = RenderPlan(scenes[r.scene], [r.cam], r.width, r.height,
                          pair_capacity=capacity[(r.scene, r.width, r.height)])
        plan.run()
        plan.check()
        r.output = plan.rgba.view(r.height, r.width, 4).clone()
        torch.cuda.synchronize()
        r.done = time.perf_counter() - t0
        del plan
    return reqs


def latency_report(reqs):
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    px = sum(r.width * r.height for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
            "mpix_per_s": round(px / span / 1e6, 2), "span_s": round(span, 3)}


def make_requests(trace, cams_fn):
    """trace entries (t, scene, (W,H), az, el) -> Request list; cams_fn(scene, W, H, az, el)."""
    return [Request(i, t, s, wh[0], wh[1], cams_fn(s, wh[0], wh[1], az, el))
            for i, (t, s, wh, az, el) in enumerate(trace)]

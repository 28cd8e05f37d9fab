"""Continuous-batching render server over resident textured scenes.

Test-time rendering of optimised scenes is the use the paper builds its texture atlases for
(Sec. 3.4, Supp. Sec. 1). Several scenes stay resident on one GPU and a stream of render
requests (scene, camera, resolution) is served.

Plans. One preallocated plan per (scene, resolution) instance holds every buffer of one
render. Plans stay resident between requests (a plan cache) and are counted against the
memory budget whether busy or idle; when a new plan would not fit, idle plans are evicted
least recently used first; a request whose key already has plans (all busy) waits for one of
them instead of evicting, and a request whose plan cannot be made to fit waits (a request alone
on the device is always admitted, or it could never run).

Two ways of running admitted requests on the device:

* mode "batch" (continuous batching): a request's front part (preprocess -> depth sort and
  tile lists), captured once per plan as a HIP graph, is replayed on one of several prep
  streams as soon as the request is admitted; the requests whose front parts are enqueued
  form the next batch, and every batch is rendered (raster with fused shading) by ONE
  persistent launch over a shared (request, view, tile) work queue (ts_raster_batch), replayed
  from a graph captured once per batch slot (the launch does not depend on the batch; its
  table is rewritten per batch). Requests that arrive while a batch renders join the next
  one, so batches grow with the load. Up to `batch_depth` batches are in flight, each on its
  own raster stream.
* mode "request": each request replays its plan's graph of the whole path on one of `slots`
  streams, so requests overlap on the device but no launch carries two of them.

Completion is detected from events; latency = completion - arrival. A pair-list overflow (a
camera producing more tile entries than the plan's capacity) is seen in the plan's status
word (copied to pinned host memory behind the request's work) and the request is rendered
again with a plan sized from the reported need.

`serve_sequential` renders the same stream one request at a time without graphs (the plain
renderer) for comparison. Python here only schedules; all rendering runs in the HIP kernels."""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _ffi as F
from .render import BatchRaster, RenderPlan, cameras_tensor


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
    batch: int = -1         # index of the batch that rendered it (mode "batch")


@dataclass
class _Plan:
    key: tuple
    plan: RenderPlan | None
    graph: object | None           # mode "request": the whole path; "batch": the front part
    cam_host: torch.Tensor | None
    nbytes: int
    job: object | None = None      # the plan's ts_raster_job (mode "batch")
    status_host: torch.Tensor | None = None
    busy: bool = False
    last_used: int = 0


def plan_bytes(plan: RenderPlan) -> int:
    """Device bytes held by a plan's buffers."""
    ts = [plan.rec, plan.rect, plan.depth_key, plan.ws, plan.sorted_ids, plan.tile_ranges,
          plan.pair_ids, plan.n_pairs, plan.status, plan.rgba, plan.gbuf, plan.t_final,
          plan.n_contrib, plan.n_blend, plan.lind, plan.gbuf_ind, plan.cams]
    return int(sum(t.numel() * t.element_size() for t in ts if t is not None))


def estimate_capacity(scene, width, height, samples, margin=1.5):
    """Pair capacity for a (scene, resolution): the largest count over sample cameras."""
    best = 0
    for cam in samples:
        probe = RenderPlan(scene, [cam], width, height, pair_capacity=None)
        best = max(best, probe.cap)
        del probe
    return int(best * margin) + 65536


def _capture(fn, stream):
    """A graph of fn()'s launches on `stream`, captured without synchronising the device
    (the plans' buffers are preallocated, so the capture allocates nothing)."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        g.capture_begin(capture_error_mode="thread_local")
        fn()
        g.capture_end()
    return g


class Server:
    def __init__(self, scenes, slots=4, mem_budget=16 << 30, use_graphs=True,
                 capacity_samples=None, keep_outputs=False, mode="batch", max_batch=16,
                 batch_depth=3, max_inflight=48):
        if mode not in ("batch", "request"):
            raise ValueError(f"unknown mode {mode}")
        self.scenes = scenes
        self.mode = mode
        self.slots = self._make_streams(slots)
        self.free_slots = list(range(slots))
        self.mem_budget = int(mem_budget)
        self.resident = 0                 # bytes of every plan, busy or idle
        self.use_graphs = use_graphs
        self.plans = collections.defaultdict(list)     # (scene, W, H) -> [_Plan]
        self.capacity = {}
        self.capacity_samples = capacity_samples or {}
        self.keep_outputs = keep_outputs
        self.max_batch = int(max_batch)
        self.batch_depth = int(batch_depth)
        self.max_inflight = int(max_inflight) if mode == "batch" else slots
        self.inflight = []        # mode "request": (req, slot, plan, handle)
        self.staged = []          # mode "batch": (req, plan, slot) with the front enqueued
        self.batches = []         # mode "batch": (batch slot, [(req, plan)], handle)
        self.n_busy = 0
        self._pinned = []
        self._tick = 0
        self._serving = False
        self._next_prep = 0
        self.stats = {"graph_replays": 0, "plans": 0, "plans_in_stream": 0, "evictions": 0,
                      "overflow_retries": 0, "max_inflight": 0, "batches": 0,
                      "max_batch_size": 0, "max_resident": 0}
        self._setup_batching()

    # -- device resources (a test substitutes a simulated executor) -----------------------
    def _make_streams(self, n):
        return [torch.cuda.Stream() for _ in range(n)]

    def _setup_batching(self):
        if self.mode == "batch":
            # one raster stream per batch slot: batches in flight may overlap on the device
            self.raster_streams = [torch.cuda.Stream() for _ in range(self.batch_depth)]
            self.batcher = BatchRaster(slots=self.batch_depth, use_graphs=self.use_graphs)
            self.free_batch_slots = list(range(self.batch_depth))

    def _clock(self):
        return time.perf_counter()

    def _sync(self):
        torch.cuda.synchronize()

    def _idle(self):
        time.sleep(20e-6)

    # -- plans ---------------------------------------------------------------------------
    def _capacity(self, s, W, H):
        key = (s, W, H)
        if key not in self.capacity:
            samples = self.capacity_samples.get(key)
            if not samples:
                raise KeyError(f"no capacity samples for {key}")
            self.capacity[key] = estimate_capacity(self.scenes[s], W, H, samples)
        return self.capacity[key]

    def _plan_size(self, s, W, H):
        """Bytes a new plan for (s, W, H) will hold."""
        return RenderPlan.bytes_for(self.scenes[s], 1, W, H, self._capacity(s, W, H))

    def _make_plan(self, s, W, H, cam):
        key = (s, W, H)
        cap = self._capacity(s, W, H)
        plan = RenderPlan(self.scenes[s], [cam], W, H, pair_capacity=cap)
        cam_host, status_host = self._pinned_pair()
        batchable = self.mode == "batch" and plan.batchable()
        graph = None
        if self.use_graphs:
            stream = self.slots[0]
            if not self._serving:
                # before serving: one eager run first (every kernel loaded before any capture)
                with torch.cuda.stream(stream):
                    plan.run()
                stream.synchronize()
            if self.mode == "batch":
                graph = _capture(plan.front if batchable else plan.run, stream)
            else:
                graph = _capture(plan.run, stream)
        p = _Plan(key, plan, graph, cam_host, plan_bytes(plan),
                  job=plan.raster_job() if batchable else None, status_host=status_host)
        self._add_plan(p)
        return p

    def _pinned_pair(self):
        """Pinned host words for a plan's camera and status (pinned allocations are slow, so
        those of evicted plans are reused)."""
        if self._pinned:
            return self._pinned.pop()
        return (torch.empty(16, dtype=torch.float32).pin_memory(),
                torch.zeros(1, dtype=torch.int32).pin_memory())

    def _add_plan(self, p):
        self.plans[p.key].append(p)
        self.resident += p.nbytes
        self.stats["plans"] += 1
        self.stats["plans_in_stream"] += int(self._serving)
        self.stats["max_resident"] = max(self.stats["max_resident"], self.resident)

    def _evict_one(self):
        """Drop the least recently used idle plan; False if every plan is busy."""
        idle = [p for ps in self.plans.values() for p in ps if not p.busy]
        if not idle:
            return False
        victim = min(idle, key=lambda p: p.last_used)
        self.plans[victim.key].remove(victim)
        self.resident -= victim.nbytes
        if victim.cam_host is not None:
            self._pinned.append((victim.cam_host, victim.status_host))
        self.stats["evictions"] += 1
        return True

    def prepare(self, keys_and_cams, per_key=2):
        """Create plans (and capture graphs) before serving, per_key instances each, within the
        memory budget."""
        for (s, W, H), cam in keys_and_cams:
            while len(self.plans[(s, W, H)]) < per_key:
                if self.resident + self._plan_size(s, W, H) > self.mem_budget:
                    break
                self._make_plan(s, W, H, cam)
        self._sync()

    def _plan_for(self, req):
        """An idle plan for the request, made (evicting idle plans) if none exists and it fits;
        None if the request has to wait."""
        key = (req.scene, req.width, req.height)
        for p in self.plans[key]:
            if not p.busy:
                return p
        need = self._plan_size(*key)
        if self.plans[key] and self.resident + need > self.mem_budget:
            # the key has plans, all busy: wait for one rather than evict another key's plan
            return None
        while self.resident + need > self.mem_budget and self._evict_one():
            pass
        if self.resident + need > self.mem_budget and self.n_busy > 0:
            return None
        return self._make_plan(req.scene, req.width, req.height, req.cam)

    # -- request life cycle ----------------------------------------------------------------
    def _try_admit(self, req):
        if self.n_busy >= self.max_inflight:
            return False
        if self.mode == "request" and not self.free_slots:
            return False
        p = self._plan_for(req)
        if p is None:
            return False
        p.busy = True
        self._tick += 1
        p.last_used = self._tick
        self.n_busy += 1
        self.stats["max_inflight"] = max(self.stats["max_inflight"], self.n_busy)
        if self.mode == "request":
            slot = self.free_slots.pop(0)
            self.inflight.append((req, slot, p, self._launch(req, p, slot)))
        else:
            slot = self._next_prep
            self._next_prep = (self._next_prep + 1) % len(self.slots)
            self._enqueue_front(req, p, slot)
            self.staged.append((req, p, slot))
        return True

    def _copy_camera(self, req, p, stream):
        cam = cameras_tensor([req.cam], "cpu")[0]
        p.cam_host.copy_(cam)
        p.plan.cams.view(-1).copy_(p.cam_host, non_blocking=True)

    def _launch(self, req, p, slot):
        """Mode "request": copy the camera into the plan and replay its graph of the whole path
        on the slot's stream."""
        stream = self.slots[slot]
        with torch.cuda.stream(stream):
            self._copy_camera(req, p, stream)
            if p.graph is not None:
                p.graph.replay()
                self.stats["graph_replays"] += 1
            else:
                p.plan.run()
            p.status_host.copy_(p.plan.status, non_blocking=True)
            if self.keep_outputs:
                req.output = p.plan.rgba.view(req.height, req.width, 4).clone()
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def _enqueue_front(self, req, p, slot):
        """Mode "batch": camera copy and the plan's front part on a prep stream; the event that
        the batch launch waits for is recorded on that stream."""
        stream = self.slots[slot]
        with torch.cuda.stream(stream):
            self._copy_camera(req, p, stream)
            if p.graph is not None:
                p.graph.replay()
                self.stats["graph_replays"] += 1
            elif p.job is not None:
                p.plan.front()
            else:
                p.plan.run()
            p.status_host.copy_(p.plan.status, non_blocking=True)
            req._front_done = torch.cuda.Event()
            req._front_done.record(stream)

    def _launch_batch(self, bslot, items):
        """One persistent raster launch over every batchable request of `items` on the raster
        stream, after their front parts; other requests (rendered whole on their prep
        streams) only join the batch's completion event."""
        rs = self.raster_streams[bslot]
        for req, p in items:
            rs.wait_event(req._front_done)
        jobs = [p.job for req, p in items if p.job is not None]
        if len(jobs) == 1:
            # a batch of one is the plain launch (the persistent grid only pays off when it
            # carries several renders)
            with torch.cuda.stream(rs):
                next(p for req, p in items if p.job is not None).plan.raster()
        elif jobs:
            self.batcher.launch(bslot, jobs, rs)
            if self.use_graphs:
                self.stats["graph_replays"] += 1
        with torch.cuda.stream(rs):
            if self.keep_outputs:
                for req, p in items:
                    req.output = p.plan.rgba.view(req.height, req.width, 4).clone()
            ev = torch.cuda.Event()
            ev.record(rs)
        return ev

    def _maybe_launch_batch(self):
        if not self.staged or not self.free_batch_slots:
            return False
        items = [(req, p) for req, p, _ in self.staged[:self.max_batch]]
        self.staged = self.staged[self.max_batch:]
        bslot = self.free_batch_slots.pop(0)
        handle = self._launch_batch(bslot, items)
        for req, _ in items:
            req.batch = self.stats["batches"]
        self.batches.append((bslot, items, handle))
        self.stats["batches"] += 1
        self.stats["max_batch_size"] = max(self.stats["max_batch_size"], len(items))
        return True

    def _is_done(self, handle):
        return handle.query()

    def _overflowed(self, p):
        return int(p.status_host[0]) != 0

    def _finish(self, req, p, now_fn):
        if self._overflowed(p):
            self._rerender(req, p)
        req.done = now_fn()
        p.busy = False
        self.n_busy -= 1

    def _poll(self, now_fn):
        done = []
        if self.mode == "request":
            still = []
            for item in self.inflight:
                req, slot, p, handle = item
                if self._is_done(handle):
                    self._finish(req, p, now_fn)
                    self.free_slots.append(slot)
                    done.append(req)
                else:
                    still.append(item)
            self.inflight = still
        else:
            still = []
            for item in self.batches:
                bslot, items, handle = item
                if self._is_done(handle):
                    for req, p in items:
                        self._finish(req, p, now_fn)
                        done.append(req)
                    self.free_batch_slots.append(bslot)
                else:
                    still.append(item)
            self.batches = still
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
        # the stale plan (and graph) is dropped; a plan with the new capacity is made on demand
        self.plans[key].remove(p)
        self.resident -= p.nbytes
        del plan

    def serve(self, requests, realtime=True):
        """Serve requests (sorted by arrival). Returns the list with completion times."""
        pending = collections.deque()
        reqs = sorted(requests, key=lambda r: r.arrival)
        i, n_done = 0, 0
        self._sync()
        self._serving = True
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
            if self.mode == "batch":
                progressed |= self._maybe_launch_batch()
            done = self._poll(now)
            n_done += len(done)
            if not progressed and not done:
                self._idle()
        self._serving = False
        return reqs


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


def latency_report(reqs, warmup=0.0):
    """p50/p99/mean/max latency (ms) of the requests arriving at or after `warmup` seconds, and
    Mpix/s over the same requests (their pixels over the span from the first arrival to the
    last completion)."""
    reqs = [r for r in reqs if r.arrival >= warmup]
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

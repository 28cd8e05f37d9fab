"""The render server on an MI355X: requests overlapping on the device (batched into persistent
launches, or one graph replay per request) give the same image as each request rendered alone
(and as the oracle); a memory budget that binds evicts idle plans and keeps every result."""
import numpy as np
import pytest

import oracle
import synth
from parity import e2e_bound, gather, pixel_match, report_failures, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _scenes():
    import paper_2506_13348_amd as P
    P._ffi.lib()
    raw = [synth.make_scene("sq100k", seed=21, n=8000, env_res=32),
           synth.make_scene("shell2k", seed=22, n=1500)]
    raw[0]["env_levels"] = 3
    return raw, [P.DeviceScene.from_dict(r, device="cuda") for r in raw]


def _trace(rng, n, res):
    out = []
    for i in range(n):
        s = int(rng.integers(2))
        W, H = res[int(rng.integers(len(res)))]
        cam = synth.serving_camera("superquadric", W, H, rng.uniform(0, 6.283), rng.uniform(0, 40))
        if s == 1:
            cam = synth.look_at_camera((0.3 * rng.normal(), 0.3 * rng.normal(), 3.0), (0, 0, 0), W, H)
        out.append((0.0005 * i, s, (W, H), cam))
    return out


@pytest.mark.parametrize("mode", ["batch", "request"])
def test_requests_in_the_mix_equal_requests_alone(mode):
    import paper_2506_13348_amd as P
    from paper_2506_13348_amd.serve import Request, Server
    print(f"serve mix, mode {mode}", flush=True)
    raw, scenes = _scenes()
    rng = np.random.default_rng(5)
    res = [(64, 64), (96, 80), (128, 128)]
    trace = _trace(rng, 40, res)
    samples = {}
    for t, s, (W, H), cam in trace:
        samples.setdefault((s, W, H), []).append(cam)
    srv = Server(scenes, slots=4, capacity_samples=samples, keep_outputs=True, mode=mode)
    srv.prepare([((s, W, H), c[0]) for (s, W, H), c in samples.items()], per_key=2)
    reqs = [Request(i, t, s, wh[0], wh[1], cam) for i, (t, s, wh, cam) in enumerate(trace)]
    srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    assert srv.stats["max_inflight"] >= 2, srv.stats
    if mode == "batch":
        # all requests arrive at once: some launch carried several of them
        assert srv.stats["max_batch_size"] >= 2 and srv.stats["batches"] < len(reqs), srv.stats
    assert srv.stats["graph_replays"] >= len(reqs) - srv.stats["overflow_retries"]
    n_exact = 0
    for r in reqs:
        alone = P.render(scenes[r.scene], [r.cam], r.width, r.height)["rgba"][0]
        d = (alone - r.output).abs()
        assert float(d[..., :3].max()) <= 1e-4 and float(d[..., 3].max()) <= 1e-5
        n_exact += int(torch.equal(alone, r.output))
    print(f"[serve] {len(reqs)} requests, {n_exact} bit-identical alone vs mix, stats {srv.stats}")
    assert n_exact == len(reqs)
    # two of them against the oracle: the same request rendered with G-buffers gives the
    # served RGBA bit for bit, and its G-buffer and shading pass the two-stage check
    for r in reqs[:2]:
        full = P.render(scenes[r.scene], [r.cam], r.width, r.height, gbuf=True)
        assert torch.equal(full["rgba"][0], r.output)
        pix = sample_pixels(np.random.default_rng(r.rid), r.width, r.height, 40)
        ref = oracle.render(raw[r.scene], r.cam, pixels=pix)
        rgba, gb = gather(full, 0, pix)
        tabs = oracle.tables(raw[r.scene]["env"], raw[r.scene]["env_levels"])
        ok, info = pixel_match(rgba, gb, ref, r.cam, pix, tabs)
        print(info)
        report_failures(ok, pix, rgba, gb, ref)
        assert info["fail"] == 0 and e2e_bound(info), info


def test_a_binding_memory_budget_evicts_idle_plans():
    """A budget of about two plans over six (scene, resolution) keys: idle plans are evicted
    least recently used first, resident plan bytes never exceed the budget, and every request
    still equals the same request rendered alone."""
    import paper_2506_13348_amd as P
    from paper_2506_13348_amd.serve import Request, Server, plan_bytes
    raw, scenes = _scenes()
    rng = np.random.default_rng(8)
    res = [(64, 64), (96, 80), (128, 128)]
    trace = _trace(rng, 30, res)
    samples = {}
    for t, s, (W, H), cam in trace:
        samples.setdefault((s, W, H), []).append(cam)
    srv = Server(scenes, slots=2, capacity_samples=samples, keep_outputs=True, mode="batch")
    sizes = {k: srv._plan_size(*k) for k in samples}
    srv.mem_budget = 2 * max(sizes.values()) + 1024
    reqs = [Request(i, t, s, wh[0], wh[1], cam) for i, (t, s, wh, cam) in enumerate(trace)]
    srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    print(f"[serve budget] budget {srv.mem_budget} stats {srv.stats}", flush=True)
    assert srv.stats["evictions"] > 0
    assert srv.stats["max_resident"] <= srv.mem_budget
    # the byte count a plan is admitted with is the bytes it holds
    for ps in srv.plans.values():
        for p in ps:
            assert p.nbytes == plan_bytes(p.plan) == sizes[p.key]
    for r in reqs:
        alone = P.render(scenes[r.scene], [r.cam], r.width, r.height)["rgba"][0]
        assert torch.equal(alone, r.output)


def test_pair_overflow_is_rerendered():
    import paper_2506_13348_amd as P
    from paper_2506_13348_amd.serve import Request, Server
    raw, scenes = _scenes()
    cam = synth.serving_camera("superquadric", 128, 128, 0.3, 10.0)
    srv = Server(scenes, slots=2, capacity_samples={(0, 128, 128): [cam]}, keep_outputs=True)
    srv.capacity[(0, 128, 128)] = 64          # far too small: the graph's lists overflow
    reqs = [Request(0, 0.0, 0, 128, 128, cam)]
    srv.serve(reqs, realtime=False)
    assert srv.stats["overflow_retries"] == 1 and reqs[0].retried
    alone = P.render(scenes[0], [cam], 128, 128)["rgba"][0]
    assert torch.equal(alone, reqs[0].output)


def test_serving_scenes_with_the_indirect_term_and_xy_normals():
    """Resident scenes of the other kinds in the same server: one with per-splat SH (the
    indirect evaluation captured in the graph), one with the two-component normal atlas;
    every request equals the same request rendered alone, bit for bit."""
    import paper_2506_13348_amd as P
    from paper_2506_13348_amd.serve import Request, Server
    P._ffi.lib()
    a = synth.make_scene("shell2k", seed=23, n=1200)
    a["sh"] = synth.indirect_sh(np.random.default_rng(1), 1200, 2)
    a["sh_degree"] = 2
    b = synth.make_scene("shell2k", seed=24, n=900)
    scenes = [P.DeviceScene.from_dict(a, device="cuda"),
              P.DeviceScene.from_dict(b, device="cuda", tex_format=1)]
    rng = np.random.default_rng(6)
    trace = _trace(rng, 20, [(64, 64), (96, 80)])
    samples = {}
    for t, s, (W, H), cam in trace:
        samples.setdefault((s, W, H), []).append(cam)
    srv = Server(scenes, slots=3, capacity_samples=samples, keep_outputs=True)
    srv.prepare([((s, W, H), c[0]) for (s, W, H), c in samples.items()], per_key=2)
    reqs = [Request(i, t, s, wh[0], wh[1], cam) for i, (t, s, wh, cam) in enumerate(trace)]
    srv.serve(reqs, realtime=False)
    torch.cuda.synchronize()
    assert srv.stats["graph_replays"] >= len(reqs) - srv.stats["overflow_retries"]
    for r in reqs:
        alone = P.render(scenes[r.scene], [r.cam], r.width, r.height)["rgba"][0]
        assert torch.equal(alone, r.output), (r.scene, r.width, r.height)
    print(f"[serve variants] {len(reqs)} requests bit-identical alone vs mix, stats {srv.stats}")

"""Batched persistent raster launches (ts_raster_batch): every job of a batch (its own scene,
views, resolution and outputs) comes out bit for bit equal to the same render by
ts_raster_fwd, for batches of mixed scenes and ragged resolutions, batches launched back to
back (the work counters reset themselves), an empty batch, and batches replayed from one
captured graph with new tables written between the replays. One job is also checked against
the oracle in two stages."""
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
    raw = [synth.make_scene("sq100k", seed=31, n=8000, env_res=32),
           synth.make_scene("shell2k", seed=32, n=1500),
           synth.make_scene("sq100k", seed=33, n=3000, tex_res=4, env_res=16)]
    raw[0]["env_levels"] = 3
    return raw, [P.DeviceScene.from_dict(r, device="cuda") for r in raw]


def _jobs(scenes, rng):
    """(scene index, cameras, W, H) of a mixed batch: ragged sizes, one two-view job."""
    out = []
    for s, (W, H), nv in [(0, (64, 64), 1), (1, (96, 80), 1), (2, (130, 70), 2), (0, (47, 33), 1),
                          (1, (128, 128), 1), (2, (64, 64), 1)]:
        geo = "superquadric" if s != 1 else "shell"
        cams = [synth.serving_camera("superquadric", W, H, rng.uniform(0, 6.283),
                                     rng.uniform(0, 40)) for _ in range(nv)]
        if geo == "shell":
            cams = [synth.look_at_camera((0.3 * rng.normal(), 0.3 * rng.normal(), 3.0), (0, 0, 0),
                                         W, H) for _ in range(nv)]
        out.append((s, cams, W, H))
    return out


def _plans(scenes, jobs):
    import paper_2506_13348_amd as P
    plans, refs = [], []
    for s, cams, W, H in jobs:
        ref = P.render(scenes[s], cams, W, H, aux=True)
        pl = ref["plan"]
        refs.append((ref["rgba"].clone(), ref["t_final"].clone()))
        pl.rgba.fill_(-1.0)
        pl.t_final.fill_(-1.0)
        plans.append(pl)
    torch.cuda.synchronize()
    return plans, refs


def _check_equal(plans, refs, which):
    torch.cuda.synchronize()
    for k in which:
        rgba, tf = refs[k]
        assert torch.equal(plans[k].rgba.view_as(rgba), rgba), f"job {k}: rgba differs"
        assert torch.equal(plans[k].t_final.view_as(tf), tf), f"job {k}: t_final differs"


def _clear(plans):
    for p in plans:
        p.rgba.fill_(-1.0)
        p.t_final.fill_(-1.0)


def test_batched_launch_equals_single_renders():
    import paper_2506_13348_amd as P
    raw, scenes = _scenes()
    rng = np.random.default_rng(3)
    jobs = _jobs(scenes, rng)
    print(f"batch of {len(jobs)} jobs: " + ", ".join(f"s{s} {W}x{H}x{len(c)}" for s, c, W, H in jobs),
          flush=True)
    plans, refs = _plans(scenes, jobs)
    br = P.BatchRaster(slots=2, use_graphs=False)
    br.launch(0, [p.raster_job() for p in plans])
    _check_equal(plans, refs, range(len(plans)))
    # back to back on the same queue: a subset in another order, then an empty batch
    _clear(plans)
    order = [4, 0, 2]
    br.launch(0, [plans[k].raster_job() for k in order])
    br.launch(0, [])
    _check_equal(plans, refs, order)
    for k in set(range(len(plans))) - set(order):
        assert float(plans[k].rgba.max()) == -1.0, "a job outside the batch was written"
    # the work counters are back at zero
    assert int(br.queue[0].abs().sum()) == 0


def test_batched_graph_replays_take_new_tables():
    import paper_2506_13348_amd as P
    raw, scenes = _scenes()
    rng = np.random.default_rng(4)
    jobs = _jobs(scenes, rng)
    plans, refs = _plans(scenes, jobs)
    br = P.BatchRaster(slots=2, use_graphs=True)
    batches = [[0, 1, 2], [3, 4, 5], [5, 0], list(range(len(plans)))]
    for rep, which in enumerate(batches):
        print(f"graph replay {rep}: jobs {which}", flush=True)
        _clear(plans)
        torch.cuda.synchronize()
        br.launch(rep % 2, [plans[k].raster_job() for k in which])
        torch.cuda.synchronize()
        _check_equal(plans, refs, which)
        # eager work of the program between replays
        _ = (plans[0].rgba * 2.0).sum().item()
    assert all(int(q.abs().sum()) == 0 for q in br.queue)


def test_batched_job_against_the_oracle():
    import paper_2506_13348_amd as P
    raw, scenes = _scenes()
    rng = np.random.default_rng(5)
    jobs = _jobs(scenes, rng)
    plans, refs = _plans(scenes, jobs)
    br = P.BatchRaster(slots=1, use_graphs=False)
    br.launch(0, [p.raster_job() for p in plans])
    torch.cuda.synchronize()
    k = 2                                    # the two-view ragged job (130x70)
    s, cams, W, H = jobs[k]
    full = P.render(scenes[s], cams, W, H, gbuf=True)
    assert torch.equal(full["rgba"].reshape(-1), plans[k].rgba)
    for v in range(len(cams)):
        pix = sample_pixels(np.random.default_rng(v), W, H, 60)
        ref = oracle.render(raw[s], cams[v], pixels=pix)
        rgba, gb = gather(full, v, pix)
        tabs = oracle.tables(raw[s]["env"], raw[s]["env_levels"])
        ok, info = pixel_match(rgba, gb, ref, cams[v], pix, tabs)
        report_failures(ok, pix, rgba, gb, ref)
        assert info["fail"] == 0 and e2e_bound(info), info


def test_batch_encode_refuses_variants_and_too_many_jobs():
    import paper_2506_13348_amd as P
    from paper_2506_13348_amd import _ffi as F
    raw, scenes = _scenes()
    plan = P.RenderPlan(scenes[1], [synth.look_at_camera((0, 0, 3.0), (0, 0, 0), 32, 32)], 32, 32)
    job = plan.raster_job()
    host = torch.empty(F.ts_raster_batch_table_bytes(), dtype=torch.uint8)
    with pytest.raises(RuntimeError, match="bad argument"):
        F.ts_raster_batch_encode([job] * 65, host)
    job.params.sampler = F.SAMPLER_TRILINEAR
    with pytest.raises(RuntimeError, match="default atlas path"):
        F.ts_raster_batch_encode([job], host)

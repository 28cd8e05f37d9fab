"""Throughput of the textured planar-Gaussian render on one MI355X.

Headline step (the JSON line's value): the 100,000-splat superquadric scene with 8x8 textures
per primitive, rendered from all 64 orbit cameras at 800x800 (preprocess -> depth sort + tile
lists -> raster with texture sampling, normal mapping, G-buffer blending and fused split-sum
shading), inputs and shading tables resident in HBM.

Further legs, reported in the same JSON object: the step with locality-packed charts;
forward+backward training steps (300k splats x 8 views at 800x800, and the 1M-splat
1600x1064 unbounded frame); the 2k-splat 128x128 frame's latency; texture-sampling cost
against the untextured primitive (the paper's Tab. 3); the serving loop against sequential
renders; and the FP64 oracle timed on a bounded pixel sample on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-fwd-bwd]
                  [--no-tab3] [--no-serving] [--serving-seconds S] [--profile-run | --profile-train]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd and fwd+bwd vs plain at 1e-4 tol; serving p50/p99 latency"
# FP32 operations of one blended splat-pixel evaluation in the definition (FMA = 2):
# (u,v) 17, Gaussian 5, alpha/transmittance/weight 5, texel coordinates 8, bilinear
# weights 6 + 8 channels x 7, normal normalisation 9, rotation 15, accumulation 16.
FLOPS_PER_BLEND = 137
# MI355X's published fp32 vector peak (packed-fp32 instructions: two lanes' worth per issue)
PEAK_FP32 = 157.3
# the same without packed-fp32 instructions, which this build does not emit:
# 256 CU x 64 lanes x 2 flops x 2.4 GHz
PEAK_FP32_UNPACKED = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_fwd(scene, cam, pix, threads, tabs=None):
    """Seconds and contributing evaluations of the oracle forward on pixels pix."""
    import oracle
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    out = oracle.render(scene, cam, pixels=pix, tabs=tabs)
    return time.perf_counter() - t0, float(out["stat"][:, 0].sum())


def _oracle_fwd_bwd(scene, cam, pix, threads, tabs):
    """Seconds of the float64 forward + backward (dense autograd reference) on pixels pix."""
    import numpy as np
    import torch
    from oracle import grad as og
    torch.set_num_threads(threads)
    d = np.random.default_rng(1).normal(size=(len(pix), 4))
    t0 = time.perf_counter()
    og.grads(scene, cam, pix, d, tabs)
    return time.perf_counter() - t0


def cpu_baseline(scene, cam, n_pix=200000, seed=0):
    """The FP64 oracle timed on the host cores. Headline value: the forward on a bounded random
    sample of pixels of one view of the headline scene (tables precomputed), every thread.
    Beside it (about 20 s more of oracle work): the same view on one core, the 2k-splat
    128x128 frame in full, a pixel sample of the 1M-splat unbounded frame, and forward +
    backward (the float64 reference gradients) on the 64x64 crop of 500 splats and on a pixel
    sample of a 300k-splat training view."""
    import numpy as np
    import oracle
    import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = oracle.set_threads(threads)
    tabs = oracle.tables(scene["env"], scene["env_levels"])
    rng = np.random.default_rng(seed)

    def sample(c, k):
        return np.stack([rng.integers(0, c["width"], k), rng.integers(0, c["height"], k)],
                        1).astype(np.int32)

    pix = sample(cam, n_pix)
    dt, ev = _oracle_fwd(scene, cam, pix, threads, tabs)
    detail = {}
    k1 = 3000
    log("cpu baseline: one core ...")
    dt1, ev1 = _oracle_fwd(scene, cam, pix[:k1], 1, tabs)
    detail["sq100k_view0_fwd_1core"] = {"pixels": k1, "s": round(dt1, 2),
                                        "mpix_per_s": round(k1 / dt1 / 1e6, 6),
                                        "evals_per_s": round(ev1 / dt1, 1)}
    s1 = synth.make_scene("shell2k")
    c1 = synth.config_cameras("shell2k")[0]
    t1 = oracle.tables(s1["env"], s1["env_levels"])
    full = oracle.all_pixels(c1["width"], c1["height"])
    for th in (threads, 1):
        d1, e1 = _oracle_fwd(s1, c1, full, th, t1)
        detail[f"shell2k_frame_fwd_{th}threads"] = {"ms_per_frame": round(d1 * 1e3, 2),
                                                    "mpix_per_s": round(len(full) / d1 / 1e6, 4),
                                                    "evals_per_s": round(e1 / d1, 1)}
    log("cpu baseline: 1M-splat frame sample ...")
    s4 = synth.make_scene("field1m")
    c4 = synth.config_cameras("field1m")[0]
    k4 = 2000
    # G-buffers only: the FP64 prefiltering of this scene's 256^2 environment alone takes
    # minutes on the host, and shading is a small part of a pixel's oracle work
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    o4 = oracle.render(s4, c4, pixels=sample(c4, k4), shade=False)
    d4 = time.perf_counter() - t0
    e4 = float(o4["stat"][:, 0].sum())
    detail["field1m_fwd_sample_gbuffers"] = {"pixels": k4, "of": "1600x1064, 1M splats",
                                             "s": round(d4, 2),
                                             "mpix_per_s": round(k4 / d4 / 1e6, 6),
                                             "evals_per_s": round(e4 / d4, 1)}
    del s4, o4
    log("cpu baseline: float64 forward + backward ...")
    s3 = synth.make_scene("sq300k_train")
    c3 = synth.config_cameras("sq300k_train")[0]
    t3 = oracle.tables(s3["env"], s3["env_levels"])
    log("cpu baseline: tables ready")
    crop, ccam = synth.fd_crop_scene(s3, c3, 368, 368, 64, 64, n_keep=500)
    cpix = oracle.all_pixels(64, 64)
    for th in (threads, 1):
        dc = _oracle_fwd_bwd(crop, ccam, cpix, th, t3)
        detail[f"crop64_500splats_fwd_bwd_{th}threads"] = {
            "s": round(dc, 3), "mpix_per_s": round(len(cpix) / dc / 1e6, 5)}
    k3 = 32
    d3 = _oracle_fwd_bwd(s3, c3, sample(c3, k3), threads, t3)
    detail["sq300k_view0_fwd_bwd_sample"] = {"pixels": k3, "of": "800x800, 300k splats",
                                             "s": round(d3, 2),
                                             "mpix_per_s": round(k3 / d3 / 1e6, 8)}
    oracle.set_threads(threads)
    return {"value": round(n_pix / dt / 1e6, 6), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_pix} random pixels of orbit view 0 (800x800, 100k splats), "
                      f"{dt:.1f} s, shading tables precomputed",
            "evals_per_s": round(ev / dt, 1),
            "host": {"cpu_model": _cpu_model(), "cpus_visible": os.cpu_count()},
            "detail": detail}


FWD_BWD_WORKLOADS = {
    "sq300k_train": "sq300k: 300k splats T=8, 8 orbit views 800x800 per step, L1 to a seeded "
                    "U(0,1) target, gradients to means/quats/scales/opacity/texels",
    "field1m": "field1m: 1M splats T=8 (height field + boxes + far shell), one 1600x1064 view "
               "per step, 256^2 env with 4 levels, L1 to a seeded U(0,1) target, gradients to "
               "means/quats/scales/opacity/texels",
}


def bench_fwd_bwd(cfg, steps, warmup, sh_degree=None, mips=False, charts=False):
    """One training step: forward of the config's batch of views, L1 loss to a seeded target,
    hand-written backward to all splat parameters. With sh_degree, the indirect term is on
    (per-splat SH of that degree, mixed visibility) and the SH coefficients get gradients;
    with mips, the atlas holds each chart's mip chain and sampling is trilinear (gradients to
    the level-0 texels and, through the level, to the geometry); with charts, each splat's
    chart has its own side by primitive size (1..8, through a chart table)."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan
    from paper_2506_13348_amd.autograd import BackwardRunner

    sc = synth.make_scene(cfg)
    cams = synth.config_cameras(cfg)
    V, W, H = len(cams), cams[0]["width"], cams[0]["height"]
    vis = None
    if sh_degree is not None:
        sc["sh"] = synth.indirect_sh(np.random.default_rng(11), len(sc["opac"]), sh_degree)
        sc["sh_degree"] = sh_degree
        vis = torch.as_tensor(synth.visibility(np.random.default_rng(12), V, H, W)).cuda()
    kw = dict(mips=mips)
    if charts:
        log2 = synth.texture_sides(sc["scales"], base_log2=3, max_log2=3)
        sc["textures"] = synth.adaptive_textures(np.random.default_rng(3), log2)
        kw["chart_log2"] = log2
    ds = DeviceScene.from_dict(sc, device="cuda", **kw)
    del sc
    target = torch.as_tensor(synth.target_image(W, H, seed=1, n_views=V)).cuda()
    plan = RenderPlan(ds, cams, W, H, gbuf=True, aux=True, vis=vis)
    run = BackwardRunner(plan)
    grads = (torch.empty_like(ds.means), torch.empty_like(ds.quats), torch.empty_like(ds.scales),
             torch.empty_like(ds.opac), torch.empty_like(ds.atlas))
    if sh_degree is not None:
        grads = grads + (torch.empty_like(ds.sh),)
    d_rgba = torch.zeros(V, H, W, 4, device="cuda")
    inv_n = 1.0 / (V * H * W * 3)

    def step(retry):
        plan.run()
        rgb = plan.rgba.view(V, H, W, 4)[..., :3]
        loss = (rgb - target).abs().sum() * inv_n
        d_rgba[..., :3] = torch.sign(rgb - target) * inv_n
        run.run(d_rgba, grads, 0.0, retry=retry)
        return loss

    for _ in range(max(warmup, 1)):
        step(True)
    plan.check()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        plan.run()
        ev[k][1].record()
        rgb = plan.rgba.view(V, H, W, 4)[..., :3]
        d_rgba[..., :3] = torch.sign(rgb - target) * inv_n
        run.run(d_rgba, grads, 0.0, retry=False)
        ev[k][2].record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    plan.check()
    if int(run.status.item()) != 0:
        raise RuntimeError("backward partial buffer overflow in the timed steps")
    fwd_ms = float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]))
    bwd_ms = float(np.mean([ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]))
    # gradients of the same loss w.r.t. the environment-table texels (learnable environment),
    # timed on their own after the step
    from paper_2506_13348_amd.autograd import EnvBackward
    eb = EnvBackward(plan)
    eb.run(d_rgba)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        eb.run(d_rgba)
    e1.record()
    torch.cuda.synchronize()
    env_ms = e0.elapsed_time(e1) / 3
    del eb
    ind_ms = None
    if sh_degree is not None:
        # ts_indirect_bwd alone (the last kernel of the step's backward)
        from paper_2506_13348_amd import _ffi as F
        e0.record()
        for _ in range(3):
            F.ts_indirect_bwd(V, plan.cams, ds.n, ds.means, ds.quats, ds.sh, sh_degree, plan.lind,
                              run.d_lind, 0.0, grads[5], grads[0], grads[1], plan.stream)
        e1.record()
        torch.cuda.synchronize()
        ind_ms = e0.elapsed_time(e1) / 3
    # algorithmic HBM bytes of two backward kernels, for their rooflines (k_bwd_gather's
    # duration comes from the kernel trace, ts_env_bwd's from the events above)
    used = int(run.used.item())
    gather_bytes = (used * 4 + plan.cap * 16 + V * ds.n * (16 + 8) + V * ds.n * 19 * 4
                    + ds.atlas.numel() * 4)
    env_bytes = V * W * H * (32 + 4 + 16) + (0 if vis is None else V * W * H * 4)
    env_gbs = env_bytes / (env_ms * 1e-3) / 1e9
    out = {"value": round(V * W * H / dt / 1e6, 2), "unit": "Mpix/s",
           "ms_per_step": round(dt * 1e3, 3), "steps": steps, "views_per_step": V,
           "width": W, "height": H, "splats": ds.n,
           "per_phase_ms": {"forward": round(fwd_ms, 3), "loss_and_backward": round(bwd_ms, 3)},
           "workload": FWD_BWD_WORKLOADS[cfg] + (
               "" if sh_degree is None else
               f"; indirect term: degree-{sh_degree} SH per splat, mixed visibility, gradients "
               "to the SH coefficients too") + (
               "; trilinear sampling over each chart's box-filtered mip chain" if mips else "") + (
               "; per-splat chart sides 1..8 by primitive size through a chart table"
               if charts else ""),
           "env_tables_bwd_ms": round(env_ms, 3),
           # G-buffers, transmittance, dL/dC (and visibility) read once per pixel; the tables'
           # gradients are a few MB
           "env_tables_bwd_hbm": {"algorithmic_bytes": env_bytes, "achieved": round(env_gbs, 1),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(env_gbs / HBM_PEAK_GBS, 4)},
           # partials and slot table read once, rectangles and offsets, record and texel
           # gradients written once
           "bwd_gather_algorithmic_bytes": gather_bytes,
           "partial_buffer_floats_used": used}
    if ind_ms is not None:
        out["indirect_bwd_ms"] = round(ind_ms, 4)
    del plan, run, grads, d_rgba, target, ds
    torch.cuda.empty_cache()
    return out


def bench_unfused_shade(ds, cams, W, H, cap, reps=10):
    """ts_shade on its own over the headline step's G-buffers (64 views x 800x800): per pixel
    32 B of G-buffer + 4 B of transmittance read and 16 B of RGBA written (the tables, a few
    MB, stay cache resident); HBM-bound. Its duration: `reps` launches back to back."""
    import torch
    from paper_2506_13348_amd import RenderPlan
    from paper_2506_13348_amd import _ffi as F
    plan = RenderPlan(ds, cams, W, H, gbuf=True, pair_capacity=cap)
    plan.run()
    plan.check()
    V = len(cams)
    env = ds.tables.struct

    def shade():
        F.ts_shade(V, W, H, plan.cams, plan.params, env, plan.gbuf, plan.t_final, plan.rgba)

    shade()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        shade()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = V * W * H * (32 + 4 + 16)
    gbs = nbytes / (ms / 1e3) / 1e9
    del plan
    torch.cuda.empty_cache()
    return {"kernel": "k_shade", "bound": "hbm", "algorithmic_bytes": nbytes,
            "ms_per_launch": round(ms, 4), "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def bench_indirect(sc, cams, W, H, cap, steps, warmup, degree=3):
    """The forward step with the indirect term (Eq. 9, Eq. 12): per-splat SH of degree 3
    evaluated per view, the blended L_ind map and the visibility mix in the fused shading,
    on the same scene and views as the headline step. Visibility is a seeded per-pixel input
    (mesh ray tracing is not part of the path)."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan
    dev = torch.device("cuda:0")
    V = len(cams)
    sci = dict(sc)
    sci["sh"] = synth.indirect_sh(np.random.default_rng(11), len(sc["opac"]), degree)
    sci["sh_degree"] = degree
    vis = torch.as_tensor(synth.visibility(np.random.default_rng(8), V, H, W)).to(dev)
    ds = DeviceScene.from_dict(sci, device=dev)
    plan = RenderPlan(ds, cams, W, H, pair_capacity=cap, vis=vis)
    for _ in range(warmup):
        plan.run()
    plan.check()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        plan.preprocess()
        ev[k][1].record()
        plan.indirect_eval()
        ev[k][2].record()
        plan.bin_sort()
        ev[k][3].record()
        plan.raster()
        ev[k][4].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    plan.check()
    ph = [float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)]))
          for i in range(4)]
    n = ds.n
    K = (degree + 1) ** 2
    # algorithmic bytes of one ts_indirect_eval launch: centres, quaternions and coefficients
    # read once, one float4 per (view, splat) written
    ind_bytes = n * (12 + 16 + 12 * K) + V * n * 16
    # the kernel's own duration: 20 launches back to back on the plan's stream (inside the
    # step the phase events also catch the launch gap between kernels)
    s = plan.stream if plan.stream is not None else torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record()
        for _ in range(20):
            plan.indirect_eval()
        e1.record()
    torch.cuda.synchronize()
    ind_ms = e0.elapsed_time(e1) / 20
    gbs = ind_bytes / (ind_ms / 1e3) / 1e9
    return {"workload": f"sq100k forward with the indirect term: degree-{degree} SH per splat, "
                        "per-pixel visibility (40% 1, 30% 0, 30% U(0,1))",
            "ms_per_step": round(ms, 3), "mpix_per_s": round(V * W * H / (ms / 1e3) / 1e6, 2),
            "per_kernel_ms": {"preprocess": round(ph[0], 4), "indirect_eval": round(ph[1], 4),
                              "bin_sort": round(ph[2], 4), "raster_fwd_shade": round(ph[3], 4)},
            "indirect_eval_roofline": {"bound": "hbm", "achieved": round(gbs, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(gbs / HBM_PEAK_GBS, 4),
                                       "algorithmic_bytes": ind_bytes,
                                       "ms_per_launch": round(ind_ms, 4)}}


def bench_atlas_variants(sc, cams, W, H, cap, steps, base_ms, base_bytes):
    """The headline step with the atlas variants: two-component normals (7-float texels),
    trilinear sampling over mip chains, per-splat resolutions by primitive size (sides 1..8:
    the median splat keeps 8 x 8, smaller ones get fewer texels; texture_sides), and the last
    two combined with two-component normals."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan
    dev = torch.device("cuda:0")
    V = len(cams)
    log2 = synth.texture_sides(sc["scales"], base_log2=3, max_log2=3)
    flat = synth.adaptive_textures(np.random.default_rng(3), log2)
    cases = {
        "normals_xy": (sc, dict(tex_format=1)),
        "trilinear": (sc, dict(mips=True)),
        "normals_xy_trilinear": (sc, dict(tex_format=1, mips=True)),
        "adaptive_sides": (dict(sc, textures=flat), dict(chart_log2=log2)),
        "adaptive_sides_xy_trilinear": (dict(sc, textures=flat),
                                        dict(chart_log2=log2, tex_format=1, mips=True)),
    }
    out = {"default": {"ms_per_step": round(base_ms, 3), "atlas_mb": round(base_bytes / 1e6, 1)}}
    for name, (scn, kw) in cases.items():
        ds = DeviceScene.from_dict(scn, device=dev, **kw)
        plan = RenderPlan(ds, cams, W, H, pair_capacity=cap)
        plan.run()
        plan.check()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        plan.check()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"ms_per_step": round(ms, 3),
                     "mpix_per_s": round(V * W * H / (ms / 1e3) / 1e6, 2),
                     "atlas_mb": round(ds.atlas.numel() * 4 / 1e6, 1),
                     "vs_default": round(base_ms / ms, 3)}
        del plan, ds
        torch.cuda.empty_cache()
    out["mean_texels_adaptive"] = round(float(np.mean((1 << log2) ** 2)), 2)
    return out


def bench_small_frame(reps=200):
    """The 2,000-splat shell, one 128x128 view, T = 4: a launch-latency-bound frame; median
    of per-frame times over reps renders."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan

    sc = synth.make_scene("shell2k")
    cams = synth.config_cameras("shell2k")
    ds = DeviceScene.from_dict(sc, device="cuda")
    plan = RenderPlan(ds, cams, 128, 128)
    for _ in range(10):
        plan.run()
    plan.check()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        plan.run()
        e1.record()
    torch.cuda.synchronize()
    ts = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    med = float(np.median(ts))
    # the same frame replayed from a HIP graph (as the serving loop does): one launch per frame
    eager = plan.rgba.clone()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        plan.run()
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        plan.run()
    stream.synchronize()
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    with torch.cuda.stream(stream):
        for e0, e1 in gev:
            e0.record()
            graph.replay()
            e1.record()
    torch.cuda.synchronize()
    gts = np.array([e0.elapsed_time(e1) for e0, e1 in gev])
    gmed = float(np.median(gts))
    if not torch.equal(plan.rgba, eager):
        raise RuntimeError("graph replay of the small frame differs from the eager render")
    return {"workload": "shell2k: 2k splats T=4, one 128x128 view, 32^2 env",
            "median_us": round(med * 1e3, 1), "p90_us": round(float(np.percentile(ts, 90)) * 1e3, 1),
            "mpix_per_s": round(128 * 128 / (med / 1e3) / 1e6, 2),
            "graph_replay_median_us": round(gmed * 1e3, 1),
            "graph_replay_mpix_per_s": round(128 * 128 / (gmed / 1e3) / 1e6, 2)}


def bench_tab3(steps=5):
    """Texture-sampling cost as in the paper's Tab. 3: the same 100k-splat superquadric
    geometry and 64 orbit views rendered untextured (one attribute per splat) and with
    software-bilinear textures at T = 2, 4, 8, 16; frame-rate ratios to the untextured run."""
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan

    cams = synth.config_cameras("sq100k")

    def timed(T, sampler):
        sc = synth.make_scene("sq100k", tex_res=T)
        ds = DeviceScene.from_dict(sc, device="cuda")
        del sc
        plan = RenderPlan(ds, cams, 800, 800, params={"sampler": sampler})
        plan.run()
        plan.check()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        plan.check()
        return e0.elapsed_time(e1) / steps

    base = timed(1, 1)
    out = {"workload": "sq100k geometry, 64 views 800x800 per step", "untextured_ms": round(base, 3),
           "T": [], "bilinear_ms": [], "fps_ratio_bilinear": []}
    for T in (2, 4, 8, 16):
        ms = timed(T, 0)
        out["T"].append(T)
        out["bilinear_ms"].append(round(ms, 3))
        out["fps_ratio_bilinear"].append(round(base / ms, 3))
        torch.cuda.empty_cache()
    out["hardware_sampler"] = "unavailable: the gfx950 toolchain has no image/texture instructions"
    out["paper_tab3_rtx_a6000"] = {"software_bilinear": [0.90, 0.86, 0.85, 0.79],
                                   "hardware_texture_atlas": [0.92, 0.93, 0.94, 0.91]}
    return out


def bench_serving(duration, rate=200.0, warm=3.0, saturation=300):
    """Serving: 4 resident scenes (50k, 200k, 500k superquadric splats, 1M height-field
    splats; T=8), a seeded Poisson stream at `rate` req/s for `duration` s (latencies of the
    first `warm` s excluded), scene uniform, resolution uniform over {256^2, 512^2, 800^2,
    1920x1080}, random orbit cameras. Three ways of serving the same stream: the
    continuous-batching server (front parts on prep streams, each batch rendered by one
    persistent launch replayed from a graph), the per-request server (one graph replay of the
    whole path per request, 4 streams), and the plain renderer one request at a time. Then a
    closed loop (`saturation` requests all arriving at once) gives each one's saturation
    throughput. The plan-cache budget is 3x the bytes of one plan per (scene, resolution): the
    Poisson stream rarely reaches it, the closed loop does (requests then wait for plans of
    their key, or evict idle plans of other keys)."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene
    from paper_2506_13348_amd.serve import Request, Server, latency_report, serve_sequential

    t0 = time.perf_counter()
    scenes, geos = [], []
    for i, (geo, n, seed) in enumerate(synth.SERVING_SCENES):
        raw = synth.serving_scene(i)
        scenes.append(DeviceScene.from_dict(raw, device="cuda"))
        geos.append(geo)
        del raw
    log(f"serving scenes ready in {time.perf_counter() - t0:.1f}s")
    rng = np.random.default_rng(7)
    trace = synth.poisson_requests(rng, rate, duration, len(scenes), synth.SERVING_RESOLUTIONS)
    cams = [synth.serving_camera(geos[s], wh[0], wh[1], az, el) for (t, s, wh, az, el) in trace]
    srng = np.random.default_rng(8)
    samples = {}
    for s in range(len(scenes)):
        for (W, H) in synth.SERVING_RESOLUTIONS:
            samples[(s, W, H)] = [synth.serving_camera(geos[s], W, H, srng.uniform(0, 2 * np.pi),
                                                       srng.uniform(0, 40)) for _ in range(3)]
    capacity, budget = None, None
    servers = {}
    for mode in ("batch", "request"):
        srv = Server(scenes, slots=4, mem_budget=1 << 62, capacity_samples=samples, mode=mode)
        if capacity is not None:
            srv.capacity = dict(capacity)
        for k in samples:
            srv._capacity(*k)
        capacity = dict(srv.capacity)
        if budget is None:
            budget = int(3.0 * sum(srv._plan_size(*k) for k in samples))
        srv.mem_budget = budget
        srv.prepare([(k, v[0]) for k, v in samples.items()], per_key=1)
        servers[mode] = srv
        log(f"{mode} server plans ready in {time.perf_counter() - t0:.1f}s: {srv.stats}")

    def fresh(closed=False):
        if closed:
            return [Request(i, 0.0, s, wh[0], wh[1], cams[i])
                    for i, (t, s, wh, az, el) in enumerate(trace[:saturation])]
        return [Request(i, t, s, wh[0], wh[1], cams[i]) for i, (t, s, wh, az, el) in enumerate(trace)]

    out = {"workload": f"4 resident scenes (50k/200k/500k/1M splats, T=8), Poisson {rate:g} req/s "
                       f"for {duration:g} s (first {warm:g} s excluded from the latencies), "
                       "resolutions 256^2/512^2/800^2/1920x1080, random orbit cameras; "
                       f"closed loop: the first {saturation} requests all at t=0",
           "plan_budget_bytes": budget}
    for mode, srv in servers.items():
        reqs = srv.serve(fresh())
        rep = latency_report(reqs, warm)
        log(f"{mode} server: {rep}")
        sat = latency_report(srv.serve(fresh(closed=True)))
        log(f"{mode} server, closed loop: {sat}")
        out[f"server_{mode}"] = rep
        out[f"server_{mode}_saturation_mpix_per_s"] = sat["mpix_per_s"]
        out[f"server_{mode}_stats"] = dict(srv.stats)
    del servers
    torch.cuda.empty_cache()
    out["raster_launch_forms"] = bench_batch_launch(scenes, geos, capacity)
    log(f"raster launch forms: {out['raster_launch_forms']}")
    seq = serve_sequential(scenes, fresh(), capacity)
    rep_seq = latency_report(seq, warm)
    log(f"sequential: {rep_seq}")
    sat_seq = latency_report(serve_sequential(scenes, fresh(closed=True), capacity))
    out["sequential_plain"] = rep_seq
    out["sequential_plain_saturation_mpix_per_s"] = sat_seq["mpix_per_s"]
    out["p99_speedup_batch_vs_sequential"] = round(rep_seq["p99_ms"] / out["server_batch"]["p99_ms"], 2)
    out["saturation_speedup_batch_vs_sequential"] = round(
        out["server_batch_saturation_mpix_per_s"] / sat_seq["mpix_per_s"], 2)
    return out


def bench_batch_launch(scenes, geos, capacity, reps=20):
    """The raster of 16 requests, one per (scene, resolution) of the serving mix, three ways:
    16 ts_raster_fwd launches on one stream, the same spread over 4 streams, and one
    ts_raster_batch launch (fronts done beforehand; each timed over `reps` repetitions)."""
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import BatchRaster, RenderPlan
    rng = np.random.default_rng(9)
    plans = []
    for s in range(len(scenes)):
        for (W, H) in synth.SERVING_RESOLUTIONS:
            cam = synth.serving_camera(geos[s], W, H, rng.uniform(0, 2 * np.pi), rng.uniform(0, 40))
            p = RenderPlan(scenes[s], [cam], W, H, pair_capacity=capacity[(s, W, H)])
            p.run()
            plans.append(p)
    for p in plans:
        p.check()
    jobs = [p.raster_job() for p in plans]
    br = BatchRaster(slots=1, use_graphs=True)
    streams = [torch.cuda.Stream() for _ in range(4)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def four_streams():
        cur = torch.cuda.current_stream()
        for i, p in enumerate(plans):
            st = streams[i % 4]
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                p.raster()
        for st in streams:
            cur.wait_stream(st)

    t_seq = timed(lambda: [p.raster() for p in plans])
    t_4 = timed(four_streams)
    t_b = timed(lambda: br.launch(0, jobs))
    px = sum(p.W * p.H for p in plans)
    del plans, br
    torch.cuda.empty_cache()
    return {"workload": "raster + shading of 16 requests (4 scenes x 256^2/512^2/800^2/1920x1080)",
            "mpix": round(px / 1e6, 3), "ms_launches_one_stream": round(t_seq, 3),
            "ms_launches_four_streams": round(t_4, 3), "ms_one_batched_launch": round(t_b, 3),
            "batched_speedup_vs_four_streams": round(t_4 / t_b, 2)}


def calibration_copy(dev):
    """A 256 MiB device-to-device copy: the counter reading per byte moved that scales the
    FETCH_SIZE / WRITE_SIZE passes."""
    import torch
    src = torch.empty(64 << 20, device=dev, dtype=torch.float32).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-tab3", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=30.0)
    ap.add_argument("--profile-train", action="store_true",
                    help="only a few forward+backward steps of the 300k-splat training batch "
                         "(for counter collection)")
    ap.add_argument("--locality", action="store_true",
                    help="with --profile-run: the atlas packed in Morton order of the centres")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the forward workload (few steps) plus a 256 MiB device copy that "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2506_13348_amd import DeviceScene, RenderPlan, _ffi

    _ffi.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_train:
        out = bench_fwd_bwd("sq300k_train", args.steps, args.warmup)
        calibration_copy(dev)
        print(json.dumps({"profile_train": True, **out}), flush=True)
        return
    t0 = time.perf_counter()
    sc = synth.make_scene("sq100k")
    cams = synth.config_cameras("sq100k")
    W, H, V = 800, 800, len(cams)
    log(f"scene drawn in {time.perf_counter() - t0:.1f}s")
    ds = DeviceScene.from_dict(sc, device=dev, locality=args.profile_run and args.locality)
    plan = RenderPlan(ds, cams, W, H)
    torch.cuda.synchronize()
    log(f"plan ready: {ds.n} splats, {V} views, pair capacity {plan.cap}")
    for _ in range(args.warmup):
        plan.run()
    n_pairs = plan.check()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(K):
        ev[k][0].record()
        plan.preprocess()
        ev[k][1].record()
        plan.bin_sort()
        ev[k][2].record()
        plan.raster()
        ev[k][3].record()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    plan.check()
    if args.profile_run:
        nbytes = calibration_copy(dev)
        print(json.dumps({"profile_run": True, "steps": K, "views": V,
                          "calibration_copy_bytes": nbytes}), flush=True)
        return
    ms_step = t_total / K * 1e3
    pre_ms = float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)]))
    bin_ms = float(np.mean([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)]))
    ras_ms = float(np.mean([ev[k][2].elapsed_time(ev[k][3]) for k in range(K)]))
    mpix = V * W * H / (ms_step / 1e3) / 1e6
    log(f"step {ms_step:.3f} ms: preprocess {pre_ms:.3f} bin_sort {bin_ms:.3f} raster {ras_ms:.3f}")

    # contributing evaluations of one step, counted by the same kernel (outside the timing)
    aux = RenderPlan(ds, cams, W, H, aux=True, pair_capacity=plan.cap)
    aux.run()
    aux.check()
    n_blend = int(aux.n_blend.to(torch.int64).sum().item())
    del aux
    achieved = n_blend * FLOPS_PER_BLEND / (ras_ms / 1e3) / 1e12
    shade_line = bench_unfused_shade(ds, cams, W, H, plan.cap)
    log(f"unfused shading: {shade_line}")
    # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, only while the
    # kernel's sources are the ones the counters were taken on
    from paper_2506_13348_amd.profiling import read_traffic
    traffic = read_traffic(os.path.join(ROOT, "profiles", "raster_fwd_sq100k_counters.md"),
                           "k_raster_fwd")
    result = {
        "metric": METRIC,
        "value": round(mpix, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sq100k forward: 100k textured planar Gaussians (8x8 texels x 8 "
                               "channels) on a random superquadric, 64 orbit views 800x800, "
                               "128^2 env with 4 prefiltered levels, fused split-sum shading",
                   "views_per_step": V, "width": W, "height": H, "splats": ds.n, "tex_res": 8,
                   "pairs_per_step": n_pairs},
        "evals_per_s": round(n_blend / (ms_step / 1e3), 1),
        "per_kernel_ms": {"preprocess": round(pre_ms, 4), "bin_sort": round(bin_ms, 4),
                          "raster_fwd_shade": round(ras_ms, 4)},
        "roofline": {"kernel": "k_raster_fwd", "bound": "alu",
                     "achieved": round(achieved, 3), "peak": PEAK_FP32,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32, 4),
                     "traffic": traffic,
                     "peak_unpacked": round(PEAK_FP32_UNPACKED, 2),
                     "frac_unpacked": round(achieved / PEAK_FP32_UNPACKED, 4),
                     "note": f"{n_blend} blended evaluations x {FLOPS_PER_BLEND} flops per launch; "
                             "peak = published fp32 vector rate (packed), peak_unpacked = the "
                             "rate without packed-fp32 instructions, which the build disables"},
    }
    result["shade_unfused"] = shade_line
    # the two phases before the raster against HBM, from the same events: k_preprocess reads
    # 40 B of parameters per splat once and writes a 112 B record, 16 B rectangle and 4 B key
    # per (view, splat); ts_bin_sort moves its keys 4 times (16 B each way per key and pass),
    # reads rectangles and ids (2 x 20 B per (view, splat)) and writes 4 B per list entry
    vn = V * ds.n
    for name, nbytes, ms in (("preprocess", 40 * ds.n + 132 * vn, pre_ms),
                             ("bin_sort", 4 * 16 * vn + 2 * 20 * vn + 4 * n_pairs, bin_ms)):
        gbs = nbytes / (ms * 1e-3) / 1e9
        result[f"{name}_hbm"] = {"algorithmic_bytes": nbytes, "ms": round(ms, 4),
                                 "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    # the same step with charts packed in Morton order of the centres (locality-aware atlas),
    # and both packings again with the splats first shuffled into a random order (the order a
    # scene has after densification), where chart order and space are unrelated
    def step_ms(scene, locality):
        ds_l = DeviceScene.from_dict(scene, device=dev, locality=locality)
        plan_l = RenderPlan(ds_l, cams, W, H, pair_capacity=plan.cap)
        for _ in range(2):
            plan_l.run()
        plan_l.check()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            plan_l.run()
        e1.record()
        torch.cuda.synchronize()
        plan_l.check()
        del plan_l, ds_l
        return e0.elapsed_time(e1) / K

    loc_ms = step_ms(sc, True)
    n_s = len(sc["opac"])
    shuf = np.random.default_rng(5).permutation(n_s)
    sc_shuf = {k: (val[shuf] if isinstance(val, np.ndarray) and val.shape[:1] == (n_s,)
                   and k != "chart_of" else val) for k, val in sc.items()}
    shuf_id_ms, shuf_loc_ms = step_ms(sc_shuf, False), step_ms(sc_shuf, True)
    del sc_shuf
    result["locality_packing"] = {"ms_per_step": round(loc_ms, 3),
                                  "mpix_per_s": round(V * W * H / (loc_ms / 1e3) / 1e6, 2),
                                  "speedup_vs_identity_packing": round(ms_step / loc_ms, 3),
                                  "shuffled_order_identity_ms": round(shuf_id_ms, 3),
                                  "shuffled_order_morton_ms": round(shuf_loc_ms, 3),
                                  "shuffled_speedup": round(shuf_id_ms / shuf_loc_ms, 3)}
    log(f"locality packing: {result['locality_packing']}")
    result["indirect"] = bench_indirect(sc, cams, W, H, plan.cap, K, args.warmup)
    log(f"indirect: {result['indirect']}")
    result["atlas_variants"] = bench_atlas_variants(sc, cams, W, H, plan.cap, max(3, K // 2),
                                                    ms_step, ds.atlas.numel() * 4)
    log(f"atlas variants: {result['atlas_variants']}")
    if not args.no_fwd_bwd:
        del plan
        torch.cuda.empty_cache()
        log("forward+backward ...")
        result["fwd_bwd"] = bench_fwd_bwd("sq300k_train", max(3, K // 2), 1)
        log(f"fwd+bwd: {result['fwd_bwd']}")
        result["fwd_bwd_field1m"] = bench_fwd_bwd("field1m", max(3, K // 2), 1)
        log(f"fwd+bwd field1m: {result['fwd_bwd_field1m']}")
        result["fwd_bwd_indirect"] = bench_fwd_bwd("sq300k_train", max(3, K // 2), 1,
                                                   sh_degree=3)
        log(f"fwd+bwd indirect: {result['fwd_bwd_indirect']}")
        result["fwd_bwd_trilinear"] = bench_fwd_bwd("sq300k_train", max(3, K // 2), 1,
                                                    mips=True)
        log(f"fwd+bwd trilinear: {result['fwd_bwd_trilinear']}")
        result["fwd_bwd_adaptive_sides"] = bench_fwd_bwd("sq300k_train", max(3, K // 2), 1,
                                                         charts=True)
        log(f"fwd+bwd adaptive sides: {result['fwd_bwd_adaptive_sides']}")
    result["small_frame"] = bench_small_frame()
    log(f"small frame: {result['small_frame']}")
    if not args.no_tab3:
        torch.cuda.empty_cache()
        log("texture sampling cost (Tab. 3 analog) ...")
        result["tab3"] = bench_tab3()
        log(f"tab3: {result['tab3']}")
    if not args.no_serving:
        torch.cuda.empty_cache()
        log("serving ...")
        result["serving"] = bench_serving(args.serving_seconds)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(sc, cams[0])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

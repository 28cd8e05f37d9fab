"""The indirect term on the HIP path against the FP64 oracle (run on an MI355X).

Per-(view, splat) SH evaluation (ts_indirect_eval), the blended L_ind map and the
visibility-weighted specular mix fused into ts_raster_fwd (Eq. 9, Eq. 12), and the same mix
in the standalone ts_shade; ragged frames, the constant sampler, full-size sampled frames and
the degenerate splats."""
import numpy as np
import pytest

import oracle
import synth
from parity import TOL_RGB, e2e_bound, gather, gather_ind, pixel_match, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pkg():
    import paper_2506_13348_amd as P
    P._ffi.lib()
    return P


def _print(name, info):
    print(f"[{name}] " + " ".join(f"{k}={v}" for k, v in info.items()), flush=True)


def _with_sh(sc, degree, seed=11):
    sc = dict(sc)
    sc["sh"] = synth.indirect_sh(np.random.default_rng(seed), len(sc["opac"]), degree)
    sc["sh_degree"] = degree
    return sc


def _eval_gpu(sc, cams, degree):
    P = _pkg()
    n = len(sc["opac"])
    V = len(cams)
    lind = torch.empty(V * n * 4, device="cuda")
    P._ffi.ts_indirect_eval(V, P.cameras_tensor(cams), n, torch.as_tensor(sc["means"]).cuda(),
                            torch.as_tensor(sc["quats"]).cuda(),
                            torch.as_tensor(sc["sh"]).cuda().contiguous(), degree, lind)
    torch.cuda.synchronize()
    return lind.view(V, n, 4).double().cpu().numpy()


def _close_f32(got, ref, sh):
    """float32 evaluation: the direction to a few ulp, each basis value to about 1e-6, the sum
    of 16 products rounded at each step, so |got - ref| <= 2e-6 sum_j |c_j| + 1e-7 per
    channel (sh: the splats' coefficients [n, K, 3])."""
    err = np.abs(got - ref)
    bound = 2e-6 * np.abs(sh.astype(np.float64)).sum(axis=1) + 1e-7
    assert (err <= bound).all(), float((err / bound).max())
    print(f"[indirect eval] max err {err.max():.3e}, max err / bound {(err / bound).max():.3f}",
          flush=True)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_indirect_eval_matches_oracle(degree):
    sc = _with_sh(synth.make_scene("shell2k"), degree)
    cams = synth.orbit_cameras(3, 64, 64, dist=2.5, el_deg=35.0)
    got = _eval_gpu(sc, cams, degree)
    for v, cam in enumerate(cams):
        ref = oracle.indirect_eval(sc, cam, sc["sh"], degree)
        _close_f32(got[v, :, :3], ref, sc["sh"])
        assert (got[v, :, 3] == 0).all()
    assert (got[..., :3] == 0).any() or degree == 0   # the clamp at zero is reached


def test_indirect_eval_all_orbit_views_sampled_splats():
    """The 100k-splat superquadric with degree-3 SH over all 64 orbit views (the launch the
    benchmark times), checked on 4,000 sampled splats per view."""
    sc = _with_sh(synth.make_scene("sq100k"), 3)
    cams = synth.config_cameras("sq100k")
    got = _eval_gpu(sc, cams, 3)
    idx = np.sort(np.random.default_rng(2).choice(len(sc["opac"]), 4000, replace=False))
    sub = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (len(sc["opac"]),) else v)
           for k, v in sc.items()}
    for v in range(0, 64, 3):
        ref = oracle.indirect_eval(sub, cams[v], sub["sh"], 3)
        _close_f32(got[v, idx, :3], ref, sub["sh"])


def test_indirect_eval_degenerate_splats():
    """A zero quaternion gives l_ind = 0 (no normal); a centre at the camera (to float32
    rounding) stays finite."""
    sc = _with_sh(synth.make_scene("shell2k", n=64), 2)
    cam = synth.config_cameras("shell2k")[0]
    w2c = np.asarray(cam["w2c"], np.float64)
    centre = -w2c[:, :3].T @ w2c[:, 3]
    sc["quats"] = sc["quats"].copy()
    sc["quats"][5] = 0.0
    sc["means"] = sc["means"].copy()
    sc["means"][9] = centre.astype(np.float32)
    got = _eval_gpu(sc, [cam], 2)
    assert (got[0, 5] == 0).all() and np.isfinite(got).all()
    keep = np.ones(64, bool)
    keep[[5, 9]] = False
    ref = oracle.indirect_eval(sc, cam, sc["sh"], 2)
    _close_f32(got[0, keep, :3], ref[keep], sc["sh"][keep])


# --------------------------------------------------------------------------- frames

def _render(sc, cams, W, H, vis=None, **kw):
    P = _pkg()
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    out = P.render(ds, cams, W, H, vis=None if vis is None else torch.as_tensor(vis).cuda(),
                   **kw)
    torch.cuda.synchronize()
    return ds, out


def _frame_parity(sc, cam, out, vis, v=0, pixels=None, name="frame", max_fail=0):
    W, H = cam["width"], cam["height"]
    if pixels is None:
        pixels = oracle.all_pixels(W, H)
    li = oracle.indirect_eval(sc, cam, sc["sh"], sc["sh_degree"])
    pv = None if vis is None else vis[v][pixels[:, 1], pixels[:, 0]]
    ref = oracle.render(sc, cam, pixels=pixels, lind=li, vis=pv)
    rgba, gb = gather(out, v, pixels)
    gi = gather_ind(out, v, pixels)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    ok, info = pixel_match(rgba, gb, ref, cam, pixels, tabs, gpu_gind=gi, vis=pv)
    _print(name, info)
    for b in np.nonzero(~ok)[0][:5]:
        print("  fail", pixels[b], "gpu", rgba[b], "ref", ref["rgba"][b], "stat", ref["stat"][b])
    assert info["fail"] <= max_fail, info
    assert e2e_bound(info), info
    assert gi is None or np.abs(ref["gind"]).max() > 0.1
    return info


def test_shell2k_indirect_full_frame():
    """The 2,000-splat shell, 128x128, degree-3 SH, mixed visibility: every pixel."""
    sc = _with_sh(synth.make_scene("shell2k"), 3)
    cam = synth.config_cameras("shell2k")[0]
    vis = synth.visibility(np.random.default_rng(5), 1, 128, 128)
    ds, out = _render(sc, [cam], 128, 128, vis=vis, gbuf=True, aux=True)
    _frame_parity(sc, cam, out, vis, name="shell2k indirect")


def test_indirect_ragged_multi_view():
    sc = _with_sh(synth.make_scene("sq100k", n=4000, tex_res=8, env_res=32), 2)
    sc["env_levels"] = 3
    cams = synth.orbit_cameras(3, 61, 47, dist=2.4, el_deg=30.0)
    vis = synth.visibility(np.random.default_rng(6), 3, 47, 61)
    ds, out = _render(sc, cams, 61, 47, vis=vis, gbuf=True)
    for v in range(3):
        _frame_parity(sc, cams[v], out, vis, v=v, name=f"indirect ragged v{v}")


def test_indirect_constant_sampler():
    sc = _with_sh(synth.make_scene("shell2k", n=900, tex_res=1), 1)
    cam = synth.crop_camera(synth.config_cameras("shell2k")[0], 30, 30, 70, 60)
    vis = synth.visibility(np.random.default_rng(7), 1, 60, 70)
    ds, out = _render(sc, [cam], 70, 60, vis=vis, params={"sampler": 1}, gbuf=True)
    _frame_parity(sc, cam, out, vis, name="indirect constant sampler")


def test_indirect_full_size_sampled():
    """The benchmark's indirect workload: 100k splats, all 64 orbit views at 800x800 in one
    launch, degree-3 SH and mixed visibility; two views checked at sampled pixels."""
    sc = _with_sh(synth.make_scene("sq100k"), 3)
    cams = synth.config_cameras("sq100k")
    vis = synth.visibility(np.random.default_rng(8), 64, 800, 800)
    ds, out = _render(sc, cams, 800, 800, vis=vis, gbuf=True)
    rng = np.random.default_rng(9)
    for v in (0, 37):
        pix = sample_pixels(rng, 800, 800, 160)
        _frame_parity(sc, cams[v], out, vis, v=v, pixels=pix, name=f"sq100k indirect v{v}")


def test_full_visibility_is_the_plain_render():
    """V = 1: the indirect variant's image equals the plain render (the mix reduces to the
    direct light; same blend order), and its G-buffer is the same."""
    sc = synth.make_scene("sq100k", n=6000, env_res=16)
    cams = synth.orbit_cameras(2, 96, 80)
    _, plain = _render(sc, cams, 96, 80, gbuf=True)
    _, ind = _render(_with_sh(sc, 3), cams, 96, 80, vis=np.ones((2, 80, 96), np.float32),
                     gbuf=True)
    dg = float((plain["gbuf"] - ind["gbuf"]).abs().max())
    dc = float((plain["rgba"] - ind["rgba"]).abs().max())
    print(f"[full visibility] gbuf diff {dg:.3e} rgba diff {dc:.3e}", flush=True)
    assert dg <= 1e-6 and dc <= 1e-6


def test_shade_with_indirect_on_synthetic_gbuffer():
    P = _pkg()
    rng = np.random.default_rng(10)
    V, H, W = 2, 40, 56
    g, a = synth.random_gbuffer(rng, V, H, W)
    gind = (rng.uniform(0, 2, size=(V, 3, H, W)) * a[:, None]).astype(np.float32)
    vis = synth.visibility(rng, V, H, W)
    env = synth.make_env(rng, 32)
    tabs_g = P.EnvTables(env, 3, device="cuda")
    cams = synth.orbit_cameras(V, W, H)
    rgba = torch.empty(V * H * W * 4, device="cuda")
    P._ffi.ts_shade(V, W, H, P.cameras_tensor(cams), P._ffi.make_params(8), tabs_g.struct,
                    torch.as_tensor(g).cuda(), torch.as_tensor(1.0 - a).cuda(), rgba,
                    gbuf_ind=torch.as_tensor(gind).cuda(), vis=torch.as_tensor(vis).cuda())
    torch.cuda.synchronize()
    rgba = rgba.view(V, H, W, 4).double().cpu().numpy()
    tabs = oracle.tables(env, 3)
    pix = oracle.all_pixels(W, H)
    for v in range(V):
        gg = g[v].reshape(8, -1).T.astype(np.float64)
        aa = (1.0 - (1.0 - a[v].astype(np.float32))).reshape(-1).astype(np.float64)
        ref, gap = oracle.shade_gbuffer(gg, aa, cams[v], pix, tabs,
                                        gind=gind[v].reshape(3, -1).T, vis=vis[v].reshape(-1))
        err = np.abs(rgba[v].reshape(-1, 4)[:, :3] - ref).max(axis=1)
        tie = gap < 1e-5
        assert (err[~tie] <= TOL_RGB).all(), err.max()
        print(f"[shade indirect v{v}] max err {err[~tie].max():.3e}", flush=True)


@pytest.mark.parametrize("degree", [1, 3])
def test_indirect_bwd_matches_float64_autograd(degree):
    """ts_indirect_bwd alone: with dL/dl_ind given per (view, splat), the coefficient, centre
    and rotation gradients against float64 autograd of the indirect term (the reference's own
    differentiable SH), summed over 3 views; 100 splats with a negative band 0 so that some
    channels are clamped at zero (no gradient through them). Upstream values of channels
    within 1e-5 of the clamp are zeroed (either side of the kink is valid)."""
    from oracle import grad as og
    P = _pkg()
    sc = _with_sh(synth.make_scene("shell2k", n=1500), degree, seed=40 + degree)
    sc["sh"][:100, 0, :] = -2.0
    cams = synth.orbit_cameras(3, 64, 64, dist=2.6, el_deg=15.0)
    n, V = len(sc["opac"]), len(cams)
    rng = np.random.default_rng(7)
    d_lind = rng.normal(size=(V, n, 4))
    DT = torch.float64
    ref_l = []
    for v, cam in enumerate(cams):
        w2c = torch.as_tensor(np.asarray(cam["w2c"], np.float64))
        o = -(w2c[:, :3].T @ w2c[:, 3])
        with torch.no_grad():
            l = og._indirect(torch.as_tensor(sc["means"], dtype=DT),
                             torch.as_tensor(sc["quats"], dtype=DT),
                             torch.as_tensor(sc["sh"], dtype=DT), degree, o).numpy()
        ref_l.append(l)
        d_lind[v, :, :3][np.abs(l) < 1e-5] = 0.0
    assert sum(int((l == 0).sum()) for l in ref_l) > 100     # clamped channels present
    leaves = {k: torch.tensor(np.asarray(sc[k], np.float32), dtype=DT, requires_grad=True)
              for k in ("means", "quats", "sh")}
    loss = 0.0
    for v, cam in enumerate(cams):
        w2c = torch.as_tensor(np.asarray(cam["w2c"], np.float64))
        o = -(w2c[:, :3].T @ w2c[:, 3])
        l = og._indirect(leaves["means"], leaves["quats"], leaves["sh"], degree, o)
        loss = loss + (l * torch.as_tensor(d_lind[v, :, :3])).sum()
    loss.backward()
    ref = {k: t.grad.numpy() for k, t in leaves.items()}

    dev = dict(device="cuda")
    means = torch.as_tensor(sc["means"]).cuda()
    quats = torch.as_tensor(sc["quats"]).cuda()
    sh = torch.as_tensor(sc["sh"]).cuda().contiguous()
    camt = P.cameras_tensor(cams)
    lind = torch.empty(V * n * 4, **dev)
    P._ffi.ts_indirect_eval(V, camt, n, means, quats, sh, degree, lind)
    d_sh = torch.full_like(sh, 7.0)          # overwritten (beta 0)
    d_means = torch.zeros(n * 3, **dev)
    d_quats = torch.zeros(n * 4, **dev)
    dl = torch.as_tensor(d_lind.astype(np.float32)).cuda().contiguous()
    P._ffi.ts_indirect_bwd(V, camt, n, means, quats, sh, degree, lind, dl, 0.0, d_sh, d_means,
                           d_quats)
    torch.cuda.synchronize()
    got = {"sh": d_sh.double().cpu().numpy(), "means": d_means.view(n, 3).double().cpu().numpy(),
           "quats": d_quats.view(n, 4).double().cpu().numpy()}
    # the clamped channels pass nothing: the coefficient gradients of those channels are 0
    clamped = np.stack([l <= 0 for l in ref_l]).all(axis=0)          # [n, 3] in every view
    assert (got["sh"].transpose(0, 2, 1)[clamped] == 0).all()
    for k in ("sh", "means", "quats"):
        a, b = got[k].reshape(-1), ref[k].reshape(-1)
        scale = np.abs(b).max()
        err = np.abs(a - b).max() / scale
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        print(f"[indirect bwd degree {degree}] {k}: rel {err:.2e} cos {cos:.8f}", flush=True)
        assert err <= 1e-4, (k, err)
        assert cos >= 0.99999, (k, cos)
    # beta = 1 adds the coefficient gradient onto d_sh; centres and rotations always add
    P._ffi.ts_indirect_bwd(V, camt, n, means, quats, sh, degree, lind, dl, 1.0, d_sh, d_means,
                           d_quats)
    torch.cuda.synchronize()
    assert torch.equal(d_sh.double().cpu(), torch.as_tensor(2 * got["sh"]))
    torch.testing.assert_close(d_means.view(n, 3).double().cpu(),
                               torch.as_tensor(2 * got["means"]), rtol=1e-6, atol=1e-9)

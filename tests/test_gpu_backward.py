"""HIP backward (ts_raster_bwd) against the float64 autograd reference (run on an MI355X).

Tolerance per gradient element (float32 path vs float64 definition):
|g - g_ref| <= 1e-3 max |g_ref| + 1e-7 + 2 spread, and cosine similarity >= 0.9999 per tensor.
Upstream gradients are zero at pixels the oracle marks as near a discrete decision (there both
branches are valid renders) and at pixels where a blended splat is seen at grazing incidence
(|cos| < 1e-3: there (u,v) has a condition number above 1e3).

spread: the render is piecewise smooth. Every bilinear lookup (texels, environment cube,
split-sum table) has a kink at each cell boundary where the derivative jumps, so at a lookup
within float32 rounding of a boundary the gradient is set-valued and the side a float32
evaluation lands on is decided by its rounding. spread is the largest change of the float64
reference gradient when the splat parameters are moved by +-2^-23 (relative, random
direction), i.e. by what float32 rounding of the inputs alone does; it is zero except at such
kinks. Computed from the reference only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import grad as og

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ("means", "quats", "scales", "opac", "textures")


def _pkg():
    import paper_2506_13348_amd as P
    P._ffi.lib()
    return P


def _gpu_grads(sc, cams, W, H, d_rgba, partial_floats=None, beta=0.0, grads=None, runner=None):
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    plan = P.RenderPlan(ds, cams, W, H, gbuf=True, aux=True)
    plan.run()
    plan.check()
    if grads is None:
        grads = (torch.zeros_like(ds.means), torch.zeros_like(ds.quats),
                 torch.zeros_like(ds.scales), torch.zeros_like(ds.opac),
                 torch.zeros_like(ds.atlas))
    run = BackwardRunner(plan, partial_floats)
    run.run(torch.as_tensor(np.asarray(d_rgba, np.float32)).cuda().contiguous(), grads, beta)
    torch.cuda.synchronize()
    return grads, run


def _np(grads):
    return {k: g.double().cpu().numpy() for k, g in zip(NAMES, grads)}


def _perturbed(sc, sign, seed):
    """Scene with means, quats and scales moved by sign * 2^-23 relative in a random direction."""
    r = np.random.default_rng(seed)
    out = dict(sc)
    for k in ("means", "quats", "scales"):
        x = np.asarray(sc[k], np.float64)
        out[k] = x * (1.0 + sign * 2.0 ** -23 * r.choice([-1.0, 1.0], size=x.shape))
    return out


def _reference(sc, cams, pix, ds, tabs):
    """Summed float64 reference gradients over views and their spread under +-2^-23 moves."""
    def total(scene):
        acc = {k: 0.0 for k in NAMES}
        for cam, d in zip(cams, ds):
            r = og.grads(scene, cam, pix, d, tabs)
            for k in NAMES:
                acc[k] = acc[k] + r[k]
        return acc
    ref = total(sc)
    spread = {k: np.zeros_like(ref[k]) for k in NAMES}
    for seed in (11, 12):
        for sign in (1.0, -1.0):
            alt = total(_perturbed(sc, sign, seed))
            for k in NAMES:
                spread[k] = np.maximum(spread[k], np.abs(alt[k] - ref[k]))
    return ref, spread


def _compare(g, ref, name, spread=None):
    out = {}
    for k in NAMES:
        a, b = g[k].reshape(-1), ref[k].reshape(-1)
        sp = np.zeros_like(b) if spread is None else spread[k].reshape(-1)
        scale = np.abs(b).max()
        tol = 1e-3 * scale + 1e-7 + 2.0 * sp
        d = np.abs(a - b)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))
        out[k] = (d.max() / max(scale, 1e-300), cos, int((sp > 1e-3 * scale).sum()))
        if (d > tol).any():
            i = int(np.argmax(d - tol))
            print(f"[{name}] worst {k}[{i}] gpu {a[i]:.6g} ref {b[i]:.6g} spread {sp[i]:.3g}",
                  flush=True)
        assert (d <= tol).all(), (name, k, float(d.max()), float(scale))
        assert cos >= 0.9999, (name, k, cos)
    print(f"[{name}] " + " ".join(f"{k}: rel {e:.2e} cos {c:.7f} kinks {n}"
                                  for k, (e, c, n) in out.items()), flush=True)


def _upstream(rng, ref, shape):
    d = rng.normal(size=(ref["rgba"].shape[0], 4))
    skip = (ref["stat"][:, 2] > 0) | (ref["stat"][:, 3] > 0)
    d[skip] = 0.0
    print(f"[upstream] {int(skip.sum())} of {len(skip)} pixels excluded "
          f"({int((ref['stat'][:, 3] > 0).sum())} grazing)", flush=True)
    return d, d.reshape(shape)


@pytest.fixture(scope="module")
def fd_case():
    sc = synth.make_scene("sq300k_train", n=20000, env_res=32)
    sc["env_levels"] = 3
    cam = synth.config_cameras("sq300k_train")[0]
    sub, crop = synth.fd_crop_scene(sc, cam, 368, 368, 64, 64, n_keep=500)
    return sub, crop


def test_grads_fd_crop(fd_case):
    """The 64x64 crop with the 500 front-most splats of the 300k-splat scene."""
    sub, crop = fd_case
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    ref_f = oracle.render(sub, crop, pixels=pix, tabs=tabs)
    d, d4 = _upstream(np.random.default_rng(1), ref_f, (1, 64, 64, 4))
    ref = og.grads(sub, crop, pix, d, tabs)
    g, _ = _gpu_grads(sub, [crop], 64, 64, d4)
    _compare(_np(g), ref, "fd crop")


def test_grads_multi_view_ragged():
    sc = synth.make_scene("shell2k", n=700, tex_res=4)
    cams = synth.orbit_cameras(3, 45, 37, dist=2.8, el_deg=10.0)
    rng = np.random.default_rng(4)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(45, 37)
    d_all = np.zeros((3, 37, 45, 4))
    ds = []
    for v, cam in enumerate(cams):
        ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs)
        d, d4 = _upstream(rng, ref_f, (37, 45, 4))
        d_all[v] = d4
        ds.append(d)
    ref, spread = _reference(sc, cams, pix, ds, tabs)
    g, _ = _gpu_grads(sc, cams, 45, 37, d_all)
    _compare(_np(g), ref, "3 views", spread)


def _full_size_sampled(cfg, n_views, per_view, seed, variant=None):
    """Full-size frame(s) of a config with dL/dC nonzero only at sampled pixels: the GPU runs the
    whole backward over every tile and view; the float64 reference needs only those pixels.
    variant: DeviceScene keyword arguments of an atlas variant (mips=True: trilinear)."""
    from parity import sample_pixels
    sc = synth.make_scene(cfg)
    if variant and variant.get("mips"):
        sc["trilinear"] = True
    cams = synth.config_cameras(cfg)
    W, H = cams[0]["width"], cams[0]["height"]
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    rng = np.random.default_rng(seed)
    d_all = np.zeros((len(cams), H, W, 4))
    pix_v, ds, used = [], [], []
    for v in range(min(n_views, len(cams))):
        pix = np.unique(sample_pixels(rng, W, H, per_view), axis=0)
        ref_f = oracle.render(sc, cams[v], pixels=pix, tabs=tabs)
        d = rng.normal(size=(len(pix), 4))
        skip = (ref_f["stat"][:, 2] > 0) | (ref_f["stat"][:, 3] > 0)
        d[skip] = 0.0
        d_all[v, pix[:, 1], pix[:, 0]] = d
        pix_v.append(pix)
        ds.append(d)
        used.append(cams[v])
    print(f"[{cfg}] {sum(len(p) for p in pix_v)} pixels with dL/dC over {len(used)} views",
          flush=True)

    def total(scene):
        acc = {k: 0.0 for k in NAMES}
        for cam, pix, d in zip(used, pix_v, ds):
            r = og.grads(scene, cam, pix, d, tabs)
            for k in NAMES:
                acc[k] = acc[k] + r[k]
        return acc
    ref = total(sc)
    spread = {k: np.zeros_like(ref[k]) for k in NAMES}
    for sign in (1.0, -1.0):
        alt = total(_perturbed(sc, sign, 11))
        for k in NAMES:
            spread[k] = np.maximum(spread[k], np.abs(alt[k] - ref[k]))
    if variant:
        flat = lambda r: dict(r, textures=r["textures"].reshape(-1, 8))
        g = _gpu_grads_variant(sc, variant, cams, W, H, d_all)
        _compare(g, flat(ref), f"{cfg} {variant}", flat(spread))
        return
    g, run = _gpu_grads(sc, cams, W, H, d_all)
    _compare(_np(g), ref, cfg, spread)


def test_grads_sq300k_training_batch_sampled():
    """The 300k-splat, 8-view 800x800 training batch through the whole backward."""
    _full_size_sampled("sq300k_train", 8, 10, 5)


def test_grads_sq300k_training_batch_trilinear_sampled():
    """The 300k-splat, 8-view training batch with trilinear sampling (the bench's trilinear
    training leg) through the whole backward, checked at sampled pixels."""
    _full_size_sampled("sq300k_train", 8, 10, 15, variant=dict(mips=True))


def test_grads_field1m_sampled():
    """The 1M-splat 1600x1064 unbounded frame through the whole backward."""
    _full_size_sampled("field1m", 1, 24, 6)


@pytest.mark.parametrize("T", [1, 16])
def test_grads_texture_resolution(T):
    sc = synth.make_scene("shell2k", n=500, tex_res=T)
    cam = synth.crop_camera(synth.config_cameras("shell2k")[0], 40, 40, 40, 40)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(40, 40)
    ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs)
    d, d4 = _upstream(np.random.default_rng(T), ref_f, (1, 40, 40, 4))
    ref, spread = _reference(sc, [cam], pix, [d], tabs)
    g, _ = _gpu_grads(sc, [cam], 40, 40, d4)
    _compare(_np(g), ref, f"T={T}", spread)


def test_deterministic_beta_and_overflow_retry():
    sc = synth.make_scene("sq100k", n=6000, env_res=16)
    cams = synth.orbit_cameras(2, 80, 64)
    d = np.random.default_rng(0).normal(size=(2, 64, 80, 4))
    g1, run1 = _gpu_grads(sc, cams, 80, 64, d)
    g2, _ = _gpu_grads(sc, cams, 80, 64, d)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    # a 1024-float partial buffer overflows; the retry sized from the reported need matches
    g3, run3 = _gpu_grads(sc, cams, 80, 64, d, partial_floats=1024)
    assert run3.partials.numel() > 1024
    for a, b in zip(g1, g3):
        assert torch.equal(a, b)
    # beta = 1 adds onto the previous contents
    acc = tuple(t.clone() for t in g1)
    _gpu_grads(sc, cams, 80, 64, d, beta=1.0, grads=acc)
    for a, b in zip(g1, acc):
        assert torch.equal(2 * a, b)


def test_autograd_function_matches_runner():
    P = _pkg()
    from paper_2506_13348_amd.autograd import render_rgba
    sc = synth.make_scene("shell2k", n=800)
    cam = synth.config_cameras("shell2k")[0]
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                       ds.atlas)]
    cams = P.cameras_tensor([cam])
    target = torch.rand(1, 128, 128, 3, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    rgba = render_rgba(*leaves, ds.chart_of, cams, 128, 128, ds.tables)
    loss = (rgba[..., :3] - target).abs().mean()
    loss.backward()
    d = (torch.sign(rgba[..., :3].detach() - target) / target.numel())
    d4 = torch.cat([d, torch.zeros_like(d[..., :1])], -1)
    g, _ = _gpu_grads(sc, [cam], 128, 128, d4.cpu().numpy())
    for leaf, ref in zip(leaves, g):
        torch.testing.assert_close(leaf.grad, ref, rtol=0, atol=0)


# ------------------------------------------------------------ environment-table gradients

def _env_ref(sc, cams, pix_list, ds, tabs, vis_list=None):
    """Summed float64 reference of the table gradients over views, and their spread under
    +-2^-23 moves of the splat parameters (taps at a texel boundary). vis_list: per view the
    visibility of the listed pixels (scenes with the indirect term), or None."""
    if vis_list is None:
        vis_list = [None] * len(cams)

    def total(scene):
        irr, spec = 0.0, None
        for cam, pix, d, pv in zip(cams, pix_list, ds, vis_list):
            r = og.grads(scene, cam, pix, d, tabs, env=True, vis=pv)
            irr = irr + r["irr"]
            spec = r["spec"] if spec is None else [a + b for a, b in zip(spec, r["spec"])]
        return [irr] + spec
    ref = total(sc)
    spread = [np.zeros_like(x) for x in ref]
    for sign in (1.0, -1.0):
        alt = total(_perturbed(sc, sign, 11))
        spread = [np.maximum(s, np.abs(a - b)) for s, a, b in zip(spread, alt, ref)]
    return ref, spread


def _gpu_env_grads(sc, cams, W, H, d_rgba, beta_twice=False, vis=None):
    P = _pkg()
    from paper_2506_13348_amd.autograd import EnvBackward
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    plan = P.RenderPlan(ds, cams, W, H, gbuf=True, aux=True,
                        vis=None if vis is None else torch.as_tensor(vis).cuda())
    plan.run()
    plan.check()
    eb = EnvBackward(plan)
    d = torch.as_tensor(np.asarray(d_rgba, np.float32)).cuda().contiguous()
    eb.run(d)
    torch.cuda.synchronize()
    out = [eb.d_irr.clone()]
    first = [eb.d_irr.clone(), eb.d_spec.clone()]
    if beta_twice:
        eb.run(d, beta=1.0)
        torch.cuda.synchronize()
    tabs = ds.tables
    r_irr = tabs.irr_res
    irr = eb.d_irr.view(6, r_irr, r_irr, 4)
    spec, off = [], 0
    for l in range(tabs.levels):
        rl = max(tabs.res >> l, 1)
        m = 6 * rl * rl * 4
        spec.append(eb.d_spec[off:off + m].view(6, rl, rl, 4))
        off += m
    return [irr] + spec, first, eb


def _compare_env(g, ref, spread, name):
    for k, (a, b, sp) in enumerate(zip(g, ref, spread)):
        a4 = a.double().cpu().numpy()
        assert np.all(a4[..., 3] == 0.0)
        a, b, sp = a4[..., :3].reshape(-1), b.reshape(-1), sp.reshape(-1)
        scale = np.abs(b).max()
        tol = 1e-3 * scale + 1e-7 + 2.0 * sp
        d = np.abs(a - b)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))
        if (d > tol).any():
            i = int(np.argmax(d - tol))
            print(f"[{name}] table {k} worst [{i}] gpu {a[i]:.6g} ref {b[i]:.6g} spread {sp[i]:.3g}",
                  flush=True)
        print(f"[{name}] table {k}: rel {d.max() / max(scale, 1e-300):.2e} cos {cos:.7f} "
              f"nonzero {int((b != 0).sum())}", flush=True)
        assert (d <= tol).all(), (name, k)
        if scale == 0.0:
            assert np.all(a == 0.0), (name, k)   # a level no pixel reads gets no gradient
        else:
            assert cos >= 0.9999, (name, k, cos)


def test_env_grads_multi_view():
    sc = synth.make_scene("sq300k_train", n=3000, env_res=16)
    sc["env_levels"] = 3
    cams = [synth.crop_camera(c, 330, 340, 45, 37) for c in synth.config_cameras("sq300k_train")[:2]]
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(45, 37)
    rng = np.random.default_rng(8)
    d_all = np.zeros((2, 37, 45, 4))
    ds = []
    for v, cam in enumerate(cams):
        ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs)
        d, d4 = _upstream(rng, ref_f, (37, 45, 4))
        d_all[v] = d4
        ds.append(d)
    ref, spread = _env_ref(sc, cams, [pix, pix], ds, tabs)
    g, first, _ = _gpu_env_grads(sc, cams, 45, 37, d_all, beta_twice=True)
    # beta = 1 added the same gradients once more
    for a, b in zip([first[0]], [g[0]]):
        assert torch.equal(2 * a, b.reshape(-1))
    g2, _, _ = _gpu_env_grads(sc, cams, 45, 37, d_all)
    for a, b in zip(g, g2):
        assert torch.equal(a, 2 * b)
    _compare_env(g2, ref, spread, "env 2 views")


def test_env_grads_fixed_point_scale_and_degenerate_upstream():
    """The sums are taken in fixed point at a scale set by the largest contribution, so an
    upstream scaled by a power of two scales every output texel by exactly that power; a zero
    upstream gives exact zeros; a non-finite one makes every texel's rgb NaN. Dense upstream on the
    8-view 800x800 batch: two calls are bit-identical."""
    sc = synth.make_scene("sq300k_train", n=3000, env_res=16)
    sc["env_levels"] = 3
    cams = [synth.crop_camera(c, 330, 340, 45, 37) for c in synth.config_cameras("sq300k_train")[:2]]
    rng = np.random.default_rng(18)
    d = rng.normal(size=(2, 37, 45, 4))
    g, _, eb = _gpu_env_grads(sc, cams, 45, 37, d)
    base = [t.clone() for t in g]
    assert any(float(t.abs().max()) > 0 for t in base)
    dd = torch.as_tensor(d.astype(np.float32)).cuda()
    for k in (-40, 17):
        eb.run((dd * 2.0 ** k).contiguous())
        torch.cuda.synchronize()
        assert torch.equal(eb.d_irr, base[0].reshape(-1) * 2.0 ** k), k
    eb.run(torch.zeros_like(dd))
    torch.cuda.synchronize()
    assert float(eb.d_irr.abs().max()) == 0.0 and float(eb.d_spec.abs().max()) == 0.0
    bad = dd.clone()
    ys, xs = np.nonzero(eb.plan.t_final.view(2, 37, 45)[0].cpu().numpy() < 1.0)
    bad[0, ys[0], xs[0], 0] = float("nan")
    eb.run(bad.contiguous())
    torch.cuda.synchronize()
    for t in (eb.d_irr, eb.d_spec):   # rgb of every texel; the fourth component stays 0
        assert bool(torch.isnan(t.view(-1, 4)[:, :3]).all()) and float(t.view(-1, 4)[:, 3].abs().max()) == 0.0
    # dense upstream over the training batch: run to run identical
    sc = synth.make_scene("sq300k_train")
    cams = synth.config_cameras("sq300k_train")
    d = np.random.default_rng(19).normal(size=(len(cams), 800, 800, 4)) * 1e-6
    g1, first, eb = _gpu_env_grads(sc, cams, 800, 800, d)
    eb.run(torch.as_tensor(d.astype(np.float32)).cuda().contiguous())
    torch.cuda.synchronize()
    assert torch.equal(first[0], eb.d_irr) and torch.equal(first[1], eb.d_spec)


def test_env_grads_many_texels_per_workgroup():
    """Random tangent normals per texel and roughness near 0 on a 64-texel environment: the
    reflected lookups of one 16x16 pixel block reach more distinct table texels than the
    accumulation's LDS table has slots (1024), so part of every block's contributions goes to
    the global accumulators directly; the sums still match the float64 reference."""
    sc = synth.make_scene("sq300k_train", n=3000, env_res=64)
    sc["env_levels"] = 5
    tex = np.array(sc["textures"], np.float64)
    rng = np.random.default_rng(5)
    nrm = rng.normal(size=tex.shape[:-1] + (3,))
    nrm[..., 2] = np.abs(nrm[..., 2]) + 0.05
    tex[..., 4:7] = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    tex[..., 3] = 0.02
    sc["textures"] = tex.astype(np.float32)
    cam = synth.crop_camera(synth.config_cameras("sq300k_train")[0], 330, 340, 45, 37)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(45, 37)
    # the first 16x16 block alone reaches more texels than a workgroup's table holds
    block = (pix[:, 0] < 16) & (pix[:, 1] < 16)
    d0 = np.where(block[:, None], rng.normal(size=(len(pix), 4)), 0.0)
    r0 = og.grads(sc, cam, pix, d0, tabs, env=True)
    reached = int((np.abs(r0["irr"]).sum(-1) > 0).sum()) + sum(
        int((np.abs(t).sum(-1) > 0).sum()) for t in r0["spec"])
    assert reached > 1024, reached
    ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs)
    d, d4 = _upstream(rng, ref_f, (1, 37, 45, 4))
    ref, spread = _env_ref(sc, [cam], [pix], [d], tabs)
    g, _, _ = _gpu_env_grads(sc, [cam], 45, 37, d4)
    _compare_env(g, ref, spread, "env many texels")


def test_env_grads_sq300k_training_batch_sampled():
    """The 8-view 800x800 training batch with dL/dC at sampled pixels only."""
    from parity import sample_pixels
    sc = synth.make_scene("sq300k_train")
    cams = synth.config_cameras("sq300k_train")
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    rng = np.random.default_rng(9)
    d_all = np.zeros((len(cams), 800, 800, 4))
    pix_v, ds = [], []
    for v in range(3):
        pix = np.unique(sample_pixels(rng, 800, 800, 12), axis=0)
        ref_f = oracle.render(sc, cams[v], pixels=pix, tabs=tabs)
        d = rng.normal(size=(len(pix), 4))
        d[(ref_f["stat"][:, 2] > 0) | (ref_f["stat"][:, 3] > 0)] = 0.0
        d_all[v, pix[:, 1], pix[:, 0]] = d
        pix_v.append(pix)
        ds.append(d)
    ref, spread = _env_ref(sc, cams[:3], pix_v, ds, tabs)
    g, _, _ = _gpu_env_grads(sc, cams, 800, 800, d_all)
    _compare_env(g, ref, spread, "env sq300k")


def test_env_grads_with_indirect_term_and_visibility():
    """A frame shaded with the indirect term and mixed visibility: the specular levels receive
    V (F0 A + B) dL/dC through their lookups (the direct light is weighted by V in Eq. 12),
    the irradiance cube what it receives without the term. Two ragged crops against the
    float64 reference with the same visibility."""
    sc = synth.make_scene("sq300k_train", n=3000, env_res=16)
    sc["env_levels"] = 3
    sc["sh"] = synth.indirect_sh(np.random.default_rng(51), 3000, 2)
    sc["sh_degree"] = 2
    cams = [synth.crop_camera(c, 330, 340, 45, 37) for c in synth.config_cameras("sq300k_train")[:2]]
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(45, 37)
    vis = synth.visibility(np.random.default_rng(52), 2, 37, 45)
    rng = np.random.default_rng(53)
    d_all = np.zeros((2, 37, 45, 4))
    ds, vs = [], []
    for v, cam in enumerate(cams):
        li = oracle.indirect_eval(sc, cam, sc["sh"], sc["sh_degree"])
        pv = vis[v][pix[:, 1], pix[:, 0]].astype(np.float64)
        ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs, lind=li, vis=pv)
        d, d4 = _upstream(rng, ref_f, (37, 45, 4))
        d_all[v] = d4
        ds.append(d)
        vs.append(pv)
    ref, spread = _env_ref(sc, cams, [pix, pix], ds, tabs, vis_list=vs)
    g, _, _ = _gpu_env_grads(sc, cams, 45, 37, d_all, vis=vis)
    _compare_env(g, ref, spread, "env indirect+vis")
    # the visibility matters: the specular levels' reference differs from the V = 1 one
    ref1, _ = _env_ref(sc, cams, [pix, pix], ds, tabs, vis_list=[np.ones(len(pix))] * 2)
    assert np.abs(ref1[1] - ref[1]).max() > 0.1 * np.abs(ref[1]).max()


# ------------------------------------------------------------ indirect-term gradients

NAMES_IND = NAMES + ("sh",)


def _with_sh(sc, degree, seed):
    out = dict(sc)
    out["sh"] = synth.indirect_sh(np.random.default_rng(seed), sc["means"].shape[0], degree)
    out["sh_degree"] = degree
    return out


def _gpu_grads_ind(sc, cams, W, H, d_rgba, vis, beta=0.0, grads=None):
    """ts_raster_bwd with the indirect arguments, then ts_indirect_bwd (d_sh; d_means and
    d_quats gain the reflected-direction terms)."""
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    plan = P.RenderPlan(ds, cams, W, H, gbuf=True, aux=True, vis=torch.as_tensor(vis).cuda())
    plan.run()
    plan.check()
    if grads is None:
        grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                    ds.atlas, ds.sh))
    BackwardRunner(plan).run(torch.as_tensor(np.asarray(d_rgba, np.float32)).cuda().contiguous(),
                             grads, beta)
    torch.cuda.synchronize()
    return grads


def _compare_ind(grads, ref, name, spread=None):
    """The bar of the plain backward, over the five splat tensors and the SH coefficients."""
    g = {k: t.double().cpu().numpy() for k, t in zip(NAMES_IND, grads)}
    for k in NAMES_IND:
        a, b = g[k].reshape(-1), ref[k].reshape(-1)
        sp = np.zeros_like(b) if spread is None else spread[k].reshape(-1)
        scale = np.abs(b).max()
        tol = 1e-3 * scale + 1e-7 + 2.0 * sp
        d = np.abs(a - b)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))
        if (d > tol).any():
            i = int(np.argmax(d - tol))
            print(f"[{name}] worst {k}[{i}] gpu {a[i]:.6g} ref {b[i]:.6g} spread {sp[i]:.3g}",
                  flush=True)
        print(f"[{name}] {k}: rel {d.max() / max(scale, 1e-300):.2e} cos {cos:.7f}", flush=True)
        assert (d <= tol).all(), (name, k, float(d.max()), float(scale))
        assert cos >= 0.9999, (name, k, cos)


def _ind_upstream(sc, cams, pix, vis, tabs, rng, H, W):
    """Per view: the upstream gradient (zero at the oracle's decision and grazing pixels) and
    the pixels' visibility."""
    d_all = np.zeros((len(cams), H, W, 4))
    ds, vs = [], []
    for v, cam in enumerate(cams):
        li = oracle.indirect_eval(sc, cam, sc["sh"], sc["sh_degree"])
        pv = vis[v][pix[:, 1], pix[:, 0]].astype(np.float64)
        ref_f = oracle.render(sc, cam, pixels=pix, tabs=tabs, lind=li, vis=pv)
        d, d4 = _upstream(rng, ref_f, (H, W, 4))
        d_all[v] = d4
        ds.append(d)
        vs.append(pv)
    return d_all, ds, vs


def _ind_reference(sc, cams, pix, ds, vs, tabs, spread=True):
    def total(scene):
        acc = {k: 0.0 for k in NAMES_IND}
        for cam, d, pv in zip(cams, ds, vs):
            r = og.grads(scene, cam, pix, d, tabs, vis=pv)
            for k in NAMES_IND:
                acc[k] = acc[k] + r[k]
        return acc
    ref = total(sc)
    if not spread:
        return ref, None
    sp = {k: np.zeros_like(ref[k]) for k in NAMES_IND}
    for sign in (1.0, -1.0):
        alt = total(_perturbed(sc, sign, 11))
        for k in NAMES_IND:
            sp[k] = np.maximum(sp[k], np.abs(alt[k] - ref[k]))
    return ref, sp


def test_indirect_grads_fd_crop(fd_case):
    """The 64x64 crop of the 300k-splat scene with degree-3 SH and mixed visibility: every
    gradient, the SH coefficients' included, against the float64 reference."""
    sub, crop = fd_case
    sc = _with_sh(sub, 3, 21)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(64, 64)
    vis = synth.visibility(np.random.default_rng(22), 1, 64, 64)
    d_all, ds, vs = _ind_upstream(sc, [crop], pix, vis, tabs, np.random.default_rng(23), 64, 64)
    ref, sp = _ind_reference(sc, [crop], pix, ds, vs, tabs)
    g = _gpu_grads_ind(sc, [crop], 64, 64, d_all, vis)
    _compare_ind(g, ref, "indirect fd crop", sp)


@pytest.mark.parametrize("degree", [0, 2])
def test_indirect_grads_multi_view_ragged(degree):
    sc = _with_sh(synth.make_scene("shell2k", n=700, tex_res=4), degree, 30 + degree)
    cams = synth.orbit_cameras(3, 45, 37, dist=2.8, el_deg=10.0)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(45, 37)
    vis = synth.visibility(np.random.default_rng(40 + degree), 3, 37, 45)
    d_all, ds, vs = _ind_upstream(sc, cams, pix, vis, tabs, np.random.default_rng(4), 37, 45)
    ref, sp = _ind_reference(sc, cams, pix, ds, vs, tabs)
    g = _gpu_grads_ind(sc, cams, 45, 37, d_all, vis)
    _compare_ind(g, ref, f"indirect 3 views degree {degree}", sp)


def test_indirect_grads_deterministic_and_beta():
    sc = _with_sh(synth.make_scene("sq100k", n=6000, env_res=16), 3, 50)
    cams = synth.orbit_cameras(2, 80, 64)
    vis = synth.visibility(np.random.default_rng(51), 2, 64, 80)
    d = np.random.default_rng(52).normal(size=(2, 64, 80, 4))
    g1 = _gpu_grads_ind(sc, cams, 80, 64, d, vis)
    g2 = _gpu_grads_ind(sc, cams, 80, 64, d, vis)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    assert float(g1[5].abs().max()) > 0
    acc = tuple(t.clone() for t in g1)
    _gpu_grads_ind(sc, cams, 80, 64, d, vis, beta=1.0, grads=acc)
    # the raster terms double exactly; d_means and d_quats gain the indirect terms after the
    # raster pass's beta, so they are compared to the rounding of one more sum
    for k, (a, b) in enumerate(zip(g1, acc)):
        if k in (0, 1):
            torch.testing.assert_close(b, 2 * a, rtol=1e-6, atol=1e-6 * float(a.abs().max()))
        else:
            assert torch.equal(2 * a, b), NAMES_IND[k]


def test_indirect_autograd_function_matches_runner():
    P = _pkg()
    from paper_2506_13348_amd.autograd import render_rgba
    sc = _with_sh(synth.make_scene("shell2k", n=800), 3, 60)
    cam = synth.config_cameras("shell2k")[0]
    vis = synth.visibility(np.random.default_rng(61), 1, 96, 96)
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                       ds.atlas, ds.sh)]
    cams = P.cameras_tensor([cam])
    rgba = render_rgba(*leaves[:5], ds.chart_of, cams, 96, 96, ds.tables, sh=leaves[5],
                       sh_degree=3, vis=torch.as_tensor(vis).cuda())
    d4 = torch.randn(1, 96, 96, 4, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    (rgba * d4).sum().backward()
    g = _gpu_grads_ind(sc, [cam], 96, 96, d4.cpu().numpy(), vis)
    for leaf, ref in zip(leaves, g):
        torch.testing.assert_close(leaf.grad, ref, rtol=0, atol=0)


def test_indirect_full_visibility_gradients_are_the_plain_ones():
    """With V = 1 everywhere the indirect light has no weight: the coefficients get exactly zero
    gradient, and the splat gradients equal those of the plain backward (the indirect kernel
    variant evaluates the same terms plus exact zeros)."""
    sc = synth.make_scene("sq100k", n=5000, env_res=16)
    cams = synth.orbit_cameras(2, 72, 56)
    d = np.random.default_rng(70).normal(size=(2, 56, 72, 4))
    plain, _ = _gpu_grads(sc, cams, 72, 56, d)
    ind = _gpu_grads_ind(_with_sh(sc, 2, 71), cams, 72, 56, d, np.ones((2, 56, 72), np.float32))
    assert float(ind[5].abs().max()) == 0.0
    for k, (a, b) in enumerate(zip(plain, ind[:5])):
        torch.testing.assert_close(b, a, rtol=1e-5, atol=1e-6 * max(float(a.abs().max()), 1e-30),
                                   msg=NAMES[k])


def test_backward_degenerate_frames():
    """No pairs (every splat behind the camera): every gradient is written as zero (beta 0,
    over a buffer holding 3.0); a scene without splats is a no-op; a 1x1 frame matches the
    float64 reference."""
    sc = synth.make_scene("shell2k", n=50)
    cam = synth.config_cameras("shell2k")[0]
    behind = dict(sc)
    behind["means"] = sc["means"] + np.float32([0, 0, 10])
    d = np.random.default_rng(80).normal(size=(1, 32, 32, 4))
    P = _pkg()
    ds = P.DeviceScene.from_dict(behind, device="cuda")
    full = tuple(torch.full_like(t, 3.0) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                   ds.atlas))
    g, _ = _gpu_grads(behind, [cam], 32, 32, d, grads=full)
    for k, t in zip(NAMES, g):
        assert torch.all(t == 0), k
    empty = {k: (v[:0] if isinstance(v, np.ndarray) and v.shape[:1] == (50,) else v)
             for k, v in sc.items()}
    g0, _ = _gpu_grads(empty, [cam], 32, 32, d)
    assert all(t.numel() == 0 for t in g0)
    big = synth.make_scene("shell2k", n=500)
    one = synth.crop_camera(synth.config_cameras("shell2k")[0], 48, 44, 1, 1)   # 7 blends
    tabs = oracle.tables(big["env"], big["env_levels"])
    pix = oracle.all_pixels(1, 1)
    ref_f = oracle.render(big, one, pixels=pix, tabs=tabs)
    assert ref_f["rgba"][0, 3] > 0.5                      # the pixel is covered
    clean = (ref_f["stat"][:, 2] == 0) & (ref_f["stat"][:, 3] == 0)
    d1 = np.array([[0.3, -0.7, 0.5, 0.2]]) * clean[:, None]
    ref = og.grads(big, one, pix, d1, tabs)
    g1, _ = _gpu_grads(big, [one], 1, 1, d1.reshape(1, 1, 1, 4))
    _compare(_np(g1), ref, "1x1")


# ------------------------------------------------ two-component tangent normals (7-float texels)

def _n2(tex):
    return np.ascontiguousarray(np.concatenate([tex[..., 0:6], tex[..., 7:8]], -1))


def _gpu_grads_xy(sc, cams, W, H, d_rgba):
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    ds = P.DeviceScene.from_dict(sc, device="cuda", tex_format=1)
    plan = P.RenderPlan(ds, cams, W, H, gbuf=True, aux=True)
    plan.run()
    plan.check()
    grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                ds.atlas))
    BackwardRunner(plan).run(torch.as_tensor(np.asarray(d_rgba, np.float32)).cuda().contiguous(),
                             grads)
    torch.cuda.synchronize()
    T = int(sc["textures"].shape[1])
    out = {k: g.double().cpu().numpy() for k, g in zip(NAMES[:4], grads[:4])}
    out["textures"] = grads[4].double().cpu().numpy().reshape(ds.n, T, T, 7)
    return out


def _seven(ref):
    """Reference texture gradients in the 7-float layout (the stored n_z is not read)."""
    r = dict(ref)
    assert np.all(ref["textures"][..., 6] == 0)
    r["textures"] = ref["textures"][..., [0, 1, 2, 3, 4, 5, 7]]
    return r


def test_xy_normal_grads_fd_crop(fd_case):
    """Two-component normals (n_z rebuilt after filtering): every gradient on the 64x64 crop
    against the float64 reference, texel gradients in the 7-float layout."""
    sub, crop = fd_case
    sc = dict(sub, tex_format=1)
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    ref_f = oracle.render(dict(sc, textures=_n2(sub["textures"])), crop, pixels=pix, tabs=tabs)
    d, d4 = _upstream(np.random.default_rng(81), ref_f, (1, 64, 64, 4))
    ref = og.grads(sc, crop, pix, d, tabs)
    g = _gpu_grads_xy(sub, [crop], 64, 64, d4)
    _compare(g, _seven(ref), "xy normals fd crop")


def test_xy_normal_grads_multi_view_ragged():
    sc = synth.make_scene("shell2k", n=700, tex_res=4)
    cams = synth.orbit_cameras(3, 45, 37, dist=2.8, el_deg=10.0)
    rng = np.random.default_rng(82)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(45, 37)
    sc1 = dict(sc, tex_format=1)
    d_all = np.zeros((3, 37, 45, 4))
    ds = []
    for v, cam in enumerate(cams):
        ref_f = oracle.render(dict(sc1, textures=_n2(sc["textures"])), cam, pixels=pix, tabs=tabs)
        d, d4 = _upstream(rng, ref_f, (37, 45, 4))
        d_all[v] = d4
        ds.append(d)
    ref, spread = _reference(sc1, cams, pix, ds, tabs)
    g = _gpu_grads_xy(sc, cams, 45, 37, d_all)
    _compare(g, _seven(ref), "xy normals 3 views", _seven(spread))


def test_xy_normal_autograd_function_matches_runner():
    P = _pkg()
    from paper_2506_13348_amd.autograd import render_rgba
    sc = synth.make_scene("shell2k", n=600)
    cam = synth.config_cameras("shell2k")[0]
    ds = P.DeviceScene.from_dict(sc, device="cuda", tex_format=1)
    T = ds.tex_res
    leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                       ds.atlas.view(ds.n, T, T, 7))]
    rgba = render_rgba(*leaves, ds.chart_of, P.cameras_tensor([cam]), 96, 96, ds.tables)
    d4 = torch.randn(1, 96, 96, 4, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    (rgba * d4).sum().backward()
    g = _gpu_grads_xy(sc, [cam], 96, 96, d4.cpu().numpy())
    for k, leaf in zip(NAMES, leaves):
        torch.testing.assert_close(leaf.grad.double().cpu().reshape(g[k].shape),
                                   torch.as_tensor(g[k]), rtol=0, atol=0, msg=k)


def test_xy_normals_with_indirect_term_grads_fd_crop(fd_case):
    """Both at once: two-component normals and degree-2 SH with mixed visibility on the crop
    (the backward kernel's <indirect, 7-float texel> variant)."""
    sub, crop = fd_case
    sc = dict(_with_sh(sub, 2, 90), tex_format=1)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(64, 64)
    vis = synth.visibility(np.random.default_rng(91), 1, 64, 64)
    osc = dict(sc, textures=_n2(sub["textures"]))
    d_all, ds, vs = _ind_upstream(osc, [crop], pix, vis, tabs, np.random.default_rng(92), 64, 64)
    ref, sp = _ind_reference(sc, [crop], pix, ds, vs, tabs, spread=False)
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    dsc = P.DeviceScene.from_dict(sc, device="cuda", tex_format=1)
    plan = P.RenderPlan(dsc, [crop], 64, 64, gbuf=True, aux=True, vis=torch.as_tensor(vis).cuda())
    plan.run()
    plan.check()
    grads = tuple(torch.zeros_like(t) for t in (dsc.means, dsc.quats, dsc.scales, dsc.opac,
                                                dsc.atlas, dsc.sh))
    BackwardRunner(plan).run(torch.as_tensor(d_all.astype(np.float32)).cuda().contiguous(), grads)
    torch.cuda.synchronize()
    T = int(sub["textures"].shape[1])
    g = list(grads)
    g[4] = g[4].view(dsc.n, T, T, 7)
    _compare_ind(g, _seven(ref), "xy normals + indirect fd crop")


# ------------------------------- atlas variants: per-chart resolutions, trilinear sampling

def _charted(sub, seed=11):
    """The crop scene with each chart box-downsampled to its own side (1 to T texels), level-0
    texels back to back in splat order, and the table of (level-0 offset, log2 side)."""
    tex = np.asarray(sub["textures"], np.float32)
    n, T = tex.shape[0], tex.shape[1]
    log2 = np.random.default_rng(seed).integers(0, int(np.log2(T)) + 1, size=n).astype(np.int32)
    parts, table, off = [], np.zeros((n, 2), np.int32), 0
    for c in range(n):
        s = 1 << int(log2[c])
        b = T // s
        parts.append(tex[c].reshape(s, b, s, b, 8).mean(axis=(1, 3)).astype(np.float32)
                     .reshape(-1, 8))
        table[c] = (off, log2[c])
        off += s * s
    return np.concatenate(parts), table, log2


def _zoomed_crop():
    """The training view with focal lengths / 10, a 64x64 crop at its centre and its 1500
    nearest splats: samples there cover several texels per pixel, so trilinear sampling blends
    levels (and some reach the last level)."""
    sc = synth.make_scene("sq300k_train", n=20000, env_res=32)
    sc["env_levels"] = 3
    cam = dict(synth.config_cameras("sq300k_train")[0])
    cam["fx"], cam["fy"] = cam["fx"] / 10, cam["fy"] / 10
    return synth.fd_crop_scene(sc, cam, 368, 368, 64, 64, n_keep=1500)


def _variant_case(sub, fmt, charts, tri):
    """(reference scene for oracle/grad.py, C-oracle scene, DeviceScene keyword arguments,
    device-side texture input) of one variant of the crop scene."""
    ref_sc = dict(sub, trilinear=tri, tex_format=fmt)
    kw = dict(tex_format=fmt, mips=tri)
    dev_sc = dict(sub)
    if charts:
        flat, table, log2 = _charted(sub)
        ref_sc.update(textures=flat, chart_table=table)
        kw["chart_log2"] = log2
        dev_sc["textures"] = flat
    c_sc = dict(ref_sc, textures=_n2(ref_sc["textures"]) if fmt else ref_sc["textures"])
    return ref_sc, c_sc, kw, dev_sc


def _gpu_grads_variant(dev_sc, kw, cams, W, H, d_rgba):
    """GPU gradients with the texel gradients taken out of the atlas layout: level 0 of each
    splat's chart, in the reference's layout (8 channels, channel 6 zero with 7-float texels);
    the chain's coarser levels must hold exact zeros."""
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    ds = P.DeviceScene.from_dict(dev_sc, device="cuda", **kw)
    plan = P.RenderPlan(ds, cams, W, H, gbuf=True, aux=True)
    plan.run()
    plan.check()
    grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac))
    grads = grads + (torch.full_like(ds.atlas, 7.0),)     # every atlas texel must be written
    BackwardRunner(plan).run(torch.as_tensor(np.asarray(d_rgba, np.float32)).cuda().contiguous(),
                             grads)
    torch.cuda.synchronize()
    out = {k: g.double().cpu().numpy() for k, g in zip(NAMES[:4], grads[:4])}
    C = 7 if kw.get("tex_format", 0) else 8
    ga = grads[4].double().cpu().numpy().reshape(-1, C)
    chart_of = ds.chart_of.cpu().numpy()
    mips = kw.get("mips", False)
    if ds.chart_table is not None:
        tab = ds.chart_table.cpu().numpy()
        ents = [(int(tab[c, 0]), 1 << int(tab[c, 1])) for c in chart_of]
    else:
        T = ds.tex_res
        stride = (4 * T * T - 1) // 3 if mips else T * T
        ents = [(int(c) * stride, T) for c in chart_of]
    lv0, coarse = [], []
    for off, side in ents:
        lv0.append(ga[off:off + side * side])
        if mips:
            coarse.append(ga[off + side * side:off + (4 * side * side - 1) // 3])
    lv0 = np.concatenate(lv0)
    if C == 7:
        lv0 = np.concatenate([lv0[:, :6], np.zeros((len(lv0), 1)), lv0[:, 6:]], 1)
    if coarse:
        assert all(np.all(c == 0) for c in coarse), "coarser chain levels got a gradient"
    out["textures"] = lv0
    return out


def _variant_compare(sub, crop, fmt, charts, tri, seed, name):
    ref_sc, c_sc, kw, dev_sc = _variant_case(sub, fmt, charts, tri)
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    ref_f = oracle.render(c_sc, crop, pixels=pix, tabs=tabs)
    d, d4 = _upstream(np.random.default_rng(seed), ref_f, (1, 64, 64, 4))
    ref, spread = _reference(ref_sc, [crop], pix, [d], tabs)
    ref = dict(ref, textures=ref["textures"].reshape(-1, 8))
    spread = dict(spread, textures=spread["textures"].reshape(-1, 8))
    g = _gpu_grads_variant(dev_sc, kw, [crop], 64, 64, d4)
    _compare(g, ref, name, spread)


@pytest.mark.parametrize("fmt", [0, 1])
def test_chart_table_grads_fd_crop(fd_case, fmt):
    """Per-chart sides 1..8 in one table-addressed atlas (level-0 bilinear) on the 64x64 crop."""
    sub, crop = fd_case
    _variant_compare(sub, crop, fmt, True, False, 101 + fmt, f"chart table fmt={fmt}")


@pytest.mark.parametrize("fmt,charts", [(0, False), (1, False), (0, True), (1, True)])
def test_trilinear_grads_zoomed_crop(fmt, charts):
    """Trilinear sampling over each chart's box-filtered chain (uniform charts or a chart
    table) where most samples blend two levels: the level's gradient reaches the centres,
    rotations and scales through the footprint, and every level's texel gradient is folded
    into level 0."""
    sub, crop = _zoomed_crop()
    _variant_compare(sub, crop, fmt, charts, True, 111 + fmt + 2 * charts,
                     f"trilinear fmt={fmt} charts={charts}")


def test_trilinear_grads_multi_view_ragged():
    """Three ragged views of a 700-splat shell with 8-texel charts: most samples blend two
    levels, some sit at the last level (1 texel), a few at level 0."""
    sc = synth.make_scene("shell2k", n=700, tex_res=8)
    cams = synth.orbit_cameras(3, 45, 37, dist=2.8, el_deg=10.0)
    rng = np.random.default_rng(121)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(45, 37)
    ref_sc = dict(sc, trilinear=True)
    d_all = np.zeros((3, 37, 45, 4))
    ds = []
    for v, cam in enumerate(cams):
        ref_f = oracle.render(ref_sc, cam, pixels=pix, tabs=tabs)
        d, d4 = _upstream(rng, ref_f, (37, 45, 4))
        d_all[v] = d4
        ds.append(d)
    ref, spread = _reference(ref_sc, cams, pix, ds, tabs)
    ref = dict(ref, textures=ref["textures"].reshape(-1, 8))
    spread = dict(spread, textures=spread["textures"].reshape(-1, 8))
    g = _gpu_grads_variant(sc, dict(mips=True), cams, 45, 37, d_all)
    _compare(g, ref, "trilinear 3 views", spread)


@pytest.mark.parametrize("charts", [False, True])
def test_variant_autograd_matches_runner_and_trains(charts):
    """render_rgba over a trilinear atlas (uniform or chart table) given the scene's atlas_spec:
    its gradients equal the runner's bit for bit, and a few gradient steps on the level-0
    texels (chains rebuilt by ts_atlas_mips after each) bring the render back towards a target
    rendered from the original texels."""
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner, render_rgba
    sc = synth.make_scene("shell2k", n=600, tex_res=8)
    cam = synth.orbit_cameras(1, 96, 96, dist=2.8, el_deg=10.0)[0]
    kw = dict(mips=True)
    dev_sc = sc
    if charts:
        log2 = synth.texture_sides(sc["scales"], max_log2=3)
        dev_sc = dict(sc, textures=synth.adaptive_textures(np.random.default_rng(5), log2))
        kw["chart_log2"] = log2
    ds = P.DeviceScene.from_dict(dev_sc, device="cuda", **kw)
    cams = P.cameras_tensor([cam])
    leaves = [t.clone().requires_grad_(True) for t in (ds.means, ds.quats, ds.scales, ds.opac,
                                                       ds.atlas)]
    rgba = render_rgba(*leaves, ds.chart_of, cams, 96, 96, ds.tables, atlas_spec=ds.atlas_spec())
    d4 = torch.randn(1, 96, 96, 4, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    (rgba * d4).sum().backward()
    plan = P.RenderPlan(ds, [cam], 96, 96, gbuf=True, aux=True)
    plan.run()
    plan.check()
    grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac, ds.atlas))
    BackwardRunner(plan).run(d4.reshape(-1).contiguous(), grads)
    torch.cuda.synchronize()
    for k, leaf, ref in zip(NAMES, leaves, grads):
        assert torch.equal(leaf.grad, ref), k
    assert float(leaves[4].grad.abs().max()) > 0
    # a short fit of the level-0 texels to a target from the original atlas
    with torch.no_grad():
        target = render_rgba(ds.means, ds.quats, ds.scales, ds.opac, ds.atlas, ds.chart_of, cams,
                             96, 96, ds.tables, atlas_spec=ds.atlas_spec()).clone()
        noise = torch.randn(ds.atlas.shape, device="cuda",
                            generator=torch.Generator("cuda").manual_seed(8))
        ds.atlas += 0.2 * noise
        ds.rebuild_mips()
    atlas = ds.atlas.requires_grad_(True)
    opt = torch.optim.Adam([atlas], lr=0.02)
    losses = []
    for it in range(30):
        out = render_rgba(ds.means, ds.quats, ds.scales, ds.opac, atlas, ds.chart_of, cams, 96, 96,
                          ds.tables, atlas_spec=ds.atlas_spec())
        loss = (out - target).square().mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            ds.rebuild_mips()
        losses.append(float(loss.detach()))
    print(f"[trilinear fit charts={charts}] loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.3 * losses[0], losses
    if not charts:
        # the rebuilt chains are the block means of the fitted level 0
        T, n = ds.tex_res, ds.n
        a = ds.atlas.detach().view(n, (4 * T * T - 1) // 3, 8).double().cpu().numpy()
        l0 = a[:, :T * T].reshape(n, T // 2, 2, T // 2, 2, 8).mean(axis=(2, 4))
        l1 = a[:, T * T:T * T + (T // 2) ** 2].reshape(n, T // 2, T // 2, 8)
        np.testing.assert_allclose(l1, l0, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("charts,tri", [(False, True), (True, False), (True, True)])
def test_variant_with_indirect_term_grads_zoomed_crop(charts, tri):
    """An atlas variant and degree-2 SH with mixed visibility at once on the zoomed crop (the
    backward kernel's <indirect, 8-float texel, chart table / trilinear> variants); texel
    gradients taken out of the atlas layout at level 0."""
    sub, crop = _zoomed_crop()
    sc = dict(_with_sh(sub, 2, 131), trilinear=tri)
    dev_sc, kw = dict(sc), dict(mips=tri)
    if charts:
        flat, table, log2 = _charted(sub)
        sc.update(textures=flat, chart_table=table)
        dev_sc["textures"] = flat
        kw["chart_log2"] = log2
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(64, 64)
    vis = synth.visibility(np.random.default_rng(132), 1, 64, 64)
    d_all, ds, vs = _ind_upstream(sc, [crop], pix, vis, tabs, np.random.default_rng(133), 64, 64)
    ref, sp = _ind_reference(sc, [crop], pix, ds, vs, tabs)
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    dsc = P.DeviceScene.from_dict(dev_sc, device="cuda", **kw)
    plan = P.RenderPlan(dsc, [crop], 64, 64, gbuf=True, aux=True, vis=torch.as_tensor(vis).cuda())
    plan.run()
    plan.check()
    grads = tuple(torch.zeros_like(t) for t in (dsc.means, dsc.quats, dsc.scales, dsc.opac,
                                                dsc.atlas, dsc.sh))
    BackwardRunner(plan).run(torch.as_tensor(d_all.astype(np.float32)).cuda().contiguous(), grads)
    torch.cuda.synchronize()
    ga = grads[4].view(-1, 8)
    if charts:
        tab = dsc.chart_table.cpu().numpy()
        ents = [(int(tab[c, 0]), 1 << int(tab[c, 1])) for c in dsc.chart_of.cpu().numpy()]
    else:
        T = dsc.tex_res
        ents = [(int(c) * ((4 * T * T - 1) // 3), T) for c in dsc.chart_of.cpu().numpy()]
    lv0 = []
    for o, side in ents:
        lv0.append(ga[o:o + side * side])
        if tri:
            assert float(ga[o + side * side:o + (4 * side * side - 1) // 3].abs().max()
                         if side > 1 else 0.0) == 0.0
    g = list(grads)
    g[4] = torch.cat(lv0)
    ref = dict(ref, textures=ref["textures"].reshape(-1, 8))
    sp = dict(sp, textures=sp["textures"].reshape(-1, 8))
    _compare_ind(g, ref, f"variant charts={charts} tri={tri} + indirect zoomed crop", sp)


def _window_splats(sc, cam, x0, y0, w, h, S=3.0, margin=2.0):
    """Indices (ascending) of the splats whose support square |u|,|v| <= S can reach a pixel
    of the window [x0, x0+w) x [y0, y0+h) of the camera: the bounding box of the square's four
    projected corners, widened by a margin; a square with a corner at or behind the near plane
    is kept (conservative). The other splats cannot touch the window's pixels."""
    q = np.asarray(sc["quats"], np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w_, x, y, z = q.T
    tu = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w_ * z), 2 * (x * z - w_ * y)], 1)
    tv = np.stack([2 * (x * y - w_ * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w_ * x)], 1)
    mu = np.asarray(sc["means"], np.float64)
    s = np.asarray(sc["scales"], np.float64)
    w2c = np.asarray(cam["w2c"], np.float64)
    xs, ys, bad = [], [], np.zeros(len(mu), bool)
    for a in (-S, S):
        for b in (-S, S):
            p = mu + a * s[:, :1] * tu + b * s[:, 1:2] * tv
            pc = p @ w2c[:, :3].T + w2c[:, 3]
            bad |= pc[:, 2] <= 0.2
            zc = np.where(pc[:, 2] > 0.2, pc[:, 2], 1.0)
            xs.append(cam["fx"] * pc[:, 0] / zc + cam["cx"])
            ys.append(cam["fy"] * pc[:, 1] / zc + cam["cy"])
    xs, ys = np.stack(xs), np.stack(ys)
    hit = ((xs.max(0) >= x0 - margin) & (xs.min(0) <= x0 + w + margin) &
           (ys.max(0) >= y0 - margin) & (ys.min(0) <= y0 + h + margin))
    return np.nonzero(hit | bad)[0]


def test_grads_sq300k_dense_window():
    """The full-size 8-view sq300k training launch with dL/dC dense (every pixel) over a 64x64
    window of two views, zero elsewhere: the partials of every splat touching the windows are
    gathered at full size. Gradients of those splats match the float64 reference (rendered
    from the splats that can reach the window, in their original order; with its spread under
    +-2^-23 moves, as the other full-size tests); every other splat's gradient is exactly
    zero."""
    sc = synth.make_scene("sq300k_train")
    cams = synth.config_cameras("sq300k_train")
    W, H = cams[0]["width"], cams[0]["height"]
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    rng = np.random.default_rng(141)
    d_all = np.zeros((len(cams), H, W, 4))
    pix = oracle.all_pixels(64, 64)
    ref = {k: 0.0 for k in NAMES}
    spread = {k: 0.0 for k in NAMES}
    touched = np.zeros(len(sc["opac"]), bool)
    for v, (x0, y0) in ((0, (368, 368)), (5, (300, 420))):
        crop = synth.crop_camera(cams[v], x0, y0, 64, 64)
        idx = _window_splats(sc, cams[v], x0, y0, 64, 64)
        sub = {k: (val[idx] if isinstance(val, np.ndarray) and val.shape[:1] == (len(sc["opac"]),)
                   else val) for k, val in sc.items()}
        sub["chart_of"] = np.arange(len(idx), dtype=np.int32)
        ref_f = oracle.render(sub, crop, pixels=pix, tabs=tabs)
        assert (ref_f["rgba"][:, 3] > 0).mean() > 0.5
        d, d4 = _upstream(rng, ref_f, (64, 64, 4))
        d_all[v, y0:y0 + 64, x0:x0 + 64] = d4
        r, sp = _reference(sub, [crop], pix, [d], tabs)
        print(f"[dense window] view {v}: {len(idx)} splats can reach it", flush=True)
        for k in NAMES:
            full = np.zeros((len(sc["opac"]),) + r[k].shape[1:])
            full[idx] = r[k]
            ref[k] = ref[k] + full
            full = np.zeros((len(sc["opac"]),) + r[k].shape[1:])
            full[idx] = sp[k]
            spread[k] = spread[k] + full
        touched[idx] = True
    g, run = _gpu_grads(sc, cams, W, H, d_all)
    g = _np(g)
    for k in NAMES:
        assert np.all(g[k][~touched] == 0.0), k
    _compare({k: g[k][touched] for k in NAMES}, {k: ref[k][touched] for k in NAMES},
             "sq300k dense windows", {k: spread[k][touched] for k in NAMES})


@pytest.mark.parametrize("tri", [False, True])
def test_chart_outside_the_atlas_backward(fd_case, tri):
    """A chart-table entry reaching past the atlas samples as zero texels in the forward; its
    backward gives the other parameters the gradients of that zero-texture render (the float64
    reference with the chart's texels zeroed) and leaves the chart's texel gradients unwritten
    (the caller's buffer keeps its contents). Trilinear on the zoomed-out crop, where the
    moved chart's samples blend levels."""
    sub, crop = _zoomed_crop() if tri else fd_case
    flat, table, log2 = _charted(sub)
    sc = dict(sub, textures=flat, chart_table=table, trilinear=tri)
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    # the splat whose texels matter most on the crop goes out of the atlas
    d0 = np.random.default_rng(150).normal(size=(len(pix), 4))
    g0 = og.grads(sc, crop, pix, d0, tabs)
    per_chart = np.array([np.abs(g0["textures"][o:o + (1 << (2 * l))]).sum() for o, l in table])
    k = int(np.argmax(per_chart))
    o, l = int(table[k, 0]), int(table[k, 1])
    ref_sc = dict(sc, textures=flat.copy())
    ref_sc["textures"][o:o + (1 << (2 * l))] = 0.0
    ref_f = oracle.render(ref_sc, crop, pixels=pix, tabs=tabs)
    d, d4 = _upstream(np.random.default_rng(151), ref_f, (1, 64, 64, 4))
    ref, spread = _reference(ref_sc, [crop], pix, [d], tabs)
    P = _pkg()
    from paper_2506_13348_amd.autograd import BackwardRunner
    ds = P.DeviceScene.from_dict(dict(sub, textures=flat), device="cuda", chart_log2=log2,
                                 mips=tri)
    o_dev = int(ds.chart_table[k, 0])
    ds.chart_table[k, 0] = int(ds.atlas_texels)          # past the end of the atlas
    plan = P.RenderPlan(ds, [crop], 64, 64, gbuf=True, aux=True)
    plan.run()
    plan.check()
    from parity import gather, pixel_match
    rgba, gb = gather(plan.outputs(), 0, pix)
    ok, info = pixel_match(rgba, gb, ref_f, crop, pix, tabs)
    print(f"[chart outside the atlas tri={tri}] forward " + " ".join(f"{a}={b}" for a, b in
                                                                  info.items()), flush=True)
    assert info["fail"] == 0, info
    grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac))
    grads = grads + (torch.full_like(ds.atlas, 5.0),)
    BackwardRunner(plan).run(torch.as_tensor(d4.astype(np.float32)).cuda().contiguous(), grads)
    torch.cuda.synchronize()
    g = {n: t.double().cpu().numpy() for n, t in zip(NAMES[:4], grads[:4])}
    # the chart moved out takes no texel gradient: its old place (level 0 and, with mip
    # chains, the coarser levels) keeps the caller's contents
    tab = ds.chart_table.cpu().numpy()
    ga = grads[4].view(-1, 8).double().cpu().numpy()
    C = (4 * (1 << (2 * l)) - 1) // 3 if tri else (1 << (2 * l))
    assert np.all(ga[o_dev:o_dev + C] == 5.0), "the moved chart's texels were written"
    lv0 = []
    for c in range(ds.n):
        if c == k:
            lv0.append(np.zeros((1 << (2 * l), 8)))
            continue
        side = 1 << int(tab[c, 1])
        lv0.append(ga[int(tab[c, 0]):int(tab[c, 0]) + side * side])
        if tri:
            coarse = ga[int(tab[c, 0]) + side * side:int(tab[c, 0]) + (4 * side * side - 1) // 3]
            assert np.all(coarse == 0.0), "coarser chain levels got a gradient"
    g["textures"] = np.concatenate(lv0)
    ref = dict(ref, textures=ref["textures"].reshape(-1, 8))
    ref["textures"][o:o + (1 << (2 * l))] = 0.0           # not a parameter the GPU writes
    spread = dict(spread, textures=spread["textures"].reshape(-1, 8))
    _compare(g, ref, f"chart outside the atlas tri={tri}", spread)

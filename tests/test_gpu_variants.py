"""The atlas variants on the HIP path against the FP64 oracle (run on an MI355X).

Two-component tangent normals (7-float texels), per-chart resolutions through a chart table,
trilinear sampling over each chart's box-filtered mip chain (built on the GPU by
ts_atlas_pack2 / ts_atlas_mips and checked against numpy block means), alone and combined;
ragged multi-view frames and the 64-view sq100k launch at sampled pixels."""
import numpy as np
import pytest

import oracle
import synth
from parity import e2e_bound, gather, pixel_match, sample_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pkg():
    import paper_2506_13348_amd as P
    P._ffi.lib()
    return P


def _print(name, info):
    print(f"[{name}] " + " ".join(f"{k}={v}" for k, v in info.items()), flush=True)


def _n2(tex):
    return np.ascontiguousarray(np.concatenate([tex[..., 0:6], tex[..., 7:8]], -1))


def _oracle_scene(sc, fmt=0, tri=False, log2=None, flat=None):
    """The oracle's view of a variant scene: its own level-0 layout (no chains)."""
    o = dict(sc, tex_format=fmt, trilinear=tri)
    if log2 is not None:
        sides = 1 << log2.astype(np.int64)
        offs = np.concatenate([[0], np.cumsum(sides * sides)])[:-1]
        o["chart_table"] = np.stack([offs, log2], 1).astype(np.int32)
        o["textures"] = _n2(flat) if fmt else flat
    elif fmt:
        o["textures"] = _n2(sc["textures"])
    return o


def _frame(osc, cam, out, v=0, pixels=None, name="frame", graze=None):
    """graze: for charts of 16 texels a side a blended splat seen at |cos| below about 0.02
    turns the float32 rounding of its (u,v) into more than 1e-5 of texture (16/6 texels per
    unit of u); with graze set, pixels the oracle flags for a blended splat below that |cos|
    are kept off the G-buffer bar only (alpha and the shading of the GPU's own G-buffer still
    apply) and counted (at most 1%)."""
    W, H = cam["width"], cam["height"]
    if pixels is None:
        pixels = oracle.all_pixels(W, H)
    ref = oracle.render(osc, cam, pixels=pixels,
                        params=None if graze is None else {"graze": graze})
    rgba, gb = gather(out, v, pixels)
    tabs = oracle.tables(osc["env"], osc["env_levels"])
    ok, info = pixel_match(rgba, gb, ref, cam, pixels, tabs, skip_graze=graze is not None)
    if graze is not None:
        assert info["grazing_off_gbuf_bar"] <= 0.01 * info["pixels"], info
    _print(name, info)
    for b in np.nonzero(~ok)[0][:5]:
        print("  fail", pixels[b], "gpu", rgba[b], "ref", ref["rgba"][b], "stat", ref["stat"][b])
    assert info["fail"] == 0, info
    assert e2e_bound(info), info


def _render(sc, cams, W, H, **scene_kw):
    P = _pkg()
    ds = P.DeviceScene.from_dict(sc, device="cuda", **scene_kw)
    out = P.render(ds, cams, W, H, gbuf=True)
    torch.cuda.synchronize()
    return ds, out


def test_mip_chain_is_the_block_mean():
    P = _pkg()
    rng = np.random.default_rng(0)
    n, T = 37, 16
    tex = rng.uniform(0, 1, size=(n, T, T, 8)).astype(np.float32)
    for fmt in (0, 1):
        C = 7 if fmt else 8
        chain = (4 * T * T - 1) // 3
        atlas = torch.empty(n * chain * C, device="cuda")
        chart_of = torch.empty(n, device="cuda", dtype=torch.int32)
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32)).cuda()
        P._ffi.ts_atlas_pack2(torch.as_tensor(tex).cuda(), n, T, perm, fmt, 1, atlas, chart_of)
        torch.cuda.synchronize()
        a = atlas.view(n, chain, C).double().cpu().numpy()
        pc = perm.cpu().numpy()
        assert np.array_equal(chart_of.cpu().numpy(), pc)
        src = _n2(tex) if fmt else tex
        off, s = 0, T
        while s >= 1:
            b = T // s
            ref = src.astype(np.float64).reshape(n, s, b, s, b, C).mean(axis=(2, 4))
            got = a[pc, off:off + s * s].reshape(n, s, s, C)
            np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-7)
            off += s * s
            s //= 2


@pytest.mark.parametrize("fmt,mips", [(0, False), (1, False), (0, True), (1, True)])
def test_chart_atlas_packed_on_the_gpu(fmt, mips):
    """ts_atlas_pack_charts: chart table = (exclusive sum of the charts' sizes, log2 side) in
    primitive order, level 0 = the primitive's texels in the target layout, and with mips
    level 1 = the 2x2 block means of level 0."""
    P = _pkg()
    rng = np.random.default_rng(7 + fmt + 2 * mips)
    n = 300
    log2 = rng.integers(0, 6, n).astype(np.int32)
    sides = 1 << log2.astype(np.int64)
    flat = rng.uniform(-1, 1, size=(int((sides * sides).sum()), 8)).astype(np.float32)
    sc = synth.make_scene("shell2k", n=n)
    ds = P.DeviceScene.from_dict(dict(sc, textures=flat), device="cuda", chart_log2=log2,
                                 tex_format=fmt, mips=mips)
    torch.cuda.synchronize()
    C = 7 if fmt else 8
    chain = (4 * sides * sides - 1) // 3 if mips else sides * sides
    offs = np.concatenate([[0], np.cumsum(chain)])[:-1]
    table = ds.chart_table.cpu().numpy()
    np.testing.assert_array_equal(table[:, 0], offs)
    np.testing.assert_array_equal(table[:, 1], log2)
    atlas = ds.atlas.view(-1, C).cpu().numpy()
    src = np.concatenate([[0], np.cumsum(sides * sides)])
    lv0 = _n2(flat) if fmt else flat
    for k in range(n):
        m = int(sides[k] ** 2)
        np.testing.assert_array_equal(atlas[offs[k]:offs[k] + m], lv0[src[k]:src[k] + m])
        if mips and sides[k] > 1:
            s0 = int(sides[k])
            l1 = atlas[offs[k] + m:offs[k] + m + m // 4].reshape(s0 // 2, s0 // 2, C)
            ref = lv0[src[k]:src[k] + m].astype(np.float64).reshape(s0 // 2, 2, s0 // 2, 2, C)
            np.testing.assert_allclose(l1, ref.mean(axis=(1, 3)), rtol=1e-6, atol=1e-7)


def test_two_component_normals_full_frame():
    sc = synth.make_scene("shell2k")
    cam = synth.config_cameras("shell2k")[0]
    ds, out = _render(sc, [cam], 128, 128, tex_format=1)
    _frame(_oracle_scene(sc, fmt=1), cam, out, name="normals xy")


@pytest.mark.parametrize("T", [4, 8, 16])
def test_trilinear_ragged_views(T):
    """Orbit views from farther away (texture minification: most samples take levels > 0)."""
    sc = synth.make_scene("sq100k", n=4000, tex_res=T, env_res=32)
    sc["env_levels"] = 3
    cams = synth.orbit_cameras(3, 77, 59, dist=5.5, el_deg=25.0)
    ds, out = _render(sc, cams, 77, 59, mips=True)
    for v in range(3):
        _frame(_oracle_scene(sc, tri=True), cams[v], out, v=v, name=f"trilinear T={T} v{v}")


def test_trilinear_two_component_close_and_far():
    sc = synth.make_scene("shell2k", n=1500, tex_res=8)
    for dist in (1.6, 7.0):
        cams = synth.orbit_cameras(2, 64, 48, dist=dist, el_deg=10.0)
        ds, out = _render(sc, cams, 64, 48, mips=True, tex_format=1)
        for v in range(2):
            _frame(_oracle_scene(sc, fmt=1, tri=True), cams[v], out, v=v,
                   name=f"trilinear xy dist={dist} v{v}")


@pytest.mark.parametrize("fmt,tri", [(0, False), (1, False), (0, True), (1, True)])
def test_adaptive_resolution(fmt, tri):
    """Per-splat sides 1..16 by primitive size, one table-addressed atlas."""
    sc = synth.make_scene("sq100k", n=3000, env_res=32)
    sc["env_levels"] = 3
    log2 = synth.texture_sides(sc["scales"])
    assert len(np.unique(log2)) >= 4
    flat = synth.adaptive_textures(np.random.default_rng(3), log2)
    sc_g = dict(sc, textures=flat)
    cams = synth.orbit_cameras(2, 70, 66, dist=3.5 if tri else 2.6, el_deg=30.0)
    ds, out = _render(sc_g, cams, 70, 66, chart_log2=log2, tex_format=fmt, mips=tri)
    osc = _oracle_scene(sc, fmt=fmt, tri=tri, log2=log2, flat=flat)
    for v in range(2):
        _frame(osc, cams[v], out, v=v, name=f"adaptive fmt={fmt} tri={tri} v{v}", graze=0.02)


def test_variants_full_size_sampled():
    """100k splats, all 64 orbit views at 800x800 in one launch, two-component normals with
    trilinear sampling; two views checked at sampled pixels."""
    sc = synth.make_scene("sq100k")
    cams = synth.config_cameras("sq100k")
    P = _pkg()
    ds = P.DeviceScene.from_dict(sc, device="cuda", tex_format=1, mips=True)
    out = P.render(ds, cams, 800, 800, gbuf=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    osc = _oracle_scene(sc, fmt=1, tri=True)
    for v in (5, 40):
        pix = sample_pixels(rng, 800, 800, 160)
        _frame(osc, cams[v], out, v=v, pixels=pix, name=f"sq100k xy+trilinear v{v}")


def test_hardware_sampler_backward_is_refused():
    """The texture-unit sampler has no gfx950 path, forward or backward."""
    P = _pkg()
    from paper_2506_13348_amd import _ffi as F
    from paper_2506_13348_amd.autograd import BackwardRunner
    sc = synth.make_scene("shell2k", n=200)
    cam = synth.config_cameras("shell2k")[0]
    ds = P.DeviceScene.from_dict(sc, device="cuda")
    plan = P.RenderPlan(ds, [cam], 64, 64, gbuf=True, aux=True)
    plan.run()
    plan.check()
    plan.params.sampler = F.SAMPLER_HARDWARE
    grads = tuple(torch.zeros_like(t) for t in (ds.means, ds.quats, ds.scales, ds.opac, ds.atlas))
    with pytest.raises(RuntimeError, match="trilinear samplers are differentiated"):
        BackwardRunner(plan).run(torch.zeros(64 * 64 * 4, device="cuda"), grads)

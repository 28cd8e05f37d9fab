"""Pins of the oracle's texture variants: two-component tangent normals (Sec. 3.5.1),
per-chart texture resolution and trilinear filtering over a box-filtered mip chain (the
adaptive allocation and mipmapping of Sec. 5).

Expected values come from other routes: unit normals rebuilt from two components against the
three-component render; for a splat parallel to the image plane the texture coordinate is
affine in the pixel position with the analytic slope z / (f s) per pixel, so the mip level
lambda = log2(T z / (2 S f s)) is known in closed form, the levels are numpy block means and
the bilinear samples come from scipy.ndimage.map_coordinates (order 1, edge replication =
clamp-to-edge)."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from helpers import camera, face_on_splat, scene_from

NO_CLIP = {"alpha_max": 1.0}


def _to_n2(tex):
    """[.., 8] texels -> [.., 7] (albedo 3, roughness, n_x, n_y, metallic)."""
    return np.ascontiguousarray(np.concatenate([tex[..., 0:6], tex[..., 7:8]], -1))


def _small_scene(rng, n=150, T=4, constant=True):
    cam = camera(40, 40)
    splats = []
    for k in range(n):
        x, y = rng.integers(2, 38, 2)
        s = face_on_splat(cam, int(x), int(y), rng.uniform(2.2, 3.5),
                          scale=tuple(rng.uniform(0.03, 0.12, 2)), opac=rng.uniform(0.2, 0.9))
        # tilt the splat so the normals are not all along the view axis
        q = np.asarray(s["quat"], float) + rng.normal(0, 0.3, 4)
        s["quat"] = q / np.linalg.norm(q)
        splats.append(s)
    tex = rng.uniform(0.05, 1.0, size=(n, T, T, 8)).astype(np.float32)
    # unit normals with n_z >= 0.43 (|(n_x, n_y)| <= 0.9), n_z from the float32 n_x, n_y
    nxy = rng.normal(0, 0.35, size=(n, T, T, 2))
    r = np.linalg.norm(nxy, axis=-1, keepdims=True)
    nxy = (nxy * np.minimum(1.0, 0.9 / np.maximum(r, 1e-12))).astype(np.float32)
    nz = np.sqrt(1 - (nxy.astype(np.float64) ** 2).sum(-1))
    tex[..., 4:6] = nxy
    tex[..., 6] = nz
    if constant:
        tex[:] = tex[:, :1, :1]
    return scene_from(splats, textures=tex), cam


def test_two_component_normals_rebuild_unit_normals():
    """Unit tangent normals with n_z >= 0 stored as (n_x, n_y) give the same G-buffer as the
    three stored components when each splat's texture is constant (no filtering between
    different normals)."""
    rng = np.random.default_rng(0)
    sc, cam = _small_scene(rng)
    ref = oracle.render(sc, cam, shade=False)
    sc2 = dict(sc, textures=_to_n2(sc["textures"]), tex_format=1)
    out = oracle.render(sc2, cam, shade=False)
    assert (ref["rgba"][:, 3] > 0).sum() > 200
    # the only difference is the float32 rounding of the stored n_z (< 6e-8 relative)
    np.testing.assert_allclose(out["gbuf"], ref["gbuf"], atol=1e-7)
    np.testing.assert_array_equal(out["rgba"][:, 3], ref["rgba"][:, 3])


def test_two_component_normals_clamp_outside_the_unit_disk():
    """|(n_x, n_y)| > 1 rebuilds n_z = 0: the normal of the stored (n_x, n_y, 0)."""
    rng = np.random.default_rng(1)
    sc, cam = _small_scene(rng, n=60)
    tex = sc["textures"].copy()
    tex[..., 4] = 0.8
    tex[..., 5] = -0.9
    tex[..., 6] = 0.0
    ref = oracle.render(dict(sc, textures=tex), cam, shade=False)
    out = oracle.render(dict(sc, textures=_to_n2(tex), tex_format=1), cam, shade=False)
    np.testing.assert_allclose(out["gbuf"], ref["gbuf"], atol=1e-12)


def test_two_component_normals_filter_before_rebuilding():
    """With varying normals the rebuilt n_z follows the filtered (n_x, n_y), which is not
    the filtered n_z: the two encodings differ inside a texel cell."""
    rng = np.random.default_rng(2)
    sc, cam = _small_scene(rng, n=80, constant=False)
    ref = oracle.render(sc, cam, shade=False)
    out = oracle.render(dict(sc, textures=_to_n2(sc["textures"]), tex_format=1), cam, shade=False)
    np.testing.assert_allclose(out["gbuf"][:, :5], ref["gbuf"][:, :5], atol=1e-12)
    assert np.abs(out["gbuf"][:, 5:8] - ref["gbuf"][:, 5:8]).max() > 1e-4


def _levels(tex):
    """Box-filtered mip chain of a [T,T,C] texture by block means."""
    T = tex.shape[0]
    out = [tex.astype(np.float64)]
    b = 2
    while b <= T:
        out.append(tex.astype(np.float64).reshape(T // b, b, T // b, b, -1).mean(axis=(1, 3)))
        b *= 2
    return out


def _bilinear(level, s, t):
    Tl = level.shape[0]
    coords = np.array([[t * Tl - 0.5], [s * Tl - 0.5]])
    return np.array([ndimage.map_coordinates(level[..., c], coords, order=1, mode="nearest")[0]
                     for c in range(level.shape[2])])


def _trilinear_expected(tex, s, t, lam):
    lv = _levels(tex)
    L = len(lv) - 1
    if lam <= 0:
        return _bilinear(lv[0], s, t)
    l0 = int(math.floor(lam))
    if l0 >= L:
        return _bilinear(lv[L], s, t)
    f = lam - l0
    return (1 - f) * _bilinear(lv[l0], s, t) + f * _bilinear(lv[l0 + 1], s, t)


@pytest.mark.parametrize("T,lam", [(8, -0.4), (8, 0.5), (8, 1.5), (8, 2.7), (8, 3.6),
                                   (4, 1.25), (2, 0.8), (16, 3.3)])
def test_trilinear_level_and_blend_against_closed_form(T, lam):
    """A splat parallel to the image plane at depth z with s_u = s_v = sc and t_u, t_v along
    the image axes: s = 1/2 + (X - x) z / (2 S f sc) at pixel X, so every pixel of it has the
    footprint rho = z / (2 S f sc) and lambda = log2(T rho)."""
    cam = camera(33, 33)
    f, S, z = cam["fx"], 3.0, 2.5
    sc_ = T * z / (2 * S * f * 2.0 ** lam)
    spl = face_on_splat(cam, 16, 16, z, scale=(sc_, sc_), opac=0.9)
    rng = np.random.default_rng(int(T * 10 + lam * 7 + 50))
    tex = rng.uniform(0.0, 1.0, size=(1, T, T, 8)).astype(np.float32)
    tex[..., 4:7] = (0.0, 0.0, 1.0)
    sc = scene_from([spl], textures=tex)
    sc["trilinear"] = True
    # pixels whose s, t stay inside the support (|u|, |v| <= 2.5)
    step = 2 * S * 2.0 ** lam / T / (2 * S)          # change of s per pixel
    r = int(min(3, math.floor(2.5 / (2 * S) / step)))
    pts = np.array([[16 + dx, 16 + dy] for dy in range(-r, r + 1) for dx in range(-r, r + 1)],
                   np.int32)
    out = oracle.render(sc, cam, pixels=pts, shade=False, params=NO_CLIP)
    mean = np.asarray(spl["mean"], np.float32).astype(np.float64)
    w2c = np.asarray(cam["w2c"], np.float64)
    pc = w2c[:, :3] @ mean + w2c[:, 3]
    px = f * pc[0] / pc[2] + cam["cx"]
    py = cam["fy"] * pc[1] / pc[2] + cam["cy"]
    zc = pc[2]
    for p, (X, Y) in enumerate(pts):
        A = out["rgba"][p, 3]
        assert A > 0
        s = 0.5 + (X + 0.5 - px) * zc / (f * float(np.float32(sc_))) / (2 * S)
        t = 0.5 + (Y + 0.5 - py) * zc / (cam["fy"] * float(np.float32(sc_))) / (2 * S)
        lam_p = math.log2(T * zc / (2 * S * f * float(np.float32(sc_))))
        exp = _trilinear_expected(tex[0], s, t, lam_p)
        np.testing.assert_allclose(out["gbuf"][p, 0:3] / A, exp[0:3], atol=1e-6)
        np.testing.assert_allclose(out["gbuf"][p, 4] / A, exp[3], atol=1e-6)


def test_chart_table_with_uniform_charts_is_the_uniform_atlas():
    """Every chart T x T but stored at permuted offsets of a flat texel array and addressed
    through the table: the same image as the uniform atlas."""
    rng = np.random.default_rng(3)
    sc, cam = _small_scene(rng, n=90, T=4, constant=False)
    n, T = 90, 4
    perm = rng.permutation(n)
    flat = np.zeros((n * T * T, 8), np.float32)
    table = np.zeros((n, 2), np.int32)
    for c in range(n):
        slot = perm[c]
        flat[slot * T * T:(slot + 1) * T * T] = sc["textures"][c].reshape(-1, 8)
        table[c] = (slot * T * T, 2)
    ref = oracle.render(sc, cam)
    out = oracle.render(dict(sc, textures=flat, chart_table=table), cam)
    for k in ("rgba", "gbuf"):
        np.testing.assert_array_equal(out[k], ref[k])


def test_one_texel_charts_are_constant_attributes():
    """Charts of resolution 1 in a mixed-resolution atlas equal constant textures."""
    rng = np.random.default_rng(4)
    sc, cam = _small_scene(rng, n=70, T=4, constant=True)
    n = 70
    res = rng.choice([0, 1, 2], size=n)              # log2 T per chart
    parts, table, off = [], np.zeros((n, 2), np.int32), 0
    for c in range(n):
        Tc = 1 << res[c]
        parts.append(np.repeat(sc["textures"][c, :1, :1].reshape(1, 8), Tc * Tc, 0))
        table[c] = (off, res[c])
        off += Tc * Tc
    flat = np.concatenate(parts).astype(np.float32)
    ref = oracle.render(sc, cam)
    out = oracle.render(dict(sc, textures=flat, chart_table=table), cam)
    np.testing.assert_allclose(out["gbuf"], ref["gbuf"], atol=1e-12)
    np.testing.assert_allclose(out["rgba"], ref["rgba"], atol=1e-12)


def test_mixed_resolutions_with_trilinear_use_each_charts_own_chain():
    """Two splats parallel to the image plane with charts of 2 and 8 texels a side in one
    table-addressed atlas: each follows its own closed-form level (the 2-texel chart stops at
    its last level)."""
    cam = camera(40, 24)
    f, S, z = cam["fx"], 3.0, 2.5
    rng = np.random.default_rng(5)
    specs = [(2, 1.6, 10), (8, 1.3, 30)]              # (T, lambda, pixel x)
    splats, parts, table, off, texs = [], [], np.zeros((2, 2), np.int32), 0, []
    for c, (T, lam, x) in enumerate(specs):
        sc_ = T * z / (2 * S * f * 2.0 ** lam)
        splats.append(face_on_splat(cam, x, 12, z, scale=(sc_, sc_), opac=0.8))
        tex = rng.uniform(0, 1, size=(T, T, 8)).astype(np.float32)
        tex[..., 4:7] = (0.0, 0.0, 1.0)
        texs.append(tex)
        parts.append(tex.reshape(-1, 8))
        table[c] = (off, int(math.log2(T)))
        off += T * T
    sc = scene_from(splats, textures=np.zeros((2, 1, 1, 8), np.float32))
    sc.update(textures=np.concatenate(parts), chart_table=table, trilinear=True)
    pts = np.array([[10, 12], [30, 12]], np.int32)
    out = oracle.render(sc, cam, pixels=pts, shade=False, params=NO_CLIP)
    for p, (T, lam, x) in enumerate(specs):
        spl = splats[p]
        sc_ = float(np.float32(spl["scale"][0]))
        mean = np.asarray(spl["mean"], np.float32).astype(np.float64)
        w2c = np.asarray(cam["w2c"], np.float64)
        pc = w2c[:, :3] @ mean + w2c[:, 3]
        px = f * pc[0] / pc[2] + cam["cx"]
        py = cam["fy"] * pc[1] / pc[2] + cam["cy"]
        s = 0.5 + (x + 0.5 - px) * pc[2] / (f * sc_) / (2 * S)
        t = 0.5 + (12 + 0.5 - py) * pc[2] / (cam["fy"] * sc_) / (2 * S)
        lam_p = math.log2(T * pc[2] / (2 * S * f * sc_))
        exp = _trilinear_expected(texs[p], s, t, lam_p)
        A = out["rgba"][p, 3]
        np.testing.assert_allclose(out["gbuf"][p, 0:3] / A, exp[0:3], atol=1e-6)

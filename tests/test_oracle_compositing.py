"""Pins of the FP64 oracle's geometry, texturing and compositing against closed forms.

Each check derives its expected value by a route other than the oracle's own code: the
forward map of Eq. 1 plus the pinhole projection, quaternion Hamilton products, closed-form
products of (1 - alpha), texture fields whose bilinear interpolant is known exactly."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import (cam_axes, camera, face_on_splat, quat_of_frame, quat_rotate, scene_from)

NO_CLIP = {"alpha_max": 1.0}


def px(x, y):
    return np.array([[x, y]], np.int32)


def test_single_face_on_splat_centre():
    """u = v = 0 at the pixel whose ray hits the centre: G = 1 and alpha = min(0.99, o); the
    bilinear sample at s = t = 1/2 of an even-resolution texture is the mean of its four
    central texels (Eq. 2, Eq. 5, Eq. 6, Eq. 8)."""
    cam = camera(32, 32)
    rng = np.random.default_rng(3)
    T = 4
    tex = rng.uniform(0.1, 1.0, size=(1, T, T, 8)).astype(np.float32)
    s = face_on_splat(cam, 13, 17, 2.5, opac=0.7)
    sc = scene_from([s], textures=tex)
    out = oracle.render(sc, cam, pixels=px(13, 17), shade=False)
    a = float(np.float32(0.7))
    centre = tex[0, 1:3, 1:3].astype(np.float64).mean(axis=(0, 1))
    g = out["gbuf"][0]
    # the centre is stored in float32, so (u, v) is zero only to ~1e-7
    assert out["rgba"][0, 3] == pytest.approx(a, abs=1e-12)
    np.testing.assert_allclose(g[0:3], a * centre[0:3], atol=1e-7)
    assert g[3] == pytest.approx(a * centre[7], abs=1e-7)      # metallic
    assert g[4] == pytest.approx(a * centre[3], abs=1e-7)      # roughness
    right, down, fwd, o = cam_axes(cam)
    nt = centre[4:7] / np.linalg.norm(centre[4:7])
    n = np.cross(right, down)                                  # t_u x t_v
    sigma = 1.0 if np.dot(n, o - s["mean"]) >= 0 else -1.0
    nw = sigma * (nt[0] * right + nt[1] * down + nt[2] * n)
    np.testing.assert_allclose(g[5:8], a * nw, atol=1e-7)
    assert out["stat"][0, 0] == 1


def test_alpha_clamp_and_cutoff():
    cam = camera(16, 16)
    s1 = face_on_splat(cam, 8, 8, 2.0, opac=1.0)
    out = oracle.render(scene_from([s1]), cam, pixels=px(8, 8), shade=False)
    assert out["rgba"][0, 3] == pytest.approx(float(np.float32(0.99)), abs=1e-12)
    s2 = face_on_splat(cam, 8, 8, 2.0, opac=0.9 / 255)
    out = oracle.render(scene_from([s2]), cam, pixels=px(8, 8), shade=False)
    assert out["rgba"][0, 3] == 0.0 and out["stat"][0, 0] == 0


def test_two_splat_occlusion_order_by_depth_not_index():
    """X = c1 a1 + c2 a2 (1 - a1) with splat 1 nearer, whatever the index order (Eq. 3)."""
    cam = camera(16, 16)
    near = face_on_splat(cam, 5, 6, 2.0, opac=0.6)
    far = face_on_splat(cam, 5, 6, 2.7, opac=0.5)
    T = 2
    for order in ([near, far], [far, near]):
        tex = np.zeros((2, T, T, 8), np.float32)
        tex[..., 6] = 1
        i_near = 0 if order[0] is near else 1
        tex[i_near, ..., 0] = 0.25
        tex[1 - i_near, ..., 0] = 0.75
        out = oracle.render(scene_from(order, textures=tex), cam, pixels=px(5, 6), shade=False)
        a1, a2 = float(np.float32(0.6)), 0.5
        exp_x = 0.25 * a1 + 0.75 * a2 * (1 - a1)
        assert out["gbuf"][0, 0] == pytest.approx(exp_x, abs=1e-12)
        assert out["rgba"][0, 3] == pytest.approx(1 - (1 - a1) * (1 - a2), abs=1e-12)


def test_equal_depth_ties_go_by_index():
    """Splats whose depths round to the same float32 key blend in index order."""
    cam = camera(16, 16)
    a = face_on_splat(cam, 7, 7, 2.0, opac=0.5)
    b = face_on_splat(cam, 7, 7, 2.0, opac=0.5)
    b = dict(b, scale=(0.2, 0.2))
    tex = np.zeros((2, 2, 2, 8), np.float32)
    tex[..., 6] = 1
    tex[0, ..., 0] = 1.0
    out = oracle.render(scene_from([a, b], textures=tex), cam, pixels=px(7, 7), shade=False)
    assert out["gbuf"][0, 0] == pytest.approx(0.5, abs=1e-12)  # index 0 in front
    out = oracle.render(scene_from([b, a], textures=tex[::-1].copy()), cam, pixels=px(7, 7),
                        shade=False)
    assert out["gbuf"][0, 0] == pytest.approx(0.5 * 0.5, abs=1e-12)


def test_termination_before_transmittance_threshold():
    """Twenty alpha = 1/2 layers: blending stops before the first splat that would take T
    below 1e-4, i.e. after 13 layers (0.5^13 >= 1e-4 > 0.5^14)."""
    cam = camera(16, 16)
    layers = [face_on_splat(cam, 4, 9, 2.0 + 0.01 * k, opac=0.5) for k in range(20)]
    out = oracle.render(scene_from(layers), cam, pixels=px(4, 9), shade=False)
    assert out["stat"][0, 0] == 13
    assert out["rgba"][0, 3] == pytest.approx(1 - 0.5 ** 13, abs=1e-15)


def test_near_plane_cull():
    cam = camera(16, 16)
    s = face_on_splat(cam, 8, 8, 0.15, opac=0.9, scale=(0.01, 0.01))
    out = oracle.render(scene_from([s]), cam, pixels=px(8, 8), shade=False)
    assert out["rgba"][0, 3] == 0.0


def _round_trip_setup(u, v, q, cam, mu, s_uv):
    """Shift the principal point so that the pixel-centre ray of (10, 10) passes through
    P(u, v) = mu + s_u t_u u + s_v t_v v (Eq. 1). Frame from quaternion Hamilton products."""
    tu = quat_rotate(q, [1.0, 0, 0])
    tv = quat_rotate(q, [0, 1.0, 0])
    P = mu + s_uv[0] * u * tu + s_uv[1] * v * tv
    w2c = np.asarray(cam["w2c"], np.float64)
    pc = w2c[:, :3] @ P + w2c[:, 3]
    xp = cam["fx"] * pc[0] / pc[2] + cam["cx"]
    yp = cam["fy"] * pc[1] / pc[2] + cam["cy"]
    c = dict(cam)
    c["cx"] = cam["cx"] + (10.5 - xp)
    c["cy"] = cam["cy"] + (10.5 - yp)
    return c


@pytest.mark.parametrize("seed", range(6))
def test_round_trip_uv_oblique(seed):
    """For an oblique splat, pick (u, v), place the pixel-centre ray through P(u, v) and
    check alpha = o exp(-(u^2+v^2)/2) and the texture value at (s, t) of Eq. 5 for an affine
    texel field, which bilinear filtering reproduces exactly inside [1/2T, 1-1/2T]."""
    rng = np.random.default_rng(seed)
    cam = camera(24, 24)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    tu, tv, n = (quat_rotate(q, e) for e in np.eye(3))
    _, _, fwd, o = cam_axes(cam)
    if abs(np.dot(n, fwd)) < 0.3:  # keep the view well away from grazing
        q = quat_of_frame(tu, np.cross(fwd, tu) / np.linalg.norm(np.cross(fwd, tu)),
                          np.cross(tu, np.cross(fwd, tu) / np.linalg.norm(np.cross(fwd, tu))))
        tu, tv, n = (quat_rotate(q, e) for e in np.eye(3))
    mu = rng.uniform(-0.3, 0.3, size=3)
    s_uv = rng.uniform(0.05, 0.2, size=2)
    u, v = rng.uniform(-2.2, 2.2, size=2)
    c = _round_trip_setup(u, v, q, cam, mu, s_uv)
    T = 8
    ii, jj = np.meshgrid(np.arange(T), np.arange(T), indexing="xy")
    tex = np.zeros((1, T, T, 8), np.float32)
    tex[0, :, :, 0] = 0.1 + 0.05 * ii + 0.02 * jj     # affine in (i, j)
    tex[0, :, :, 6] = 1.0
    op = float(np.float32(0.8))
    sc = scene_from([{"mean": mu, "quat": q, "scale": s_uv, "opac": op}], textures=tex)
    out = oracle.render(sc, c, pixels=px(10, 10), shade=False, params=NO_CLIP)
    alpha = op * math.exp(-0.5 * (u * u + v * v))
    sc_mu = sc["means"][0].astype(np.float64)
    assert out["rgba"][0, 3] == pytest.approx(alpha, rel=1e-5)
    X = (u + 3) / 6 * T - 0.5
    Y = (v + 3) / 6 * T - 0.5
    assert out["gbuf"][0, 0] == pytest.approx(alpha * (0.1 + 0.05 * X + 0.02 * Y), rel=1e-5)
    assert sc_mu is not None


def test_constant_texture_reduces_to_single_attribute():
    """Stage-two initialisation (Sec. 4.1): textures holding each splat's single attribute
    render exactly as 1x1 textures (the untextured primitive)."""
    sc = synth.make_scene("shell2k", n=300, tex_res=4)
    cam = synth.config_cameras("shell2k")[0]
    cam = synth.crop_camera(cam, 40, 40, 48, 48)
    rng = np.random.default_rng(5)
    attr = rng.uniform(0.05, 1.0, size=(300, 8)).astype(np.float32)
    attr[:, 4:7] = synth._normalize(rng.normal(size=(300, 3)) + [0, 0, 2]).astype(np.float32)
    tex4 = np.broadcast_to(attr[:, None, None, :], (300, 4, 4, 8)).copy()
    tex1 = attr[:, None, None, :].copy()
    a = oracle.render(dict(sc, textures=tex4), cam, shade=False)
    b = oracle.render(dict(sc, textures=tex1, tex_res=1), cam, shade=False)
    np.testing.assert_allclose(a["gbuf"], b["gbuf"], atol=1e-12)
    np.testing.assert_array_equal(a["rgba"][:, 3], b["rgba"][:, 3])
    assert (a["stat"][:, 0] > 0).sum() > 200


def test_weights_telescope_to_alpha():
    """sum_i alpha_i T_i = 1 - prod_i (1 - alpha_i): a unit albedo texture blends to A."""
    sc = synth.make_scene("shell2k", n=600)
    cam = synth.crop_camera(synth.config_cameras("shell2k")[0], 32, 32, 64, 64)
    tex = sc["textures"].copy()
    tex[..., 0] = 1.0
    out = oracle.render(dict(sc, textures=tex), cam, shade=False)
    np.testing.assert_allclose(out["gbuf"][:, 0], out["rgba"][:, 3], atol=1e-12)
    A = out["rgba"][:, 3]
    assert A.min() >= 0.0 and A.max() <= 1 - 1e-4 + 1e-15


def test_transmittance_monotone_in_splat_prefix():
    """Adding splats never raises transmittance: A over the first k splats is
    non-decreasing in k when the extra splats lie behind the first ones."""
    cam = camera(16, 16)
    rng = np.random.default_rng(2)
    sp = [face_on_splat(cam, 8, 8, 2.0 + 0.1 * k, opac=float(rng.uniform(0.1, 0.6)),
                        scale=tuple(rng.uniform(0.05, 0.3, 2))) for k in range(12)]
    pix = np.stack(np.meshgrid(np.arange(16), np.arange(16)), -1).reshape(-1, 2).astype(np.int32)
    prev = np.zeros(len(pix))
    for k in range(1, 13):
        A = oracle.render(scene_from(sp[:k]), cam, pixels=pix, shade=False)["rgba"][:, 3]
        assert np.all(A >= prev - 1e-15)
        prev = A


def test_flat_tangent_normal_gives_primitive_normal():
    """n^t = (0,0,1) maps to n_w = sigma R e_z = sigma t_u x t_v (Eq. 7 with n = t_u x t_v)."""
    rng = np.random.default_rng(11)
    cam = camera(24, 24)
    _, _, fwd, o = cam_axes(cam)
    for trial in range(5):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        tu, tv = quat_rotate(q, [1.0, 0, 0]), quat_rotate(q, [0, 1.0, 0])
        n = np.cross(tu, tv)
        if abs(np.dot(n, fwd)) < 0.2:
            continue
        mu = rng.uniform(-0.2, 0.2, 3)
        c = _round_trip_setup(0.0, 0.0, q, cam, mu, (0.1, 0.1))
        sc = scene_from([{"mean": mu, "quat": q, "scale": (0.1, 0.1), "opac": 0.5}])
        out = oracle.render(sc, c, pixels=px(10, 10), shade=False)
        sigma = 1.0 if np.dot(n, o - mu) >= 0 else -1.0
        np.testing.assert_allclose(out["gbuf"][0, 5:8], 0.5 * sigma * n, atol=1e-6)


def test_depth_key_is_float32_of_camera_depth():
    """Sort keys: depth along the optical axis from the camera centre, rounded to float32."""
    sc = synth.make_scene("shell2k")
    cam = synth.config_cameras("shell2k")[0]
    d32, keep, _ = oracle.splat_setup(sc, cam)
    _, _, fwd, o = cam_axes(cam)
    z = (sc["means"].astype(np.float64) - o) @ fwd
    same = d32 == z.astype(np.float32)
    assert same.mean() > 0.999
    np.testing.assert_allclose(d32, z, rtol=1.2e-7)
    np.testing.assert_array_equal(keep, z > 0.2)


def test_support_edge_is_flagged_with_both_outcomes():
    """A pixel landing exactly on u = S is a decision a rounding can flip: it is recorded and
    the alternate render takes the other branch."""
    cam = camera(24, 24)
    q = quat_of_frame(*[np.asarray(v) for v in cam_axes(cam)[:2]],
                      np.cross(cam_axes(cam)[0], cam_axes(cam)[1]))
    mu = np.array([0.05, -0.03, 0.1])
    c = _round_trip_setup(3.0, 0.4, q, cam, mu, (0.1, 0.1))
    sc = scene_from([{"mean": mu, "quat": q, "scale": (0.1, 0.1), "opac": 0.9}])
    out = oracle.render(sc, c, pixels=px(10, 10), shade=False)
    assert out["stat"][0, 2] >= 1 and out["stat"][0, 5] >= 1
    both = {round(out["rgba"][0, 3], 9), round(out["alt_rgba"][0, 0, 3], 9)}
    expected_in = float(np.float32(0.9)) * math.exp(-0.5 * (9 + 0.16))
    assert 0.0 in both and any(abs(b - expected_in) < 1e-5 for b in both)

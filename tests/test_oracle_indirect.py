"""Pins of the oracle's indirect term (Eq. 9 and Eq. 12) and of its spherical harmonics.

Expected values come from other routes than the oracle's code: scipy's complex spherical
harmonics turned into the real basis, Gauss-Legendre quadrature of the basis products, the
addition theorem, the reflection law checked through Hamilton-product normals, the albedo
blend of the same scene (a second, already pinned, route through Eq. 9), and identities of
the specular mix that hold for any tables."""
import math

import numpy as np
import pytest
import scipy.special as sps

import oracle
import synth
from helpers import cam_axes, camera, quat_rotate


def _unit_dirs(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _scipy_real_sh(l, m, d):
    """Real orthonormal SH from scipy's complex Y_l^m (which carries the Condon-Shortley
    phase): sqrt(2) (-1)^m Re Y_l^m for m > 0, sqrt(2) (-1)^m Im Y_l^|m| for m < 0."""
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    y = sps.sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return y.real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * y.real
    return math.sqrt(2) * (-1) ** m * y.imag


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = _unit_dirs(rng, 200)
    B = oracle.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(B[:, l * l + l + m], _scipy_real_sh(l, m, d), atol=1e-12,
                                       err_msg=f"l={l} m={m}")


def test_sh_band_one_is_the_direction():
    """Band 1 is sqrt(3/(4 pi)) (y, z, x): the index order l*l + l + m with no phase sign."""
    rng = np.random.default_rng(1)
    d = _unit_dirs(rng, 50)
    B = oracle.sh_basis(1, d)
    c = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(B[:, 0], 0.5 / math.sqrt(math.pi), atol=1e-14)
    np.testing.assert_allclose(B[:, 1:4], c * d[:, [1, 2, 0]], atol=1e-14)


def test_sh_orthonormal_by_quadrature():
    """Gram matrix of the degree-3 basis over the sphere by Gauss-Legendre in cos(theta)
    times uniform phi (exact for these polynomial degrees) is the identity."""
    x, wx = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    B = oracle.sh_basis(3, d)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_addition_theorem():
    """sum_m Y_lm(w)^2 = (2l+1)/(4 pi) for every direction."""
    rng = np.random.default_rng(2)
    B = oracle.sh_basis(3, _unit_dirs(rng, 100))
    for l in range(4):
        np.testing.assert_allclose((B[:, l * l:(l + 1) ** 2] ** 2).sum(1),
                                   (2 * l + 1) / (4 * math.pi), rtol=1e-12)


def _small_scene(n=60, seed=4):
    sc = synth.make_scene("shell2k", seed=seed, n=n)
    return sc


def test_indirect_direction_is_the_mirror_reflection():
    """Coefficients chosen so that channel c reads 2 + w_r[c] (band 0 = 2, band 1 picks x, y,
    z): the recovered w_r is a unit vector with w_r.n = -d.n and w_r - d parallel to n, d the
    unit camera-to-centre direction and n the splat normal (rotated z axis)."""
    sc = _small_scene()
    cam = camera(32, 32, eye=(0.3, -0.4, 3.0))
    n = len(sc["opac"])
    sh = np.zeros((n, 4, 3), np.float32)
    sh[:, 0, :] = 2.0 * 2.0 * math.sqrt(math.pi)        # Y_00 = 1/(2 sqrt(pi))
    k1 = 1.0 / math.sqrt(3 / (4 * math.pi))
    sh[:, 3, 0] = k1    # x
    sh[:, 1, 1] = k1    # y
    sh[:, 2, 2] = k1    # z
    li = oracle.indirect_eval(sc, cam, sh, 1)
    sh32 = sh.astype(np.float64)
    wr = li - sh32[:, 0, :] * (0.5 / math.sqrt(math.pi))
    wr = wr / (sh32[:, 3, 0][:, None] * math.sqrt(3 / (4 * math.pi)))
    o = cam_axes(cam)[3]
    for k in range(n):
        q = sc["quats"][k].astype(np.float64)
        nk = quat_rotate(q, np.array([0.0, 0.0, 1.0]))
        d = sc["means"][k].astype(np.float64) - o
        d /= np.linalg.norm(d)
        assert np.linalg.norm(wr[k]) == pytest.approx(1.0, abs=1e-6)
        assert np.dot(wr[k], nk) == pytest.approx(-np.dot(d, nk), abs=1e-6)
        np.testing.assert_allclose(np.cross(wr[k] - d, nk), 0.0, atol=1e-6)


def test_indirect_sign_of_normal_does_not_matter_and_clamps_at_zero():
    sc = _small_scene()
    cam = camera(32, 32)
    rng = np.random.default_rng(5)
    sh = synth.indirect_sh(rng, len(sc["opac"]), 3)
    a = oracle.indirect_eval(sc, cam, sh, 3)
    # a half turn about t_u flips n (and t_v): q -> q * (0, 1, 0, 0)
    w, x, y, z = sc["quats"].astype(np.float64).T
    flipped = dict(sc)
    flipped["quats"] = np.stack([-x, w, z, -y], 1).astype(np.float32)
    b = oracle.indirect_eval(flipped, cam, sh, 3)
    np.testing.assert_allclose(a, b, atol=1e-5)
    neg = -np.abs(sh)
    neg[:, 1:] = 0
    assert (oracle.indirect_eval(sc, cam, neg, 3) == 0).all()
    # degree 2 equals degree 3 with the third band removed
    sh2 = sh[:, :9].copy()
    sh3 = sh.copy()
    sh3[:, 9:] = 0
    np.testing.assert_array_equal(oracle.indirect_eval(sc, cam, sh2, 2),
                                  oracle.indirect_eval(sc, cam, sh3, 3))


def _scene_and_lind(seed=6):
    sc = synth.make_scene("shell2k", seed=seed, n=300)
    cam = camera(40, 36)
    rng = np.random.default_rng(seed)
    li = oracle.indirect_eval(sc, cam, synth.indirect_sh(rng, len(sc["opac"]), 3), 3)
    return sc, cam, li


def test_indirect_map_blends_like_a_constant_albedo():
    """Eq. 9: L_ind = sum_i l_i alpha_i T_i, the blend of any other map. With the albedo
    texels of every splat set to its l_ind, the albedo map must equal the L_ind map."""
    sc, cam, li = _scene_and_lind()
    out = oracle.render(sc, cam, shade=False, lind=li)
    sc2 = dict(sc)
    tex = sc["textures"].copy()
    tex[..., 0:3] = li.astype(np.float32)[:, None, None, :]
    sc2["textures"] = tex
    li32 = li.astype(np.float32).astype(np.float64)
    out_li32 = oracle.render(sc, cam, shade=False, lind=li32)
    ref = oracle.render(sc2, cam, shade=False)
    assert (out["gind"] != 0).any()
    np.testing.assert_allclose(out_li32["gind"], ref["gbuf"][:, 0:3], atol=1e-12)
    np.testing.assert_allclose(out["rgba"][:, 3], ref["rgba"][:, 3], atol=0)


def test_full_visibility_is_the_plain_split_sum():
    sc, cam, li = _scene_and_lind()
    plain = oracle.render(sc, cam)
    vis1 = oracle.render(sc, cam, lind=li, vis=np.ones(cam["width"] * cam["height"]))
    np.testing.assert_array_equal(vis1["rgba"], plain["rgba"])


def _const_tables(sc, value):
    t = oracle.tables(sc["env"], sc["env_levels"])
    return {"spec": [np.full_like(l, 0.0) + np.asarray(value) for l in t["spec"]],
            "irr": t["irr"], "lut": t["lut"]}


def test_occluded_pixels_take_the_indirect_light_through_the_brdf_table():
    """V = 0 and L_ind = c A (every splat radiating c): the specular term becomes
    (F0 a + b) c A, i.e. A times the specular term of an environment whose prefiltered
    levels are the constant c, while the diffuse term is untouched."""
    sc, cam, _ = _scene_and_lind()
    c = np.array([0.7, 1.3, 0.4])
    n = len(sc["opac"])
    P = cam["width"] * cam["height"]
    occl = oracle.render(sc, cam, lind=np.tile(c, (n, 1)), vis=np.zeros(P),
                         tabs=_const_tables(sc, 0.0))
    dark = oracle.render(sc, cam, tabs=_const_tables(sc, 0.0))
    lit = oracle.render(sc, cam, tabs=_const_tables(sc, c))
    A = dark["rgba"][:, 3:4]
    assert (A > 0.3).any()
    np.testing.assert_allclose(occl["rgba"][:, :3] - dark["rgba"][:, :3],
                               A * (lit["rgba"][:, :3] - dark["rgba"][:, :3]), atol=1e-12)


def test_shading_is_affine_in_visibility():
    """C(V) = (1 - V) C(0) + V C(1) for given G-buffers (Eq. 12 mixes the two lights by V)."""
    rng = np.random.default_rng(8)
    H, W = 6, 7
    g, a = synth.random_gbuffer(rng, 1, H, W)
    gind = rng.uniform(0, 2, size=(H * W, 3)) * a.reshape(-1, 1)
    sc = _small_scene()
    cam = camera(W, H)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(W, H)
    gb = g[0].reshape(8, -1).T
    V = rng.uniform(0, 1, H * W)
    c0, _ = oracle.shade_gbuffer(gb, a.reshape(-1), cam, pix, tabs, gind=gind, vis=np.zeros(H * W))
    c1, _ = oracle.shade_gbuffer(gb, a.reshape(-1), cam, pix, tabs, gind=gind, vis=np.ones(H * W))
    cv, _ = oracle.shade_gbuffer(gb, a.reshape(-1), cam, pix, tabs, gind=gind, vis=V)
    np.testing.assert_allclose(cv, (1 - V)[:, None] * c0 + V[:, None] * c1, atol=1e-12)
    plain, _ = oracle.shade_gbuffer(gb, a.reshape(-1), cam, pix, tabs)
    np.testing.assert_array_equal(c1, plain)

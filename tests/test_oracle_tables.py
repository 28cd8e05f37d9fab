"""Pins of the oracle's cube-map addressing, pre-integrated tables and shading.

References used: the exact solid angle of the sphere (4 pi), Lambert's cosine integral
(pi c for a constant environment, pi a + 2 pi/3 b.n for a linear one), Schlick's Fresnel at
zero roughness, numerical quadrature (scipy) of the continuous split-sum and GGX-prefilter
integrals, and a mirror reflecting a face-constant environment."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from helpers import camera


@pytest.fixture(scope="module")
def lut():
    return oracle.brdf_lut(256, 4096)


def test_cube_solid_angles_sum_to_sphere():
    for r in (1, 4, 16, 33):
        _, solid = oracle.cube_texels(r)
        assert solid.sum() == pytest.approx(4 * math.pi, abs=1e-12)
        assert solid.min() > 0


def test_cube_texel_round_trip_and_faces():
    """Looking up a texel's own centre direction returns that texel exactly; the major axis
    selects faces +X,-X,+Y,-Y,+Z,-Z."""
    r = 8
    dirs, _ = oracle.cube_texels(r)
    cube = np.arange(6 * r * r * 3, dtype=np.float64).reshape(6, r, r, 3)
    got = oracle.cube_sample(cube, dirs.reshape(-1, 3))
    np.testing.assert_allclose(got, cube.reshape(-1, 3), atol=1e-9)
    face_cube = np.repeat(np.arange(6, dtype=np.float64), r * r * 3).reshape(6, r, r, 3)
    probes = np.array([[1, .3, -.2], [-1, .5, .4], [.2, 1, -.6], [.1, -1, .7], [.4, -.2, 1],
                       [-.5, .6, -1]], np.float64)
    np.testing.assert_array_equal(oracle.cube_sample(face_cube, probes)[:, 0], np.arange(6))
    # ties go X, then Y, then Z
    ties = np.array([[1, 1, 0.2], [0.3, 1, 1], [1, -0.5, -1]], np.float64)
    np.testing.assert_array_equal(oracle.cube_sample(face_cube, ties)[:, 0], [0, 2, 0])


def test_irradiance_constant_and_linear_environment():
    r = 32
    dirs, _ = oracle.cube_texels(r)
    E = oracle.irradiance(np.full((6, r, r, 3), 2.0, np.float32), 8)
    np.testing.assert_allclose(E, 2.0 * math.pi, rtol=2e-3)
    a, b = 1.5, np.array([0.3, -0.2, 0.5])
    env = (a + dirs @ b)[..., None].repeat(3, axis=-1).astype(np.float32)
    E = oracle.irradiance(env, 8)
    ndirs, _ = oracle.cube_texels(8)
    expect = math.pi * a + 2 * math.pi / 3 * (ndirs @ b)
    np.testing.assert_allclose(E[..., 0], expect, rtol=3e-3)


def test_prefilter_levels():
    r = 16
    env = np.full((6, r, r, 3), 0.7, np.float32)
    lv = oracle.prefilter(env, 4)
    assert [l.shape[1] for l in lv] == [16, 8, 4, 2]
    for l in lv:
        np.testing.assert_allclose(l, float(np.float32(0.7)), rtol=1e-12)
    rng = np.random.default_rng(0)
    env = rng.uniform(0.5, 2.0, size=(6, r, r, 3)).astype(np.float32)
    lv = oracle.prefilter(env, 3)
    np.testing.assert_array_equal(lv[0], env.astype(np.float64))
    # a weighted mean: every value lies within the environment's range
    assert lv[1].min() >= env.min() - 1e-12 and lv[2].max() <= env.max() + 1e-12


def _pref_continuous(L, rdir, alpha):
    """Continuous GGX prefilter with N = V = R: int L (r.w) D(h) dw / int (r.w) D(h) dw,
    over the hemisphere around r, by scipy quadrature."""
    rdir = rdir / np.linalg.norm(rdir)
    helper = np.array([1.0, 0, 0]) if abs(rdir[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(rdir, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(rdir, e1)
    a2 = alpha * alpha

    def D(c):
        d = c * c * (a2 - 1) + 1
        return a2 / (math.pi * d * d)

    def f(th, ph, with_L):
        w = math.sin(th) * (math.cos(ph) * e1 + math.sin(ph) * e2) + math.cos(th) * rdir
        h = w + rdir
        h /= np.linalg.norm(h)
        val = math.cos(th) * D(float(np.dot(h, rdir))) * math.sin(th)
        return val * (L(w) if with_L else 1.0)

    num = integrate.dblquad(lambda th, ph: f(th, ph, True), 0, 2 * math.pi, 0, math.pi / 2,
                            epsabs=1e-9, epsrel=1e-7)[0]
    den = integrate.dblquad(lambda th, ph: f(th, ph, False), 0, 2 * math.pi, 0, math.pi / 2,
                            epsabs=1e-9, epsrel=1e-7)[0]
    return num / den


@pytest.mark.parametrize("level,alpha_rough", [(2, 2 / 3), (3, 1.0)])
def test_prefilter_matches_continuous_integral(level, alpha_rough):
    """Level l of L = 4 is the GGX prefilter at roughness l/3 (alpha = roughness^2)."""
    r = 48
    dirs, _ = oracle.cube_texels(r)

    def L(w):
        return 1.0 + 0.5 * w[0] + 2.0 * w[2] * w[2]

    env = (1.0 + 0.5 * dirs[..., 0] + 2.0 * dirs[..., 2] ** 2)[..., None].repeat(3, -1)
    lv = oracle.prefilter(env.astype(np.float32), 4)
    rl = r >> level
    ldirs, _ = oracle.cube_texels(rl)
    for (f, j, i) in [(4, rl // 2, rl // 2), (0, 1, rl - 2), (2, 0, 0)]:
        want = _pref_continuous(L, ldirs[f, j, i], alpha_rough ** 2)
        assert lv[level][f, j, i, 0] == pytest.approx(want, rel=3e-3)


def test_lut_zero_roughness_is_schlick(lut):
    """At roughness -> 0 every half vector is the normal and G = 1: A = 1 - (1-N.V)^5,
    B = (1-N.V)^5."""
    nv = (np.arange(256) + 0.5) / 256
    fc = (1 - nv) ** 5
    ok = nv > 0.02   # the Smith term at k = 2e-6 departs from 1 only for N.V ~ k
    np.testing.assert_allclose(lut[0, ok, 0], 1 - fc[ok], atol=2e-4)
    np.testing.assert_allclose(lut[0, ok, 1], fc[ok], atol=2e-4)


def test_lut_bounds(lut):
    assert lut.min() >= 0.0
    assert (lut[..., 0] + lut[..., 1]).max() <= 1.0 + 2e-3


def _lut_continuous(nv, rough):
    """A, B of the split-sum BRDF integral by quadrature over the light hemisphere."""
    a = rough * rough
    k = a / 2
    v = np.array([math.sqrt(1 - nv * nv), 0.0, nv])

    def g1(x):
        return x / (x * (1 - k) + k)

    def integrand(th, ph, which):
        l = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        h = v + l
        h /= np.linalg.norm(h)
        nh, vh, nl = h[2], max(float(np.dot(v, h)), 0.0), l[2]
        d = nh * nh * (a * a - 1) + 1
        D = a * a / (math.pi * d * d)
        G = g1(nv) * g1(nl)
        fc = (1 - vh) ** 5
        w = fc if which else (1 - fc)
        return w * D * G / (4 * nv) * math.sin(th)

    A = integrate.dblquad(lambda th, ph: integrand(th, ph, 0), 0, 2 * math.pi, 0, math.pi / 2,
                          epsabs=1e-8)[0]
    B = integrate.dblquad(lambda th, ph: integrand(th, ph, 1), 0, 2 * math.pi, 0, math.pi / 2,
                          epsabs=1e-8)[0]
    return A, B


@pytest.mark.parametrize("nv,rough", [(0.25, 0.5), (0.7, 0.35), (0.9, 0.8)])
def test_lut_matches_quadrature(lut, nv, rough):
    """The 4096-sample Hammersley estimate at a texel centre agrees with the integral."""
    i = int(round(nv * 256 - 0.5))
    j = int(round(rough * 256 - 0.5))
    nv_c, r_c = (i + 0.5) / 256, (j + 0.5) / 256
    A, B = _lut_continuous(nv_c, r_c)
    assert lut[j, i, 0] == pytest.approx(A, abs=4e-3)
    assert lut[j, i, 1] == pytest.approx(B, abs=2e-3)


def _const_tables(c, lut, r=16, levels=3):
    env = np.full((6, r, r, 3), c, np.float32)
    return {"spec": oracle.prefilter(env, levels), "irr": oracle.irradiance(env, 8), "lut": lut}


def test_shading_empty_pixel_is_background(lut):
    cam = camera(8, 8)
    tabs = _const_tables(1.0, lut)
    rgb, _ = oracle.shade_gbuffer(np.zeros((1, 8)), np.zeros(1), cam, np.array([[3, 4]]), tabs,
                                  params={"bg": (0.2, 0.3, 0.4)})
    np.testing.assert_allclose(rgb[0], np.float32([0.2, 0.3, 0.4]), atol=1e-12)


def test_shading_constant_environment(lut):
    """Constant radiance c: E = pi c, so L_d = albedo (1-M) c; at roughness 0 the split sum
    gives c (F0 (1 - (1-N.V)^5) + (1-N.V)^5) with F0 = 0.04 (1-M) + albedo M (Eq. 10-12)."""
    cam = camera(16, 16)
    c = 1.7
    tabs = _const_tables(c, lut)
    rng = np.random.default_rng(1)
    pix = rng.integers(0, 16, size=(20, 2)).astype(np.int32)
    w2c = np.asarray(cam["w2c"], np.float64)
    g = np.zeros((20, 8))
    g[:, 0:3] = rng.uniform(0, 1, (20, 3))
    g[:, 3] = rng.uniform(0, 1, 20)
    g[:, 4] = 0.0
    # normals facing the viewer with a random tilt
    for p in range(20):
        x, y = pix[p]
        d = w2c[:, :3].T @ np.array([(x + 0.5 - cam["cx"]) / cam["fx"],
                                     (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
        wo = -d / np.linalg.norm(d)
        nrm = wo + 0.4 * rng.normal(size=3)
        g[p, 5:8] = nrm / np.linalg.norm(nrm) * 0.8
    rgb, _ = oracle.shade_gbuffer(g, np.ones(20), cam, pix, tabs)
    for p in range(20):
        x, y = pix[p]
        d = w2c[:, :3].T @ np.array([(x + 0.5 - cam["cx"]) / cam["fx"],
                                     (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
        wo = -d / np.linalg.norm(d)
        N = g[p, 5:8] / np.linalg.norm(g[p, 5:8])
        ndv = min(max(float(N @ wo), 0.0), 1.0)
        fc = (1 - ndv) ** 5
        M = g[p, 3]
        F0 = 0.04 * (1 - M) + g[p, 0:3] * M
        cc = float(np.float32(c))
        want = g[p, 0:3] * (1 - M) * cc + cc * (F0 * (1 - fc) + fc)
        np.testing.assert_allclose(rgb[p], want, rtol=3e-3)


def test_shading_mirror_returns_environment_radiance(lut):
    """Metallic 1, albedo 1, roughness 0, normal along the view vector: the reflection
    direction is the view vector itself and the pixel returns the radiance of that face."""
    cam = camera(16, 16)
    r = 16
    face_val = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    env = np.repeat(face_val, r * r * 3).reshape(6, r, r, 3).astype(np.float32)
    tabs = {"spec": oracle.prefilter(env, 1), "irr": oracle.irradiance(env, 4), "lut": lut}
    w2c = np.asarray(cam["w2c"], np.float64)
    pix = np.array([[2, 3], [8, 8], [14, 1]], np.int32)
    g = np.zeros((3, 8))
    g[:, 0:3] = 1.0
    g[:, 3] = 1.0
    faces = []
    for p, (x, y) in enumerate(pix):
        d = w2c[:, :3].T @ np.array([(x + 0.5 - cam["cx"]) / cam["fx"],
                                     (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
        wo = -d / np.linalg.norm(d)
        g[p, 5:8] = wo
        ax = int(np.argmax(np.abs(wo)))
        faces.append(2 * ax + (0 if wo[ax] >= 0 else 1))
    rgb, _ = oracle.shade_gbuffer(g, np.ones(3), cam, pix, tabs)
    np.testing.assert_allclose(rgb[:, 0], face_val[faces], rtol=2e-4)

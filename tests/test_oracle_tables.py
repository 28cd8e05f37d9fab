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


# ----------------------------------------------------------------------------------------
# pins of the cube-face orientation and of the roughness-selected level blend
# ----------------------------------------------------------------------------------------

def _opengl_face_st(d):
    """Face and (s,t) of direction d from the public OpenGL cube-map table (major axis ma,
    in-face coordinates sc, tc; s = (sc/|ma| + 1)/2, t = (tc/|ma| + 1)/2), written out here
    independently of the oracle."""
    x, y, z = d
    ax, ay, az = abs(x), abs(y), abs(z)
    if ax >= ay and ax >= az:
        face, sc, tc, ma = (0, -z, -y, ax) if x >= 0 else (1, z, -y, ax)
    elif ay >= az:
        face, sc, tc, ma = (2, x, z, ay) if y >= 0 else (3, x, -z, ay)
    else:
        face, sc, tc, ma = (4, x, -y, az) if z >= 0 else (5, -x, -y, az)
    return face, 0.5 * (sc / ma + 1.0), 0.5 * (tc / ma + 1.0)


def _coordinate_cube(r):
    """Cube whose texel [f][row j][col i] holds (f, (i+1/2)/r, (j+1/2)/r): bilinear filtering
    of these affine fields returns the face and the exact (s,t) of any lookup that lands
    between texel centres."""
    cube = np.zeros((6, r, r, 3))
    c = (np.arange(r) + 0.5) / r
    cube[..., 0] = np.arange(6)[:, None, None]
    cube[..., 1] = c[None, None, :]
    cube[..., 2] = c[None, :, None]
    return cube


def test_cube_orientation_matches_opengl_table():
    """For several directions on every face, the oracle's lookup lands on the face and the
    in-face (s,t) of the OpenGL table (column s, row t), so no face is mirrored, rotated or
    transposed."""
    r = 16
    cube = _coordinate_cube(r)
    rng = np.random.default_rng(3)
    dirs = []
    for axis in range(3):
        for sign in (1.0, -1.0):
            for _ in range(6):
                d = rng.uniform(-0.7, 0.7, 3)
                d[axis] = sign
                dirs.append(d * rng.uniform(0.5, 2.0))
    dirs = np.array(dirs)
    got = oracle.cube_sample(cube, dirs)
    for d, g in zip(dirs, got):
        face, s, t = _opengl_face_st(d)
        assert int(round(g[0])) == face, (d, g)
        assert g[1] == pytest.approx(s, abs=1e-12), (d, g, s, t)
        assert g[2] == pytest.approx(t, abs=1e-12), (d, g, s, t)


def test_cube_orientation_hand_picked():
    """A few directions whose table values are written by hand: e.g. +X with y, z < 0 lands in
    the lower half of neither axis (sc = -z > 0, tc = -y > 0)."""
    cube = _coordinate_cube(8)
    cases = [  # direction, face, s, t
        ((1.0, -0.2, -0.4), 0, 0.7, 0.6),
        ((-1.0, -0.2, -0.4), 1, 0.3, 0.6),
        ((0.4, 1.0, 0.2), 2, 0.7, 0.6),
        ((0.4, -1.0, 0.2), 3, 0.7, 0.4),
        ((0.4, 0.2, 1.0), 4, 0.7, 0.4),
        ((0.4, 0.2, -1.0), 5, 0.3, 0.4),
    ]
    got = oracle.cube_sample(cube, np.array([c[0] for c in cases]))
    for (d, f, s, t), g in zip(cases, got):
        np.testing.assert_allclose(g, [f, s, t], atol=1e-12, err_msg=str(d))


def _level_tables(levels, r, lut_ab, irr_val):
    """Hand-built shading tables: specular level l constant with channel values
    (1 + l, 10 + 3 l, 0.5 l) at resolution r >> l; irradiance constant; split-sum table lut_ab
    [n][n][2]."""
    spec = []
    for l in range(levels):
        rl = max(r >> l, 1)
        lv = np.empty((6, rl, rl, 3))
        lv[...] = [1.0 + l, 10.0 + 3.0 * l, 0.5 * l]
        spec.append(lv)
    irr = np.full((6, 4, 4, 3), irr_val)
    return {"spec": spec, "irr": irr, "lut": lut_ab}


def _pixel_dirs(cam, pix):
    w2c = np.asarray(cam["w2c"], np.float64)
    out = []
    for x, y in pix:
        d = w2c[:, :3].T @ np.array([(x + 0.5 - cam["cx"]) / cam["fx"],
                                     (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
        out.append(d / np.linalg.norm(d))
    return np.array(out)


@pytest.mark.parametrize("levels", [2, 3, 4, 5])
def test_shading_level_blend_closed_form(levels):
    """Eq. 12 with roughness selecting the prefiltered level (reading: level = clamp(R,0,1)
    (L-1), linear between the two levels around it). With constant levels c_l, a constant
    split-sum table (A, B) and constant irradiance E the shaded colour is exactly
    albedo/pi (1-M) E + lerp(c_floor, c_ceil, frac) (F0 A + B), F0 = 0.04 (1-M) + albedo M.
    Roughness values sit on every level boundary, between them, and outside [0,1] (clamped).
    A wrong mapping (R^2, R L, reversed levels) or a wrong level offset picks other
    constants."""
    n = 8
    A, B = 0.63, 0.21
    lut_ab = np.empty((n, n, 2))
    lut_ab[..., 0], lut_ab[..., 1] = A, B
    E = np.array([0.9, 1.3, 2.1])
    tabs = _level_tables(levels, 32, lut_ab, 1.0)
    tabs["irr"][...] = E
    cam = camera(16, 16)
    rough = sorted(set([l / (levels - 1) for l in range(levels)] +
                       [(l + f) / (levels - 1) for l in range(levels - 1)
                        for f in (0.25, 0.5, 0.9)] + [-0.3, 1.4]))
    P = len(rough)
    rng = np.random.default_rng(levels)
    pix = rng.integers(2, 14, size=(P, 2)).astype(np.int32)
    g = np.zeros((P, 8))
    g[:, 0:3] = rng.uniform(0.1, 0.9, (P, 3))
    g[:, 3] = rng.uniform(0, 1, P)
    g[:, 4] = rough
    g[:, 5:8] = -_pixel_dirs(cam, pix) + 0.2 * rng.normal(size=(P, 3))
    rgb, _ = oracle.shade_gbuffer(g, np.ones(P), cam, pix, tabs)
    for p in range(P):
        lev = min(max(rough[p], 0.0), 1.0) * (levels - 1)
        l0 = min(int(np.floor(lev)), levels - 1)
        l1 = min(l0 + 1, levels - 1)
        f = lev - l0
        c0 = np.array([1.0 + l0, 10.0 + 3.0 * l0, 0.5 * l0])
        c1 = np.array([1.0 + l1, 10.0 + 3.0 * l1, 0.5 * l1])
        Lp = (1 - f) * c0 + f * c1
        M = g[p, 3]
        F0 = 0.04 * (1 - M) + g[p, 0:3] * M
        want = g[p, 0:3] / math.pi * (1 - M) * E + Lp * (F0 * A + B)
        np.testing.assert_allclose(rgb[p], want, rtol=1e-12, atol=1e-12,
                                   err_msg=f"R={rough[p]} L={levels}")


def test_shading_lut_axes_closed_form():
    """The split-sum table is read at (column = clamp(N.V,0,1), row = clamp(R,0,1)), bilinear at
    texel centres: with A affine in the column and B affine in the row, interior lookups return
    the affine values exactly, so transposed or flipped axes fail. One level (L = 1), constant
    radiance c: colour = albedo/pi (1-M) E + c (F0 A + B)."""
    n = 16
    xc = (np.arange(n) + 0.5) / n
    lut_ab = np.empty((n, n, 2))
    lut_ab[..., 0] = (0.2 + 0.5 * xc)[None, :]     # A(N.V): varies along columns
    lut_ab[..., 1] = (0.05 + 0.3 * xc)[:, None]    # B(R): varies along rows
    c = 1.6
    tabs = _level_tables(1, 8, lut_ab, 0.0)
    tabs["spec"][0][...] = c
    cam = camera(16, 16)
    rng = np.random.default_rng(5)
    P = 24
    pix = rng.integers(0, 16, size=(P, 2)).astype(np.int32)
    d = _pixel_dirs(cam, pix)
    wo = -d
    g = np.zeros((P, 8))
    g[:, 0:3] = rng.uniform(0.1, 0.9, (P, 3))
    g[:, 3] = rng.uniform(0, 1, P)
    g[:, 4] = rng.uniform(0.1, 0.9, P)
    # normals tilted away from the view vector so that N.V spans the table's interior
    for p in range(P):
        axis = np.cross(wo[p], [0.0, 1.0, 0.0])
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(0.3, 1.3)
        nrm = math.cos(ang) * wo[p] + math.sin(ang) * axis
        g[p, 5:8] = nrm * rng.uniform(0.3, 1.0)
    rgb, _ = oracle.shade_gbuffer(g, np.ones(P), cam, pix, tabs)
    for p in range(P):
        N = g[p, 5:8] / np.linalg.norm(g[p, 5:8])
        ndv = float(N @ wo[p])
        assert 0.5 / n < ndv < 1 - 0.5 / n
        A = 0.2 + 0.5 * ndv
        B = 0.05 + 0.3 * g[p, 4]
        M = g[p, 3]
        F0 = 0.04 * (1 - M) + g[p, 0:3] * M
        np.testing.assert_allclose(rgb[p], c * (F0 * A + B), rtol=1e-12, atol=1e-12)

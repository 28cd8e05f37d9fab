"""Seeded synthetic inputs for textured planar-Gaussian rendering.

This module only draws inputs: splat parameters, per-primitive textures, environment
cubemaps, cameras, G-buffers and request streams. It holds none of the rendering
arithmetic (no projection, compositing, filtering, shading or table precompute), and it
imports neither the HIP library nor the oracle, so both sides may use it.

The distributions follow the workloads the method is evaluated on (object-centred scenes
seen from orbit cameras, and unbounded scenes with a far background), with the paper's
texture channels: albedo RGB, roughness, metallic and a tangent-space normal (Sec. 3.5.1).

Conventions shared by every consumer:
  * means [N,3], quats [N,4] (w,x,y,z, unit here but any non-zero length is allowed),
    scales [N,2] linear (s_u, s_v), opac [N] in (0,1), all float32;
  * textures [N,T,T,8] float32, indexed [k][row j (t)][col i (s)][channel], channels
    (albedo r,g,b, roughness, normal x,y,z, metallic);
  * env [6,r,r,3] float32, faces +X,-X,+Y,-Y,+Z,-Z, texel [face][row][col];
  * camera dict: w2c [3,4] (row-major [R|t], x right, y down, z forward), fx, fy, cx, cy,
    width, height; horizontal field of view, square pixels, principal point at the centre.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CONFIGS", "SceneConfig", "make_scene", "make_env", "look_at_camera", "orbit_cameras",
    "config_cameras", "crop_camera", "random_gbuffer", "poisson_requests", "target_image",
    "cameras_array", "fd_crop_scene", "serving_camera", "serving_scene", "SERVING_SCENES",
    "SERVING_RESOLUTIONS", "indirect_sh", "visibility", "texture_sides", "adaptive_textures",
]


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _normalize(v, axis=-1):
    n = np.linalg.norm(v, axis=axis, keepdims=True)
    n = np.where(n == 0.0, 1.0, n)
    return v / n


def _quat_from_frames(tu, tv, n):
    """Unit quaternion (w,x,y,z) of the rotation whose columns are (tu, tv, n)."""
    m = np.stack([tu, tv, n], axis=-1)  # [N,3,3], columns
    m00, m11, m22 = m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]
    tr = m00 + m11 + m22
    q = np.zeros((m.shape[0], 4))
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr + 1.0, 1e-300)) * 2
    q[c0, 0] = 0.25 * s[c0]
    q[c0, 1] = (m[c0, 2, 1] - m[c0, 1, 2]) / s[c0]
    q[c0, 2] = (m[c0, 0, 2] - m[c0, 2, 0]) / s[c0]
    q[c0, 3] = (m[c0, 1, 0] - m[c0, 0, 1]) / s[c0]
    c1 = (~c0) & (m00 > m11) & (m00 > m22)
    s = np.sqrt(np.maximum(1.0 + m00 - m11 - m22, 1e-300)) * 2
    q[c1, 0] = (m[c1, 2, 1] - m[c1, 1, 2]) / s[c1]
    q[c1, 1] = 0.25 * s[c1]
    q[c1, 2] = (m[c1, 0, 1] + m[c1, 1, 0]) / s[c1]
    q[c1, 3] = (m[c1, 0, 2] + m[c1, 2, 0]) / s[c1]
    c2 = (~c0) & (~c1) & (m11 > m22)
    s = np.sqrt(np.maximum(1.0 + m11 - m00 - m22, 1e-300)) * 2
    q[c2, 0] = (m[c2, 0, 2] - m[c2, 2, 0]) / s[c2]
    q[c2, 1] = (m[c2, 0, 1] + m[c2, 1, 0]) / s[c2]
    q[c2, 2] = 0.25 * s[c2]
    q[c2, 3] = (m[c2, 1, 2] + m[c2, 2, 1]) / s[c2]
    c3 = (~c0) & (~c1) & (~c2)
    s = np.sqrt(np.maximum(1.0 + m22 - m00 - m11, 1e-300)) * 2
    q[c3, 0] = (m[c3, 1, 0] - m[c3, 0, 1]) / s[c3]
    q[c3, 1] = (m[c3, 0, 2] + m[c3, 2, 0]) / s[c3]
    q[c3, 2] = (m[c3, 1, 2] + m[c3, 2, 1]) / s[c3]
    q[c3, 3] = 0.25 * s[c3]
    return _normalize(q)


def _frames_from_normals(rng, normals):
    """Random tangent t_u in the plane orthogonal to each normal, t_v = n x t_u."""
    n = _normalize(normals)
    r = rng.normal(size=n.shape)
    tu = r - np.sum(r * n, axis=1, keepdims=True) * n
    bad = np.linalg.norm(tu, axis=1) < 1e-6
    if bad.any():
        alt = np.where(np.abs(n[bad, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        tu[bad] = alt - np.sum(alt * n[bad], axis=1, keepdims=True) * n[bad]
    tu = _normalize(tu)
    tv = np.cross(n, tu)
    return tu, tv, n


def _textures(rng, n, T):
    """Per-primitive material textures, drawn albedo, roughness, metallic, normal
    (float32 draws: millions of texels per scene)."""
    tex = np.empty((n, T, T, 8), np.float32)
    tex[..., 0:3] = rng.random(size=(n, T, T, 3), dtype=np.float32)
    tex[..., 3] = np.float32(0.05) + np.float32(0.95) * rng.random(size=(n, T, T), dtype=np.float32)
    tex[..., 7] = (rng.random(size=(n, T, T), dtype=np.float32) < 0.3).astype(np.float32)
    nxy = np.float32(0.2) * rng.standard_normal(size=(n, T, T, 2), dtype=np.float32)
    inv = 1.0 / np.sqrt(1.0 + nxy[..., 0] ** 2 + nxy[..., 1] ** 2)
    tex[..., 4] = nxy[..., 0] * inv
    tex[..., 5] = nxy[..., 1] * inv
    tex[..., 6] = inv
    return tex


def make_env(rng, res):
    """Environment cubemap [6,res,res,3], radiance log-normal(0,1) per texel and channel."""
    return np.exp(rng.normal(0.0, 1.0, size=(6, res, res, 3))).astype(np.float32)


# ---------------------------------------------------------------------------------------
# geometry generators
# ---------------------------------------------------------------------------------------

def _shell_centres(rng, n, r0, r1):
    d = _normalize(rng.normal(size=(n, 3)))
    r = np.cbrt(rng.uniform(r0 ** 3, r1 ** 3, size=(n, 1)))
    return d * r


def _superquadric(rng, n):
    """Samples of a random superquadric surface with jittered normals."""
    a = rng.uniform(0.6, 1.0, size=3)
    e1, e2 = rng.uniform(0.3, 1.5, size=2)
    eta = np.arcsin(rng.uniform(-1.0, 1.0, size=n))
    om = rng.uniform(-math.pi, math.pi, size=n)

    def spow(x, p):
        return np.sign(x) * np.abs(x) ** p

    ce, se, co, so = np.cos(eta), np.sin(eta), np.cos(om), np.sin(om)
    x = a[0] * spow(ce, e1) * spow(co, e2)
    y = a[1] * spow(ce, e1) * spow(so, e2)
    z = a[2] * spow(se, e1)
    pts = np.stack([x, y, z], axis=1)
    # gradient of the implicit function ((x/a1)^(2/e2)+(y/a2)^(2/e2))^(e2/e1)+(z/a3)^(2/e1)
    X, Y, Z = np.abs(x / a[0]), np.abs(y / a[1]), np.abs(z / a[2])
    A = X ** (2 / e2) + Y ** (2 / e2)
    with np.errstate(divide="ignore", invalid="ignore"):
        ca = (2 / e1) * np.power(np.maximum(A, 1e-30), e2 / e1 - 1.0)
        gx = ca * X ** (2 / e2 - 1) * np.sign(x) / a[0]
        gy = ca * Y ** (2 / e2 - 1) * np.sign(y) / a[1]
        gz = (2 / e1) * Z ** (2 / e1 - 1) * np.sign(z) / a[2]
    g = np.stack([gx, gy, gz], axis=1)
    bad = ~np.all(np.isfinite(g), axis=1) | (np.linalg.norm(g, axis=1) < 1e-12)
    g[bad] = pts[bad]
    g = _normalize(g) + rng.normal(0.0, 0.1, size=(n, 3))
    return pts, _normalize(g)


def _height_field_scene(rng, n):
    """Ground height field over [-6,6]^2 with 6 boxes (70%) and a far shell (30%)."""
    n_fg = int(round(0.7 * n))
    n_bg = n - n_fg
    amp = rng.uniform(0.05, 0.3, size=4)
    freq = rng.uniform(0.3, 2.0, size=(4, 2)) * np.sign(rng.uniform(-1, 1, size=(4, 2)))
    ph = rng.uniform(0, 2 * math.pi, size=4)
    boxes_c = np.concatenate([rng.uniform(-4, 4, size=(6, 1)), np.zeros((6, 1)),
                              rng.uniform(-4, 4, size=(6, 1))], axis=1)
    boxes_s = rng.uniform(0.3, 1.2, size=(6, 3))

    def height(xz):
        h = np.zeros(xz.shape[0])
        for k in range(4):
            h += amp[k] * np.sin(xz @ freq[k] + ph[k])
        return h

    def dheight(xz):
        g = np.zeros_like(xz)
        for k in range(4):
            g += amp[k] * np.cos(xz @ freq[k] + ph[k])[:, None] * freq[k][None, :]
        return g

    # area of the boxes' five visible faces versus the ground
    face_area = []
    for b in range(6):
        sx, sy, sz = boxes_s[b]
        face_area += [sx * sz, sy * sz, sy * sz, sx * sy, sx * sy]
    face_area = np.array(face_area)
    ground_area = 144.0
    p_face = face_area / (face_area.sum() + ground_area)
    choice = rng.choice(len(face_area) + 1, size=n_fg,
                        p=np.concatenate([p_face, [ground_area / (face_area.sum() + ground_area)]]))
    pts = np.zeros((n_fg, 3))
    nrm = np.zeros((n_fg, 3))
    g = choice == len(face_area)
    xz = rng.uniform(-6, 6, size=(int(g.sum()), 2))
    pts[g, 0], pts[g, 2] = xz[:, 0], xz[:, 1]
    pts[g, 1] = height(xz)
    dh = dheight(xz)
    nrm[g] = _normalize(np.stack([-dh[:, 0], np.ones(len(xz)), -dh[:, 1]], axis=1))
    uv = rng.uniform(-0.5, 0.5, size=(n_fg, 2))
    for f in range(len(face_area)):
        m = choice == f
        if not m.any():
            continue
        b, side = divmod(f, 5)
        c, s = boxes_c[b].copy(), boxes_s[b]
        base = c + np.array([0.0, height(c[None, [0, 2]])[0], 0.0])
        q = uv[m]
        if side == 0:   # top
            p = base + np.stack([q[:, 0] * s[0], np.full(len(q), s[1]), q[:, 1] * s[2]], axis=1)
            nn = np.array([0, 1.0, 0])
        elif side in (1, 2):  # +-x
            sg = 1.0 if side == 1 else -1.0
            p = base + np.stack([np.full(len(q), sg * s[0] / 2), (q[:, 0] + 0.5) * s[1],
                                 q[:, 1] * s[2]], axis=1)
            nn = np.array([sg, 0, 0.0])
        else:           # +-z
            sg = 1.0 if side == 3 else -1.0
            p = base + np.stack([q[:, 0] * s[0], (q[:, 1] + 0.5) * s[1],
                                 np.full(len(q), sg * s[2] / 2)], axis=1)
            nn = np.array([0, 0, sg])
        pts[m] = p
        nrm[m] = nn
    bg_dir = _normalize(rng.normal(size=(n_bg, 3)))
    bg_r = rng.uniform(5.0, 50.0, size=(n_bg, 1))
    bg_pts = bg_dir * bg_r
    bg_nrm = _normalize(rng.normal(size=(n_bg, 3)))
    return (np.concatenate([pts, bg_pts]), np.concatenate([nrm, bg_nrm]), n_fg,
            bg_r[:, 0])


# ---------------------------------------------------------------------------------------
# cameras
# ---------------------------------------------------------------------------------------

def look_at_camera(eye, target, width, height, fov_deg=50.0, up=(0.0, 1.0, 0.0)):
    """Pinhole camera looking from eye at target; fov is horizontal, fy = fx."""
    eye = np.asarray(eye, np.float64)
    f = _normalize(np.asarray(target, np.float64) - eye)
    r = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(r) < 1e-9:
        r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r = _normalize(r)
    d = np.cross(f, r)
    rot = np.stack([r, d, f], axis=0)  # world->camera rows
    t = -rot @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    w2c = np.concatenate([rot, t[:, None]], axis=1).astype(np.float32)
    return {"w2c": w2c, "fx": float(np.float32(fx)), "fy": float(np.float32(fx)),
            "cx": width / 2.0, "cy": height / 2.0, "width": int(width), "height": int(height)}


def orbit_cameras(n, width, height, dist=3.0, el_deg=20.0, fov_deg=50.0, az0=0.0,
                  target=(0.0, 0.0, 0.0)):
    cams = []
    for k in range(n):
        az = az0 + 2 * math.pi * k / n
        el = math.radians(el_deg)
        eye = np.array(target) + dist * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                                  math.cos(el) * math.cos(az)])
        cams.append(look_at_camera(eye, target, width, height, fov_deg))
    return cams


def crop_camera(cam, x0, y0, w, h):
    """The same camera restricted to the pixel window [x0,x0+w) x [y0,y0+h)."""
    c = dict(cam)
    c["cx"] = cam["cx"] - x0
    c["cy"] = cam["cy"] - y0
    c["width"], c["height"] = int(w), int(h)
    return c


def cameras_array(cams):
    """Pack cameras as float32 [V,16]: w2c (12, row-major), fx, fy, cx, cy."""
    out = np.zeros((len(cams), 16), np.float32)
    for i, c in enumerate(cams):
        out[i, :12] = np.asarray(c["w2c"], np.float32).reshape(12)
        out[i, 12:16] = [c["fx"], c["fy"], c["cx"], c["cy"]]
    return out


# ---------------------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------------------

@dataclass
class SceneConfig:
    name: str
    n: int
    tex_res: int
    geometry: str           # "shell" | "superquadric" | "heightfield"
    env_res: int
    env_levels: int
    width: int
    height: int
    n_views: int
    seed: int = 0
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # 2k splats in a shell, one 128x128 view.
    "shell2k": SceneConfig("shell2k", 2000, 4, "shell", 32, 1, 128, 128, 1),
    # 100k splats on a superquadric, 64 orbit views of 800x800.
    "sq100k": SceneConfig("sq100k", 100_000, 8, "superquadric", 128, 4, 800, 800, 64),
    # 300k splats, a batch of 8 orbit views per step, L1 loss to a seeded target.
    "sq300k_train": SceneConfig("sq300k_train", 300_000, 8, "superquadric", 128, 4, 800, 800, 8),
    # 1M splats, ground + boxes + far shell, one 1600x1064 view.
    "field1m": SceneConfig("field1m", 1_000_000, 8, "heightfield", 256, 4, 1600, 1064, 1),
}


def make_scene(cfg: SceneConfig | str, seed: int | None = None, n: int | None = None,
               tex_res: int | None = None, env_res: int | None = None):
    """Draw one scene. Draw order: centres, scales, rotations, opacity, textures, env."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    seed = cfg.seed if seed is None else seed
    n = cfg.n if n is None else n
    T = cfg.tex_res if tex_res is None else tex_res
    env_res = cfg.env_res if env_res is None else env_res
    rng = np.random.default_rng(seed)
    bg_r = None
    normals = None
    if cfg.geometry == "shell":
        means = _shell_centres(rng, n, 0.8, 1.0)
    elif cfg.geometry == "superquadric":
        means, normals = _superquadric(rng, n)
    elif cfg.geometry == "heightfield":
        means, normals, _, bg_r = _height_field_scene(rng, n)
    else:
        raise ValueError(cfg.geometry)
    log_s = rng.uniform(-4.0, -2.5, size=(n, 2))
    if bg_r is not None:
        log_s[-len(bg_r):] += np.log(bg_r / 3.0)[:, None]
    scales = np.exp(log_s)
    if normals is None:
        quats = _normalize(rng.normal(size=(n, 4)))
    else:
        if bg_r is not None:  # background splats take a random orientation
            nb = len(bg_r)
            normals = normals.copy()
            normals[-nb:] = _normalize(rng.normal(size=(nb, 3)))
        tu, tv, nn = _frames_from_normals(rng, normals)
        quats = _quat_from_frames(tu, tv, nn)
    opac = _sigmoid(rng.normal(size=n))
    tex = _textures(rng, n, T)
    env = make_env(rng, env_res)
    return {
        "means": means.astype(np.float32),
        "quats": quats.astype(np.float32),
        "scales": scales.astype(np.float32),
        "opac": opac.astype(np.float32),
        "textures": tex,
        "chart_of": np.arange(n, dtype=np.int32),
        "env": env,
        "tex_res": T,
        "env_levels": cfg.env_levels,
    }


def config_cameras(cfg: SceneConfig | str, n_views: int | None = None):
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    V = cfg.n_views if n_views is None else n_views
    if cfg.geometry == "shell":
        return [look_at_camera((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), cfg.width, cfg.height)]
    if cfg.geometry == "heightfield":
        cams = []
        for k in range(V):
            az = 2 * math.pi * k / max(V, 1)
            eye = (4.0 * math.sin(az), 1.5, 4.0 * math.cos(az))
            cams.append(look_at_camera(eye, (0.0, 0.5, 0.0), cfg.width, cfg.height))
        return cams
    if cfg.name == "sq300k_train":
        return orbit_cameras(V, cfg.width, cfg.height)
    return orbit_cameras(V, cfg.width, cfg.height)


def serving_camera(geometry, width, height, az, el_deg):
    """A random serving view: orbit at distance 3 around the object scenes, or a view from
    radius 4 at height 1.5 + el/40 towards (0, 0.5, 0) for the height-field scene."""
    if geometry == "heightfield":
        eye = (4.0 * math.sin(az), 1.5 + el_deg / 40.0, 4.0 * math.cos(az))
        return look_at_camera(eye, (0.0, 0.5, 0.0), width, height)
    el = math.radians(el_deg)
    eye = 3.0 * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return look_at_camera(eye, (0.0, 0.0, 0.0), width, height)


SERVING_SCENES = [("superquadric", 50_000, 10), ("superquadric", 200_000, 11),
                  ("superquadric", 500_000, 12), ("heightfield", 1_000_000, 13)]
SERVING_RESOLUTIONS = [(256, 256), (512, 512), (800, 800), (1920, 1080)]


def serving_scene(i, n=None):
    geo, count, seed = SERVING_SCENES[i]
    base = "field1m" if geo == "heightfield" else "sq100k"
    return make_scene(base, seed=seed, n=count if n is None else n)


def target_image(width, height, seed=1, n_views=1):
    """Seeded L1 target: U(0,1) RGB per pixel, [V,H,W,3]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n_views, height, width, 3)).astype(np.float32)


def random_gbuffer(rng, n_views, height, width, empty_frac=0.1):
    """A seeded G-buffer [V,8,H,W] (albedo 3, metallic, roughness, normal 3) and alpha [V,H,W].

    Values are premultiplied by a coverage alpha; a fraction of pixels is left empty."""
    a = rng.uniform(0.05, 1.0, size=(n_views, height, width))
    a[rng.uniform(size=a.shape) < empty_frac] = 0.0
    g = np.empty((n_views, 8, height, width))
    g[:, 0:3] = rng.uniform(0, 1, size=(n_views, 3, height, width))
    g[:, 3] = (rng.uniform(size=(n_views, height, width)) < 0.3)
    g[:, 4] = rng.uniform(0.0, 1.0, size=(n_views, height, width))
    nrm = _normalize(rng.normal(size=(n_views, height, width, 3)))
    g[:, 5:8] = np.moveaxis(nrm, -1, 1) * rng.uniform(0.3, 1.0, size=(n_views, 1, height, width))
    g *= a[:, None]
    return g.astype(np.float32), a.astype(np.float32)


def indirect_sh(rng, n, degree=3):
    """Per-splat spherical-harmonic coefficients of the indirect light, [n,(degree+1)^2,3]
    float32: the constant band drawn U(0.5, 3.5) (a positive mean radiance), band l >= 1
    drawn N(0, (0.3/l)^2) (smoother light for the higher bands)."""
    K = (degree + 1) ** 2
    c = np.empty((n, K, 3))
    c[:, 0] = rng.uniform(0.5, 3.5, size=(n, 3))
    for l in range(1, degree + 1):
        c[:, l * l:(l + 1) * (l + 1)] = rng.normal(0.0, 0.3 / l, size=(n, 2 * l + 1, 3))
    return c.astype(np.float32)


def texture_sides(scales, base_log2=3, max_log2=4):
    """Per-splat texture side exponents for an adaptive atlas: larger primitives get more
    texels, log2 T_k = clip(round(log2(s_k / median s) + base_log2), 0, max_log2) with s_k the
    larger scale (an allocation by primitive size, the policy the paper suggests)."""
    s = np.asarray(scales, np.float64).max(axis=1)
    med = np.median(s) if len(s) else 1.0
    return np.clip(np.round(np.log2(s / med) + base_log2), 0, max_log2).astype(np.int32)


def adaptive_textures(rng, log2):
    """Level-0 texels of every splat at its own side 2^log2[k], back to back in splat order
    ([sum 4^log2, 8] float32; channel distributions as the uniform textures)."""
    parts = [_textures(rng, 1, 1 << int(l)).reshape(-1, 8) for l in log2]
    return (np.concatenate(parts) if parts else np.zeros((0, 8), np.float32)).astype(np.float32)


def visibility(rng, n_views, height, width):
    """Per-pixel visibility V in [0,1], [V,H,W] float32: 40% of pixels fully visible (1),
    30% occluded (0), 30% partial U(0,1) (pixels on an occluder's edge)."""
    u = rng.uniform(size=(n_views, height, width))
    v = rng.uniform(size=(n_views, height, width))
    return np.where(u < 0.4, 1.0, np.where(u < 0.7, 0.0, v)).astype(np.float32)


def fd_crop_scene(scene, cam, x0, y0, w, h, n_keep=500):
    """Splats whose centres project into the crop window, the n_keep nearest by depth."""
    w2c = np.asarray(cam["w2c"], np.float64)
    pc = scene["means"].astype(np.float64) @ w2c[:, :3].T + w2c[:, 3]
    z = pc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        px = cam["fx"] * pc[:, 0] / z + cam["cx"]
        py = cam["fy"] * pc[:, 1] / z + cam["cy"]
    inside = (z > 0.2) & (px >= x0) & (px < x0 + w) & (py >= y0) & (py < y0 + h)
    idx = np.nonzero(inside)[0]
    idx = idx[np.argsort(z[idx], kind="stable")][:n_keep]
    idx = np.sort(idx)
    out = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (len(z),) else v)
           for k, v in scene.items()}
    out["chart_of"] = np.arange(len(idx), dtype=np.int32)
    return out, crop_camera(cam, x0, y0, w, h)


def poisson_requests(rng, rate, duration, n_scenes, resolutions):
    """Arrival times (s), scene ids and (W,H) of a Poisson request stream."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = int(rng.integers(n_scenes))
        wh = resolutions[int(rng.integers(len(resolutions)))]
        az = rng.uniform(0, 2 * math.pi)
        el = rng.uniform(0.0, 40.0)
        out.append((t, s, wh, az, el))
    return out

"""FP64 oracle for textured planar-Gaussian rendering — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package. The product path never does, and this package imports nothing from it.

`oracle.c` holds the forward definition (per pixel, every splat against every pixel) and the
pre-integrated shading tables; `grad.py` holds the gradient reference (float64 autograd of a
dense formulation). Both follow the paper's equations; see the headers of those files.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MAX_ALT = 4

DEFAULT_PARAMS = {
    "s_sigma": 3.0,
    "alpha_min": 1.0 / 255.0,
    "alpha_max": 0.99,
    "t_min": 1e-4,
    "near_z": 0.2,
    "bg": (0.0, 0.0, 0.0),
    "amb_eps": 2e-5,     # relative margin below which a threshold decision counts as ambiguous
    "graze": 1e-3,       # |cos(ray, normal)| below which a blended splat counts as grazing
}

LUT_RES = 256
LUT_SAMPLES = 4096
IRR_RES = 16


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            for name in ["or_irradiance", "or_prefilter", "or_brdf_lut", "or_render", "or_shade",
                         "or_cube_sample", "or_cube_texels", "or_lut_sample", "or_splat_setup",
                         "or_sh_basis", "or_indirect_eval", "or_set_threads"]:
                getattr(L, name).restype = ctypes.c_int
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n=0):
    """Host threads of the oracle's OpenMP loops (n > 0 sets them); returns the count in use."""
    return int(lib().or_set_threads(int(n)))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam16(cam) -> np.ndarray:
    """Camera as float64 [16]: w2c (12, row-major) then fx, fy, cx, cy (float32 values)."""
    c = np.zeros(16, np.float64)
    c[:12] = np.asarray(cam["w2c"], np.float32).reshape(12).astype(np.float64)
    c[12:16] = np.asarray([cam["fx"], cam["fy"], cam["cx"], cam["cy"]], np.float32)
    return c


def params_vec(params=None) -> np.ndarray:
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    bg = p["bg"]
    v = [p["s_sigma"], p["alpha_min"], p["alpha_max"], p["t_min"], p["near_z"], bg[0], bg[1],
         bg[2], p["amb_eps"], p["graze"]]
    return np.asarray(np.asarray(v, np.float32), np.float64)


# ----------------------------------------------------------------------------------------
# tables
# ----------------------------------------------------------------------------------------

def irradiance(env, out_res=IRR_RES):
    env = _f32(env)
    r = env.shape[1]
    out = np.zeros((6, out_res, out_res, 3))
    assert lib().or_irradiance(_p(env), r, out_res, _p(out)) == 0
    return out


def prefilter(env, levels):
    """Levels 0..L-1 as a list of [6, r>>l, r>>l, 3] arrays."""
    env = _f32(env)
    r = env.shape[1]
    sizes = [max(r >> l, 1) for l in range(levels)]
    flat = np.zeros(sum(6 * s * s * 3 for s in sizes))
    assert lib().or_prefilter(_p(env), r, levels, _p(flat)) == 0
    out, off = [], 0
    for s in sizes:
        out.append(flat[off:off + 6 * s * s * 3].reshape(6, s, s, 3))
        off += 6 * s * s * 3
    return out


def brdf_lut(n=LUT_RES, samples=LUT_SAMPLES):
    out = np.zeros((n, n, 2))
    assert lib().or_brdf_lut(n, samples, _p(out)) == 0
    return out


_table_cache = {}


def tables(env, levels, irr_res=IRR_RES, lut_res=LUT_RES, lut_samples=LUT_SAMPLES):
    """All shading tables of one environment (cached by content)."""
    env = _f32(env)
    key = (env.shape, levels, irr_res, lut_res, lut_samples, hash(env.tobytes()))
    if key not in _table_cache:
        lkey = ("lut", lut_res, lut_samples)
        if lkey not in _table_cache:
            _table_cache[lkey] = brdf_lut(lut_res, lut_samples)
        _table_cache[key] = {
            "spec": prefilter(env, levels),
            "irr": irradiance(env, irr_res),
            "lut": _table_cache[lkey],
        }
    return _table_cache[key]


def cube_sample(cube, dirs):
    cube = _f64(cube)
    dirs = _f64(dirs).reshape(-1, 3)
    out = np.zeros_like(dirs)
    assert lib().or_cube_sample(_p(cube), cube.shape[1], _p(dirs), len(dirs), _p(out)) == 0
    return out


def cube_texels(r):
    dirs = np.zeros((6, r, r, 3))
    solid = np.zeros((6, r, r))
    assert lib().or_cube_texels(r, _p(dirs), _p(solid)) == 0
    return dirs, solid


def lut_sample(lut, xy):
    lut = _f64(lut)
    xy = _f64(xy).reshape(-1, 2)
    out = np.zeros_like(xy)
    assert lib().or_lut_sample(_p(lut), lut.shape[0], _p(xy), len(xy), _p(out)) == 0
    return out


# ----------------------------------------------------------------------------------------
# rendering
# ----------------------------------------------------------------------------------------

def splat_setup(scene, cam, params=None):
    """Per-splat depth rounded to float32 (sort key), keep flag, facing sign."""
    n = len(scene["opac"])
    depth = np.zeros(n, np.float32)
    keep = np.zeros(n, np.int32)
    sigma = np.zeros(n)
    m, q, s, o = (_f32(scene[k]) for k in ("means", "quats", "scales", "opac"))
    assert lib().or_splat_setup(n, _p(m), _p(q), _p(s), _p(o), _p(cam16(cam)),
                                _p(params_vec(params)), _p(depth), _p(keep), _p(sigma)) == 0
    return depth, keep.astype(bool), sigma


def all_pixels(width, height):
    ys, xs = np.mgrid[0:height, 0:width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


GB = 11   # G-buffer channels of the oracle: albedo 3, metallic, roughness, normal 3, L_ind 3


def render(scene, cam, pixels=None, params=None, tabs=None, shade=True, lind=None, vis=None):
    """Render the listed pixels ([P,2] x,y; default: the whole frame).

    Texture variants read from the scene dict: "tex_format" 1 = textures with 7 channels
    (albedo 3, roughness, normal x, y, metallic; n_z rebuilt), "trilinear" = filter over the
    box-filtered mip chain, "chart_table" [n_charts,2] = (level-0 texel offset, log2 T) of
    each chart with "textures" then a flat [texels, C] array.

    lind: per-splat indirect radiance [n,3] of this view (indirect_eval), or None;
    vis: visibility V per listed pixel [P], or None (V = 1).

    Returns dict with rgba [P,4], gbuf [P,8] (albedo 3, metallic, roughness, normal 3),
    gind [P,3] (blended L_ind), stat [P,7] (n_blend, n_support, n_ambiguous, grazing,
    min cube-face gap, n_alt, shading sensitivity = sum over G-buffer channels of
    max_rgb |dC/dg_c|), alt_rgba [P,MAX_ALT,4], alt_gbuf [P,MAX_ALT,8], alt_gind [P,MAX_ALT,3]."""
    if pixels is None:
        pixels = all_pixels(cam["width"], cam["height"])
    pixels = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    P = len(pixels)
    n = len(scene["opac"])
    m, q, s, o, tex = (_f32(scene[k]) for k in ("means", "quats", "scales", "opac", "textures"))
    chart = np.ascontiguousarray(scene["chart_of"], dtype=np.int32)
    # texture variants: two-component normals, trilinear mips, per-chart resolutions
    fmt = int(scene.get("tex_format", 0))
    tri = 1 if scene.get("trilinear", False) else 0
    ctab = scene.get("chart_table")
    if ctab is not None:
        ctab = np.ascontiguousarray(ctab, dtype=np.int32).reshape(-1, 2)
        T = 1
    else:
        T = int(scene["textures"].shape[1])
    assert tex.shape[-1] == (7 if fmt else 8)
    gbuf = np.zeros((P, GB))
    alt_gbuf = np.zeros((P, MAX_ALT, GB))
    out = {"rgba": np.zeros((P, 4)), "stat": np.zeros((P, 7)),
           "alt_rgba": np.zeros((P, MAX_ALT, 4))}
    li = None if lind is None else _f64(lind).reshape(n, 3)
    vi = None if vis is None else _f64(vis).reshape(P)
    if shade:
        if tabs is None:
            tabs = tables(scene["env"], scene["env_levels"])
        spec = np.concatenate([l.ravel() for l in tabs["spec"]])
        spec_res, levels = tabs["spec"][0].shape[1], len(tabs["spec"])
        irr, lut = _f64(tabs["irr"]), _f64(tabs["lut"])
        env_args = (_p(spec), spec_res, levels, _p(irr), irr.shape[1], _p(lut), lut.shape[0])
    else:
        env_args = (None, 0, 0, None, 0, None, 0)
    rc = lib().or_render(n, T, _p(m), _p(q), _p(s), _p(o), _p(tex), _p(chart), fmt, tri,
                         None if ctab is None else _p(ctab), _p(cam16(cam)), _p(params_vec(params)), *env_args,
                         None if li is None else _p(li), None if vi is None else _p(vi),
                         _p(pixels), P, _p(out["rgba"]), _p(gbuf), _p(out["stat"]),
                         _p(out["alt_rgba"]), _p(alt_gbuf))
    assert rc == 0
    out["gbuf"], out["gind"] = gbuf[:, :8], gbuf[:, 8:]
    out["alt_gbuf"], out["alt_gind"] = alt_gbuf[:, :, :8], alt_gbuf[:, :, 8:]
    return out


def shade_gbuffer(gbuf, alpha, cam, pixels, tabs, params=None, gind=None, vis=None):
    """Shade given G-buffer values: gbuf [P,8], alpha [P] at pixels [P,2] -> rgb [P,3];
    gind [P,3] blended indirect radiance (default 0), vis [P] visibility (default 1)."""
    g8 = _f64(gbuf).reshape(-1, 8)
    P0 = len(g8)
    gbuf = np.zeros((P0, GB))
    gbuf[:, :8] = g8
    if gind is not None:
        gbuf[:, 8:] = _f64(gind).reshape(P0, 3)
    vi = None if vis is None else _f64(vis).reshape(P0)
    alpha = _f64(alpha).reshape(-1)
    pixels = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    P = len(pixels)
    spec = np.concatenate([l.ravel() for l in tabs["spec"]])
    irr, lut = _f64(tabs["irr"]), _f64(tabs["lut"])
    rgb = np.zeros((P, 3))
    gap = np.zeros(P)
    assert lib().or_shade(_p(gbuf), _p(alpha), None if vi is None else _p(vi), _p(pixels), P,
                          _p(cam16(cam)),
                          _p(params_vec(params)), _p(spec), tabs["spec"][0].shape[1],
                          len(tabs["spec"]), _p(irr), irr.shape[1], _p(lut), lut.shape[0],
                          _p(rgb), _p(gap)) == 0
    return rgb, gap


# ----------------------------------------------------------------------------------------
# indirect light (per-splat spherical harmonics)
# ----------------------------------------------------------------------------------------

def sh_basis(degree, dirs):
    """Real orthonormal SH basis values at directions [P,3] -> [P,(degree+1)^2]."""
    dirs = _f64(dirs).reshape(-1, 3)
    K = (degree + 1) ** 2
    out = np.zeros((len(dirs), K))
    assert lib().or_sh_basis(int(degree), _p(dirs), len(dirs), _p(out)) == 0
    return out


def indirect_eval(scene, cam, sh, degree):
    """Per-splat indirect radiance [n,3] for one camera from sh [n,(degree+1)^2,3]."""
    n = len(scene["opac"])
    K = (degree + 1) ** 2
    sh = _f32(sh).reshape(n, K, 3)
    m, q = _f32(scene["means"]), _f32(scene["quats"])
    out = np.zeros((n, 3))
    assert lib().or_indirect_eval(n, _p(m), _p(q), _p(sh), int(degree), _p(cam16(cam)),
                                  _p(out)) == 0
    return out

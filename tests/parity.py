"""Comparison of HIP outputs with the FP64 oracle, pixel by pixel.

Tolerances (float32 path against the float64 definition): alpha max-abs 1e-5, G-buffer
channels max-abs 1e-5, linear RGB max-abs 1e-4 plus the first-order effect of the G-buffer
tolerance, sens * 1e-5, where sens = sum_c max_rgb |dC/dg_c| is the oracle's own
finite-difference sensitivity of the shading to the blended maps. Where sens * 1e-5 exceeds
1e-4 the pixel is counted as ill-conditioned (typically a low-coverage pixel, whose normal is
normalised from a short blended vector, in front of a high-contrast environment texel).
A pixel whose oracle result has near-threshold decisions (support edge, alpha cut-off,
termination) passes if the HIP value matches the primary oracle result or one of the
alternates with that decision flipped."""
import numpy as np

TOL_RGB = 1e-4
TOL_A = 1e-5
TOL_G = 1e-5


def pixel_match(gpu_rgba, gpu_gbuf, ref, tol_rgb=TOL_RGB, tol_a=TOL_A, tol_g=TOL_G,
                check_rgb=True, gpu_gind=None, skip_graze=False):
    """gpu_rgba [P,4], gpu_gbuf [P,8] or None, gpu_gind [P,3] (blended indirect map) or None,
    ref = oracle.render output for the same pixels. Returns (ok [P] bool, info dict).

    skip_graze: pixels that blend a splat seen nearly edge-on (the oracle's grazing flag,
    |cos(ray, normal)| below its `graze` parameter) are not held to the G-buffer bar: the
    float32 closed-form (u,v) loses about 1/|cos| of its precision there, and a
    high-resolution chart turns that into texture error. They are counted in the info."""
    P = len(ref["rgba"])
    sens = ref["stat"][:, 6]
    tol_pix = tol_rgb + sens * tol_g

    def ok_against(rr, gg, gi):
        ok = np.abs(gpu_rgba[:, 3] - rr[:, 3]) <= tol_a
        if check_rgb:
            ok &= np.abs(gpu_rgba[:, :3] - rr[:, :3]).max(axis=1) <= tol_pix
        if gpu_gbuf is not None:
            ok &= np.abs(gpu_gbuf - gg).max(axis=1) <= tol_g
        if gpu_gind is not None:
            ok &= np.abs(gpu_gind - gi).max(axis=1) <= tol_g
        return ok

    ok_primary = ok_against(ref["rgba"], ref["gbuf"], ref["gind"])
    ok = ok_primary.copy()
    n_alt = ref["stat"][:, 5].astype(int)
    for a in range(ref["alt_rgba"].shape[1]):
        has = n_alt > a
        if not has.any():
            continue
        ok |= has & ok_against(ref["alt_rgba"][:, a], ref["alt_gbuf"][:, a],
                               ref["alt_gind"][:, a])
    graze = ref["stat"][:, 3] > 0
    matched_alt = int((ok & ~ok_primary).sum())
    if skip_graze:
        ok |= graze
    err_rgb = np.abs(gpu_rgba[:, :3] - ref["rgba"][:, :3]).max(axis=1)
    err_a = np.abs(gpu_rgba[:, 3] - ref["rgba"][:, 3])
    clear = ref["stat"][:, 2] == 0
    well = clear & (sens * tol_g <= tol_rgb)
    info = {
        "pixels": P,
        "fail": int((~ok).sum()),
        "ambiguous": int((~clear).sum()),
        "matched_alternate": matched_alt,
        "ill_conditioned": int((clear & ~well).sum()),
        "over_strict_rgb_tol": int((err_rgb > tol_rgb).sum()),
        "max_err_rgb_well_conditioned": float(err_rgb[well].max(initial=0.0)),
        "p99_err_rgb": float(np.percentile(err_rgb[clear], 99)) if clear.any() else 0.0,
        "max_err_alpha_unambiguous": float(err_a[clear].max(initial=0.0)),
    }
    if skip_graze:
        info["grazing_excluded"] = int(graze.sum())
    if gpu_gbuf is not None:
        err_g = np.abs(gpu_gbuf - ref["gbuf"]).max(axis=1)
        info["max_err_gbuf_unambiguous"] = float(err_g[clear].max(initial=0.0))
        info["p99_err_gbuf"] = float(np.percentile(err_g[clear], 99)) if clear.any() else 0.0
    if gpu_gind is not None:
        err_i = np.abs(gpu_gind - ref["gind"]).max(axis=1)
        info["max_err_gind_unambiguous"] = float(err_i[clear].max(initial=0.0))
    return ok, info


def gather(out, v, pixels):
    """GPU outputs of view v at pixels [P,2] (x,y) as float64 numpy."""
    xs, ys = pixels[:, 0], pixels[:, 1]
    rgba = out["rgba"][v].double().cpu().numpy()[ys, xs] if "rgba" in out else None
    gb = None
    if "gbuf" in out:
        g = out["gbuf"][v].double().cpu().numpy()
        gb = g[:, ys, xs].T
    return rgba, gb


def gather_ind(out, v, pixels):
    """The blended indirect map of view v at pixels [P,2] as float64 [P,3] (or None)."""
    if "gbuf_ind" not in out:
        return None
    g = out["gbuf_ind"][v].double().cpu().numpy()
    return g[:, pixels[:, 1], pixels[:, 0]].T


def sample_pixels(rng, width, height, n, tile=16):
    """Random pixels plus the corners of random tiles (tile seams) and the image corners."""
    pts = [rng.integers(0, width, n), rng.integers(0, height, n)]
    px = np.stack(pts, 1)
    tx = rng.integers(0, (width + tile - 1) // tile, n // 4)
    ty = rng.integers(0, (height + tile - 1) // tile, n // 4)
    seams = np.stack([np.minimum(tx * tile + 15, width - 1), np.minimum(ty * tile, height - 1)], 1)
    corners = np.array([[0, 0], [width - 1, 0], [0, height - 1], [width - 1, height - 1]])
    return np.unique(np.concatenate([px, seams, corners]), axis=0).astype(np.int32)

"""Pins of the gradient reference (oracle/grad.py).

* its forward equals the C oracle's forward (two independent codes of the same definition);
* its autograd gradients equal float64 central finite differences of that forward on the
  64x64 crop / 500-splat configuration, away from discontinuities (a perturbation that
  crosses a support edge, the alpha cut-off or the termination threshold changes the h and
  h/2 differences; such parameters are skipped and counted);
* with constant textures, the texel gradients of a splat summed over its T x T texels equal
  the gradient of the same attribute rendered with 1x1 textures (the untextured primitive);
* with per-chart resolutions (a table-addressed flat atlas) and with trilinear filtering over
  the box-filtered mip chain (on a zoomed-out crop whose samples blend levels), the forward
  equals the C oracle's and every parameter group's gradient equals central differences;
  a level fraction taken without gradient fails the trilinear case.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as og


@pytest.fixture(scope="module")
def fd_case():
    sc = synth.make_scene("sq300k_train", n=20000, env_res=32)
    sc["env_levels"] = 3
    cam = synth.config_cameras("sq300k_train")[0]
    sub, crop = synth.fd_crop_scene(sc, cam, 368, 368, 64, 64, n_keep=500)
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    rng = np.random.default_rng(1)
    d = rng.normal(size=(len(pix), 4))
    return sub, crop, tabs, pix, d


def test_forward_matches_c_oracle(fd_case):
    sub, crop, tabs, pix, d = fd_case
    ref = oracle.render(sub, crop, pixels=pix, tabs=tabs)
    g = og.grads(sub, crop, pix, d, tabs)
    assert (ref["rgba"][:, 3] > 0).mean() > 0.5
    np.testing.assert_allclose(g["rgba"], ref["rgba"], atol=1e-10)
    np.testing.assert_allclose(g["gbuf"], ref["gbuf"], atol=1e-12)


def _loss(sub, crop, pix, d, tabs, name, idx, val):
    leaves = {k: torch.tensor(np.asarray(sub[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures")}
    leaves[name].view(-1)[idx] = val
    rgba, _ = og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], sub["chart_of"], crop, pix, tabs)
    return float((rgba * torch.as_tensor(d)).sum())


def test_gradients_match_central_differences(fd_case):
    sub, crop, tabs, pix, d = fd_case
    g = og.grads(sub, crop, pix, d, tabs)
    rng = np.random.default_rng(7)
    checked, skipped = 0, 0
    for name in ("means", "quats", "scales", "opac", "textures"):
        arr = np.asarray(sub[name], np.float64).reshape(-1)
        gg = g[name].reshape(-1)
        # parameters with a non-negligible gradient, plus random ones
        cand = np.argsort(-np.abs(gg))[:40]
        picks = list(rng.choice(cand, 4, replace=False)) + list(rng.integers(0, len(arr), 2))
        for idx in picks:
            x0 = arr[idx]
            h = 1e-6 * max(1.0, abs(x0))
            f = lambda dx: _loss(sub, crop, pix, d, tabs, name, idx, x0 + dx)
            d1 = (f(h) - f(-h)) / (2 * h)
            d2 = (f(h / 2) - f(-h / 2)) / h
            scale = max(abs(gg[idx]), 1e-3 * np.abs(gg).max(), 1e-8)
            if abs(d1 - d2) > 1e-4 * scale:
                skipped += 1          # a discrete decision moved inside [-h, h]
                continue
            assert abs(d1 - gg[idx]) <= 2e-5 * scale + 1e-7, (name, idx, d1, gg[idx])
            checked += 1
    print(f"checked {checked}, skipped {skipped}")
    assert checked >= 20 and skipped <= 6, (checked, skipped)


def test_texel_gradients_sum_to_single_attribute_gradient():
    sc = synth.make_scene("shell2k", n=200, tex_res=4)
    cam = synth.crop_camera(synth.config_cameras("shell2k")[0], 48, 48, 32, 32)
    rng = np.random.default_rng(3)
    attr = rng.uniform(0.1, 0.9, size=(200, 8)).astype(np.float32)
    attr[:, 4:7] = synth._normalize(rng.normal(size=(200, 3)) + [0, 0, 2]).astype(np.float32)
    tabs = oracle.tables(sc["env"], 1)
    pix = oracle.all_pixels(32, 32)
    d = rng.normal(size=(len(pix), 4))
    g4 = og.grads(dict(sc, textures=np.broadcast_to(attr[:, None, None], (200, 4, 4, 8)).copy()),
                  cam, pix, d, tabs)
    g1 = og.grads(dict(sc, textures=attr[:, None, None].copy(), tex_res=1), cam, pix, d, tabs)
    np.testing.assert_allclose(g4["textures"].sum(axis=(1, 2)), g1["textures"][:, 0, 0],
                               atol=1e-9)
    for k in ("means", "quats", "scales", "opac"):
        np.testing.assert_allclose(g4[k], g1[k], atol=1e-8 * max(1.0, np.abs(g1[k]).max()))
    assert np.abs(g1["textures"]).max() > 0


# ---------------------------------------------------------------- environment-table gradients

@pytest.fixture(scope="module")
def env_case():
    sc = synth.make_scene("sq300k_train", n=3000, env_res=16)
    sc["env_levels"] = 3
    cam = synth.crop_camera(synth.config_cameras("sq300k_train")[0], 360, 360, 24, 24)
    tabs = oracle.tables(sc["env"], sc["env_levels"])
    pix = oracle.all_pixels(24, 24)
    d = np.random.default_rng(3).normal(size=(len(pix), 4))
    g = og.grads(sc, cam, pix, d, tabs, env=True)
    return sc, cam, tabs, pix, d, g


def _env_loss(sc, cam, pix, d, tabs, which, level, idx, val):
    t = dict(tabs)
    if which == "irr":
        a = np.array(tabs["irr"], np.float64)
        a.reshape(-1)[idx] = val
        t["irr"] = a
    else:
        levels = [np.array(l, np.float64) for l in tabs["spec"]]
        levels[level].reshape(-1)[idx] = val
        t["spec"] = levels
    leaves = {k: torch.tensor(np.asarray(sc[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures")}
    rgba, _ = og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], sc["chart_of"], cam, pix, t)
    return float((rgba * torch.as_tensor(d)).sum())


def test_env_gradients_equal_unit_differences(env_case):
    """The render is linear in every table texel (faces and taps depend on directions only),
    so a central difference with a step of 1 is the exact derivative."""
    sc, cam, tabs, pix, d, g = env_case
    rng = np.random.default_rng(5)
    checked = 0
    cases = [("irr", 0, g["irr"], tabs["irr"])]
    cases += [("spec", l, g["spec"][l], tabs["spec"][l]) for l in range(len(tabs["spec"]))]
    for which, level, grad, base in cases:
        flat = grad.reshape(-1)
        hit = np.nonzero(np.abs(flat) > 0)[0]
        assert len(hit) > 0, (which, level)
        for idx in list(rng.choice(hit, min(4, len(hit)), replace=False)) + [int(np.argmax(np.abs(flat)))]:
            x0 = float(np.asarray(base).reshape(-1)[idx])
            fd = (_env_loss(sc, cam, pix, d, tabs, which, level, idx, x0 + 1.0) -
                  _env_loss(sc, cam, pix, d, tabs, which, level, idx, x0 - 1.0)) / 2.0
            assert abs(fd - flat[idx]) <= 1e-9 * max(1.0, abs(fd)), (which, level, idx, fd, flat[idx])
            checked += 1
    assert checked >= 10


def test_irradiance_gradients_partition_of_unity(env_case):
    """Bilinear weights sum to one, so the irradiance-texel gradients of each channel sum to
    sum_pixels dL/dC_c * albedo_c (1 - M) / pi over the covered pixels (Eq. 11)."""
    sc, cam, tabs, pix, d, g = env_case
    ref = oracle.render(sc, cam, pixels=pix, tabs=tabs)
    gb, A = ref["gbuf"], ref["rgba"][:, 3]
    cov = A > 0
    expect = (d[cov, :3] * gb[cov, 0:3] * (1 - gb[cov, 3:4]) / np.pi).sum(0)
    got = g["irr"].reshape(-1, 3).sum(0)
    np.testing.assert_allclose(got, expect, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------ indirect term (Eq. 9, 12)

@pytest.fixture(scope="module")
def ind_case(fd_case):
    sub, crop, tabs, pix, d = fd_case
    rng = np.random.default_rng(21)
    sc = dict(sub)
    sc["sh"] = synth.indirect_sh(rng, len(sub["opac"]), 3)
    sc["sh_degree"] = 3
    vis = synth.visibility(rng, 1, 64, 64)[0].reshape(-1)
    return sc, crop, tabs, pix, d, vis


def test_sh_basis_two_codes():
    """The differentiable basis of the gradient reference (Legendre-polynomial derivatives
    and powers of x + iy) equals the C oracle's (associated-Legendre recurrence, atan2)."""
    rng = np.random.default_rng(0)
    w = rng.normal(size=(100, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    np.testing.assert_allclose(og._sh_basis(torch.as_tensor(w), 3).numpy(),
                               oracle.sh_basis(3, w), atol=1e-14)


def test_indirect_forward_matches_c_oracle(ind_case):
    sc, crop, tabs, pix, d, vis = ind_case
    li = oracle.indirect_eval(sc, crop, sc["sh"], 3)
    ref = oracle.render(sc, crop, pixels=pix, tabs=tabs, lind=li, vis=vis)
    g = og.grads(sc, crop, pix, d, tabs, vis=vis)
    np.testing.assert_allclose(g["rgba"], ref["rgba"], atol=1e-10)
    np.testing.assert_allclose(g["gind"], ref["gind"], atol=1e-12)
    assert np.abs(ref["gind"]).max() > 0.1


def _loss_ind(sc, crop, pix, d, tabs, vis, name, idx, val):
    leaves = {k: torch.tensor(np.asarray(sc[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures", "sh")}
    leaves[name].view(-1)[idx] = val
    rgba, _ = og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], sc["chart_of"], crop, pix, tabs,
                              sh=leaves["sh"], degree=3, vis=vis)
    return float((rgba * torch.as_tensor(d)).sum())


def test_sh_gradients_equal_unit_differences(ind_case):
    """The shaded colour is linear in L_ind, L_ind in each l_ind, and l_ind in each coefficient
    while the clamp at zero does not switch: a finite step gives the gradient exactly."""
    sc, crop, tabs, pix, d, vis = ind_case
    g = og.grads(sc, crop, pix, d, tabs, vis=vis)["sh"].reshape(-1)
    arr = np.asarray(sc["sh"], np.float64).reshape(-1)
    rng = np.random.default_rng(3)
    picks = list(np.argsort(-np.abs(g))[:6]) + list(rng.integers(0, len(arr), 4))
    base = _loss_ind(sc, crop, pix, d, tabs, vis, "sh", 0, arr[0])
    for idx in picks:
        h = 1e-3
        fd = (_loss_ind(sc, crop, pix, d, tabs, vis, "sh", idx, arr[idx] + h) - base) / h
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx])), (idx, fd, g[idx])
    assert np.abs(g).max() > 1e-3


def test_indirect_gradients_match_central_differences(ind_case):
    """Centres and rotations move the reflected direction the SH is read at: their gradients
    (and those of the other parameters) with the indirect term on against central
    differences, as for the plain render."""
    sc, crop, tabs, pix, d, vis = ind_case
    g = og.grads(sc, crop, pix, d, tabs, vis=vis)
    rng = np.random.default_rng(8)
    checked, skipped = 0, 0
    for name in ("means", "quats", "opac", "sh"):
        arr = np.asarray(sc[name], np.float64).reshape(-1)
        gg = g[name].reshape(-1)
        cand = np.argsort(-np.abs(gg))[:40]
        for idx in list(rng.choice(cand, 5, replace=False)):
            x0 = arr[idx]
            h = 1e-6 * max(1.0, abs(x0))
            f = lambda dx: _loss_ind(sc, crop, pix, d, tabs, vis, name, idx, x0 + dx)
            d1 = (f(h) - f(-h)) / (2 * h)
            d2 = (f(h / 2) - f(-h / 2)) / h
            scale = max(abs(gg[idx]), 1e-3 * np.abs(gg).max(), 1e-8)
            if abs(d1 - d2) > 1e-4 * scale:
                skipped += 1
                continue
            assert abs(d1 - gg[idx]) <= 2e-5 * scale + 1e-7, (name, idx, d1, gg[idx])
            checked += 1
    print(f"checked {checked}, skipped {skipped}")
    assert checked >= 15 and skipped <= 5, (checked, skipped)


# ------------------------------------------------------------- two-component tangent normals

def _n2(tex):
    return np.ascontiguousarray(np.concatenate([tex[..., 0:6], tex[..., 7:8]], -1))


def test_two_component_forward_matches_c_oracle(fd_case):
    """The reference with tex_format 1 (n_z rebuilt after filtering) equals the C oracle
    rendering the 7-channel atlas of the same scene."""
    sub, crop, tabs, pix, d = fd_case
    sc2 = dict(sub, tex_format=1)
    ref = oracle.render(dict(sc2, textures=_n2(sub["textures"])), crop, pixels=pix, tabs=tabs)
    g = og.grads(sc2, crop, pix, d, tabs)
    np.testing.assert_allclose(g["rgba"], ref["rgba"], atol=1e-10)
    np.testing.assert_allclose(g["gbuf"], ref["gbuf"], atol=1e-12)
    assert np.all(g["textures"][..., 6] == 0)          # the stored n_z is not read
    # and it differs from the three-component render (the rebuilt n_z is not the stored one)
    g3 = og.grads(sub, crop, pix, d, tabs)
    assert np.abs(g["gbuf"] - g3["gbuf"]).max() > 1e-6


def _loss2(sub, crop, pix, d, tabs, name, idx, val):
    leaves = {k: torch.tensor(np.asarray(sub[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures")}
    leaves[name].view(-1)[idx] = val
    rgba, _ = og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], sub["chart_of"], crop, pix, tabs, tex_format=1)
    return float((rgba * torch.as_tensor(d)).sum())


def test_two_component_gradients_match_central_differences(fd_case):
    """Texel gradients of the two encoded normal channels (and centres, through the
    rebuilt n_z of the filtered sample) against central differences."""
    sub, crop, tabs, pix, d = fd_case
    g = og.grads(dict(sub, tex_format=1), crop, pix, d, tabs)
    rng = np.random.default_rng(9)
    checked, skipped = 0, 0
    tex = np.asarray(sub["textures"], np.float64)
    gt = g["textures"]
    for name, pool in (("textures", [4, 5]), ("means", None)):
        arr = np.asarray(sub[name], np.float64).reshape(-1)
        gg = g[name].reshape(-1)
        if pool is None:
            cand = np.argsort(-np.abs(gg))[:30]
        else:
            mask = np.zeros(tex.shape, bool)
            mask[..., pool] = True
            flat = np.nonzero(mask.reshape(-1))[0]
            cand = flat[np.argsort(-np.abs(gt.reshape(-1)[flat]))[:30]]
        for idx in rng.choice(cand, 6, replace=False):
            x0 = arr[idx]
            # a smaller step than the plain pin's: some centres sit where the render is
            # smooth but steeply curved, and 1e-6 leaves a third-order error near 3e-5
            h = 1e-7 * max(1.0, abs(x0))
            f = lambda dx: _loss2(sub, crop, pix, d, tabs, name, idx, x0 + dx)
            d1 = (f(h) - f(-h)) / (2 * h)
            d2 = (f(h / 2) - f(-h / 2)) / h
            scale = max(abs(gg[idx]), 1e-3 * np.abs(gg).max(), 1e-8)
            if abs(d1 - d2) > 1e-4 * scale:
                skipped += 1
                continue
            assert abs(d1 - gg[idx]) <= 2e-5 * scale + 1e-7, (name, idx, d1, gg[idx])
            checked += 1
    assert checked >= 9 and skipped <= 3, (checked, skipped)


# ------------------------------------------- per-chart resolutions and trilinear filtering

def _charted(sub, seed=11):
    """The crop scene with each chart box-downsampled to its own side (1 to 8 texels) in a
    table-addressed flat atlas."""
    tex = np.asarray(sub["textures"], np.float32)
    n, T = tex.shape[0], tex.shape[1]
    rng = np.random.default_rng(seed)
    log2 = rng.integers(0, int(np.log2(T)) + 1, size=n)
    parts, table, off = [], np.zeros((n, 2), np.int32), 0
    for c in range(n):
        s = 1 << int(log2[c])
        b = T // s
        lv = tex[c].reshape(s, b, s, b, 8).mean(axis=(1, 3)).astype(np.float32)
        parts.append(lv.reshape(-1, 8))
        table[c] = (off, log2[c])
        off += s * s
    return dict(sub, textures=np.concatenate(parts), chart_table=table)


def _variant_loss(sc, crop, pix, d, tabs, name, idx, val):
    leaves = {k: torch.tensor(np.asarray(sc[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures")}
    leaves[name].view(-1)[idx] = val
    rgba, _ = og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], sc["chart_of"], crop, pix, tabs,
                              chart_table=sc.get("chart_table"),
                              trilinear=bool(sc.get("trilinear", False)))
    return float((rgba * torch.as_tensor(d)).sum())


@pytest.fixture(scope="module")
def tri_case():
    """The training view zoomed out ten times (focal lengths / 10) and cropped to 64x64 around
    its centre, the 1500 nearest splats: most samples there cover several texels per pixel,
    so trilinear filtering blends levels, where the full-resolution crop only magnifies."""
    sc = synth.make_scene("sq300k_train", n=20000, env_res=32)
    sc["env_levels"] = 3
    cam = dict(synth.config_cameras("sq300k_train")[0])
    cam["fx"], cam["fy"] = cam["fx"] / 10, cam["fy"] / 10
    sub, crop = synth.fd_crop_scene(sc, cam, 368, 368, 64, 64, n_keep=1500)
    tabs = oracle.tables(sub["env"], sub["env_levels"])
    pix = oracle.all_pixels(64, 64)
    d = np.random.default_rng(2).normal(size=(len(pix), 4))
    return sub, crop, tabs, pix, d


VARIANTS = {"charts": dict(tri=False, charts=True), "trilinear": dict(tri=True, charts=False),
            "charts+trilinear": dict(tri=True, charts=True)}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variant_forward_matches_c_oracle(fd_case, tri_case, variant):
    """Per-chart resolutions (flat table-addressed atlas) and trilinear filtering over the
    box-filtered chain: the differentiable reference equals the C oracle's forward."""
    v = VARIANTS[variant]
    sub, crop, tabs, pix, d = tri_case if v["tri"] else fd_case
    sc = _charted(sub) if v["charts"] else dict(sub)
    sc["trilinear"] = v["tri"]
    ref = oracle.render(sc, crop, pixels=pix, tabs=tabs)
    g = og.grads(sc, crop, pix, d, tabs)
    np.testing.assert_allclose(g["rgba"], ref["rgba"], atol=1e-10)
    np.testing.assert_allclose(g["gbuf"], ref["gbuf"], atol=1e-12)
    # the variant changes the image (it is not the plain uniform bilinear render)
    base = oracle.render(sub, crop, pixels=pix, tabs=tabs)
    assert np.abs(base["gbuf"] - ref["gbuf"]).max() > 1e-4
    assert g["textures"].shape == np.asarray(sc["textures"]).shape


def test_trilinear_crop_exercises_every_level_rule(tri_case):
    """The trilinear pins below are meaningful only if the crop has samples below level 0's
    threshold, blending two levels, and clamped at the last level; count them from the
    footprint the reference differentiates."""
    sub, crop, tabs, pix, d = tri_case
    sc = dict(sub, trilinear=True)
    leaves = {k: torch.tensor(np.asarray(sc[k], np.float32), dtype=torch.float64)
              for k in ("means", "quats", "scales", "opac", "textures")}
    stats = {}
    og.render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                    leaves["textures"], sc["chart_of"], crop, pix, tabs, trilinear=True,
                    info=stats)
    print(stats)
    assert stats["blend"] > 10000 and stats["level0"] > 10000 and stats["last"] > 0, stats


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variant_gradients_match_central_differences(fd_case, tri_case, variant):
    """Gradients of every parameter group under the variant against central differences;
    with trilinear filtering the centres, rotations and scales also move the level (the
    blend fraction lambda - floor(lambda) carries gradient through the footprint)."""
    v = VARIANTS[variant]
    sub, crop, tabs, pix, d = tri_case if v["tri"] else fd_case
    sc = _charted(sub) if v["charts"] else dict(sub)
    sc["trilinear"] = v["tri"]
    g = og.grads(sc, crop, pix, d, tabs)
    rng = np.random.default_rng(13)
    checked, skipped = 0, 0
    for name in ("means", "quats", "scales", "opac", "textures"):
        arr = np.asarray(sc[name], np.float64).reshape(-1)
        gg = g[name].reshape(-1)
        cand = np.argsort(-np.abs(gg))[:40]
        picks = list(rng.choice(cand, 4, replace=False)) + list(rng.integers(0, len(arr), 1))
        for idx in picks:
            x0 = arr[idx]
            h = 1e-7 * max(1.0, abs(x0))
            f = lambda dx: _variant_loss(sc, crop, pix, d, tabs, name, idx, x0 + dx)
            d1 = (f(h) - f(-h)) / (2 * h)
            d2 = (f(h / 2) - f(-h / 2)) / h
            scale = max(abs(gg[idx]), 1e-3 * np.abs(gg).max(), 1e-8)
            if abs(d1 - d2) > 1e-4 * scale:
                skipped += 1
                continue
            assert abs(d1 - gg[idx]) <= 2e-5 * scale + 1e-7, (name, idx, d1, gg[idx])
            checked += 1
    print(f"{variant}: checked {checked}, skipped {skipped}")
    assert checked >= 18 and skipped <= 5, (checked, skipped)

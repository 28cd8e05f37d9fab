"""Gradient reference — TEST INFRASTRUCTURE ONLY.

A dense float64 formulation of the same per-pixel definition as oracle.c (Sec. 3.1 Eq. 1-3,
Sec. 3.2-3.3 Eq. 4-6, Sec. 3.5 Eq. 7-12), written with plain PyTorch CPU ops so that autograd
gives the gradient of any scalar of the rendered RGBA with respect to the splat centres, the
(unnormalised) quaternions, the linear scales, the opacities and the texels — the quantities
the paper optimises (Sec. 3.6) — and, on request, to the texels of the environment's shading
tables (irradiance cube and prefiltered levels taken as learnable, as the environment is
optimised end to end in Sec. 3.5-3.6) and to the per-splat spherical-harmonic coefficients of
the indirect light (Eq. 9, Eq. 12, also learned end to end in Sec. 3.6).

Discrete decisions are taken from values and carry no gradient, exactly as in the forward
definition: the near-plane drop, the hit in front of the camera, the square support, the alpha
cut-off, the termination threshold (a splat blends iff the running transmittance after it
stays >= t_min), the depth order (float32 depth, then index), the texel taps and the cube
face. Everything continuous between those decisions is differentiated: alpha = min(alpha_max,
o G) passes no gradient when clamped.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import DEFAULT_PARAMS, cam16

DT = torch.float64


def _quat_rot(q):
    qn = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = qn.unbind(1)
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)
    return R.view(-1, 3, 3)


def _cube_face(d):
    """Face index and (sc, tc, ma) of directions d [M,3] (OpenGL major-axis rule)."""
    ad = d.abs().detach()
    ax, ay, az = ad[:, 0], ad[:, 1], ad[:, 2]
    isx = (ax >= ay) & (ax >= az)
    isy = (~isx) & (ay >= az)
    isz = (~isx) & (~isy)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pos = torch.where(isx, x >= 0, torch.where(isy, y >= 0, z >= 0)).detach()
    face = torch.where(isx, 0, torch.where(isy, 2, 4)) + (~pos).long()
    sc = torch.where(face == 0, -z, torch.where(face == 1, z, torch.where(face == 5, -x, x)))
    tc = torch.where(face <= 1, -y, torch.where(face == 2, z, torch.where(face == 3, -z, -y)))
    ma = torch.where(isx, x.abs(), torch.where(isy, y.abs(), z.abs()))
    return face, sc, tc, ma


def _bilinear(flat, base, H, W, X, Y):
    """Bilinear sample of images stored in flat [K, C] (row-major H x W each, image m starting
    at row base[m]) at texel coordinates X, Y [M] (centres at integers), clamp-to-edge."""
    x0 = torch.floor(X.detach())
    y0 = torch.floor(Y.detach())
    fx, fy = X - x0, Y - y0
    i0 = x0.long().clamp(0, W - 1)
    i1 = (x0.long() + 1).clamp(0, W - 1)
    j0 = y0.long().clamp(0, H - 1)
    j1 = (y0.long() + 1).clamp(0, H - 1)
    v00, v10 = flat[base + j0 * W + i0], flat[base + j0 * W + i1]
    v01, v11 = flat[base + j1 * W + i0], flat[base + j1 * W + i1]
    fx, fy = fx[:, None], fy[:, None]
    return (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11)


def _bilinear_var(flat, base, side, X, Y):
    """Bilinear samples of square images in flat [K, C], image m of side[m] texels starting at
    row base[m] (per-sample long tensors), at texel coordinates X, Y (centres at integers),
    clamp-to-edge."""
    x0 = torch.floor(X.detach())
    y0 = torch.floor(Y.detach())
    fx, fy = X - x0, Y - y0
    top = side - 1
    i0 = torch.minimum(torch.clamp(x0.long(), min=0), top)
    i1 = torch.minimum(torch.clamp(x0.long() + 1, min=0), top)
    j0 = torch.minimum(torch.clamp(y0.long(), min=0), top)
    j1 = torch.minimum(torch.clamp(y0.long() + 1, min=0), top)
    v00, v10 = flat[base + j0 * side + i0], flat[base + j0 * side + i1]
    v01, v11 = flat[base + j1 * side + i0], flat[base + j1 * side + i1]
    fx, fy = fx[:, None], fy[:, None]
    return (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11)


def _mip_chain(flat, off0, log2):
    """Every chart's box-filtered mip chain (Sec. 5 mipmapping: level l texel = mean of the
    2^l x 2^l level-0 texels it covers), built from the level-0 texels in flat [K, 8] (chart c
    at row off0[c], 2^log2[c] a side) with differentiable means. Returns the chain texels
    [K', 8] and offs [n_charts, 6] (row of level l of chart c, -1 past its last level)."""
    n = len(off0)
    offs = np.full((n, 6), -1, np.int64)
    parts, rows = [], 0
    for lg in np.unique(log2):
        cs = np.nonzero(log2 == lg)[0]
        side = 1 << int(lg)
        idx = torch.as_tensor(off0[cs][:, None] + np.arange(side * side)[None], dtype=torch.long)
        lv = flat[idx].reshape(len(cs), side, side, 8)
        for l in range(int(lg) + 1):
            sl, b = side >> l, 1 << l
            m = lv.reshape(len(cs), sl, b, sl, b, 8).mean(dim=(2, 4))
            offs[cs, l] = rows + np.arange(len(cs)) * sl * sl
            parts.append(m.reshape(-1, 8))
            rows += len(cs) * sl * sl
    return torch.cat(parts, 0), offs


def _cube_lookup(cube, d):
    """cube [6, r, r, 3] float64 tensor, directions d [M,3] -> [M,3]."""
    r = cube.shape[1]
    face, sc, tc, ma = _cube_face(d)
    X = 0.5 * (sc / ma + 1.0) * r - 0.5
    Y = 0.5 * (tc / ma + 1.0) * r - 0.5
    return _bilinear(cube.reshape(-1, 3), face * r * r, r, r, X, Y)


def _sh_basis(w, degree):
    """Real orthonormal spherical harmonics (no Condon-Shortley phase, index l*l + l + m) at
    unit directions w [M,3] -> [M,(degree+1)^2], differentiable: with z = cos(theta),
    P_l^m(z) = (1 - z^2)^(m/2) d^m P_l / dz^m (Legendre polynomial derivatives from numpy) and
    (1 - z^2)^(m/2) (cos, sin)(m phi) = (Re, Im) (x + i y)^m on the unit sphere."""
    x, y, z = w.unbind(1)
    K = (degree + 1) ** 2
    cols = [None] * K
    re, im = torch.ones_like(x), torch.zeros_like(x)     # (x + i y)^0
    pw = [(re, im)]
    for m in range(1, degree + 1):
        re, im = re * x - im * y, re * y + im * x
        pw.append((re, im))
    for l in range(degree + 1):
        Pl = np.polynomial.legendre.Legendre.basis(l)
        for m in range(0, l + 1):
            coef = Pl.deriv(m).convert(kind=np.polynomial.Polynomial).coef
            pz = torch.zeros_like(z)
            for i in range(len(coef) - 1, -1, -1):          # Horner in z
                pz = pz * z + float(coef[i])
            Klm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) /
                            math.factorial(l + m))
            if m == 0:
                cols[l * l + l] = Klm * pz
            else:
                cols[l * l + l + m] = math.sqrt(2) * Klm * pz * pw[m][0]
                cols[l * l + l - m] = math.sqrt(2) * Klm * pz * pw[m][1]
    return torch.stack(cols, 1)


def _indirect(means, quats, sh, degree, o):
    """Per-splat indirect radiance [N,3]: max(0, sum_j c_j Y_j(w_r)), w_r the mirror reflection
    of the unit camera-to-centre direction about the splat plane."""
    n = _quat_rot(quats)[:, :, 2]
    d = means - o[None]
    d = d / d.norm(dim=1, keepdim=True)
    wr = d - 2 * (d * n).sum(1, keepdim=True) * n
    wr = wr / wr.norm(dim=1, keepdim=True)
    Y = _sh_basis(wr, degree)
    return torch.clamp((Y[:, :, None] * sh).sum(1), min=0.0)


def _shade(g, A, dirs, tabs, bg, gind=None, vis=None):
    """Split-sum shading (Eq. 10-12) of blended maps g [P,8] with alpha A [P]; with the
    indirect term the specular radiance is V L_dir + (1 - V) L_ind (gind [P,3], vis [P])."""
    P = g.shape[0]
    wo = -dirs / dirs.norm(dim=1, keepdim=True)
    N = g[:, 5:8]
    nn = N.norm(dim=1, keepdim=True)
    zero = (nn[:, 0] == 0).detach()
    Nh = torch.where(zero[:, None], wo, N / torch.where(zero[:, None], torch.ones_like(nn), nn))
    ndv = (Nh * wo).sum(1)
    wr = 2 * ndv[:, None] * Nh - wo
    M, R = g[:, 3], g[:, 4]
    irr = tabs["irr"] if torch.is_tensor(tabs["irr"]) else torch.as_tensor(tabs["irr"], dtype=DT)
    E = _cube_lookup(irr, Nh)
    levels = [l if torch.is_tensor(l) else torch.as_tensor(l, dtype=DT) for l in tabs["spec"]]
    L = len(levels)
    rc = R.clamp(0.0, 1.0)
    lev = rc * (L - 1)
    l0 = torch.floor(lev.detach()).long().clamp(max=L - 1)
    l1 = (l0 + 1).clamp(max=L - 1)
    fl = lev - l0.to(DT)
    P0 = torch.zeros(P, 3, dtype=DT)
    P1 = torch.zeros(P, 3, dtype=DT)
    for l in range(L):
        m0 = l0 == l
        if m0.any():
            P0 = P0.index_put((m0.nonzero()[:, 0],), _cube_lookup(levels[l], wr[m0]))
        m1 = l1 == l
        if m1.any():
            P1 = P1.index_put((m1.nonzero()[:, 0],), _cube_lookup(levels[l], wr[m1]))
    Lp = (1 - fl)[:, None] * P0 + fl[:, None] * P1
    if gind is not None:
        V = vis[:, None]
        Lp = V * Lp + (1 - V) * gind
    lut = torch.as_tensor(tabs["lut"], dtype=DT)
    n = lut.shape[0]
    x = ndv.clamp(0.0, 1.0) * n - 0.5
    y = rc * n - 0.5
    ab = _bilinear(lut.reshape(-1, 2), torch.zeros(P, dtype=torch.long), n, n, x, y)
    F0 = 0.04 * (1 - M)[:, None] + g[:, 0:3] * M[:, None]
    bgt = torch.as_tensor(bg, dtype=DT)[None]
    C = (g[:, 0:3] / math.pi * (1 - M)[:, None] * E + Lp * (F0 * ab[:, 0:1] + ab[:, 1:2])
         + (1 - A)[:, None] * bgt)
    empty = (A <= 0).detach()
    return torch.where(empty[:, None], bgt.expand(P, 3), C)


def render_dense(means, quats, scales, opac, textures, chart_of, cam, pixels, tabs=None,
                 params=None, sh=None, degree=0, vis=None, tex_format=0, chart_table=None,
                 trilinear=False, info=None):
    """Differentiable render of pixels [P,2]. Tensors are float64 (leaves may require grad).
    Returns rgba [P,4] and gbuf [P,8] (albedo 3, metallic, roughness, normal 3); with sh
    ([N,(degree+1)^2,3]) the indirect term is on (vis [P] visibility, default 1) and gbuf has
    the blended L_ind as channels 8..10. tex_format 1: two-component tangent normals, n_z
    rebuilt as sqrt(max(0, 1 - n_x^2 - n_y^2)) after filtering (texel channel 6 unused).
    chart_table [n_charts, 2] (level-0 texel offset, log2 side): per-chart resolutions, the
    textures then a flat [texels, 8] array (Sec. 5, adaptive resolution). trilinear: filter
    over each chart's box-filtered mip chain at the level lambda = log2(T rho), rho the larger
    of the pixel's texture-space steps along the image axes (derivatives of the exact
    ray-plane (u,v)); lambda <= 0 samples level 0, past the last level the last level, else
    levels floor(lambda) and floor(lambda)+1 blend by the fraction, which carries gradient
    through rho to the geometry (Sec. 5, mipmapping). info: a dict that receives the number
    of blended samples at level 0 alone, blending two levels and at the last level alone."""
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    f32 = lambda x: float(np.float32(x))
    S, amin, amax, tmin, near = (f32(p[k]) for k in ("s_sigma", "alpha_min", "alpha_max",
                                                      "t_min", "near_z"))
    bg = [f32(b) for b in p["bg"]]
    c = cam16(cam)
    Wr = torch.as_tensor(c[:12].reshape(3, 4)[:, :3], dtype=DT)
    t = torch.as_tensor(c[:12].reshape(3, 4)[:, 3], dtype=DT)
    fx, fy, cx, cy = (float(v) for v in c[12:16])
    o = -(Wr.T @ t)
    R = _quat_rot(quats)
    tu, tv, nrm = R[:, :, 0], R[:, :, 1], R[:, :, 2]
    # depth (float32 key) and near-plane drop, from values
    mu_np = means.detach().numpy()
    Wn, tn = c[:12].reshape(3, 4)[:, :3], c[:12].reshape(3, 4)[:, 3]
    z = Wn[2, 0] * mu_np[:, 0] + Wn[2, 1] * mu_np[:, 1] + Wn[2, 2] * mu_np[:, 2] + tn[2]
    keep = torch.as_tensor(z > near)
    order = np.lexsort((np.arange(len(z)), z.astype(np.float32)))
    sigma = torch.where(((nrm * (o[None] - means)).sum(1) >= 0).detach(), 1.0, -1.0).to(DT)
    pix = torch.as_tensor(np.asarray(pixels, np.float64))
    dc = torch.stack([(pix[:, 0] + 0.5 - cx) / fx, (pix[:, 1] + 0.5 - cy) / fy,
                      torch.ones(len(pix), dtype=DT)], 1)
    dirs = dc @ Wr           # rows: R_c2w d_cam = Wr^T d_cam
    # dense ray-plane intersection [P,N]
    den = dirs @ nrm.T
    mo = means - o[None]
    num = (mo * nrm).sum(1)
    safe = torch.where(den == 0, torch.ones_like(den), den)
    lam = num[None] / safe
    # P - mu = o + lam d - mu
    rel_u = (o[None] @ tu.T - (means * tu).sum(1)[None]) + lam * (dirs @ tu.T)
    rel_v = (o[None] @ tv.T - (means * tv).sum(1)[None]) + lam * (dirs @ tv.T)
    u = rel_u / scales[None, :, 0]
    v = rel_v / scales[None, :, 1]
    valid = (keep[None] & (den != 0) & (lam > 0)).detach()
    mabs = torch.maximum(u.abs(), v.abs()).detach()
    valid &= mabs <= S
    G = torch.exp(-0.5 * (u * u + v * v))
    oG = opac[None] * G
    alpha = torch.minimum(oG, torch.full_like(oG, amax))
    include = valid & (alpha.detach() >= amin)
    a_inc = torch.where(include, alpha, torch.zeros_like(alpha))
    # depth order, termination from values
    a_o = a_inc[:, order]
    inc_o = include[:, order]
    trans_after = torch.cumprod(1 - a_o.detach(), dim=1)
    blended_o = inc_o & (trans_after >= tmin)
    a_b = torch.where(blended_o, a_o, torch.zeros_like(a_o))
    one_m = 1 - a_b
    T_excl = torch.cat([torch.ones(len(pix), 1, dtype=DT), torch.cumprod(one_m, 1)[:, :-1]], 1)
    w_o = a_b * T_excl
    T_final = torch.prod(one_m, 1)
    # texture on the blended pairs only
    pi, ki = blended_o.nonzero(as_tuple=True)
    k = torch.as_tensor(order)[ki]
    uu, vv = u[pi, k], v[pi, k]
    chart = np.asarray(chart_of, np.int64)[k.numpy()]
    flat = textures.reshape(-1, 8)
    if chart_table is None:
        T = textures.shape[1]
        nch = len(textures)
        off0 = np.arange(nch, dtype=np.int64) * T * T
        log2 = np.full(nch, int(round(math.log2(T))), np.int64)
    else:
        ct = np.asarray(chart_table, np.int64).reshape(-1, 2)
        off0, log2 = ct[:, 0], ct[:, 1]
    side_b = torch.as_tensor(1 << log2[chart], dtype=torch.long)
    s_tex = (uu + S) / (2 * S)
    t_tex = (vv + S) / (2 * S)
    if not trilinear:
        sf = side_b.to(DT)
        tx = _bilinear_var(flat, torch.as_tensor(off0[chart]), side_b, s_tex * sf - 0.5,
                           t_tex * sf - 0.5)                                    # [B, 8]
    else:
        chain, offs = _mip_chain(flat, off0, log2)
        # footprint: d(s,t)/dX and d(s,t)/dY from the ray derivative d'(X) = column X of the
        # camera-to-world rotation over f, lambda' = -lambda (d'.n)/(d.n), P' = lambda' d +
        # lambda d'
        Rc2w = Wr.T
        lam_b, den_b, d_b = lam[pi, k], den[pi, k], dirs[pi]
        steps = []
        for ax, f in ((0, fx), (1, fy)):
            dd = Rc2w[:, ax] / f
            dlam = -lam_b * (nrm[k] @ dd) / den_b
            dP = lam_b[:, None] * dd[None] + dlam[:, None] * d_b
            ju = (dP * tu[k]).sum(1) / scales[k, 0] / (2 * S)
            jv = (dP * tv[k]).sum(1) / scales[k, 1] / (2 * S)
            steps.append(torch.sqrt(ju * ju + jv * jv))
        rho = torch.maximum(steps[0], steps[1])
        lamb = torch.log2(side_b.to(DT) * rho)
        Lc = torch.as_tensor(log2[chart], dtype=torch.long)
        lv = lamb.detach()
        l0 = torch.where(lv > 0, torch.floor(lv).long(), torch.zeros_like(Lc))
        last = l0 >= Lc
        blend = (lv > 0) & ~last
        la = torch.where(last, Lc, l0)
        lb = torch.where(blend, l0 + 1, la)
        fb = torch.where(blend, lamb - torch.floor(lv), torch.zeros_like(lamb))
        offs_t = torch.as_tensor(offs)
        cb = torch.as_tensor(chart, dtype=torch.long)

        def level_sample(l):
            sl = side_b >> l
            sf = sl.to(DT)
            return _bilinear_var(chain, offs_t[cb, l], sl, s_tex * sf - 0.5, t_tex * sf - 0.5)

        if info is not None:
            info.update(level0=int((lv <= 0).sum()), blend=int(blend.sum()),
                        last=int(((lv > 0) & last).sum()))
        va, vb = level_sample(la), level_sample(lb)
        tx = (1 - fb)[:, None] * va + fb[:, None] * vb
    nt = tx[:, 4:7]
    if tex_format == 1:
        r2 = 1 - tx[:, 4] * tx[:, 4] - tx[:, 5] * tx[:, 5]
        pos = (r2 > 0).detach()
        nz = torch.where(pos, torch.sqrt(torch.where(pos, r2, torch.ones_like(r2))),
                         torch.zeros_like(r2))
        nt = torch.stack([tx[:, 4], tx[:, 5], nz], 1)
    ntl = nt.norm(dim=1, keepdim=True)
    nth = torch.where(ntl > 0, nt / torch.where(ntl > 0, ntl, torch.ones_like(ntl)),
                      torch.tensor([0.0, 0.0, 1.0], dtype=DT)[None])
    nw = sigma[k][:, None] * torch.einsum("bij,bj->bi", R[k], nth)
    x8 = torch.cat([tx[:, 0:3], tx[:, 7:8], tx[:, 3:4], nw], 1)
    if sh is not None:
        x8 = torch.cat([x8, _indirect(means, quats, sh, degree, o)[k]], 1)
    wb = w_o[pi, ki]
    gbuf = torch.zeros(len(pix), x8.shape[1], dtype=DT).index_add(0, pi, wb[:, None] * x8)
    A = 1 - T_final
    if tabs is None:
        rgb = torch.zeros(len(pix), 3, dtype=DT)
    elif sh is None:
        rgb = _shade(gbuf, A, dirs, tabs, bg)
    else:
        V = (torch.ones(len(pix), dtype=DT) if vis is None
             else torch.as_tensor(np.asarray(vis, np.float64)))
        rgb = _shade(gbuf[:, :8], A, dirs, tabs, bg, gind=gbuf[:, 8:11], vis=V)
    rgba = torch.cat([rgb, A[:, None]], 1)
    return rgba, gbuf


def grads(scene, cam, pixels, d_rgba, tabs=None, params=None, env=False, vis=None):
    """Gradients of sum(d_rgba * rgba) w.r.t. means, quats, scales, opac and textures; with
    env=True also w.r.t. the texels of the irradiance cube ("irr", [6,r,r,3]) and of every
    prefiltered level ("spec", list of [6,r_l,r_l,3]), the tables taken as parameters; with
    scene["sh"] (degree scene["sh_degree"]) the indirect term is on (vis [P] per pixel) and
    the coefficients get their gradient ("sh"); scene["tex_format"] = 1 renders with
    two-component tangent normals (textures stay [N,T,T,8]; channel 6 gets no gradient)."""
    names = ["means", "quats", "scales", "opac", "textures"]
    if scene.get("sh") is not None:
        names.append("sh")
    leaves = {k: torch.tensor(np.asarray(scene[k], np.float32), dtype=DT, requires_grad=True)
              for k in names}
    t = tabs
    if env:
        t = dict(tabs)
        t["irr"] = torch.tensor(np.asarray(tabs["irr"]), dtype=DT, requires_grad=True)
        t["spec"] = [torch.tensor(np.asarray(l), dtype=DT, requires_grad=True)
                     for l in tabs["spec"]]
    rgba, gbuf = render_dense(leaves["means"], leaves["quats"], leaves["scales"], leaves["opac"],
                              leaves["textures"], scene["chart_of"], cam, pixels, t, params,
                              sh=leaves.get("sh"), degree=int(scene.get("sh_degree", 0)),
                              vis=vis, tex_format=int(scene.get("tex_format", 0)),
                              chart_table=scene.get("chart_table"),
                              trilinear=bool(scene.get("trilinear", False)))
    loss = (rgba * torch.as_tensor(np.asarray(d_rgba), dtype=DT)).sum()
    loss.backward()
    out = {k: leaves[k].grad.detach().numpy() for k in leaves}
    out["rgba"] = rgba.detach().numpy()
    out["gbuf"] = gbuf[:, :8].detach().numpy()
    if gbuf.shape[1] > 8:
        out["gind"] = gbuf[:, 8:].detach().numpy()
    if env:
        z = lambda x: (x.grad if x.grad is not None else torch.zeros_like(x)).detach().numpy()
        out["irr"] = z(t["irr"])
        out["spec"] = [z(l) for l in t["spec"]]
    return out

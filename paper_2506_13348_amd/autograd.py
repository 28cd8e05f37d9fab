"""torch.autograd.Function over ts_raster_fwd / ts_raster_bwd (and, with the indirect term,
ts_indirect_eval / ts_indirect_bwd).

`render_rgba(means, quats, scales, opac, atlas, chart_of, cams, width, height, tables)` renders
a batch of views and, under autograd, returns gradients for the five splat tensors (and the
per-splat SH coefficients of the indirect term) from the hand-written HIP backward
(deterministic, no floating-point atomics). Python here allocates buffers and enqueues the C
entry points; it performs none of the rendering arithmetic."""
from __future__ import annotations

from types import SimpleNamespace

import torch

from . import _ffi as F
from .render import RenderPlan


class _SceneView(SimpleNamespace):
    pass


def _scene_view(means, quats, scales, opac, atlas, chart_of, tables, sh=None, sh_degree=0,
                atlas_spec=None):
    if atlas_spec is None:
        # [n_charts, T, T, 8], or [n_charts, T, T, 7]: two-component tangent normals
        spec = dict(tex_res=int(atlas.shape[1]),
                    tex_format=1 if atlas.dim() == 4 and atlas.shape[-1] == 7 else 0)
    else:
        spec = dict(atlas_spec)
    return _SceneView(device=means.device, n=int(means.shape[0]), means=means.contiguous(),
                      quats=quats.contiguous(), scales=scales.contiguous(),
                      opac=opac.contiguous(), atlas=atlas.contiguous(),
                      chart_of=chart_of.contiguous(), tables=tables,
                      sh=None if sh is None else sh.contiguous(), sh_degree=int(sh_degree),
                      **spec)


class BackwardRunner:
    """Workspace and partial buffer of ts_raster_bwd for one render plan, grown on demand."""

    def __init__(self, plan: RenderPlan, partial_floats=None):
        self.plan = plan
        dev = plan.scene.device
        ws = F.ts_raster_bwd_workspace(plan.V, plan.scene.n, plan.cap)
        self.ws = torch.empty((ws + 7) // 8, device=dev, dtype=torch.int64)
        if partial_floats is None:
            partial_floats = max(1 << 20, 64 * max(plan.cap, 1))
        self.partials = torch.empty(int(partial_floats), device=dev, dtype=torch.float32)
        self.status = torch.zeros(1, device=dev, dtype=torch.int32)
        self.used = torch.zeros(1, device=dev, dtype=torch.int64)
        # the indirect term: dL/dl_ind per (view, splat), then the SH coefficients
        self.indirect = getattr(plan, "indirect", False)
        if self.indirect and plan.gbuf_ind is None:
            raise ValueError("the indirect backward needs the plan's L_ind map (gbuf=True)")
        self.d_lind = (torch.empty(plan.V * max(plan.scene.n, 1) * 4, device=dev,
                                   dtype=torch.float32) if self.indirect else None)

    def run(self, d_rgba, grads, beta=0.0, retry=True):
        """grads = (d_means, d_quats, d_scales, d_opac, d_atlas[, d_sh]); d_sh (the SH
        coefficients' gradient) only for a plan with the indirect term."""
        p, sc = self.plan, self.plan.scene
        d_means, d_quats, d_scales, d_opac, d_atlas = grads[:5]
        d_sh = grads[5] if len(grads) > 5 else None
        ind = dict(lind=p.lind, vis=p.vis, gbuf_ind=p.gbuf_ind, d_lind=self.d_lind) \
            if self.indirect else {}
        for attempt in range(2):
            self.status.zero_()
            F.ts_raster_bwd(p.V, p.W, p.H, p.cams, p.params, sc.n, sc.means, sc.quats, sc.scales,
                            sc.chart_of, p.rec, p.rect, p.tile_ranges, p.pair_ids, p.cap,
                            sc.atlas, sc.tables.struct, p.gbuf, p.t_final, p.n_contrib,
                            d_rgba.contiguous(), self.ws, self.partials, self.status, self.used,
                            beta, d_means, d_quats, d_scales, d_opac, d_atlas, p.stream, **ind)
            if not retry:
                break
            if int(self.status.item()) == 0:
                break
            # the counter reports what the frame needed: size to it and run again
            need = int(self.used.item())
            self.partials = torch.empty(need + need // 16 + 4096, device=self.partials.device,
                                        dtype=torch.float32)
        else:
            raise RuntimeError("ts_raster_bwd: partial buffer overflow after resizing")
        if self.indirect and d_sh is not None:
            F.ts_indirect_bwd(p.V, p.cams, sc.n, sc.means, sc.quats, sc.sh, sc.sh_degree, p.lind,
                              self.d_lind, beta, d_sh, d_means, d_quats, p.stream)


class EnvBackward:
    """Workspace of ts_env_bwd for one render plan: gradients of the loss with respect to the
    texels of the plan's shading tables (irradiance cube and prefiltered levels); a plan with
    the indirect term passes its visibility, which weights the specular tables' share."""

    def __init__(self, plan: RenderPlan):
        self.plan = plan
        dev = plan.scene.device
        ws = F.ts_env_bwd_workspace(plan.scene.tables.struct)
        self.ws = torch.empty((ws + 7) // 8, device=dev, dtype=torch.int64)
        tabs = plan.scene.tables
        self.d_irr = torch.zeros_like(tabs.irr)
        self.d_spec = torch.zeros_like(tabs.spec)

    def run(self, d_rgba, beta=0.0):
        p = self.plan
        if p.gbuf is None or p.t_final is None:
            raise RuntimeError("environment gradients need the plan's G-buffers (gbuf=True)")
        F.ts_env_bwd(p.V, p.W, p.H, p.cams, p.scene.tables.struct, p.gbuf, p.t_final,
                     d_rgba.contiguous(), self.ws, beta, self.d_irr, self.d_spec, p.stream,
                     vis=p.vis)
        return self.d_irr, self.d_spec


class TexSplatRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, quats, scales, opac, atlas, chart_of, cams, width, height, tables,
                params, sh, sh_degree, vis, atlas_spec):
        sv = _scene_view(means.detach(), quats.detach(), scales.detach(), opac.detach(),
                         atlas.detach(), chart_of, tables,
                         None if sh is None else sh.detach(), sh_degree, atlas_spec)
        plan = RenderPlan(sv, cams, width, height, params, shade=True, gbuf=True, aux=True,
                          vis=vis)
        plan.run()
        plan.check()
        ctx.plan = plan
        return plan.rgba.view(plan.V, plan.H, plan.W, 4).clone()

    @staticmethod
    def backward(ctx, d_rgba):
        plan = ctx.plan
        sc = plan.scene
        grads = (torch.empty_like(sc.means), torch.empty_like(sc.quats),
                 torch.empty_like(sc.scales), torch.empty_like(sc.opac),
                 torch.empty_like(sc.atlas))
        if plan.indirect:
            grads = grads + (torch.empty_like(sc.sh),)
        BackwardRunner(plan).run(d_rgba.contiguous(), grads)
        d_sh = grads[5] if plan.indirect else None
        return (*grads[:5], None, None, None, None, None, None, d_sh, None, None, None)


def render_rgba(means, quats, scales, opac, atlas, chart_of, cams, width, height, tables,
                params=None, sh=None, sh_degree=0, vis=None, atlas_spec=None):
    """[V,H,W,4] shaded RGBA + alpha, differentiable w.r.t. the first five tensors (atlas
    [n_charts,T,T,8], or [n_charts,T,T,7] with two-component tangent normals) and, with
    the indirect term (sh [n,(sh_degree+1)^2,3] per-splat SH coefficients, vis [V,H,W] optional
    visibility), w.r.t. sh as well.

    atlas_spec (DeviceScene.atlas_spec()) describes any other atlas layout: per-chart sides
    through a chart table, mip chains with trilinear sampling. The atlas gradient then has the
    atlas's layout and is w.r.t. the level-0 texels (zero on the coarser levels of a chain,
    which ts_atlas_mips rebuilds from level 0 after an update)."""
    return TexSplatRender.apply(means, quats, scales, opac, atlas, chart_of, cams, width, height,
                                tables, params, sh, sh_degree, vis, atlas_spec)

"""Device-resident scenes and render plans over the texsplat C ABI.

A `DeviceScene` holds one scene on the GPU: splat parameters, the packed texture atlas with
its indirection buffer (Supp. Sec. 1) and the shading tables of its environment (Sec. 3.5.4).
A `RenderPlan` preallocates every buffer of a batch of same-resolution views, so `run()`
enqueues the whole path (preprocess -> bin/sort -> raster with fused shading) on a stream
without allocating or synchronising; `check()` reads the pair-list status afterwards.
A scene with per-splat indirect-light SH coefficients renders with the indirect term of
Eq. 9 and Eq. 12 (per-view SH evaluation, blended L_ind map, visibility-weighted specular
mix; the visibility is an input of the plan)."""
from __future__ import annotations

import numpy as np
import torch

from . import _ffi as F

DEFAULTS = dict(s_sigma=3.0, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, near_z=0.2,
                bg=(0.0, 0.0, 0.0), sampler=0)
IRR_RES = 16
LUT_RES = 256
LUT_SAMPLES = 4096


def _dev(x, device, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x)) if isinstance(x, np.ndarray) else x
    t = t.to(device=device)
    if dtype is not None:
        t = t.to(dtype)
    return t.contiguous()


def cameras_tensor(cams, device="cuda"):
    """[V,16] float32: w2c (12, row-major), fx, fy, cx, cy."""
    if isinstance(cams, torch.Tensor):
        return cams.to(device=device, dtype=torch.float32).contiguous()
    if isinstance(cams, np.ndarray):
        return _dev(cams.astype(np.float32), device)
    arr = np.zeros((len(cams), 16), np.float32)
    for i, c in enumerate(cams):
        arr[i, :12] = np.asarray(c["w2c"], np.float32).reshape(12)
        arr[i, 12:] = [c["fx"], c["fy"], c["cx"], c["cy"]]
    return _dev(arr, device)


class EnvTables:
    """Shading tables of one environment cubemap, built by the HIP table kernels."""

    def __init__(self, env, levels, device="cuda", irr_res=IRR_RES, lut_res=LUT_RES,
                 lut_samples=LUT_SAMPLES, lut=None):
        env = _dev(np.asarray(env, np.float32) if isinstance(env, np.ndarray) else env, device,
                   torch.float32)
        r = int(env.shape[1])
        self.res, self.levels, self.irr_res, self.lut_res = r, int(levels), irr_res, lut_res
        n_spec = sum(6 * max(r >> l, 1) ** 2 for l in range(self.levels))
        self.spec = torch.empty(n_spec * 4, device=device, dtype=torch.float32)
        self.irr = torch.empty(6 * irr_res * irr_res * 4, device=device, dtype=torch.float32)
        texel_ws = torch.empty(6 * r * r * 4, device=device, dtype=torch.float64)
        F.ts_env_tables(env, r, self.levels, irr_res, self.spec, self.irr, texel_ws)
        if lut is None:
            lut = torch.empty(lut_res * lut_res * 2, device=device, dtype=torch.float32)
            F.ts_brdf_lut(lut_res, lut_samples, lut)
        self.lut = lut
        self._keep = (env, texel_ws)
        self.struct = F.make_env(self.spec, r, self.levels, self.irr, irr_res, self.lut, lut_res)

    def spec_levels(self):
        """Specular levels as a list of [6, r_l, r_l, 3] tensors (views)."""
        out, off = [], 0
        for l in range(self.levels):
            rl = max(self.res >> l, 1)
            m = 6 * rl * rl * 4
            out.append(self.spec[off:off + m].view(6, rl, rl, 4)[..., :3])
            off += m
        return out


class DeviceScene:
    """Splats + packed atlas + shading tables resident on one device."""

    def __init__(self, means, quats, scales, opac, textures, env=None, env_levels=1,
                 device="cuda", perm=None, tables=None, locality=False, sh=None, sh_degree=0,
                 tex_format=0, mips=False, chart_log2=None):
        """Atlas variants: tex_format 1 stores 7-float texels (two-component normals); mips
        builds each chart's box-filtered chain and renders with trilinear sampling;
        chart_log2 [n] gives per-splat texture sides 2^l, textures then being the level-0
        texels of all splats back to back ([sum 4^l, 8], splat order)."""
        self.device = torch.device(device)
        self.tex_format, self.mips = int(tex_format), bool(mips)
        self.chart_table, self.atlas_texels = None, 0
        self.max_log2 = 0       # largest log2 chart side
        # indirect light: [n, (degree+1)^2, 3] SH coefficients per splat, or None
        self.sh = None if sh is None else _dev(sh, device, torch.float32)
        self.sh_degree = int(sh_degree)
        self.means = _dev(means, device, torch.float32)
        self.quats = _dev(quats, device, torch.float32)
        self.scales = _dev(scales, device, torch.float32)
        self.opac = _dev(opac, device, torch.float32)
        self.n = int(self.means.shape[0])
        if chart_log2 is not None:
            self._adaptive_atlas(np.asarray(textures, np.float32), np.asarray(chart_log2))
        else:
            tex = _dev(textures, device, torch.float32)
            self.tex_res = int(tex.shape[1])
            self.max_log2 = max(self.tex_res.bit_length() - 1, 0)
            T, C = self.tex_res, (7 if self.tex_format else 8)
            chart = (4 * T * T - 1) // 3 if self.mips else T * T
            self.atlas = (torch.empty_like(tex) if not (self.tex_format or self.mips) else
                          torch.empty(max(self.n, 1) * chart * C, device=device,
                                      dtype=torch.float32))
            self.chart_of = torch.empty(self.n, device=device, dtype=torch.int32)
            permt = None if perm is None else _dev(np.asarray(perm, np.int32), device, torch.int32)
            if locality and perm is None and self.n:
                # charts in Morton order of the centres: neighbouring splats share cache lines
                permt = torch.empty(self.n, device=device, dtype=torch.int32)
                F.ts_locality_perm(self.means, self.n, permt)
            if self.n:
                if self.tex_format or self.mips:
                    F.ts_atlas_pack2(tex, self.n, T, permt, self.tex_format, self.mips,
                                     self.atlas, self.chart_of)
                else:
                    F.ts_atlas_pack(tex, self.n, T, permt, self.atlas, self.chart_of)
            del tex
        if tables is not None:
            self.tables = tables
        elif env is not None:
            self.tables = EnvTables(env, env_levels, device)
        else:
            self.tables = None

    def _adaptive_atlas(self, texels, log2):
        """Charts of per-splat sides 2^log2[k] (with their mip chains when self.mips), packed
        back to back in splat order on the GPU by ts_atlas_pack_charts; the chart table holds
        (level-0 texel offset, log2 side). Only the atlas size is worked out here."""
        n = self.n
        log2 = np.asarray(log2, np.int32)
        sides = 1 << log2.astype(np.int64)
        chain = (4 * sides * sides - 1) // 3 if self.mips else sides * sides
        total = int(chain.sum()) if n else 1
        C = 7 if self.tex_format else 8
        self.atlas = torch.zeros(max(total, 1) * C, device=self.device, dtype=torch.float32)
        self.chart_table = torch.zeros((max(n, 1), 2), device=self.device, dtype=torch.int32)
        self.atlas_texels = total
        self.chart_of = torch.arange(n, device=self.device, dtype=torch.int32)
        self.tex_res = int(sides.max()) if n else 1
        self.max_log2 = int(log2.max()) if n else 0
        if n:
            lv0 = _dev(np.asarray(texels, np.float32).reshape(-1, 8), self.device)
            ws = F.ts_atlas_pack_charts(lv0, n, _dev(log2, self.device), int(log2.max()),
                                        self.tex_format, int(self.mips), self.chart_table,
                                        self.atlas, total)
            torch.cuda.current_stream(self.device).synchronize()
            del lv0, ws

    def atlas_spec(self):
        """How the atlas is laid out (side, texel format, mip chains, chart table), for views
        of this scene's tensors such as autograd.render_rgba's."""
        return dict(tex_res=self.tex_res, tex_format=self.tex_format, mips=self.mips,
                    chart_table=self.chart_table, atlas_texels=self.atlas_texels)

    def rebuild_mips(self, stream=None):
        """Levels 1.. of every chart's chain again from its level 0 (after level 0 changed)."""
        if not self.mips:
            raise ValueError("the atlas holds no mip chains")
        F.ts_atlas_mips(self.atlas, self.n, self.tex_res, self.chart_table, self.max_log2,
                        self.atlas_texels, self.tex_format, stream)

    @classmethod
    def from_dict(cls, sc, device="cuda", **kw):
        if "sh" in sc and "sh" not in kw:
            kw = dict(kw, sh=sc["sh"], sh_degree=sc.get("sh_degree", 3))
        return cls(sc["means"], sc["quats"], sc["scales"], sc["opac"], sc["textures"],
                   sc.get("env"), sc.get("env_levels", 1), device=device, **kw)

    def bytes(self):
        b = sum(t.numel() * t.element_size() for t in
                (self.means, self.quats, self.scales, self.opac, self.atlas, self.chart_of))
        if self.tables is not None:
            b += sum(t.numel() * 4 for t in (self.tables.spec, self.tables.irr, self.tables.lut))
        if self.sh is not None:
            b += self.sh.numel() * 4
        return b


class RenderPlan:
    """All buffers for rendering `cams` (same resolution) of `scene`; run() is alloc-free."""

    def __init__(self, scene: DeviceScene, cams, width, height, params=None, shade=True,
                 gbuf=False, aux=False, pair_capacity=None, stream=None, vis=None):
        p = dict(DEFAULTS)
        if params:
            p.update(params)
        self.scene = scene
        self.W, self.H = int(width), int(height)
        self.cams = cameras_tensor(cams, scene.device)
        self.V = int(self.cams.shape[0])
        # atlas variants and the indirect term (absent on plain scene views)
        mips = getattr(scene, "mips", False)
        if mips and not (params and "sampler" in params):
            p["sampler"] = F.SAMPLER_TRILINEAR
        self.params = F.make_params(scene.tex_res, tex_format=getattr(scene, "tex_format", 0),
                                    chart_table=getattr(scene, "chart_table", None),
                                    atlas_texels=getattr(scene, "atlas_texels", 0), **p)
        self.ntx = (self.W + F.TILE - 1) // F.TILE
        self.nty = (self.H + F.TILE - 1) // F.TILE
        self.n_tiles = self.ntx * self.nty
        dev, V, n = scene.device, self.V, scene.n
        i32 = dict(device=dev, dtype=torch.int32)
        self.rec = torch.empty(V * max(n, 1) * F.REC_FLOATS, device=dev, dtype=torch.float32)
        self.rect = torch.empty(V * max(n, 1) * 4, **i32)
        self.depth_key = torch.empty(V * max(n, 1), **i32)
        ws_bytes = F.ts_workspace_size(F.TS_OP_BIN_SORT, V, n, self.W, self.H)
        self.ws = torch.empty((ws_bytes + 3) // 4, **i32)
        self.sorted_ids = torch.empty(V * max(n, 1), **i32)
        self.tile_ranges = torch.empty(V * self.n_tiles * 2, **i32)
        self.n_pairs = torch.zeros(1, device=dev, dtype=torch.int64)
        self.status = torch.zeros(1, **i32)
        self.shade = bool(shade) and scene.tables is not None
        plane = V * self.H * self.W
        self.rgba = torch.empty(plane * 4, device=dev, dtype=torch.float32) if self.shade else None
        self.gbuf = torch.empty(plane * 8, device=dev, dtype=torch.float32) if (gbuf or not self.shade) else None
        self.t_final = torch.empty(plane, device=dev, dtype=torch.float32) if (aux or gbuf or not self.shade) else None
        self.n_contrib = torch.empty(plane, **i32) if aux else None
        self.n_blend = torch.empty(plane, **i32) if aux else None
        # indirect term (on when the scene carries SH coefficients)
        self.indirect = getattr(scene, "sh", None) is not None
        self.lind = (torch.empty(V * max(n, 1) * 4, device=dev, dtype=torch.float32)
                     if self.indirect else None)
        self.gbuf_ind = (torch.empty(plane * 3, device=dev, dtype=torch.float32)
                         if self.indirect and self.gbuf is not None else None)
        if vis is not None and not (self.indirect and self.shade):
            raise ValueError("visibility needs a scene with indirect SH and shading")
        self.vis = None if vis is None else _dev(vis, dev, torch.float32).reshape(-1)
        if self.vis is not None and self.vis.numel() != plane:
            raise ValueError(f"visibility has {self.vis.numel()} values for {plane} pixels")
        self.stream = stream
        if pair_capacity is None:
            self.pair_ids = torch.empty(1, **i32)
            self.cap = 0
            self._front()
            torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
            need = int(self.n_pairs.item())
            pair_capacity = need + need // 8 + 4096
        self.cap = int(pair_capacity)
        self.pair_ids = torch.empty(max(self.cap, 1), **i32)

    def preprocess(self):
        sc = self.scene
        F.ts_preprocess(self.V, self.W, self.H, self.cams, self.params, sc.n, sc.means, sc.quats,
                        sc.scales, sc.opac, sc.chart_of, self.rec, self.rect, self.depth_key,
                        self.stream)

    def bin_sort(self):
        F.ts_bin_sort(self.V, self.W, self.H, self.scene.n, self.rect, self.depth_key, self.ws,
                      self.cap, self.sorted_ids, self.tile_ranges, self.pair_ids, self.n_pairs,
                      self.status, self.stream)

    def indirect_eval(self):
        sc = self.scene
        F.ts_indirect_eval(self.V, self.cams, sc.n, sc.means, sc.quats, sc.sh, sc.sh_degree,
                           self.lind, self.stream)

    def _front(self):
        self.preprocess()
        if self.indirect:
            self.indirect_eval()
        self.bin_sort()

    def raster(self):
        sc = self.scene
        env = sc.tables.struct if self.shade else None
        F.ts_raster_fwd(self.V, self.W, self.H, self.cams, self.params, sc.n, self.rec,
                        self.tile_ranges, self.pair_ids, self.cap, sc.atlas, env, self.rgba, self.gbuf,
                        self.t_final, self.n_contrib, self.n_blend, self.stream, lind=self.lind,
                        vis=self.vis, gbuf_ind=self.gbuf_ind)

    def run(self):
        """Enqueue preprocess, bin/sort and raster(+shade). No host synchronisation."""
        self._front()
        self.raster()

    def front(self):
        """Enqueue the steps before the raster (preprocess, indirect term, bin/sort)."""
        self._front()

    @staticmethod
    def bytes_for(scene, n_views, width, height, pair_capacity, shade=True, gbuf=False,
                  aux=False):
        """Device bytes a plan of these arguments allocates (visibility input not counted)."""
        V, n = int(n_views), max(scene.n, 1)
        n_tiles = ((width + F.TILE - 1) // F.TILE) * ((height + F.TILE - 1) // F.TILE)
        plane = V * width * height
        shade = bool(shade) and scene.tables is not None
        ind = getattr(scene, "sh", None) is not None
        b = V * n * (F.REC_FLOATS * 4 + 16 + 4 + 4)            # rec, rect, depth_key, sorted_ids
        b += (F.ts_workspace_size(F.TS_OP_BIN_SORT, V, scene.n, width, height) + 3) // 4 * 4
        b += V * n_tiles * 8 + max(int(pair_capacity), 1) * 4 + 8 + 4 + V * 64
        b += plane * 16 if shade else 0
        b += plane * 32 if (gbuf or not shade) else 0
        b += plane * 4 if (aux or gbuf or not shade) else 0
        b += plane * 8 if aux else 0
        b += V * n * 16 if ind else 0
        b += plane * 12 if ind and (gbuf or not shade) else 0
        return int(b)

    def batchable(self):
        """Whether the raster of this plan can join a batched launch (ts_raster_batch)."""
        p = self.params
        return (self.shade and not self.indirect and p.sampler == F.SAMPLER_BILINEAR
                and p.tex_format == F.TEX_RGBN3 and not p.chart_table)

    def raster_job(self):
        """This plan's raster + shading as a ts_raster_job for a batched launch (default atlas
        path, shaded, no indirect term)."""
        if not self.shade or self.indirect:
            raise ValueError("batched renders are shaded renders without the indirect term")
        sc = self.scene
        return F.make_raster_job(self.V, self.W, self.H, self.cams, self.params, sc.n, self.rec,
                                 self.tile_ranges, self.pair_ids, self.cap, sc.atlas,
                                 sc.tables.struct, self.rgba, self.t_final)

    def check(self):
        """Synchronise and verify the pair lists fit; returns the pair count."""
        (self.stream or torch.cuda.current_stream()).synchronize()
        if int(self.status.item()) != 0:
            raise RuntimeError(f"pair capacity {self.cap} < {int(self.n_pairs.item())}")
        return int(self.n_pairs.item())

    def outputs(self):
        V, H, W = self.V, self.H, self.W
        out = {}
        if self.rgba is not None:
            out["rgba"] = self.rgba.view(V, H, W, 4)
        if self.gbuf is not None:
            out["gbuf"] = self.gbuf.view(V, 8, H, W)
        if self.t_final is not None:
            out["t_final"] = self.t_final.view(V, H, W)
        if self.n_contrib is not None:
            out["n_contrib"] = self.n_contrib.view(V, H, W)
            out["n_blend"] = self.n_blend.view(V, H, W)
        if self.gbuf_ind is not None:
            out["gbuf_ind"] = self.gbuf_ind.view(V, 3, H, W)
        if self.lind is not None:
            out["lind"] = self.lind.view(V, -1, 4)[:, :self.scene.n]
        return out


class BatchRaster:
    """Batched persistent raster launches from a ring of job tables.

    Slot i owns a pinned host table, its device copy and a work-queue buffer; launch(i, jobs)
    encodes the jobs, copies the table to the device and renders the whole batch in one
    launch (optionally by replaying a graph captured once per slot: the launch does not depend
    on the batch). A slot may be reused once the stream has finished its previous batch."""

    def __init__(self, device="cuda", slots=2, use_graphs=True):
        nb = F.ts_raster_batch_table_bytes()
        self.device = torch.device(device)
        self.host = [torch.empty(nb, dtype=torch.uint8).pin_memory() for _ in range(slots)]
        self.table = [torch.empty(nb, dtype=torch.uint8, device=self.device) for _ in range(slots)]
        # work counters: zero before the first launch, left zero by every launch
        self.queue = [torch.zeros(16, dtype=torch.int32, device=self.device) for _ in range(slots)]
        self.graphs = [None] * slots
        if use_graphs:
            for i in range(slots):
                self.graphs[i] = self._capture(i)

    def _capture(self, i):
        # an empty batch first (a plain launch, outside any capture), then the capture
        F.ts_raster_batch_encode([], self.host[i])
        self.table[i].copy_(self.host[i])
        F.ts_raster_batch(self.table[i], self.queue[i])
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(self.device)
        with torch.cuda.stream(s):
            g.capture_begin(capture_error_mode="thread_local")
            F.ts_raster_batch(self.table[i], self.queue[i], s)
            g.capture_end()
        s.synchronize()
        return g

    def launch(self, i, jobs, stream=None):
        """Render `jobs` (ts_raster_job structs) in one launch on `stream` (current if None)."""
        F.ts_raster_batch_encode(jobs, self.host[i])
        stream = stream or torch.cuda.current_stream(self.device)
        with torch.cuda.stream(stream):
            self.table[i].copy_(self.host[i], non_blocking=True)
            if self.graphs[i] is not None:
                self.graphs[i].replay()
            else:
                F.ts_raster_batch(self.table[i], self.queue[i], stream)


def render(scene: DeviceScene, cams, width, height, params=None, shade=True, gbuf=False,
           aux=False, vis=None):
    """Render a batch of views; grows the pair capacity and re-runs if it overflowed."""
    plan = RenderPlan(scene, cams, width, height, params, shade=shade, gbuf=gbuf, aux=aux,
                      vis=vis)
    plan.run()
    (plan.stream or torch.cuda.current_stream()).synchronize()
    if int(plan.status.item()) != 0:
        plan = RenderPlan(scene, cams, width, height, params, shade=shade, gbuf=gbuf, aux=aux,
                          pair_capacity=2 * int(plan.n_pairs.item()) + 4096, vis=vis)
        plan.run()
        plan.check()
    out = plan.outputs()
    out["plan"] = plan
    return out

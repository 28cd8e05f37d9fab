"""ctypes binding of libtexsplat (argument marshalling only; all work runs in the HIP kernels).

The functions here take torch CUDA tensors and pass raw device pointers and the current
stream to the C ABI declared in include/texsplat.h. Nothing falls back to another
implementation: if the library is missing or a call fails, an exception is raised."""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtexsplat.so")

TS_OK = 0
TS_OP_BIN_SORT, TS_OP_RASTER_BWD, TS_OP_ENV_BWD, TS_OP_LOCALITY_PERM, TS_OP_ATLAS_CHARTS = 1, 2, 3, 4, 5
REC_FLOATS = 28
TILE = 16

c_int32, c_int64, c_float, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                                   ctypes.c_void_p, ctypes.c_size_t)


class TsParams(ctypes.Structure):
    _fields_ = [("s_sigma", c_float), ("alpha_min", c_float), ("alpha_max", c_float),
                ("t_min", c_float), ("near_z", c_float), ("bg", c_float * 3),
                ("tex_res", c_int32), ("sampler", c_int32), ("tex_format", c_int32),
                ("chart_table", c_void_p), ("atlas_texels", c_int64)]


class TsEnv(ctypes.Structure):
    _fields_ = [("spec", c_void_p), ("spec_res", c_int32), ("spec_levels", c_int32),
                ("irr", c_void_p), ("irr_res", c_int32), ("lut", c_void_p), ("lut_res", c_int32)]


class TsRasterJob(ctypes.Structure):
    _fields_ = [("n_views", c_int32), ("width", c_int32), ("height", c_int32), ("n", c_int32),
                ("cams", c_void_p), ("rec", c_void_p), ("tile_ranges", c_void_p),
                ("pair_ids", c_void_p), ("pair_capacity", c_int64), ("atlas", c_void_p),
                ("params", TsParams), ("env", TsEnv), ("rgba", c_void_p), ("t_final", c_void_p)]


_SIGS = {
    "ts_workspace_size": [c_int32, c_int32, c_int32, c_int32, c_int32, c_int64,
                          ctypes.POINTER(c_size_t)],
    "ts_preprocess": [c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(TsParams), c_int32,
                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_void_p],
    "ts_bin_sort": [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                    c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_bin_sort_noalloc": [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int64,
                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_raster_fwd": [c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(TsParams), c_int32,
                      c_void_p, c_void_p, c_void_p, c_int64, c_void_p, ctypes.POINTER(TsEnv),
                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_void_p],
    "ts_shade": [c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(TsParams),
                 ctypes.POINTER(TsEnv), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                 c_void_p],
    "ts_indirect_eval": [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                         c_void_p, c_void_p],
    "ts_raster_bwd": [c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(TsParams), c_int32,
                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_int64, c_void_p, ctypes.POINTER(TsEnv), c_void_p, c_void_p,
                      c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_int64, c_void_p,
                      c_void_p, c_float, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_indirect_bwd": [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                        c_void_p, c_void_p, c_float, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_raster_bwd_workspace": [c_int32, c_int32, c_int64, ctypes.POINTER(c_size_t)],
    "ts_env_bwd": [c_int32, c_int32, c_int32, c_void_p, ctypes.POINTER(TsEnv), c_void_p, c_void_p,
                   c_void_p, c_void_p, c_void_p, c_size_t, ctypes.c_float, c_void_p, c_void_p,
                   c_void_p],
    "ts_env_bwd_workspace": [ctypes.POINTER(TsEnv), ctypes.POINTER(c_size_t)],
    "ts_brdf_lut": [c_int32, c_int32, c_void_p, c_void_p],
    "ts_env_tables": [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_atlas_pack": [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p],
    "ts_locality_perm": [c_void_p, c_int32, c_void_p, c_size_t, c_void_p, c_void_p],
    "ts_atlas_pack2": [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                       c_void_p],
    "ts_atlas_mips": [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int64, c_int32, c_void_p],
    "ts_locality_perm_workspace": [c_int32, ctypes.POINTER(c_size_t)],
    "ts_atlas_pack_charts": [c_void_p, c_int64, c_int32, c_void_p, c_int32, c_int32, c_int32,
                             c_void_p, c_size_t, c_void_p, c_void_p, c_int64, c_void_p],
    "ts_atlas_charts_workspace": [c_int32, ctypes.POINTER(c_size_t)],
    "ts_raster_batch_encode": [ctypes.POINTER(TsRasterJob), c_int32, c_void_p, c_size_t],
    "ts_raster_batch": [c_void_p, c_void_p, c_void_p],
}

_SIZE_FNS = ("ts_bin_sort_noalloc_max_bytes", "ts_raster_batch_table_bytes")
EXPORTS = tuple(_SIGS) + ("ts_last_error",) + _SIZE_FNS

_lib = None


def lib():
    """Load libtexsplat.so (built in-tree by __graft_entry__.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"texsplat HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int32
        L.ts_last_error.restype = ctypes.c_char_p
        L.ts_last_error.argtypes = []
        for name in _SIZE_FNS:
            getattr(L, name).restype = c_size_t
            getattr(L, name).argtypes = []
        _lib = L
    return _lib


def _check(rc, name):
    if rc != TS_OK:
        msg = lib().ts_last_error().decode()
        raise RuntimeError(f"{name} failed ({rc}): {msg}")


def ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


SAMPLER_BILINEAR, SAMPLER_CONSTANT, SAMPLER_HARDWARE, SAMPLER_TRILINEAR = 0, 1, 2, 3
TEX_RGBN3, TEX_RGBN2 = 0, 1


def make_params(tex_res, s_sigma=3.0, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4,
                near_z=0.2, bg=(0.0, 0.0, 0.0), sampler=SAMPLER_BILINEAR, tex_format=0,
                chart_table=None, atlas_texels=0):
    """chart_table: device int32 tensor [n_charts, 2] or None (kept alive by the caller)."""
    p = TsParams()
    p.s_sigma, p.alpha_min, p.alpha_max, p.t_min, p.near_z = s_sigma, alpha_min, alpha_max, t_min, near_z
    for i in range(3):
        p.bg[i] = bg[i]
    p.tex_res = int(tex_res)
    p.sampler = int(sampler)
    p.tex_format = int(tex_format)
    p.chart_table = None if chart_table is None else ptr(chart_table)
    p.atlas_texels = int(atlas_texels)
    return p


def make_env(spec, spec_res, levels, irr, irr_res, lut, lut_res):
    e = TsEnv()
    e.spec, e.spec_res, e.spec_levels = spec.data_ptr(), spec_res, levels
    e.irr, e.irr_res = irr.data_ptr(), irr_res
    e.lut, e.lut_res = lut.data_ptr(), lut_res
    return e


# --------------------------------------------------------------------------------------
# one wrapper per C entry point, same names
# --------------------------------------------------------------------------------------

def ts_workspace_size(op, n_views, n, width, height, pair_capacity=0):
    out = c_size_t(0)
    _check(lib().ts_workspace_size(op, n_views, n, width, height, pair_capacity,
                                   ctypes.byref(out)),
           "ts_workspace_size")
    return int(out.value)


def ts_preprocess(n_views, width, height, cams, params, n, means, quats, scales, opac, chart_of,
                  rec, rect, depth_key, stream=None):
    _check(lib().ts_preprocess(n_views, width, height, ptr(cams), ctypes.byref(params), n,
                               ptr(means), ptr(quats), ptr(scales), ptr(opac), ptr(chart_of),
                               ptr(rec), ptr(rect), ptr(depth_key), stream_handle(stream)),
           "ts_preprocess")


def ts_bin_sort(n_views, width, height, n, rect, depth_key, ws, pair_capacity, sorted_ids,
                tile_ranges, pair_ids, n_pairs, status, stream=None):
    _check(lib().ts_bin_sort(n_views, width, height, n, ptr(rect), ptr(depth_key), ptr(ws),
                             ws.numel() * ws.element_size(), pair_capacity, ptr(sorted_ids),
                             ptr(tile_ranges), ptr(pair_ids), ptr(n_pairs), ptr(status),
                             stream_handle(stream)), "ts_bin_sort")


def ts_bin_sort_noalloc(n_views, width, height, n, rect, depth_key, pair_capacity, sorted_ids,
                        tile_ranges, pair_ids, n_pairs, status, stream=None):
    _check(lib().ts_bin_sort_noalloc(n_views, width, height, n, ptr(rect), ptr(depth_key),
                                     pair_capacity, ptr(sorted_ids), ptr(tile_ranges),
                                     ptr(pair_ids), ptr(n_pairs), ptr(status),
                                     stream_handle(stream)), "ts_bin_sort_noalloc")


def ts_bin_sort_noalloc_max_bytes():
    return int(lib().ts_bin_sort_noalloc_max_bytes())


def ts_atlas_pack_charts(texels, n, log2_side, max_log2, tex_format, mips, chart_table, atlas,
                         atlas_texels, stream=None):
    """texels: device [n_texels, 8] level-0 texels of all primitives back to back."""
    out = c_size_t(0)
    _check(lib().ts_atlas_charts_workspace(n, ctypes.byref(out)), "ts_atlas_charts_workspace")
    ws = torch.empty(max(int(out.value), 8), dtype=torch.uint8, device=atlas.device)
    _check(lib().ts_atlas_pack_charts(ptr(texels), texels.shape[0], n, ptr(log2_side), max_log2,
                                      tex_format, mips, ptr(ws), ws.numel(), ptr(chart_table),
                                      ptr(atlas), atlas_texels, stream_handle(stream)),
           "ts_atlas_pack_charts")
    return ws


def ts_raster_batch_table_bytes():
    return int(lib().ts_raster_batch_table_bytes())


def make_raster_job(n_views, width, height, cams, params, n, rec, tile_ranges, pair_ids,
                    pair_capacity, atlas, env, rgba, t_final=None):
    """A ts_raster_job of device tensors (the caller keeps them alive while the job is used)."""
    j = TsRasterJob()
    j.n_views, j.width, j.height, j.n = int(n_views), int(width), int(height), int(n)
    j.cams, j.rec, j.tile_ranges = ptr(cams), ptr(rec), ptr(tile_ranges)
    j.pair_ids, j.pair_capacity, j.atlas = ptr(pair_ids), int(pair_capacity), ptr(atlas)
    j.params, j.env = params, env
    j.rgba, j.t_final = ptr(rgba), ptr(t_final)
    return j


def ts_raster_batch_encode(jobs, table):
    """Encode a list of TsRasterJob into `table` (a host uint8 tensor, e.g. pinned)."""
    arr = (TsRasterJob * max(len(jobs), 1))(*jobs)
    if table.is_cuda or not table.is_contiguous():
        raise ValueError("the batch table is encoded in contiguous host memory")
    _check(lib().ts_raster_batch_encode(arr, len(jobs), ctypes.c_void_p(table.data_ptr()),
                                        table.numel() * table.element_size()),
           "ts_raster_batch_encode")


def ts_raster_batch(table, queue, stream=None):
    _check(lib().ts_raster_batch(ptr(table), ptr(queue), stream_handle(stream)),
           "ts_raster_batch")


def ts_raster_fwd(n_views, width, height, cams, params, n, rec, tile_ranges, pair_ids,
                  pair_capacity, atlas, env, rgba, gbuf, t_final, n_contrib, n_blend=None,
                  stream=None, lind=None, vis=None, gbuf_ind=None):
    _check(lib().ts_raster_fwd(n_views, width, height, ptr(cams), ctypes.byref(params), n,
                               ptr(rec), ptr(tile_ranges), ptr(pair_ids), pair_capacity, ptr(atlas),
                               ctypes.byref(env) if env is not None else None, ptr(rgba),
                               ptr(gbuf), ptr(t_final), ptr(n_contrib), ptr(n_blend), ptr(lind),
                               ptr(vis), ptr(gbuf_ind), stream_handle(stream)),
           "ts_raster_fwd")


def ts_indirect_eval(n_views, cams, n, means, quats, sh, sh_degree, lind, stream=None):
    _check(lib().ts_indirect_eval(n_views, ptr(cams), n, ptr(means), ptr(quats), ptr(sh),
                                  int(sh_degree), ptr(lind), stream_handle(stream)),
           "ts_indirect_eval")


def ts_env_bwd_workspace(env):
    out = c_size_t(0)
    _check(lib().ts_env_bwd_workspace(ctypes.byref(env), ctypes.byref(out)),
           "ts_env_bwd_workspace")
    return out.value


def ts_env_bwd(n_views, width, height, cams, env, gbuf, t_final, d_rgba, ws, beta, d_irr, d_spec,
               stream=None, vis=None):
    _check(lib().ts_env_bwd(n_views, width, height, ptr(cams), ctypes.byref(env), ptr(gbuf),
                            ptr(t_final), ptr(d_rgba), ptr(vis), ptr(ws),
                            ws.numel() * ws.element_size(),
                            float(beta), ptr(d_irr), ptr(d_spec), stream_handle(stream)),
           "ts_env_bwd")


def ts_raster_bwd_workspace(n_views, n, pair_capacity):
    out = c_size_t(0)
    _check(lib().ts_raster_bwd_workspace(n_views, n, pair_capacity, ctypes.byref(out)),
           "ts_raster_bwd_workspace")
    return int(out.value)


def ts_raster_bwd(n_views, width, height, cams, params, n, means, quats, scales, chart_of, rec,
                  rect, tile_ranges, pair_ids, pair_capacity, atlas, env, gbuf, t_final,
                  n_contrib, d_rgba, ws, partials, status, partial_used, beta, d_means, d_quats,
                  d_scales, d_opac, d_atlas, stream=None, lind=None, vis=None, gbuf_ind=None,
                  d_lind=None):
    _check(lib().ts_raster_bwd(n_views, width, height, ptr(cams), ctypes.byref(params), n,
                               ptr(means), ptr(quats), ptr(scales), ptr(chart_of), ptr(rec),
                               ptr(rect), ptr(tile_ranges), ptr(pair_ids), pair_capacity,
                               ptr(atlas), ctypes.byref(env), ptr(gbuf), ptr(t_final),
                               ptr(n_contrib), ptr(d_rgba), ptr(ws), ws.numel() * ws.element_size(),
                               ptr(partials), partials.numel(), ptr(status), ptr(partial_used),
                               float(beta),
                               ptr(d_means), ptr(d_quats), ptr(d_scales), ptr(d_opac),
                               ptr(d_atlas), ptr(lind), ptr(vis), ptr(gbuf_ind), ptr(d_lind),
                               stream_handle(stream)), "ts_raster_bwd")


def ts_indirect_bwd(n_views, cams, n, means, quats, sh, sh_degree, lind, d_lind, beta, d_sh,
                    d_means, d_quats, stream=None):
    _check(lib().ts_indirect_bwd(n_views, ptr(cams), n, ptr(means), ptr(quats), ptr(sh),
                                 int(sh_degree), ptr(lind), ptr(d_lind), float(beta), ptr(d_sh),
                                 ptr(d_means), ptr(d_quats), stream_handle(stream)),
           "ts_indirect_bwd")


def ts_shade(n_views, width, height, cams, params, env, gbuf, t_final, rgba, stream=None,
             gbuf_ind=None, vis=None):
    _check(lib().ts_shade(n_views, width, height, ptr(cams), ctypes.byref(params),
                          ctypes.byref(env), ptr(gbuf), ptr(t_final), ptr(rgba), ptr(gbuf_ind),
                          ptr(vis), stream_handle(stream)), "ts_shade")


def ts_brdf_lut(n, samples, lut, stream=None):
    _check(lib().ts_brdf_lut(n, samples, ptr(lut), stream_handle(stream)), "ts_brdf_lut")


def ts_env_tables(env, r, levels, irr_res, spec, irr, texel_ws, stream=None):
    _check(lib().ts_env_tables(ptr(env), r, levels, irr_res, ptr(spec), ptr(irr), ptr(texel_ws),
                               stream_handle(stream)), "ts_env_tables")


def ts_atlas_pack(textures, n, tex_res, perm, atlas, chart_of, stream=None):
    _check(lib().ts_atlas_pack(ptr(textures), n, tex_res, ptr(perm), ptr(atlas), ptr(chart_of),
                               stream_handle(stream)), "ts_atlas_pack")


def ts_locality_perm(means, n, perm, stream=None):
    nb = c_size_t(0)
    _check(lib().ts_locality_perm_workspace(n, ctypes.byref(nb)), "ts_locality_perm_workspace")
    ws = torch.empty(max(int(nb.value), 1), device=means.device, dtype=torch.uint8)
    _check(lib().ts_locality_perm(ptr(means), n, ptr(ws), ws.numel(), ptr(perm),
                                  stream_handle(stream)), "ts_locality_perm")


def ts_atlas_pack2(textures, n, tex_res, perm, tex_format, mips, atlas, chart_of, stream=None):
    _check(lib().ts_atlas_pack2(ptr(textures), n, tex_res, ptr(perm), int(tex_format), int(mips),
                                ptr(atlas), ptr(chart_of), stream_handle(stream)),
           "ts_atlas_pack2")


def ts_atlas_mips(atlas, n_charts, tex_res, chart_table, max_log2, atlas_texels, tex_format,
                  stream=None):
    _check(lib().ts_atlas_mips(ptr(atlas), n_charts, tex_res, ptr(chart_table), int(max_log2),
                               int(atlas_texels), int(tex_format), stream_handle(stream)),
           "ts_atlas_mips")

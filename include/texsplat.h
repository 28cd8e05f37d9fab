/*
 * texsplat — C ABI of a gfx950 renderer for textured planar (2D) Gaussian splats.
 *
 * What is computed (TextureSplat, arXiv 2506.13348):
 *   each splat k is a planar Gaussian P(u,v) = p_k + s_u t_u u + s_v t_v v       (Sec. 3.1, Eq. 1)
 *   a pixel's ray meets the plane at the local (u,v) in closed form             (Sec. 3.1-3.2)
 *   alpha = min(alpha_max, o_k G(u,v)), G = exp(-(u^2+v^2)/2)                     (Eq. 2, Sec. 3.1)
 *   material texels T_k, sampled bilinearly at s = (u+S)/(2S), t = (v+S)/(2S)    (Eq. 4-6)
 *   tangent normals rotated to world space, n = R_k n^t                           (Eq. 7)
 *   G-buffers X = sum_i x_i alpha_i prod_{j<i}(1 - alpha_j) over the depth order  (Eq. 8-9)
 *   deferred split-sum shading L_o = L_d + L_s against an environment cubemap    (Eq. 10-12)
 *   per-primitive textures packed into one atlas addressed through an indirection
 *   buffer prim -> chart                                                          (Sec. 3.4, Supp. Sec. 1)
 *
 * Conventions shared by every call
 *   - Array pointers are DEVICE pointers owned by the caller, C-contiguous, float32 unless
 *     noted. Camera and parameter structs marked "host" are read on the host.
 *   - Every call is ordered on `stream`, never synchronises the host and never allocates:
 *     scratch memory comes in through `ws`/`ws_bytes` (size it with ts_workspace_size).
 *   - Return value: TS_OK (0) or a negative TS_E_* code. On a negative return nothing was
 *     enqueued (argument errors) or a launch failed (TS_E_LAUNCH; the stream state is then the
 *     caller's to inspect); ts_last_error() gives a message. Conditions found on the device
 *     (pair-list overflow) go to a device status word instead, so no call needs a host sync.
 *   - Calls hold no global mutable state and may run concurrently on different streams with
 *     distinct output and workspace buffers.
 *   - Screen tiles are 16x16 pixels, row-major; n_tiles = ceil(W/16) * ceil(H/16).
 *   - A batch of n_views cameras of one resolution is processed per call; per-view arrays
 *     are laid out view-major ([V][...]).
 */
#ifndef TEXSPLAT_H
#define TEXSPLAT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TS_OK 0
#define TS_E_ARG (-1)        /* null pointer, negative or inconsistent size, unsupported T  */
#define TS_E_WORKSPACE (-2)  /* workspace smaller than ts_workspace_size reports            */
#define TS_E_LAUNCH (-3)     /* a kernel launch failed (hipGetLastError)                    */
#define TS_E_UNSUPPORTED (-4)/* feature not available on this device                        */

#define TS_TILE 16
#define TS_REC_FLOATS 28     /* floats per projected-splat record                          */

/* Pinhole camera, one per view (device array of these for the batched calls).
   w2c: row-major [R|t] world -> camera, camera axes x right, y down, z forward.
   A pixel (x,y) has its centre at (x+1/2, y+1/2); its camera ray is
   ((x+1/2-cx)/fx, (y+1/2-cy)/fy, 1). */
typedef struct ts_camera {
    float w2c[12];
    float fx, fy, cx, cy;
} ts_camera;

/* Rendering constants (host struct). Defaults in brackets. */
typedef struct ts_params {
    float s_sigma;    /* S: kernel support max(|u|,|v|) <= S, texture span [-S,S]^2 [3]    */
    float alpha_min;  /* splats with alpha below this are skipped                 [1/255] */
    float alpha_max;  /* alpha is clamped to this                                   [0.99] */
    float t_min;      /* blending stops before a splat that takes T below this      [1e-4] */
    float near_z;     /* splats with camera depth <= near_z are dropped              [0.2] */
    float bg[3];      /* background radiance of empty pixels                           [0] */
    int32_t tex_res;  /* T: texels per side of each primitive's texture, 1..32        [8] */
    int32_t sampler;  /* TS_SAMPLER_*                                          [BILINEAR] */
    int32_t tex_format;          /* TS_TEX_*: texel layout of the atlas           [RGBN3] */
    const int32_t* chart_table;  /* device [n_charts][2]: texel offset of the chart's level 0
                                    and log2 of its side (0..5), for atlases of per-chart
                                    resolutions (Sec. 5, adaptive allocation); NULL: every
                                    chart is tex_res a side, chart c at texel c * (texels of
                                    one chart with its mip chain if any)           [NULL] */
    int64_t atlas_texels;        /* texels in the atlas (bounds every chart-table entry; a
                                    chart reaching past it samples as 0); read only with
                                    chart_table                                       [0] */
} ts_params;

/* Texel layouts (ts_params.tex_format). A chart holds its texels row-major, level 0 first;
   with TS_SAMPLER_TRILINEAR its box-filtered levels 1..log2(T) follow (level l is
   (T>>l)^2 texels, level l at texel offset 4 (T^2 - (T>>l)^2) / 3 of the chart). */
#define TS_TEX_RGBN3 0   /* 8 floats: albedo rgb, roughness, tangent normal xyz, metallic    */
#define TS_TEX_RGBN2 1   /* 7 floats: albedo rgb, roughness, tangent normal xy, metallic;
                            n_z = sqrt(max(0, 1 - n_x^2 - n_y^2)) rebuilt after filtering
                            (the paper's memory encoding, Sec. 3.5.1)                       */

/* Texture sampling of ts_raster_fwd / ts_raster_bwd (ts_params.sampler). */
#define TS_SAMPLER_BILINEAR 0   /* software bilinear on the packed atlas (Eq. 5-6)             */
#define TS_SAMPLER_CONSTANT 1   /* untextured primitives: one attribute per splat (T must be 1),
                                   the baseline the paper's Tab. 3 compares against            */
#define TS_SAMPLER_HARDWARE 2   /* texture-unit bilinear on an image atlas (Supp. Sec. 1 Eq.
                                   S1-S2); the gfx950 toolchain offers no image/texture
                                   instructions, so this returns TS_E_UNSUPPORTED              */
#define TS_SAMPLER_TRILINEAR 3  /* mipmapping (Sec. 5): level lambda = log2(T rho), rho the
                                   larger of the pixel's two texture-space steps (the
                                   derivatives of (s,t) along the image axes from the closed-
                                   form (u,v)); lambda <= 0: level-0 bilinear, else bilinear on
                                   levels floor(lambda) and floor(lambda)+1 blended by the
                                   fraction, the last level alone beyond it. The atlas holds
                                   each chart's mip chain (ts_atlas_pack2 / ts_atlas_mips)     */

/* Shading tables (device pointers, produced by ts_env_tables / ts_brdf_lut). */
typedef struct ts_env {
    const float* spec;     /* specular levels back to back, level l is [6][r_l][r_l][4],
                              r_l = max(spec_res >> l, 1), rgb + pad; faces +X,-X,+Y,-Y,+Z,-Z,
                              texel [face][row][col]                                       */
    int32_t spec_res;
    int32_t spec_levels;   /* L >= 1: level l prefiltered at roughness l/(L-1)              */
    const float* irr;      /* diffuse irradiance cube [6][irr_res][irr_res][4]              */
    int32_t irr_res;
    const float* lut;      /* split-sum BRDF table [lut_res][lut_res][2]: (A,B), column =
                              N.V, row = roughness, texel centres at (i+1/2)/lut_res        */
    int32_t lut_res;
} ts_env;

/* Workspace sizing (host only): the scratch bytes of one call, written to *bytes.
     TS_OP_BIN_SORT       ts_bin_sort          (n_views, n, width, height)
     TS_OP_RASTER_BWD     ts_raster_bwd        (n_views, n, pair_capacity)
     TS_OP_ENV_BWD        ts_env_bwd           (n = texels of the environment's tables:
                                                6 irr_res^2 + 6 r_l^2 over the specular levels)
     TS_OP_LOCALITY_PERM  ts_locality_perm     (n)
     TS_OP_ATLAS_CHARTS   ts_atlas_pack_charts (n)
   Arguments an op does not use are ignored. The per-op functions below give the same sizes.
   Errors: TS_E_ARG (unknown op, null bytes, negative sizes, n_views < 1 or width/height < 1
   where the op uses them, n < 1 for TS_OP_ENV_BWD). */
#define TS_OP_BIN_SORT 1
#define TS_OP_RASTER_BWD 2
#define TS_OP_ENV_BWD 3
#define TS_OP_LOCALITY_PERM 4
#define TS_OP_ATLAS_CHARTS 5
int ts_workspace_size(int32_t op, int32_t n_views, int32_t n, int32_t width, int32_t height,
                      int64_t pair_capacity, size_t* bytes);

/*
 * ts_preprocess — per view and per splat: camera-space frame, depth, facing sign, the
 * closed-form ray-splat transform used per pixel, and a conservative screen bound.
 * (Sec. 3.1 Eq. 1-2: the pixel's (u,v) is where its ray meets the splat's plane.)
 *
 *   cams      [n_views] ts_camera (device)
 *   means     [n,3]  splat centres p_k
 *   quats     [n,4]  rotations (w,x,y,z), any non-zero length (normalised here); the
 *                    rotation's columns are t_u, t_v and n = t_u x t_v
 *   scales    [n,2]  (s_u, s_v), linear, > 0
 *   opac      [n]    o_k in (0,1]
 *   chart_of  [n]    int32 atlas chart of each primitive (Supp. Sec. 1 indirection buffer)
 *   rec       [n_views][n][TS_REC_FLOATS] out: projected records read by the rasteriser
 *   rect      [n_views][n][4] int32 out: tile rectangle [x0,x1) x [y0,y1); empty if the
 *                    splat cannot contribute to any pixel (behind the near plane, off screen,
 *                    o < alpha_min)
 *   depth_key [n_views][n] uint32 out: bits of the camera depth rounded to float32
 *                    (positive floats sort like their bits); 0xFFFFFFFF for dropped splats
 * Errors: TS_E_ARG for null pointers, n < 0, n_views < 1, width/height < 1.
 */
int ts_preprocess(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                  const ts_params* params, int32_t n, const float* means, const float* quats,
                  const float* scales, const float* opac, const int32_t* chart_of,
                  float* rec, int32_t* rect, uint32_t* depth_key, hipStream_t stream);

/*
 * ts_bin_sort — the per-view global depth order and per-tile splat lists.
 * Splats are radix-sorted per view by depth_key (stable, so equal keys keep index order),
 * then every tile's list holds the splats whose rect covers it, in that depth order
 * (the global sort the paper's rasteriser inherits from 2DGS, Supp. Sec. 3).
 *
 *   rect, depth_key  outputs of ts_preprocess for the same views
 *   ws, ws_bytes     scratch, at least ts_workspace_size(TS_OP_BIN_SORT, ...) bytes
 *   pair_capacity    length of pair_ids
 *   sorted_ids   [n_views][n] int32 out: splat indices in (depth, index) order per view
 *   tile_ranges  [n_views][n_tiles][2] int32 out: [start, end) of each tile's list in
 *                pair_ids (global offsets; view v's lists follow view v-1's)
 *   pair_ids     [pair_capacity] int32 out: splat indices of all tile lists
 *   n_pairs      [1] int64 out: total list length (also when it exceeds the capacity)
 *   status       [1] int32 out: 0 ok, 1 = n_pairs > pair_capacity (lists truncated:
 *                re-run with a larger capacity before rasterising)
 * Errors: TS_E_ARG, TS_E_WORKSPACE, TS_E_LAUNCH.
 */
int ts_bin_sort(int32_t n_views, int32_t width, int32_t height, int32_t n,
                const int32_t* rect, const uint32_t* depth_key, void* ws, size_t ws_bytes,
                int64_t pair_capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                int32_t* pair_ids, int64_t* n_pairs, int32_t* status, hipStream_t stream);

/*
 * ts_bin_sort_noalloc — ts_bin_sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels
 * and outputs, with the scratch taken from a static device array of the library instead of a
 * workspace argument. Arguments as ts_bin_sort without ws/ws_bytes; inputs and outputs are
 * still the caller's.
 *   - Allocates nothing (no hipMalloc/hipFree, no allocating library call). The array is
 *     ts_bin_sort_noalloc_max_bytes() = 128 MiB per GPU, held from the library's load until
 *     the process ends; its device address is looked up on the first call on each device.
 *   - A call whose scratch (ts_workspace_size(TS_OP_BIN_SORT, ...)) exceeds that size returns
 *     TS_E_WORKSPACE and enqueues nothing.
 *   - Every call on one GPU shares that GPU's array: calls that overlap on one GPU (concurrent
 *     streams, or host threads) race and must be serialised by the caller. Each call writes
 *     every scratch word it reads before reading it, so no clearing is needed between calls.
 * Errors: TS_E_ARG (as ts_bin_sort), TS_E_WORKSPACE (scratch above the maximum), TS_E_LAUNCH
 *         (no current device, symbol lookup or launch failure).
 */
int ts_bin_sort_noalloc(int32_t n_views, int32_t width, int32_t height, int32_t n,
                        const int32_t* rect, const uint32_t* depth_key, int64_t pair_capacity,
                        int32_t* sorted_ids, int32_t* tile_ranges, int32_t* pair_ids,
                        int64_t* n_pairs, int32_t* status, hipStream_t stream);
size_t ts_bin_sort_noalloc_max_bytes(void);

/*
 * ts_indirect_eval — per (view, splat) indirect radiance l_ind from per-splat spherical
 * harmonics (Sec. 3.5-3.6: indirect light encoded per primitive with SH, blended by Eq. 9
 * and mixed into the specular term by Eq. 12). With d the unit direction from camera v's
 * centre to the splat centre and n the splat normal (third column of R(q)), the direction is
 * the mirror reflection w_r = d - 2 (d.n) n, and per channel
 *   l_ind = max(0, sum_j sh[k][j][c] Y_j(w_r)),
 * Y_j the real orthonormal SH basis without the Condon-Shortley phase, index j = l*l + l + m:
 * Y_00 = 1/(2 sqrt(pi)), (Y_1-1, Y_10, Y_11) = sqrt(3/(4 pi)) (y, z, x), and so on to l = 3.
 * Evaluated in float32 (within about 2e-6 of sum_j |c_j| of the exact value).
 *
 *   cams      [n_views] cameras (host or device memory readable by the kernel: device)
 *   means, quats   as given to ts_preprocess
 *   sh        [n][(sh_degree+1)^2][3] float32 coefficients, device
 *   sh_degree 0..3
 *   lind      [n_views][n][4] out (rgb, 0), device; input of ts_raster_fwd
 * A splat with a zero quaternion gets l_ind = 0.
 * Errors: TS_E_ARG (degree outside 0..3, null pointers, n_views * n above 2^31-1),
 *         TS_E_LAUNCH.
 */
int ts_indirect_eval(int32_t n_views, const ts_camera* cams, int32_t n, const float* means,
                     const float* quats, const float* sh, int32_t sh_degree, float* lind,
                     hipStream_t stream);

/*
 * ts_raster_fwd — per pixel, front-to-back over its tile's list: (u,v) -> G -> alpha ->
 * bilinear texel fetch from the atlas -> normal mapping -> G-buffer blend (Eq. 2-9), with
 * the split-sum shading of Eq. 10-12 fused into the epilogue when env != NULL.
 * With lind != NULL the indirect term is on: each blended splat also adds w l_ind to a
 * blended indirect map L_ind (Eq. 9), and the fused shading takes the specular radiance as
 * V Lspec + (1 - V) L_ind (Eq. 12).
 *
 *   n       splats per view (rec is [n_views][n][TS_REC_FLOATS])
 *   rec, tile_ranges, pair_ids   from ts_preprocess / ts_bin_sort
 *   pair_capacity  length of pair_ids; list entries at or beyond it are never read (after
 *           an overflow reported by ts_bin_sort the image is incomplete, not unsafe)
 *   atlas   [n_charts][T][T][8] texels, channels (albedo r,g,b, roughness, normal x,y,z,
 *           metallic); texel [chart][row j (t)][col i (s)]
 *   env     shading tables, or NULL to skip shading (rgba must then be NULL)
 *   rgba    [n_views][H][W][4] out or NULL: linear radiance + alpha A = 1 - T
 *   gbuf    [n_views][8][H][W] out or NULL: blended albedo(3), metallic, roughness,
 *           normal(3), planar
 *   t_final [n_views][H][W] out or NULL: final transmittance T
 *   n_contrib [n_views][H][W] int32 out or NULL: list position (within the tile's list)
 *           one past the last blended splat, 0 if none
 *   n_blend [n_views][H][W] int32 out or NULL: number of splats blended into the pixel
 *           (the contributing splat-pixel evaluations)
 *   lind    [n_views][n][4] from ts_indirect_eval, or NULL: no indirect term (then vis and
 *           gbuf_ind must be NULL)
 *   vis     [n_views][H][W] visibility V in [0,1] (an input: the paper ray-traces an
 *           extracted mesh for it), or NULL: V = 1; needs rgba and env
 *   gbuf_ind [n_views][3][H][W] out or NULL: the blended L_ind map, planar
 * Errors: TS_E_ARG (null required pointer, tex_res outside 1..32, rgba without env,
 *         vis or gbuf_ind without lind, vis without rgba), TS_E_LAUNCH.
 */
int ts_raster_fwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                  const ts_params* params, int32_t n, const float* rec, const int32_t* tile_ranges,
                  const int32_t* pair_ids, int64_t pair_capacity, const float* atlas,
                  const ts_env* env,
                  float* rgba, float* gbuf, float* t_final, int32_t* n_contrib,
                  int32_t* n_blend, const float* lind, const float* vis, float* gbuf_ind,
                  hipStream_t stream);

/*
 * Batched forward renders for serving (test-time rendering from resident atlases, Sec. 3.4 and
 * Supp. Sec. 1): the ts_raster_fwd work of several jobs, each with its own scene, views,
 * resolution and outputs, in one launch of a fixed persistent grid (every compute unit's
 * resident workgroups). The (job, view, tile) work items are cut into one contiguous range
 * per XCD; workgroups take items from their XCD's queue, then from the others, until all are
 * done. Each job's output is the one ts_raster_fwd gives for the same arguments (the same
 * per-tile code). The grid does not depend on the batch, so a single captured graph of
 * ts_raster_batch serves every batch written into its table.
 *
 * A job is a shaded render on the default atlas path: sampler TS_SAMPLER_BILINEAR,
 * tex_format TS_TEX_RGBN3, no chart table, no indirect term.
 */
typedef struct ts_raster_job {
    int32_t n_views, width, height, n;   /* as ts_raster_fwd                               */
    const ts_camera* cams;               /* device [n_views]                               */
    const float* rec;                    /* device, from ts_preprocess                     */
    const int32_t* tile_ranges;          /* device, from ts_bin_sort                       */
    const int32_t* pair_ids;             /* device, from ts_bin_sort                       */
    int64_t pair_capacity;
    const float* atlas;                  /* device [n_charts][T][T][8]                     */
    ts_params params;                    /* by value (see the restriction above)           */
    ts_env env;                          /* by value: the job's shading tables (device)    */
    float* rgba;                         /* device [n_views][H][W][4] out                  */
    float* t_final;                      /* device [n_views][H][W] out, or NULL            */
} ts_raster_job;

/* Bytes of a batch table (host copy and device copy alike); it holds up to 64 jobs. */
size_t ts_raster_batch_table_bytes(void);

/*
 * ts_raster_batch_encode — host only: checks jobs[0..n_jobs) (the checks of ts_raster_fwd) and
 * writes the batch table to `table` (host memory of ts_raster_batch_table_bytes() bytes, e.g.
 * pinned, that the caller then copies to a device table). n_jobs = 0 gives an empty batch.
 * Errors: TS_E_ARG (a job's arguments, n_jobs outside 0..64, table too small, more than 2^31-1
 *         tiles), TS_E_UNSUPPORTED (a job off the default atlas path or without rgba/env).
 */
int ts_raster_batch_encode(const ts_raster_job* jobs, int32_t n_jobs, void* table,
                           size_t table_bytes);

/*
 * ts_raster_batch — renders every job of a device batch table in one persistent launch.
 *   table  device copy of a table written by ts_raster_batch_encode; read when the kernel
 *          runs, so a graph replay renders whatever the table holds at that time
 *   queue  device [16] uint32 work counters, zero before the first call (e.g. from a zeroed
 *          allocation); each launch leaves them zero for the next. Launches that share a queue
 *          must not overlap (use one queue per concurrently running launch).
 * The launch allocates nothing and never synchronises the host.
 * Errors: TS_E_ARG (null table or queue), TS_E_LAUNCH.
 */
int ts_raster_batch(const void* table, uint32_t* queue, hipStream_t stream);

/*
 * ts_shade — deferred split-sum shading of given G-buffers (Eq. 10-12): with N^ = N/|N|
 * (the view vector if |N| = 0), w_o the unit vector to the camera,
 * w_r = 2 (N^.w_o) N^ - w_o, level = clamp(R,0,1) (L-1):
 *   C = albedo/pi (1-M) E(N^) + (V Lspec(w_r, level) + (1-V) L_ind) (F0 A + B)
 *       + (1 - alpha) bg,
 *   F0 = 0.04 (1-M) + albedo M, (A,B) = lut(clamp(N^.w_o,0,1), clamp(R,0,1));
 * pixels with alpha = 0 take bg. Cube lookups pick the face by the major axis (ties X, Y,
 * Z) and filter bilinearly inside the face at texel centres with clamp-to-edge.
 *
 *   gbuf    [n_views][8][H][W] (layout of ts_raster_fwd)
 *   t_final [n_views][H][W] transmittance, alpha = 1 - T
 *   rgba    [n_views][H][W][4] out
 *   gbuf_ind [n_views][3][H][W] blended indirect map L_ind, or NULL: L_ind = 0
 *   vis     [n_views][H][W] visibility V, or NULL: V = 1
 */
int ts_shade(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
             const ts_params* params, const ts_env* env, const float* gbuf,
             const float* t_final, float* rgba, const float* gbuf_ind, const float* vis,
             hipStream_t stream);

/*
 * ts_raster_bwd — gradients of a scalar loss L of the shaded output with respect to the
 * splat parameters the paper optimises (Sec. 3.6): centres, rotations, scales, opacities and
 * texels, for the frame rendered by ts_raster_fwd with the same arguments (G-buffers,
 * t_final and n_contrib requested). Adjoint of Eq. 10-12 per pixel, then of the front-to-back
 * blend (Eq. 8) back to front from each pixel's last blended splat with T_i recovered as
 * T_{i+1}/(1-alpha_i), then of Eq. 2-7 and of the projection set-up. Gradients are w.r.t. the
 * values passed (linear scales, opacities as given, unnormalised quaternions); nothing is
 * accumulated with floating-point atomics and the result is run-to-run identical.
 *
 *   means, quats, scales, chart_of, rec, rect, tile_ranges, pair_ids, pair_capacity, atlas,
 *   env      as given to ts_preprocess / ts_bin_sort / ts_raster_fwd
 *   gbuf, t_final, n_contrib   forward outputs of the same frame
 *   d_rgba   [n_views][H][W][4] dL/d(rgb, alpha)
 *   ws       scratch, at least ts_raster_bwd_workspace(n_views, n, pair_capacity) bytes
 *   partials scratch for per-(tile entry, 8x8 block) partial sums, partial_capacity floats;
 *            if it is too small, *status is set to 2 and the gradients are incomplete
 *            (re-run with a larger buffer). A frame needs about 24 + 8 * (level-0 texels touched)
 *            floats per (entry, 8x8 block) with a blended pixel; each 8x8 block of the frame
 *            takes the buffer in chunks of 2048 floats, so up to that much more per block.
 *            At most 2^34 floats (TS_E_ARG above).
 *   status   [1] int32 device word, set to 2 on partial-buffer overflow (never cleared here);
 *            the gradient outputs are written only if it is 0 once the partials are built,
 *            so a run that overflowed can be repeated with a larger buffer for any beta
 *   partial_used [1] int64 device word or NULL: floats the frame asked for (also on overflow)
 *   beta     0: overwrite the gradient outputs; 1: add to them
 *   d_means [n,3], d_quats [n,4], d_scales [n,2], d_opac [n] out
 *   d_atlas  out, in the layout of atlas (params->tex_format, chart table, mip chains):
 *            [n_charts][T][T][8], or [n_charts][T][T][7] for TS_TEX_RGBN2 (two-component
 *            normals, Sec. 3.5.1: the rebuilt n_z's gradient goes to n_x and n_y through
 *            n_z = sqrt(1 - n_x^2 - n_y^2)); with a chart table each splat's chart at its
 *            table offset. The gradient is w.r.t. the level-0 texels: with
 *            TS_SAMPLER_TRILINEAR a level-l texel's share reaches the 2^l x 2^l level-0 texels
 *            it is the box mean of (weight 4^-l), the chain's coarser levels are written as
 *            zero gradient, and the blend fraction's gradient reaches the geometry through the
 *            level lambda = log2(T rho) (Sec. 5). Each chart belongs to one splat (as the atlas
 *            packers make it); texels of no splat's chart, and charts outside the atlas, are
 *            not written
 *   lind, vis, gbuf_ind   the indirect term of the forward (as given to / written by
 *            ts_raster_fwd), or NULL for the plain shading; with lind the shading adjoint
 *            takes the specular radiance V Lspec + (1 - V) L_ind and
 *   d_lind   [n_views][n][4] out: dL/dl_ind per (view, splat) (rgb, 0), the input of
 *            ts_indirect_bwd (written, not accumulated)
 * Errors: TS_E_ARG (also gbuf_ind or d_lind missing with lind, or given without it; the
 *         constant sampler; the forward's atlas checks), TS_E_WORKSPACE, TS_E_LAUNCH,
 *         TS_E_UNSUPPORTED (the hardware sampler).
 */
int ts_raster_bwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                  const ts_params* params, int32_t n, const float* means, const float* quats,
                  const float* scales, const int32_t* chart_of, const float* rec,
                  const int32_t* rect, const int32_t* tile_ranges, const int32_t* pair_ids,
                  int64_t pair_capacity, const float* atlas, const ts_env* env,
                  const float* gbuf, const float* t_final, const int32_t* n_contrib,
                  const float* d_rgba, void* ws, size_t ws_bytes, float* partials,
                  int64_t partial_capacity, int32_t* status, int64_t* partial_used, float beta,
                  float* d_means,
                  float* d_quats, float* d_scales, float* d_opac, float* d_atlas,
                  const float* lind, const float* vis, const float* gbuf_ind, float* d_lind,
                  hipStream_t stream);

/*
 * ts_indirect_bwd — the indirect term's share of the gradients (the SH coefficients are learned
 * end to end, Sec. 3.6): from dL/dl_ind per (view, splat) (ts_raster_bwd's d_lind) and the
 * forward's l_ind (a channel clamped at zero passes no gradient), per splat over the views in
 * order: dL/dc_j = sum_v Y_j(w_r) dL/dl_ind, and through the reflected direction
 * w_r = normalize(d - 2 (d.n) n), d = normalize(mu - o), n = R(q/|q|) e_z, to the centre and
 * the (unnormalised) quaternion. float32, one thread per splat, no atomics.
 *
 *   cams, means, quats, sh, sh_degree   as given to ts_indirect_eval
 *   lind     [n_views][n][4] the forward's ts_indirect_eval output
 *   d_lind   [n_views][n][4] from ts_raster_bwd
 *   beta     0: overwrite d_sh; 1: add to it
 *   d_sh     [n][(sh_degree+1)^2][3] out
 *   d_means [n,3], d_quats [n,4]  ADDED to (call after ts_raster_bwd, which writes them)
 * Errors: TS_E_ARG, TS_E_LAUNCH.
 */
int ts_indirect_bwd(int32_t n_views, const ts_camera* cams, int32_t n, const float* means,
                    const float* quats, const float* sh, int32_t sh_degree, const float* lind,
                    const float* d_lind, float beta, float* d_sh, float* d_means, float* d_quats,
                    hipStream_t stream);

/* Scratch bytes ts_raster_bwd needs (host only). */
int ts_raster_bwd_workspace(int32_t n_views, int32_t n, int64_t pair_capacity, size_t* bytes);

/*
 * ts_env_bwd — gradients of the same loss with respect to the texels of the environment's
 * shading tables, taken as learnable parameters (the environment is optimised end to end,
 * Sec. 3.5-3.6): the irradiance cube E of Eq. 11 and every prefiltered level of the split-sum
 * specular term of Eq. 12. The shaded colour is linear in each texel; per covered pixel the
 * irradiance lookup at N receives dL/dC * albedo (1-M)/pi and the two specular lookups at the
 * reflected direction receive dL/dC * V (F0 A + B) weighted (1-f) and f between the levels
 * around R (L-1), each spread over 4 texels by the bilinear weights (V the pixel's
 * visibility: with the indirect term the specular radiance is V L_pref + (1 - V) L_ind).
 * Empty pixels (alpha = 0, background only) contribute nothing. Summed in 64-bit fixed
 * point: each contribution x is rounded to a multiple of 2^(e+b-61), with M < 2^e the largest
 * |x| of the call and 2^b above the number of contributions (12 per pixel), so that no sum
 * leaves 2^61; the sums do not depend on the order of the additions (integer atomics), so
 * the result is run-to-run identical, within M 2^(b-61) per contribution of the exact sum.
 * A non-finite contribution makes every output texel NaN.
 *
 *   cams, env    as given to ts_raster_fwd / ts_raster_bwd
 *   gbuf, t_final  forward outputs of the same frame ([n_views][8][H][W], [n_views][H][W])
 *   d_rgba       [n_views][H][W][4] dL/d(rgb, alpha) (alpha does not reach the tables)
 *   vis          [n_views][H][W] the visibility the frame was shaded with, or NULL: V = 1
 *   ws, ws_bytes scratch, at least ts_env_bwd_workspace(env) bytes (c copies of 24 bytes
 *                per table texel, c = 16 or fewer so that they fit 64 MB but at least 1,
 *                rounded up to 256 bytes, plus 256)
 *   beta         0: overwrite the outputs; 1: add to them (any other value is TS_E_ARG)
 *   d_irr        [6][irr_res][irr_res][4] out, layout of env->irr (the 4th component is 0)
 *   d_spec       levels back to back as env->spec, [6][r_l][r_l][4] each, out
 * Errors: TS_E_ARG (null pointers, bad sizes, beta not 0 or 1, more than 2^40
 * contributions), TS_E_WORKSPACE, TS_E_LAUNCH.
 */
int ts_env_bwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
               const ts_env* env, const float* gbuf, const float* t_final, const float* d_rgba,
               const float* vis, void* ws, size_t ws_bytes, float beta, float* d_irr,
               float* d_spec, hipStream_t stream);

/* Scratch bytes ts_env_bwd needs for the tables of env (host only; reads only the
   resolutions and the level count). Errors: TS_E_ARG (null pointers, sizes < 1). */
int ts_env_bwd_workspace(const ts_env* env, size_t* bytes);

/*
 * ts_brdf_lut — the split-sum BRDF table (Sec. 3.5.4 precomputed 2D lookup; split sum of
 * Karis 2013): texel (i,j) at N.V = (i+1/2)/n, roughness r = (j+1/2)/n holds
 *   A = mean_k (1 - Fc) G_vis,  B = mean_k Fc G_vis,
 * over `samples` half vectors importance-sampled from GGX (alpha = r^2) at Hammersley
 * points (k/samples, radical_inverse_2(k)), Fc = (1 - V.H)^5,
 * G_vis = G V.H / (N.H N.V), G = Smith-Schlick with k = alpha/2; evaluated in double
 * precision and rounded to float32.
 *   lut [n][n][2] out.  Errors: TS_E_ARG for n < 1 or samples < 1.
 */
int ts_brdf_lut(int32_t n, int32_t samples, float* lut, hipStream_t stream);

/*
 * ts_env_tables — shading tables of an environment cubemap (Sec. 3.5.4 pre-integrated
 * diffuse irradiance and roughness-selected specular levels):
 *   level 0 = the environment;
 *   level l >= 1 (roughness rho = l/(L-1), alpha = rho^2, resolution r >> l):
 *     pref(w) = sum_j L_j (w.w_j)^+ D(h_j) dOmega_j / sum_j (w.w_j)^+ D(h_j) dOmega_j,
 *     h_j = normalize(w + w_j), D the GGX distribution, over all source texels j;
 *   irradiance E(n) = sum_j L_j (n.w_j)^+ dOmega_j at the irr_res texel centres;
 * with w_j the source texel centre directions and dOmega_j their exact solid angles.
 *   env     [6][r][r][3] source radiance
 *   spec    out: levels back to back, level l [6][r_l][r_l][4]
 *   irr     out: [6][irr_res][irr_res][4]
 *   texel_ws scratch of 6*r*r*32 bytes (texel directions and solid angles in double)
 * The sums run in double precision and are rounded to float32 once.
 * Errors: TS_E_ARG for null pointers, r < 1, levels < 1, irr_res < 1.
 */
int ts_env_tables(const float* env, int32_t r, int32_t levels, int32_t irr_res, float* spec,
                  float* irr, void* texel_ws, hipStream_t stream);

/*
 * ts_atlas_pack — copy per-primitive textures [n][T][T][8] into the packed atlas
 * (chart-major [n][T][T][8]) under a chart permutation: chart perm[k] receives primitive
 * k's texels and chart_of[k] = perm[k] (Supp. Sec. 1 atlas + indirection buffer).
 * perm == NULL means the identity. perm must be a permutation of 0..n-1.
 */
int ts_atlas_pack(const float* textures, int32_t n, int32_t tex_res, const int32_t* perm,
                  float* atlas, int32_t* chart_of, hipStream_t stream);

/*
 * ts_atlas_pack2 — ts_atlas_pack into a chosen texel layout: chart perm[k] receives primitive
 * k's level 0 ([n][T][T][8] input, converted to tex_format), charts at a stride of T^2
 * texels, or of the whole mip chain ((4 T^2 - 1)/3 texels) when mips != 0, in which case the
 * chain is built as by ts_atlas_mips. atlas holds n such charts (C = 8 or 7 floats a texel).
 * Errors: TS_E_ARG (null pointers, T not a power of two in 1..32, unknown format), TS_E_LAUNCH.
 */
int ts_atlas_pack2(const float* textures, int32_t n, int32_t tex_res, const int32_t* perm,
                   int32_t tex_format, int32_t mips, float* atlas, int32_t* chart_of,
                   hipStream_t stream);

/*
 * ts_atlas_mips — build levels 1..log2(T_c) of every chart in place from its level 0: texel
 * (i,j) of level l is the mean of texels (2i..2i+1, 2j..2j+1) of level l-1 (the box filter;
 * so the mean of its 2^l x 2^l level-0 block). chart_table (device [n_charts][2], as in
 * ts_params) or NULL for uniform charts of tex_res texels a side with their chains at a
 * stride of (4 T^2 - 1)/3 texels; max_log2 bounds the per-chart log2 sides (0..5);
 * atlas_texels bounds table entries (a chart past it is skipped).
 */
int ts_atlas_mips(float* atlas, int32_t n_charts, int32_t tex_res, const int32_t* chart_table,
                  int32_t max_log2, int64_t atlas_texels, int32_t tex_format, hipStream_t stream);

/*
 * ts_atlas_pack_charts — the atlas of per-chart resolutions (Sec. 5: adaptive texture
 * resolution per primitive): primitive k gets a chart of 2^log2_side[k] texels a side, the
 * charts back to back in primitive order (each followed by room for its mip chain when
 * mips != 0, which is then built as by ts_atlas_mips), and chart_table[k] = (texel offset of
 * the chart's level 0, log2 side) for ts_params.chart_table.
 *   texels     [n_texels][8] level-0 texels of all primitives back to back in primitive
 *              order (primitive k's 4^log2_side[k] texels row-major), channels as ts_atlas_pack
 *   log2_side  [n] int32 (device), clamped to 0..max_log2; max_log2 <= 5 bounds the mip passes
 *   ws         scratch of ts_atlas_charts_workspace(n) bytes
 *   chart_table [n][2] int32 out (device)
 *   atlas      out, atlas_texels texels of 8 (or 7, tex_format TS_TEX_RGBN2) floats; the caller
 *              sizes it as sum_k 4^l_k (or (4^(l_k+1) - 1)/3 with mips); charts past it, or at
 *              offsets past 2^31-1, are left out (their table entry's offset is then -1 or past
 *              atlas_texels, which the renderer samples as zero)
 * Errors: TS_E_ARG, TS_E_WORKSPACE, TS_E_LAUNCH.
 */
int ts_atlas_pack_charts(const float* texels, int64_t n_texels, int32_t n, const int32_t* log2_side,
                         int32_t max_log2, int32_t tex_format, int32_t mips, void* ws,
                         size_t ws_bytes, int32_t* chart_table, float* atlas, int64_t atlas_texels,
                         hipStream_t stream);
int ts_atlas_charts_workspace(int32_t n, size_t* bytes);

/*
 * ts_locality_perm — a chart permutation that stores the textures of nearby primitives next to
 * each other (the packing the paper leaves open, Sec. 4.4): perm[k] = rank of splat k in the
 * Morton (Z-order) sequence of its centre on a 1024^3 grid over the centres' bounding box,
 * ties by index. Pass it to ts_atlas_pack. Rendering is unchanged (a pure relabelling of
 * charts); texel fetches of neighbouring splats share cache lines and DRAM pages more often.
 *   means [n,3]; ws scratch of ts_locality_perm_workspace(n) bytes; perm [n] int32 out.
 */
int ts_locality_perm(const float* means, int32_t n, void* ws, size_t ws_bytes, int32_t* perm,
                     hipStream_t stream);
int ts_locality_perm_workspace(int32_t n, size_t* bytes);

/* Message of the last non-zero return on this thread (never NULL). */
const char* ts_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TEXSPLAT_H */

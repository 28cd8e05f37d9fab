// ts_raster_fwd / ts_shade.
//
// One 256-thread workgroup per (view, 16x16 tile); wave w covers the 8x8 quadrant
// (w&1, w>>1), one pixel per lane. The tile's list is walked front to back in batches of 256
// records staged in LDS (one record per thread, 112 B). A wave skips a splat whose pixel
// bound misses its quadrant (one scalar test) and leaves the list as soon as all 64 of its
// pixels have terminated (ballot); the workgroup stops loading batches when all 256 have.
//
// Per pixel and splat (Eq. 2-9): closed-form (u,v) from the record, square support
// max(|u|,|v|) <= S, G = exp(-(u^2+v^2)/2), alpha = min(alpha_max, o G), skip below
// alpha_min, stop before a splat taking T below t_min; then the texture (Eq. 5-6): bilinear
// on the primitive's T x T texels in the atlas at s = (u+S)/(2S), t = (v+S)/(2S), texel
// centres at (i+1/2)/T, clamp-to-edge within the chart; the tangent normal is normalised and
// rotated by sigma R (Eq. 7); the eight G-buffer channels accumulate with w = alpha T.
// With the indirect term (Eq. 9, Eq. 12) each record's l_ind (per view and splat) is staged
// beside it, a ninth to eleventh channel blends it, and the fused shading mixes the direct
// and indirect specular light by the pixel's visibility.
//
// Texture paths (template kSamp): 0 the default atlas (8-float texels, uniform charts,
// bilinear on level 0) in straight-line code; 1 one attribute per splat; 2 the atlas variants
// with bilinear sampling (two-component normals, per-chart resolutions through a chart
// table); 3 the same with trilinear sampling over each chart's mip chain, the level taken from
// the pixel's footprint on the splat (derivatives of the closed-form (u,v) along the image
// axes: du/dX = (u_x - u w_x) / den, and likewise for v and Y); 4 and 5 are 2 and 3 on the
// 7-float texels of two-component normals. The texel layout is a template argument because a
// run-time choice between the two loads around every texel fetch cost up to 43% of the step
// (per-chart sides: 32.4 against 22.6 ms).
#include <string.h>

#include <mutex>

#include "eval.h"
#include "shade.h"
#include "texture.h"
#include "ts_internal.h"

namespace ts {

struct RasterArgs {
    int V, W, H, ntx, n_tiles, T, n;
    const ts_camera* cams;
    float S, amin, amax, tmin;
    ShadeConst sc;
    EnvDev env;
    bool shade;
    const float4* rec;
    const int2* ranges;
    const int32_t* pair_ids;
    int64_t cap;
    const float4* atlas;     // [chart][T][T][2] float4
    float4* rgba;
    float* gbuf;
    float* t_final;
    int32_t* n_contrib;
    int32_t* n_blend;
    const float4* lind;      // [V][n] indirect radiance per (view, splat), kInd only
    const float* vis;        // [V][H][W] visibility or null (V = 1)
    float* gbuf_ind;         // [V][3][H][W] blended L_ind or null
    TexArgs tex;             // atlas description of the variant paths (kSamp 2, 3)
};

constexpr int kBatch = 192;   // records staged per batch (a multiple of 64)
static_assert(kBatch % kWave == 0, "the batch is walked in rows of 64");

// Waves per SIMD of the raster kernels, as measured on the 64-view headline step: the default
// path at 7 (72 VGPRs, 32 bytes of spills, a 22.5 KB record batch: seven workgroups per CU;
// 18.30 ms against 18.63 at 6); the indirect term and the atlas variants stage more per record
// (26 and 24 KB), which leaves room for six workgroups: 6 waves (the indirect term at 80 VGPRs,
// 19.33 ms against 19.40 at 5; trilinear sampling at 80 VGPRs with a few spills, 23.9 ms per
// step against 25.6 at 5 and 25.4 at 4 with 92 VGPRs).
constexpr bool samp_variant(int kSamp) { return kSamp >= 2; }
constexpr bool samp_tri(int kSamp) { return kSamp == 3 || kSamp == 5; }
constexpr int samp_fmt(int kSamp) { return kSamp >= 4 ? 1 : 0; }

// the batched launch: 6 waves per SIMD (7 measured slower there: 10.76 against 10.53 ms for
// the raster of 16 serving requests), so a grid of 6 workgroups per CU is every resident one
constexpr int kBatchWaves = 6;

template <int kSamp, bool kInd>
constexpr int raster_waves() {
    return (samp_variant(kSamp) || kInd) ? 6 : 7;
}

// A pixel's outputs: G-buffer channels, transmittance, counters and the fused shading.
template <bool kInd>
__device__ __forceinline__ void raster_outputs(const RasterArgs& a, int v, int x, int y,
                                               const float* acc, const float* ai, float Tr,
                                               int last, int nbl) {
    int64_t pix = ((int64_t)v * a.H + y) * a.W + x;
    int64_t plane = (int64_t)a.H * a.W;
    if (a.gbuf) {
        float* gb = a.gbuf + (int64_t)v * 8 * plane + (int64_t)y * a.W + x;
#pragma unroll
        for (int c = 0; c < 8; c++) gb[c * plane] = acc[c];
    }
    if (kInd && a.gbuf_ind) {
        float* gi = a.gbuf_ind + (int64_t)v * 3 * plane + (int64_t)y * a.W + x;
#pragma unroll
        for (int c = 0; c < 3; c++) gi[c * plane] = ai[c];
    }
    if (a.t_final) a.t_final[pix] = Tr;
    if (a.n_contrib) a.n_contrib[pix] = last;
    if (a.n_blend) a.n_blend[pix] = nbl;
    if (a.shade) {
        float3 d = pixel_ray(a.cams[v], (float)x + 0.5f, (float)y + 0.5f);
        float vis = (kInd && a.vis) ? a.vis[pix] : 1.0f;
        float3 C = shade_pixel<kInd>(a.env, a.sc, acc, Tr, d, ai, vis);
        a.rgba[pix] = make_float4(C.x, C.y, C.z, 1.0f - Tr);
    }
}

// Blends one texture sample t[0..7] (albedo rgb, roughness, tangent normal xyz, metallic) with
// weight ww: sigma R (t / |t|) = (sigma R t) / |t| rotates the sampled tangent normal (Eq. 7),
// scaled by ww / |t|; a zero-length sample is (0,0,1).
__device__ __forceinline__ void blend_sample(float* acc, float ww, float4 c4, float4 c5,
                                             float4 c6, float t0, float t1, float t2, float t3,
                                             float t4, float t5, float t6, float t7) {
    float nl = t4 * t4 + t5 * t5 + t6 * t6;
    bool hasn = nl > 0.f;
    float il = hasn ? __builtin_amdgcn_rsqf(nl) : 1.f;
    float tz = hasn ? t6 : 1.f;
    float wn = ww * il;
    acc[0] = fmaf(ww, t0, acc[0]);
    acc[1] = fmaf(ww, t1, acc[1]);
    acc[2] = fmaf(ww, t2, acc[2]);
    acc[3] = fmaf(ww, t7, acc[3]);   // metallic
    acc[4] = fmaf(ww, t3, acc[4]);   // roughness
    acc[5] = fmaf(wn, c4.x * t4 + c4.y * t5 + c4.z * tz, acc[5]);
    acc[6] = fmaf(wn, c4.w * t4 + c5.x * t5 + c5.y * tz, acc[6]);
    acc[7] = fmaf(wn, c5.z * t4 + c5.w * t5 + c6.x * tz, acc[7]);
}

// The whole render of tile t of view v: front-to-back walk of its list, G-buffer blend,
// outputs and the fused shading. Every thread of the workgroup calls it with the same (v, t);
// it leaves the staging arrays free (its last step is a barrier), so a workgroup can render
// several tiles in a row.
template <int kSamp, bool kInd>
__device__ __forceinline__ void raster_tile(const RasterArgs& a, int v, int t) {
    constexpr bool kTextured = kSamp != 1;
    __shared__ float4 srec[kBatch * kRec4];
    __shared__ uint32_t smask[kBatch];
    __shared__ float4 slind[kInd ? kBatch : 1];
    __shared__ int2 schart[samp_variant(kSamp) ? kBatch : 1];   // chart entries (variants)
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int bx = tx * kTile + (w & 1) * 8, by = ty * kTile + (w >> 1) * 8;
    const int x = bx + (lane & 7), y = by + (lane >> 3);
    const bool inside = x < a.W && y < a.H;
    const float X = (float)x + 0.5f, Y = (float)y + 0.5f;
    int2 range = a.ranges[(int64_t)v * a.n_tiles + t];
    // lists cut short by a capacity overflow are never read past the buffer
    range.x = (int)min((int64_t)range.x, a.cap);
    range.y = (int)min((int64_t)range.y, a.cap);
    const float4* recv = a.rec;
    const int T = a.T;
    const float tscale = (float)T / (2.0f * a.S);
    const float toff = 0.5f * (float)T - 0.5f;
    const unsigned chart4 = (unsigned)(T * T * 2);

    float Tr = 1.0f;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float ai[3] = {0.f, 0.f, 0.f};
    bool done = !inside;
    int last = 0;
    int nbl = 0;

    for (int b0 = range.x; b0 < range.y; b0 += kBatch) {
        if (__syncthreads_count(!done) == 0) break;
        int nb = min(kBatch, range.y - b0);
        uint32_t qm = 0;
        if (tid < nb) {
            int id = a.pair_ids[b0 + tid];
            const float4* src = recv + ((int64_t)v * a.n + (int64_t)id) * kRec4;
            float4 r0 = src[0], r1 = src[1], r2 = src[2], r3 = src[3];
            srec[tid * kRec4 + 0] = r0;
            srec[tid * kRec4 + 1] = r1;
            srec[tid * kRec4 + 2] = r2;
            srec[tid * kRec4 + 3] = r3;
#pragma unroll
            for (int q = 4; q < kRec4; q++) srec[tid * kRec4 + q] = src[q];
            if (kInd) slind[tid] = a.lind[(int64_t)v * a.n + id];
            if (samp_variant(kSamp))
                schart[tid] = chart_entry<samp_tri(kSamp)>(a.tex,
                                                           __float_as_int(srec[tid * kRec4 + 6].y));
            qm = quad_mask_uv(r0, r1, r2, r3, tx * kTile, ty * kTile, a.S, a.amin);
        }
        if (tid < kBatch) smask[tid] = qm;
        __syncthreads();
        if (__ballot(!done) != 0) {
            // splats of this batch whose bounds touch this wave's 8x8 block, in list order
            for (int r = 0; r < kBatch / kWave; r++) {
                uint64_t m = __ballot((smask[r * kWave + lane] >> w) & 1u);
                bool wave_done = false;
                while (m) {
                    int j = r * kWave + __builtin_ctzll(m);
                    m &= m - 1;
                    const float4* rp = srec + j * kRec4;
                    SplatEval e = eval_splat(rp, X, Y, a.S, a.amin, a.amax);
                    float u = e.u, vv = e.v, alpha = e.alpha;
                    bool ok = !done && e.hit;
                    float Tn = Tr * (1.0f - alpha);
                    if (ok && Tn < a.tmin) {
                        done = true;
                        ok = false;
                    }
                    if (ok) {
                        float4 c4 = rp[4], c5 = rp[5], c6 = rp[6];
                        // the chart is the same for the whole wave: scalar base address
                        int chart = __builtin_amdgcn_readfirstlane(__float_as_int(c6.y));
                        float t0, t1, t2, t3, t4, t5, t6, t7;
                        if (samp_variant(kSamp)) {
                            float lr = 0.f;
                            if (samp_tri(kSamp)) {
                                lr = footprint(rp[1], rp[2], rp[3], u, vv, e.inv, a.S).lr;
                            }
                            float tt[8];
                            int2 ce = schart[j];
                            ce.x = __builtin_amdgcn_readfirstlane(ce.x);
                            ce.y = __builtin_amdgcn_readfirstlane(ce.y);
                            sample_chart<samp_tri(kSamp), samp_fmt(kSamp)>(a.tex, ce, u, vv, a.S,
                                                                           lr, tt);
                            t0 = tt[0]; t1 = tt[1]; t2 = tt[2]; t3 = tt[3];
                            t4 = tt[4]; t5 = tt[5]; t6 = tt[6]; t7 = tt[7];
                        } else if (kTextured) {
                            __amdgpu_buffer_rsrc_t tr = chart_rsrc(a.atlas + (size_t)(unsigned)chart * chart4,
                                                                   chart4 * 16u);
                            float sx = fmaf(u, tscale, toff), sy = fmaf(vv, tscale, toff);
                            float fx0 = floorf(sx), fy0 = floorf(sy);
                            float fx = sx - fx0, fy = sy - fy0;
                            int i0 = (int)fx0, j0 = (int)fy0;
                            int i1 = min(max(i0 + 1, 0), T - 1), j1 = min(max(j0 + 1, 0), T - 1);
                            i0 = min(max(i0, 0), T - 1);
                            j0 = min(max(j0, 0), T - 1);
                            float4 p00, q00, p10, q10, p01, q01, p11, q11;
                            load_texel8(tr, (unsigned)(j0 * T + i0), p00, q00);
                            load_texel8(tr, (unsigned)(j0 * T + i1), p10, q10);
                            load_texel8(tr, (unsigned)(j1 * T + i0), p01, q01);
                            load_texel8(tr, (unsigned)(j1 * T + i1), p11, q11);
                            // keep the eight loads together ahead of their use (the scheduler
                            // otherwise may interleave them with the math to save registers,
                            // leaving one texel in flight at a time)
                            __builtin_amdgcn_sched_barrier(0);
                            float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy);
                            float w01 = (1.f - fx) * fy, w11 = fx * fy;
                            t0 = w00 * p00.x + w10 * p10.x + w01 * p01.x + w11 * p11.x;
                            t1 = w00 * p00.y + w10 * p10.y + w01 * p01.y + w11 * p11.y;
                            t2 = w00 * p00.z + w10 * p10.z + w01 * p01.z + w11 * p11.z;
                            t3 = w00 * p00.w + w10 * p10.w + w01 * p01.w + w11 * p11.w;
                            t4 = w00 * q00.x + w10 * q10.x + w01 * q01.x + w11 * q11.x;
                            t5 = w00 * q00.y + w10 * q10.y + w01 * q01.y + w11 * q11.y;
                            t6 = w00 * q00.z + w10 * q10.z + w01 * q01.z + w11 * q11.z;
                            t7 = w00 * q00.w + w10 * q10.w + w01 * q01.w + w11 * q11.w;
                        } else {
                            // one attribute per splat (the untextured primitive)
                            __amdgpu_buffer_rsrc_t tr = chart_rsrc(a.atlas + (size_t)(unsigned)chart * chart4,
                                                                   chart4 * 16u);
                            float4 p0, q0;
                            load_texel8(tr, 0u, p0, q0);
                            t0 = p0.x; t1 = p0.y; t2 = p0.z; t3 = p0.w;
                            t4 = q0.x; t5 = q0.y; t6 = q0.z; t7 = q0.w;
                        }
                        float ww = alpha * Tr;
                        blend_sample(acc, ww, c4, c5, c6, t0, t1, t2, t3, t4, t5, t6, t7);
                        if (kInd) {
                            float4 l4 = slind[j];
                            ai[0] = fmaf(ww, l4.x, ai[0]);
                            ai[1] = fmaf(ww, l4.y, ai[1]);
                            ai[2] = fmaf(ww, l4.z, ai[2]);
                        }
                        Tr = Tn;
                        last = b0 - range.x + j + 1;
                        nbl++;
                    }
                    if (__ballot(!done) == 0) {
                        wave_done = true;
                        break;
                    }
                }
                if (wave_done) break;
            }
        }
        __syncthreads();
    }
    if (!inside) return;
    raster_outputs<kInd>(a, v, x, y, acc, ai, Tr, last, nbl);
}

// One 256-thread workgroup per (view, tile); workgroup ids remapped so that each XCD takes a
// contiguous run of tiles of one view (shared L2).
template <int kSamp, bool kInd>
__global__ __launch_bounds__(256, (raster_waves<kSamp, kInd>())) void k_raster_fwd(RasterArgs a) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int v = bid / a.n_tiles;
    raster_tile<kSamp, kInd>(a, v, bid - v * a.n_tiles);
}

struct ShadeArgs {
    int V, W, H;
    const ts_camera* cams;
    ShadeConst sc;
    EnvDev env;
    const float* gbuf;
    const float* t_final;
    float4* rgba;
    const float* gbuf_ind;   // [V][3][H][W] or null (L_ind = 0)
    const float* vis;        // [V][H][W] or null (V = 1)
};

template <bool kInd>
__global__ __launch_bounds__(256) void k_shade(ShadeArgs a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t plane = (int64_t)a.H * a.W;
    if (i >= (int64_t)a.V * plane) return;
    int v = (int)(i / plane);
    int64_t p = i - v * plane;
    int y = (int)(p / a.W), x = (int)(p % a.W);
    float g[8];
    const float* gb = a.gbuf + (int64_t)v * 8 * plane + p;
#pragma unroll
    for (int c = 0; c < 8; c++) g[c] = gb[c * plane];
    float T = a.t_final[i];
    float3 d = pixel_ray(a.cams[v], (float)x + 0.5f, (float)y + 0.5f);
    float li[3] = {0.f, 0.f, 0.f};
    float vis = 1.0f;
    if (kInd) {
        if (a.gbuf_ind) {
            const float* gi = a.gbuf_ind + (int64_t)v * 3 * plane + p;
#pragma unroll
            for (int c = 0; c < 3; c++) li[c] = gi[c * plane];
        }
        if (a.vis) vis = a.vis[i];
    }
    float3 C = shade_pixel<kInd>(a.env, a.sc, g, T, d, li, vis);
    a.rgba[i] = make_float4(C.x, C.y, C.z, 1.0f - T);
}

static int env_from(const ts_env* e, EnvDev& d, const char* who) {
    if (!e->spec || !e->irr || !e->lut || e->spec_res < 1 || e->spec_levels < 1 || e->irr_res < 1 ||
        e->lut_res < 1) {
        set_error("%s: bad ts_env", who);
        return TS_E_ARG;
    }
    d.spec = (const float4*)e->spec;
    d.irr = (const float4*)e->irr;
    d.lut = (const float2*)e->lut;
    d.spec_res = e->spec_res;
    d.levels = e->spec_levels;
    d.irr_res = e->irr_res;
    d.lut_res = e->lut_res;
    return TS_OK;
}

// Checks the arguments of one forward render and fills its kernel arguments; `samp` is the
// texture path (template kSamp of k_raster_fwd). Nothing is enqueued.
static int make_raster_args(const char* who, int32_t n_views, int32_t width, int32_t height,
                            const ts_camera* cams, const ts_params* params, int32_t n,
                            const float* rec, const int32_t* tile_ranges,
                            const int32_t* pair_ids, int64_t pair_capacity, const float* atlas,
                            const ts_env* env, float* rgba, float* gbuf, float* t_final,
                            int32_t* n_contrib, int32_t* n_blend, const float* lind,
                            const float* vis, float* gbuf_ind, RasterArgs& a, int& samp) {
    if (n_views < 1 || width < 1 || height < 1 || n < 0 || !params || !cams || !tile_ranges ||
        (n > 0 && (!atlas || !rec || !pair_ids))) {
        set_error("%s: bad argument", who);
        return TS_E_ARG;
    }
    if (params->tex_res < 1 || params->tex_res > 32) {
        set_error("%s: tex_res %d outside 1..32", who, params->tex_res);
        return TS_E_ARG;
    }
    if (params->sampler == TS_SAMPLER_HARDWARE) {
        set_error("%s: texture-unit sampling is not available on gfx950 (no image "
                  "instructions for this target)", who);
        return TS_E_UNSUPPORTED;
    }
    if (params->sampler != TS_SAMPLER_BILINEAR && params->sampler != TS_SAMPLER_CONSTANT &&
        params->sampler != TS_SAMPLER_TRILINEAR) {
        set_error("%s: unknown sampler %d", who, params->sampler);
        return TS_E_ARG;
    }
    if (params->sampler == TS_SAMPLER_CONSTANT && params->tex_res != 1) {
        set_error("%s: the constant sampler needs tex_res 1 (got %d)", who, params->tex_res);
        return TS_E_ARG;
    }
    if (params->tex_format != TS_TEX_RGBN3 && params->tex_format != TS_TEX_RGBN2) {
        set_error("%s: unknown tex_format %d", who, params->tex_format);
        return TS_E_ARG;
    }
    // the atlas variants: another texel layout, a chart table or trilinear sampling
    const bool variant = params->tex_format != TS_TEX_RGBN3 || params->chart_table ||
                         params->sampler == TS_SAMPLER_TRILINEAR;
    if (variant && !params->chart_table &&
        (params->tex_res & (params->tex_res - 1)) != 0) {
        set_error("%s: atlas variants need a power-of-two tex_res (got %d)", who,
                  params->tex_res);
        return TS_E_ARG;
    }
    if (params->chart_table && params->atlas_texels <= 0) {
        set_error("%s: chart_table needs atlas_texels", who);
        return TS_E_ARG;
    }
    if ((rgba != nullptr) != (env != nullptr)) {
        set_error("%s: rgba and env must be given together", who);
        return TS_E_ARG;
    }
    if (!lind && (vis || gbuf_ind)) {
        set_error("%s: vis and gbuf_ind need lind (the indirect term)", who);
        return TS_E_ARG;
    }
    if (vis && !rgba) {
        set_error("%s: vis is a shading input and needs rgba and env", who);
        return TS_E_ARG;
    }
    a = RasterArgs{};
    a.V = n_views; a.W = width; a.H = height; a.n = n;
    a.ntx = tiles_x(width);
    a.n_tiles = a.ntx * tiles_y(height);
    a.T = params->tex_res;
    a.cams = cams;
    a.S = params->s_sigma; a.amin = params->alpha_min; a.amax = params->alpha_max;
    a.tmin = params->t_min;
    for (int c = 0; c < 3; c++) a.sc.bg[c] = params->bg[c];
    a.shade = env != nullptr;
    if (env) {
        int rc = env_from(env, a.env, who);
        if (rc != TS_OK) return rc;
    }
    a.rec = (const float4*)rec;
    a.ranges = (const int2*)tile_ranges;
    a.pair_ids = pair_ids;
    a.cap = pair_capacity < 0 ? 0 : pair_capacity;
    a.atlas = (const float4*)atlas;
    a.rgba = (float4*)rgba;
    a.gbuf = gbuf;
    a.t_final = t_final;
    a.n_contrib = n_contrib;
    a.n_blend = n_blend;
    a.lind = (const float4*)lind;
    a.vis = vis;
    a.gbuf_ind = gbuf_ind;
    const bool tri = params->sampler == TS_SAMPLER_TRILINEAR;
    a.tex.atlas = (const char*)atlas;
    a.tex.table = (const int2*)params->chart_table;
    a.tex.atlas_texels = params->atlas_texels;
    a.tex.T = params->tex_res;
    a.tex.L = ilog2(params->tex_res);
    a.tex.chart_texels = tri ? chain_texels(params->tex_res)
                             : (unsigned)(params->tex_res * params->tex_res);
    a.tex.fmt = params->tex_format;
    if ((int64_t)n_views * a.n_tiles > 0x7FFFFFFF) {
        set_error("%s: too many tiles", who);
        return TS_E_ARG;
    }
    samp = tri ? 3 : variant ? 2 : params->sampler == TS_SAMPLER_CONSTANT ? 1 : 0;
    if (samp >= 2 && params->tex_format == TS_TEX_RGBN2) samp += 2;
    return TS_OK;
}

// ---- batched persistent launch -------------------------------------------------------------
// The renders of several jobs (each a ts_raster_fwd call on the default atlas path: its own
// scene, views, resolution and outputs) in one launch of a fixed grid. The (job, view, tile)
// work items are numbered job by job and cut into kXcd contiguous ranges, one queue each;
// a workgroup takes items from the queue of its XCD (the hardware deals workgroups to the
// XCDs round-robin) and then from the others in turn, so each XCD mostly works on adjacent
// tiles of one job and every workgroup keeps working while any queue holds items. The grid
// and the kernel do not depend on the batch, so one captured graph serves every batch.
constexpr int kBatchMaxJobs = 64;
constexpr int kBatchQueueWords = 16;   // kXcd counters, the exit count, spare

struct BatchTable {
    int32_t n_jobs;
    int32_t pad[3];
    int32_t item_end[kBatchMaxJobs];   // inclusive prefix sums of n_views * n_tiles
    RasterArgs job[kBatchMaxJobs];
};

// Next work item for this workgroup (thread 0 only), or -1 when every queue is empty.
// `k` is the number of queues this workgroup has found empty so far (it never returns to
// them).
__device__ inline int batch_pop(uint32_t* queue, int total, int xcd, int& k) {
    for (; k < kXcd; k++) {
        int q = (xcd + k) % kXcd;
        int lo = (int)((int64_t)q * total / kXcd), hi = (int)((int64_t)(q + 1) * total / kXcd);
        if (hi <= lo) continue;
        uint32_t i = atomicAdd(&queue[q], 1u);
        if ((int64_t)lo + i < hi) return lo + (int)i;
    }
    return -1;
}

template <int kSamp, bool kInd>
__global__ __launch_bounds__(256, kBatchWaves) void k_raster_batch(
    const BatchTable* __restrict__ tab, uint32_t* __restrict__ queue) {
    __shared__ int s_item[2];
    const int n_jobs = tab->n_jobs;
    const int total = n_jobs > 0 ? tab->item_end[n_jobs - 1] : 0;
    const int xcd = blockIdx.x % kXcd;
    int k = 0;
    for (int it = 0;; it++) {
        // double-buffered broadcast: slot it&1 is rewritten two iterations later, after the
        // next barrier, by which time every thread has read it
        if (threadIdx.x == 0) s_item[it & 1] = batch_pop(queue, total, xcd, k);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item[it & 1]);
        if (item < 0) break;
        int j = 0;
        while (j < n_jobs - 1 && item >= tab->item_end[j]) j++;
        const int local = item - (j > 0 ? tab->item_end[j - 1] : 0);
        const RasterArgs& a = tab->job[j];
        const int v = local / a.n_tiles;
        raster_tile<kSamp, kInd>(a, v, local - v * a.n_tiles);
    }
    // the last workgroup to leave clears the counters for the next launch
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[kXcd], 1u) == gridDim.x - 1) {
            for (int q = 0; q <= kXcd; q++) atomicExch(&queue[q], 0u);
        }
    }
}

// Grid of the batched launch: every CU's resident workgroups, once per device.
static int batch_grid(int dev) {
    static std::mutex mu;
    static int grid[64];
    if (dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!grid[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            return 0;
        grid[dev] = cus * kBatchWaves;
    }
    return grid[dev];
}

}  // namespace ts

using namespace ts;

extern "C" int ts_raster_fwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                             const ts_params* params, int32_t n, const float* rec,
                             const int32_t* tile_ranges, const int32_t* pair_ids,
                             int64_t pair_capacity, const float* atlas, const ts_env* env,
                             float* rgba, float* gbuf, float* t_final, int32_t* n_contrib,
                             int32_t* n_blend, const float* lind, const float* vis,
                             float* gbuf_ind, hipStream_t stream) {
    RasterArgs a;
    int samp = 0;
    int rc = make_raster_args("ts_raster_fwd", n_views, width, height, cams, params, n, rec,
                              tile_ranges, pair_ids, pair_capacity, atlas, env, rgba, gbuf,
                              t_final, n_contrib, n_blend, lind, vis, gbuf_ind, a, samp);
    if (rc != TS_OK) return rc;
    const dim3 grid((unsigned)((int64_t)n_views * a.n_tiles)), block(256);
    if (lind) {
        switch (samp) {
            case 0: hipLaunchKernelGGL((k_raster_fwd<0, true>), grid, block, 0, stream, a); break;
            case 1: hipLaunchKernelGGL((k_raster_fwd<1, true>), grid, block, 0, stream, a); break;
            case 2: hipLaunchKernelGGL((k_raster_fwd<2, true>), grid, block, 0, stream, a); break;
            case 3: hipLaunchKernelGGL((k_raster_fwd<3, true>), grid, block, 0, stream, a); break;
            case 4: hipLaunchKernelGGL((k_raster_fwd<4, true>), grid, block, 0, stream, a); break;
            default: hipLaunchKernelGGL((k_raster_fwd<5, true>), grid, block, 0, stream, a); break;
        }
    } else {
        switch (samp) {
            case 0: hipLaunchKernelGGL((k_raster_fwd<0, false>), grid, block, 0, stream, a); break;
            case 1: hipLaunchKernelGGL((k_raster_fwd<1, false>), grid, block, 0, stream, a); break;
            case 2: hipLaunchKernelGGL((k_raster_fwd<2, false>), grid, block, 0, stream, a); break;
            case 3: hipLaunchKernelGGL((k_raster_fwd<3, false>), grid, block, 0, stream, a); break;
            case 4: hipLaunchKernelGGL((k_raster_fwd<4, false>), grid, block, 0, stream, a); break;
            default: hipLaunchKernelGGL((k_raster_fwd<5, false>), grid, block, 0, stream, a); break;
        }
    }
    return launch_check("ts_raster_fwd");
}

extern "C" size_t ts_raster_batch_table_bytes(void) { return sizeof(BatchTable); }

extern "C" int ts_raster_batch_encode(const ts_raster_job* jobs, int32_t n_jobs, void* table,
                                      size_t table_bytes) {
    if (!table || table_bytes < sizeof(BatchTable) || n_jobs < 0 || n_jobs > kBatchMaxJobs ||
        (n_jobs > 0 && !jobs)) {
        set_error("ts_raster_batch_encode: bad argument (table of %zu bytes needed, 0..%d jobs)",
                  sizeof(BatchTable), kBatchMaxJobs);
        return TS_E_ARG;
    }
    BatchTable* t = (BatchTable*)table;
    memset(t, 0, sizeof(BatchTable));
    int64_t total = 0;
    for (int j = 0; j < n_jobs; j++) {
        const ts_raster_job& J = jobs[j];
        int samp = 0;
        int rc = make_raster_args("ts_raster_batch_encode", J.n_views, J.width, J.height, J.cams,
                                  &J.params, J.n, J.rec, J.tile_ranges, J.pair_ids,
                                  J.pair_capacity, J.atlas, &J.env, J.rgba, nullptr, J.t_final,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, t->job[j], samp);
        if (rc != TS_OK) return rc;
        if (samp != 0 || !J.rgba) {
            set_error("ts_raster_batch_encode: job %d is not a shaded render on the default "
                      "atlas path (bilinear, 8-float texels, no chart table)", j);
            return TS_E_UNSUPPORTED;
        }
        total += (int64_t)J.n_views * t->job[j].n_tiles;
        if (total > 0x7FFFFFFF) {
            set_error("ts_raster_batch_encode: more than 2^31-1 tiles in the batch");
            return TS_E_ARG;
        }
        t->item_end[j] = (int32_t)total;
    }
    t->n_jobs = n_jobs;
    return TS_OK;
}

extern "C" int ts_raster_batch(const void* table, uint32_t* queue, hipStream_t stream) {
    if (!table || !queue) {
        set_error("ts_raster_batch: bad argument");
        return TS_E_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("ts_raster_batch: no current device");
        return TS_E_LAUNCH;
    }
    const int g = batch_grid(dev);
    if (g < 1) {
        set_error("ts_raster_batch: cannot read the compute-unit count of device %d", dev);
        return TS_E_LAUNCH;
    }
    hipLaunchKernelGGL((k_raster_batch<0, false>), dim3(g), dim3(256), 0, stream,
                       (const BatchTable*)table, queue);
    return launch_check("ts_raster_batch");
}

extern "C" int ts_shade(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                        const ts_params* params, const ts_env* env, const float* gbuf,
                        const float* t_final, float* rgba, const float* gbuf_ind,
                        const float* vis, hipStream_t stream) {
    if (n_views < 1 || width < 1 || height < 1 || !params || !cams || !env || !gbuf || !t_final ||
        !rgba) {
        set_error("ts_shade: bad argument");
        return TS_E_ARG;
    }
    ShadeArgs a = {};
    a.V = n_views; a.W = width; a.H = height; a.cams = cams;
    for (int c = 0; c < 3; c++) a.sc.bg[c] = params->bg[c];
    int rc = env_from(env, a.env, "ts_shade");
    if (rc != TS_OK) return rc;
    a.gbuf = gbuf; a.t_final = t_final; a.rgba = (float4*)rgba;
    a.gbuf_ind = gbuf_ind; a.vis = vis;
    int64_t total = (int64_t)n_views * width * height;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (gbuf_ind || vis) hipLaunchKernelGGL(k_shade<true>, grid, block, 0, stream, a);
    else hipLaunchKernelGGL(k_shade<false>, grid, block, 0, stream, a);
    return launch_check("ts_shade");
}

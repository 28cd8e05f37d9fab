// Texture sampling of the atlas variants (two-component normals, per-chart resolutions,
// trilinear over the mip chain), shared by the raster and the atlas builders. The default
// layout (8-float texels, uniform charts, bilinear on level 0) keeps its own straight-line
// path in the raster kernel.
#pragma once
#include "ts_internal.h"

namespace ts {

constexpr int kMaxTexLog2 = 5;   // charts of at most 32 x 32 texels

__host__ __device__ inline int ilog2(int x) {
    int l = 0;
    while ((1 << (l + 1)) <= x) l++;
    return l;
}
// texels of a chart of side T with its full mip chain: T^2 + (T/2)^2 + ... + 1
__host__ __device__ inline unsigned chain_texels(int T) { return (unsigned)(4 * T * T - 1) / 3u; }
// first texel of level l inside such a chart
__host__ __device__ inline unsigned level_offset(int T, int l) {
    int s = T >> l;
    return (unsigned)(4 * (T * T - s * s)) / 3u;
}

struct TexArgs {
    const char* atlas;       // texel bytes
    const int2* table;       // per chart (level-0 texel offset, log2 side) or null
    int64_t atlas_texels;    // bound of table entries
    int T, L;                // uniform side and its log2
    unsigned chart_texels;   // uniform chart stride in texels
    int fmt;                 // TS_TEX_*
};

// The eight channels of texel t (albedo rgb, roughness | normal xyz, metallic); with the
// two-component layout n_z comes back as 0 (rebuilt after filtering).
__device__ __forceinline__ void fetch_texel(__amdgpu_buffer_rsrc_t r, int fmt, unsigned t,
                                            float4& lo, float4& hi) {
    if (fmt) {
        lo = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, t * 28u, 0, 0));
        auto q = __builtin_amdgcn_raw_buffer_load_b96(r, t * 28u + 16u, 0, 0);
        hi = make_float4(__int_as_float(q[0]), __int_as_float(q[1]), 0.f, __int_as_float(q[2]));
    } else {
        load_texel8(r, t, lo, hi);
    }
}

// The four taps of bilinear filtering on a level of Tl texels a side at local (u,v)
// (s = (u+S)/(2S)): texel centres at (i+1/2)/T_l, clamp-to-edge inside the chart (Eq. 5-6).
struct Taps {
    int i0, i1, j0, j1;
    float fx, fy;
};

__device__ inline Taps bilinear_taps(int Tl, float u, float v, float S) {
    Taps k;
    const float sc = (float)Tl / (2.0f * S), off = 0.5f * (float)Tl - 0.5f;
    float sx = fmaf(u, sc, off), sy = fmaf(v, sc, off);
    float fx0 = floorf(sx), fy0 = floorf(sy);
    k.fx = sx - fx0;
    k.fy = sy - fy0;
    int i0 = (int)fx0, j0 = (int)fy0;
    k.i1 = min(max(i0 + 1, 0), Tl - 1);
    k.j1 = min(max(j0 + 1, 0), Tl - 1);
    k.i0 = min(max(i0, 0), Tl - 1);
    k.j0 = min(max(j0, 0), Tl - 1);
    return k;
}

// Footprint of the pixel on the splat: the image-axis derivatives of the closed-form
// (u,v) = (ux dx + uy dy + u0, vx dx + vy dy + v0) / (wx dx + wy dy + w0) (record rows c1..c3,
// inv = 1/den of the pixel), d(u,v)/dX = (ux - u wx, vx - v wx) inv and likewise along Y, and
// lr = log2 rho = log2 max(|d(u,v)/dX|, |d(u,v)/dY|) - log2(2S): rho in units of the whole
// chart, so a chart of side T_c takes level lambda = log2 T_c + lr (Sec. 5, mipmapping).
struct Footprint {
    float dux, duy, dvx, dvy, ax, ay, lr;
};

__device__ inline Footprint footprint(float4 c1, float4 c2, float4 c3, float u, float v,
                                      float inv, float S) {
    Footprint f;
    f.dux = (c1.z - u * c3.x) * inv;
    f.duy = (c1.w - u * c3.y) * inv;
    f.dvx = (c2.y - v * c3.x) * inv;
    f.dvy = (c2.z - v * c3.y) * inv;
    f.ax = fmaf(f.dux, f.dux, f.dvx * f.dvx);
    f.ay = fmaf(f.duy, f.duy, f.dvy * f.dvy);
    f.lr = 0.5f * __builtin_amdgcn_logf(fmaxf(f.ax, f.ay)) - __builtin_amdgcn_logf(2.0f * S);
    return f;
}

// Levels of trilinear sampling on a chain of levels 0..L at lambda = L + lr: lambda <= 0 (or
// undefined) level 0 alone; past the last level, level L alone; else levels floor(lambda) and
// floor(lambda)+1 blended by the fraction f.
struct Levels {
    int la, lb;
    float f;
    bool blend;
};

__device__ inline Levels mip_levels(int L, float lr) {
    Levels m = {0, 0, 0.f, false};
    float lam = (float)L + lr;
    if (lam > 0.f) {
        int l0 = (int)floorf(lam);
        if (l0 >= L) {
            m.la = m.lb = L;
        } else {
            m.la = l0;
            m.lb = l0 + 1;
            m.f = lam - (float)l0;
            m.blend = true;
        }
    }
    return m;
}

// Bilinear on level l of a chart of side Tc at local (u,v); fmt is a compile-time constant
// at every call (the whole function is inlined), so each texel layout gets its own loads.
__device__ __forceinline__ void bilinear_level(__amdgpu_buffer_rsrc_t r, int fmt, int Tc, int l,
                                               float u, float v, float S, float* o) {
    const int Tl = Tc >> l;
    const Taps k = bilinear_taps(Tl, u, v, S);
    const int i0 = k.i0, i1 = k.i1, j0 = k.j0, j1 = k.j1;
    const float fx = k.fx, fy = k.fy;
    const unsigned lo = level_offset(Tc, l);
    float4 p00, q00, p10, q10, p01, q01, p11, q11;
    fetch_texel(r, fmt, lo + (unsigned)(j0 * Tl + i0), p00, q00);
    fetch_texel(r, fmt, lo + (unsigned)(j0 * Tl + i1), p10, q10);
    fetch_texel(r, fmt, lo + (unsigned)(j1 * Tl + i0), p01, q01);
    fetch_texel(r, fmt, lo + (unsigned)(j1 * Tl + i1), p11, q11);
    float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy);
    float w01 = (1.f - fx) * fy, w11 = fx * fy;
    o[0] = w00 * p00.x + w10 * p10.x + w01 * p01.x + w11 * p11.x;
    o[1] = w00 * p00.y + w10 * p10.y + w01 * p01.y + w11 * p11.y;
    o[2] = w00 * p00.z + w10 * p10.z + w01 * p01.z + w11 * p11.z;
    o[3] = w00 * p00.w + w10 * p10.w + w01 * p01.w + w11 * p11.w;
    o[4] = w00 * q00.x + w10 * q10.x + w01 * q01.x + w11 * q11.x;
    o[5] = w00 * q00.y + w10 * q10.y + w01 * q01.y + w11 * q11.y;
    o[6] = w00 * q00.z + w10 * q10.z + w01 * q01.z + w11 * q11.z;
    o[7] = w00 * q00.w + w10 * q10.w + w01 * q01.w + w11 * q11.w;
}

// Where chart `chart` lives: (level-0 texel offset, log2 side); log2 side -1 marks a table
// entry outside the atlas (sampled as 0).
template <bool kTri>
__device__ inline int2 chart_entry(const TexArgs& ta, int chart) {
    if (!ta.table) return make_int2((int)((unsigned)chart * ta.chart_texels), ta.L);
    int2 e = ta.table[chart];
    bool ok = e.y >= 0 && e.y <= kMaxTexLog2 && e.x >= 0 &&
              (int64_t)e.x + (int64_t)(kTri ? chain_texels(1 << e.y) : (1u << (2 * e.y))) <=
                  ta.atlas_texels;
    return ok ? e : make_int2(0, -1);
}

// Texture of the chart at entry `ce` (the same for the whole wave) at (u,v), texels of layout
// kFmt (TS_TEX_*). lr = log2 of the pixel's footprint in units of the whole chart (log2 rho);
// the level is lambda = log2 T_c + lr.
template <bool kTri, int kFmt>
__device__ __forceinline__ void sample_chart(const TexArgs& ta, int2 ce, float u, float v,
                                             float S, float lr, float* t) {
    const bool ok = ce.y >= 0;
    const int64_t base = (unsigned)ce.x;
    const int L = ok ? ce.y : 0;
    const int Tc = 1 << L;
    constexpr unsigned tb = kFmt ? 28u : 32u;
    const unsigned n_tex = ok ? (kTri ? chain_texels(Tc) : (unsigned)(Tc * Tc)) : 0u;
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(ta.atlas + base * tb), (short)0, (int)(n_tex * tb), 0x00020000);
    if (!kTri) {
        bilinear_level(r, kFmt, Tc, 0, u, v, S, t);
    } else {
        // level a for every lane, level b only where two levels blend (one fetch of level a
        // in a wave that mixes both cases: 46.0 -> 39.3 ms on the trilinear headline step)
        const Levels m = mip_levels(L, lr);
        bilinear_level(r, kFmt, Tc, m.la, u, v, S, t);
        if (m.blend) {
            float t1[8];
            bilinear_level(r, kFmt, Tc, m.lb, u, v, S, t1);
#pragma unroll
            for (int q = 0; q < 8; q++) t[q] = fmaf(m.f, t1[q] - t[q], t[q]);
        }
    }
    if (kFmt) t[6] = sqrtf(fmaxf(0.f, 1.f - t[4] * t[4] - t[5] * t[5]));
}

}  // namespace ts

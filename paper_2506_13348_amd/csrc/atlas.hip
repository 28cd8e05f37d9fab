// Atlas variants (once per scene): texel layout conversion, chart strides with room for the
// mip chain, and the box-filtered chain itself (Sec. 3.5.1 two-component normals; Sec. 5
// adaptive resolution and mipmapping).
//
// A chart holds level 0 (T x T texels, row-major) and, for trilinear sampling, levels
// 1..log2 T after it; level l starts at texel 4 (T^2 - (T>>l)^2) / 3 of the chart. A texel is
// 8 floats (albedo rgb, roughness, normal xyz, metallic) or 7 (normal xy only).
#include "texture.h"
#include "ts_internal.h"

namespace ts {

// One thread per (primitive, level-0 texel): copy primitive k's texel into chart perm[k] in
// the target layout.
__global__ __launch_bounds__(256) void k_atlas_pack2(const float* __restrict__ tex, int n, int T,
                                                     const int32_t* __restrict__ perm, int fmt,
                                                     unsigned chart_texels,
                                                     float* __restrict__ atlas,
                                                     int32_t* __restrict__ chart_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)T * T;
    if (i >= (int64_t)n * per) return;
    int k = (int)(i / per);
    int o = (int)(i - (int64_t)k * per);
    int c = perm ? perm[k] : k;
    const float* src = tex + i * 8;
    const int C = fmt ? 7 : 8;
    float* dst = atlas + ((int64_t)c * chart_texels + o) * C;
    if (fmt) {
        // drop n_z (channel 6): albedo rgb, roughness, n_x, n_y, metallic
        for (int q = 0; q < 6; q++) dst[q] = src[q];
        dst[6] = src[7];
    } else {
        for (int q = 0; q < 8; q++) dst[q] = src[q];
    }
    if (o == 0) chart_of[k] = c;
}

// One thread per (chart, texel of level l): mean of the 2x2 texels of level l-1 below it.
__global__ __launch_bounds__(256) void k_atlas_level(float* __restrict__ atlas, int n_charts,
                                                     int T, const int2* __restrict__ table,
                                                     int64_t atlas_texels, int fmt, int l,
                                                     int side_max) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)side_max * side_max;
    if (i >= (int64_t)n_charts * per) return;
    int c = (int)(i / per);
    int o = (int)(i - (int64_t)c * per);
    int64_t base;
    int L;
    if (table) {
        int2 e = table[c];
        base = e.x;
        L = e.y;
        if (L < 0 || L > kMaxTexLog2 || base < 0 ||
            base + (int64_t)chain_texels(1 << L) > atlas_texels)
            return;
    } else {
        L = ilog2(T);
        base = (int64_t)c * chain_texels(T);
    }
    if (l > L) return;
    int Tc = 1 << L;
    int s = Tc >> l, sp = s * 2;                 // sides of level l and of level l-1
    int ox = o % side_max, oy = o / side_max;
    if (ox >= s || oy >= s) return;
    const int C = fmt ? 7 : 8;
    const float* lo = atlas + (base + level_offset(Tc, l - 1)) * C;
    float* hi = atlas + (base + level_offset(Tc, l)) * C;
    const float* a = lo + ((int64_t)(2 * oy) * sp + 2 * ox) * C;
    const float* b = a + C;
    const float* d = a + (int64_t)sp * C;
    const float* e = d + C;
    float* out = hi + ((int64_t)oy * s + ox) * C;
    for (int q = 0; q < C; q++) out[q] = 0.25f * ((a[q] + b[q]) + (d[q] + e[q]));
}

// Per-chart resolutions, set-up of the chart table: one workgroup scans the charts in order
// (chunks of 1024 with a carried sum): table[k] = (texel offset of chart k's level 0 in the
// atlas, log2 side clamped to 0..max_log2), the charts back to back, each with room for its
// mip chain when `mips`; src_off[k] = offset of primitive k's level-0 texels in the input
// (sides^2 back to back).
constexpr int kChartScan = 1024;

__global__ __launch_bounds__(kChartScan) void k_chart_table(const int32_t* __restrict__ log2_side,
                                                            int n, int max_log2, int mips,
                                                            int2* __restrict__ table,
                                                            int64_t* __restrict__ src_off) {
    __shared__ int64_t sa[kChartScan], sb[kChartScan];
    int64_t carry_a = 0, carry_b = 0;
    const int tid = threadIdx.x;
    for (int c0 = 0; c0 < n; c0 += kChartScan) {
        const int k = c0 + tid;
        const int l = k < n ? min(max(log2_side[k], 0), max_log2) : 0;
        const int64_t side = (int64_t)1 << l;
        const int64_t a = k < n ? (mips ? (int64_t)chain_texels((int)side) : side * side) : 0;
        const int64_t b = k < n ? side * side : 0;
        sa[tid] = a;
        sb[tid] = b;
        __syncthreads();
        for (int o = 1; o < kChartScan; o <<= 1) {
            int64_t ya = tid >= o ? sa[tid - o] : 0, yb = tid >= o ? sb[tid - o] : 0;
            __syncthreads();
            sa[tid] += ya;
            sb[tid] += yb;
            __syncthreads();
        }
        if (k < n) {
            const int64_t ea = carry_a + sa[tid] - a;
            // offsets past int32 are marked invalid (-1): the chart then samples as zero
            table[k] = make_int2(ea <= 0x7FFFFFFFLL ? (int)ea : -1, l);
            src_off[k] = carry_b + sb[tid] - b;
        }
        carry_a += sa[kChartScan - 1];
        carry_b += sb[kChartScan - 1];
        __syncthreads();
    }
    if (tid == 0) src_off[n] = carry_b;
}

// One thread per input level-0 texel: its primitive by binary search over src_off, then the
// copy into that chart's level 0 in the target layout (charts past atlas_texels are skipped).
__global__ __launch_bounds__(256) void k_chart_copy(const float* __restrict__ texels,
                                                    int64_t n_texels, int n,
                                                    const int64_t* __restrict__ src_off,
                                                    const int2* __restrict__ table, int fmt,
                                                    int64_t atlas_texels,
                                                    float* __restrict__ atlas) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_texels || i >= src_off[n]) return;
    int lo = 0, hi = n - 1;   // the last k with src_off[k] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (src_off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int2 e = table[lo];
    const int64_t o = i - src_off[lo];
    if (e.x < 0 || e.x + o >= atlas_texels) return;
    const float* src = texels + i * 8;
    const int C = fmt ? 7 : 8;
    float* dst = atlas + ((int64_t)e.x + o) * C;
    if (fmt) {
        for (int q = 0; q < 6; q++) dst[q] = src[q];
        dst[6] = src[7];
    } else {
        for (int q = 0; q < 8; q++) dst[q] = src[q];
    }
}

static int launch_levels(float* atlas, int n_charts, int T, const int2* table, int max_log2,
                         int64_t atlas_texels, int fmt, hipStream_t stream) {
    for (int l = 1; l <= max_log2; l++) {
        int side = (1 << max_log2) >> l;
        int64_t total = (int64_t)n_charts * side * side;
        if (total == 0) continue;
        hipLaunchKernelGGL(k_atlas_level, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           stream, atlas, n_charts, T, table, atlas_texels, fmt, l, side);
    }
    return TS_OK;
}

}  // namespace ts

using namespace ts;

static bool pow2_side(int T) { return T >= 1 && T <= (1 << kMaxTexLog2) && (T & (T - 1)) == 0; }

extern "C" int ts_atlas_pack2(const float* textures, int32_t n, int32_t tex_res,
                              const int32_t* perm, int32_t tex_format, int32_t mips, float* atlas,
                              int32_t* chart_of, hipStream_t stream) {
    if (n < 0 || !pow2_side(tex_res) || (tex_format != TS_TEX_RGBN3 && tex_format != TS_TEX_RGBN2)) {
        set_error("ts_atlas_pack2: bad argument (n=%d T=%d format=%d)", n, tex_res, tex_format);
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    if (!textures || !atlas || !chart_of) {
        set_error("ts_atlas_pack2: null array");
        return TS_E_ARG;
    }
    unsigned chart = mips ? chain_texels(tex_res) : (unsigned)(tex_res * tex_res);
    int64_t total = (int64_t)n * tex_res * tex_res;
    hipLaunchKernelGGL(k_atlas_pack2, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                       textures, n, tex_res, perm, tex_format, chart, atlas, chart_of);
    if (mips)
        launch_levels(atlas, n, tex_res, nullptr, ilog2(tex_res), 0, tex_format, stream);
    return launch_check("ts_atlas_pack2");
}

extern "C" int ts_atlas_mips(float* atlas, int32_t n_charts, int32_t tex_res,
                             const int32_t* chart_table, int32_t max_log2, int64_t atlas_texels,
                             int32_t tex_format, hipStream_t stream) {
    if (n_charts < 0 || !atlas || (tex_format != TS_TEX_RGBN3 && tex_format != TS_TEX_RGBN2) ||
        (!chart_table && !pow2_side(tex_res)) ||
        (chart_table && (max_log2 < 0 || max_log2 > kMaxTexLog2 || atlas_texels < 0))) {
        set_error("ts_atlas_mips: bad argument");
        return TS_E_ARG;
    }
    if (n_charts == 0) return TS_OK;
    int L = chart_table ? max_log2 : ilog2(tex_res);
    launch_levels(atlas, n_charts, tex_res, (const int2*)chart_table, L, atlas_texels, tex_format,
                  stream);
    return launch_check("ts_atlas_mips");
}

extern "C" int ts_atlas_charts_workspace(int32_t n, size_t* bytes) {
    if (!bytes || n < 0) {
        set_error("ts_atlas_charts_workspace: bad argument");
        return TS_E_ARG;
    }
    *bytes = ((size_t)n + 1) * sizeof(int64_t);
    return TS_OK;
}

extern "C" int ts_atlas_pack_charts(const float* texels, int64_t n_texels, int32_t n,
                                    const int32_t* log2_side, int32_t max_log2, int32_t tex_format,
                                    int32_t mips, void* ws, size_t ws_bytes, int32_t* chart_table,
                                    float* atlas, int64_t atlas_texels, hipStream_t stream) {
    if (n < 0 || n_texels < 0 || atlas_texels < 0 || max_log2 < 0 || max_log2 > kMaxTexLog2 ||
        (tex_format != TS_TEX_RGBN3 && tex_format != TS_TEX_RGBN2)) {
        set_error("ts_atlas_pack_charts: bad argument (n=%d format=%d)", n, tex_format);
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    if (!log2_side || !chart_table || !atlas || (n_texels > 0 && !texels)) {
        set_error("ts_atlas_pack_charts: null array");
        return TS_E_ARG;
    }
    if (!ws || ws_bytes < ((size_t)n + 1) * sizeof(int64_t)) {
        set_error("ts_atlas_pack_charts: workspace %zu < %zu bytes", ws_bytes,
                  ((size_t)n + 1) * sizeof(int64_t));
        return TS_E_WORKSPACE;
    }
    int64_t* src_off = (int64_t*)ws;
    hipLaunchKernelGGL(k_chart_table, dim3(1), dim3(kChartScan), 0, stream, log2_side, n,
                       max_log2, mips, (int2*)chart_table, src_off);
    if (n_texels > 0)
        hipLaunchKernelGGL(k_chart_copy, dim3((unsigned)((n_texels + 255) / 256)), dim3(256), 0,
                           stream, texels, n_texels, n, src_off, (const int2*)chart_table,
                           tex_format, atlas_texels, atlas);
    if (mips)
        launch_levels(atlas, n, 1, (const int2*)chart_table, max_log2, atlas_texels, tex_format,
                      stream);
    return launch_check("ts_atlas_pack_charts");
}

// ts_raster_bwd: gradients of a loss on the shaded RGBA with respect to the splat centres,
// rotations (unnormalised quaternions), scales, opacities and atlas texels (the parameters the
// paper optimises end to end, Sec. 3.6).
//
// 1. k_area_*: exclusive scan of the splats' tile-rectangle areas (the splat-major row of
//    each (splat, tile) pair: start[v][s] + row-major index of the tile in the rectangle);
//    k_clear_slots: every (pair, 8x8 block) slot starts empty.
// 2. k_raster_bwd: per tile, per pixel: the adjoint of the shading (dL/dX for the 8 G-buffer
//    channels, dL/dT), then the tile list back to front from the pixel's last blended splat,
//    recovering T_i = T_{i+1} / (1 - alpha_i), with
//        dL/dalpha_i = T_i (g . x_i) - (sum_{j>i} w_j g . x_j + dL/dT_final T_final) / (1 - alpha_i)
//    and the chain through alpha = o G(u,v), the bilinear texture sample at (u,v), the normal
//    normalisation and rotation (Eq. 2-9), down to the 9 coefficients of the closed-form (u,v),
//    the opacity and sigma R. On the atlas variants (per-chart sides from a chart table,
//    trilinear sampling over the box-filtered chain) the sample is taken as the forward takes
//    it; with trilinear sampling the blend fraction of two levels also carries gradient through
//    the level lambda = log2 T_c + log2 rho to the footprint, i.e. to the (u,v) coefficients
//    and the pixel's (u,v), and a level-l texel's gradient reaches the 2^l x 2^l level-0 texels
//    it is the mean of, each with weight 4^-l (the chain is derived from level 0). Each wave (8x8 pixels) sums its pixels' contributions for one
//    splat in a fixed lane order and writes one partial — 19 geometric values and the window
//    of texels it touched — into the partial buffer and records where in the pair's
//    splat-major slot row. No value is accumulated with
//    atomics; a wave takes buffer space in chunks of kChunk floats with one integer atomic.
//    With the indirect term (Eq. 9, Eq. 12) the shading adjoint also gives dL/dL_ind, each
//    blended splat's l_ind joins g . x_i, and its partial carries 3 more sums, w dL/dL_ind.
// 3. k_bwd_gather: per splat, the partials of its (view, tile, quadrant) entries summed in a
//    fixed order (its slot rows are contiguous) -> per-view record gradients and the splat's
//    level-0 texel gradients (and, with the indirect term, dL/dl_ind per view and splat); the
//    coarser levels of a chain get none (they are not parameters).
// 4. k_bwd_params: per splat, in double precision, the record gradients of every view chained
//    through the projection set-up to the splat parameters.
#include "eval.h"
#include "shade_bwd.h"
#include "texture.h"
#include "ts_internal.h"

namespace ts {

constexpr int kGeo = 19;          // px py ux uy vx vy wx wy w0 opacity sR[9]
constexpr int kHdr = 24;          // floats in a partial's header: 19 geometric + window i0 j0 wi wj + pad
// with the indirect term: 19 geometric + 3 of dL/dl_ind, window, pad to a multiple of 8 floats
// (partials start at multiples of 8 floats)
template <bool kInd> constexpr int geo_n() { return kInd ? kGeo + 3 : kGeo; }
template <bool kInd> constexpr int hdr_n() { return kInd ? 32 : kHdr; }
constexpr int kBwdBatch = 128;
constexpr int kEnt = 16;          // LDS floats per lane entry: taps (4 ints), fx, fy, q[8], pad 2
// atlas variants: taps, fx, fy of two levels, their weights over 4^level, the two levels, q[8]
constexpr int kEntVar = 24;
// texture paths of the backward: 0 the default atlas (uniform charts, level-0 bilinear), 1 a
// chart table with level-0 bilinear, 2 trilinear over each chart's chain (table or uniform)
template <int kVar> constexpr int ent_n() { return kVar ? kEntVar : kEnt; }
// resident waves per SIMD: 4 on every texture path, as measured on the 8-view sq300k training
// batch (the chart table: 26.8 ms against 32.3 at 3; trilinear, whose taps are read a row at a
// time and again after the shading adjoint so that it fits 128 registers but for a few spills:
// 32.3 ms against 37.9 at 3; with the indirect term the compiler keeps 3)
template <int kVar> constexpr int bwd_waves() { return 4; }

// bits lo..hi of a 32-bit mask (0 <= lo <= hi <= 31)
__device__ inline unsigned bit_range(int lo, int hi) {
    unsigned top = hi >= 31 ? 0xFFFFFFFFu : ((2u << hi) - 1u);
    return top & ~((1u << lo) - 1u);
}

// The four texels of a bilinear footprint on one level (first texel of the level at lo,
// Tl a side): v[tap][channel], taps 00, 10, 01, 11.
template <int kFmt>
__device__ inline void fetch_taps(__amdgpu_buffer_rsrc_t r, unsigned lo, int Tl, const Taps& k,
                                  float (&v)[4][8]) {
    float4 p[4], q[4];
    fetch_texel(r, kFmt, lo + (unsigned)(k.j0 * Tl + k.i0), p[0], q[0]);
    fetch_texel(r, kFmt, lo + (unsigned)(k.j0 * Tl + k.i1), p[1], q[1]);
    fetch_texel(r, kFmt, lo + (unsigned)(k.j1 * Tl + k.i0), p[2], q[2]);
    fetch_texel(r, kFmt, lo + (unsigned)(k.j1 * Tl + k.i1), p[3], q[3]);
#pragma unroll
    for (int t = 0; t < 4; t++) {
        v[t][0] = p[t].x; v[t][1] = p[t].y; v[t][2] = p[t].z; v[t][3] = p[t].w;
        v[t][4] = q[t].x; v[t][5] = q[t].y; v[t][6] = q[t].z; v[t][7] = q[t].w;
    }
}

// One level's bilinear sample s and its derivatives along the texel coordinates,
// ds/dfx = (1-fy)(v10 - v00) + fy (v11 - v01) and ds/dfy likewise: all that the gradient needs
// of the four texels once the sample's gradient q is known (dL/dfx = q . ds/dfx).
template <int kFmt>
__device__ inline void level_sample(__amdgpu_buffer_rsrc_t r, unsigned lo, int Tl, const Taps& k,
                                    float (&s)[8], float (&sx)[8], float (&sy)[8]) {
    float v[4][8];
    fetch_taps<kFmt>(r, lo, Tl, k, v);
    float w00 = (1.f - k.fx) * (1.f - k.fy), w10 = k.fx * (1.f - k.fy);
    float w01 = (1.f - k.fx) * k.fy, w11 = k.fx * k.fy;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        s[c] = w00 * v[0][c] + w10 * v[1][c] + w01 * v[2][c] + w11 * v[3][c];
        sx[c] = (1.f - k.fy) * (v[1][c] - v[0][c]) + k.fy * (v[3][c] - v[2][c]);
        sy[c] = (1.f - k.fx) * (v[2][c] - v[0][c]) + k.fx * (v[3][c] - v[1][c]);
    }
}

// Two of a level's four taps (0-1: row j0, 2-3: row j1) as 8-channel values.
template <int kFmt>
__device__ __forceinline__ void fetch_row(__amdgpu_buffer_rsrc_t r, unsigned lo, int Tl,
                                          const Taps& k, int row, float (&v)[2][8]) {
    const int j = row ? k.j1 : k.j0;
    float4 p[2], q[2];
    fetch_texel(r, kFmt, lo + (unsigned)(j * Tl + k.i0), p[0], q[0]);
    fetch_texel(r, kFmt, lo + (unsigned)(j * Tl + k.i1), p[1], q[1]);
#pragma unroll
    for (int t = 0; t < 2; t++) {
        v[t][0] = p[t].x; v[t][1] = p[t].y; v[t][2] = p[t].z; v[t][3] = p[t].w;
        v[t][4] = q[t].x; v[t][5] = q[t].y; v[t][6] = q[t].z; v[t][7] = q[t].w;
    }
}

// One level's bilinear sample only (trilinear backward: the taps are read again once q is
// known, so that no level's texels or derivatives stay in registers across the shading
// adjoint; a row of two taps at a time keeps 16 of them in flight, not 32).
template <int kFmt>
__device__ inline void level_value(__amdgpu_buffer_rsrc_t r, unsigned lo, int Tl, const Taps& k,
                                   float (&s)[8]) {
    const float wx0 = 1.f - k.fx, wx1 = k.fx;
#pragma unroll
    for (int row = 0; row < 2; row++) {
        float v[2][8];
        fetch_row<kFmt>(r, lo, Tl, k, row, v);
        const float wy = row ? k.fy : 1.f - k.fy;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float h = wx0 * v[0][c] + wx1 * v[1][c];
            s[c] = row ? fmaf(wy, h, s[c]) : wy * h;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// With the sample's gradient q: the tap dot products D_t = q . v_t of one level, and from them
// q . ds/dfx, q . ds/dfy and q . s (the same sums as from level_sample's outputs, reordered).
template <int kFmt>
__device__ inline void level_dots(__amdgpu_buffer_rsrc_t r, unsigned lo, int Tl, const Taps& k,
                                  const float (&q)[8], float& gX, float& gY, float& qs) {
    float D[4];
#pragma unroll
    for (int row = 0; row < 2; row++) {
        float v[2][8];
        fetch_row<kFmt>(r, lo, Tl, k, row, v);
#pragma unroll
        for (int t = 0; t < 2; t++) {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 8; c++) d = fmaf(q[c], v[t][c], d);
            D[2 * row + t] = d;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    gX = (1.f - k.fy) * (D[1] - D[0]) + k.fy * (D[3] - D[2]);
    gY = (1.f - k.fx) * (D[2] - D[0]) + k.fx * (D[3] - D[1]);
    qs = (1.f - k.fx) * (1.f - k.fy) * D[0] + k.fx * (1.f - k.fy) * D[1] +
         (1.f - k.fx) * k.fy * D[2] + k.fx * k.fy * D[3];
}
constexpr int kChunk = 2048;      // floats of the partial buffer a wave takes at a time

struct BwdArgs {
    int V, W, H, ntx, n_tiles, T, n;
    const ts_camera* cams;
    float S, amin, amax, tmin;
    ShadeConst sc;
    EnvDev env;
    const float4* rec;
    const int2* ranges;
    const int32_t* pair_ids;
    int64_t cap;
    const float4* atlas;
    const float* gbuf;
    const float* t_final;
    const int32_t* n_contrib;
    const float4* d_rgba;
    int32_t* slots;          // [cap][4], splat-major: entry start[v][s] + k, block 0..3
    const int4* rect;        // [V][n] tile rectangles
    const int64_t* start;    // [V][n] exclusive scan of the rectangle areas
    float* part;             // partial buffer
    int64_t part_cap;        // floats
    unsigned long long* part_top;
    int32_t* status;
    const float4* lind;      // [V][n] per (view, splat) l_ind (indirect term) or null
    const float* gind;       // [V][3][H][W] the forward's blended L_ind
    const float* vis;        // [V][H][W] visibility or null (V = 1)
    TexArgs tex;             // atlas description of the variant paths
};

// Texel formats: kFmt 0 = 8 floats (normal xyz), 1 = 7 floats (normal xy, n_z rebuilt as
// sqrt(max(0, 1 - n_x^2 - n_y^2)) after filtering: its gradient folds into n_x and n_y).

// 4 waves per SIMD (at most 128 VGPRs): enough resident waves to cover the texel and
// record loads measured faster than 3 waves with more registers; also for the indirect
// variant (three more sums and the L_ind channel), whose few register spills at 4 waves cost
// less than the fourth wave gains (training step with the indirect term 37.4 -> 33.0 ms)
template <bool kInd, int kFmt, int kVar>
__global__ __launch_bounds__(256, (bwd_waves<kVar>())) void k_raster_bwd(BwdArgs a) {
    constexpr int kGeoN = geo_n<kInd>();
    constexpr int kHdrN = hdr_n<kInd>();
    constexpr int kEntN = ent_n<kVar>();
    __shared__ float4 srec[kBwdBatch * kRec4];
    __shared__ float4 slind[kInd ? kBwdBatch : 1];
    __shared__ float ent[4][kWave * kEntN];
    __shared__ int smax[4];
    __shared__ uint32_t smask[kBwdBatch];
    __shared__ int32_t sslot[kBwdBatch];
    const int g = gridDim.x;
    const int bid = xcd_remap(blockIdx.x, g);
    const int v = bid / a.n_tiles;
    const int t = bid - v * a.n_tiles;
    const int tx = t % a.ntx, ty = t / a.ntx;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int bx = tx * kTile + (w & 1) * 8, by = ty * kTile + (w >> 1) * 8;
    const int x = bx + (lane & 7), y = by + (lane >> 3);
    const bool inside = x < a.W && y < a.H;
    const float X = (float)x + 0.5f, Y = (float)y + 0.5f;
    int2 range = a.ranges[(int64_t)v * a.n_tiles + t];
    range.x = (int)min((int64_t)range.x, a.cap);
    range.y = (int)min((int64_t)range.y, a.cap);
    const int T = a.T;
    const float tscale = (float)T / (2.0f * a.S);
    const float toff = 0.5f * (float)T - 0.5f;
    const int chart4 = T * T * 2;
    float* E = ent[w];

    // per-pixel adjoint of the shading
    int64_t pix = ((int64_t)v * a.H + (inside ? y : 0)) * a.W + (inside ? x : 0);
    int64_t plane = (int64_t)a.H * a.W;
    float gx[8];
    float gli[3] = {0.f, 0.f, 0.f};   // dL/dL_ind (indirect term)
    float Tf = 1.f, dLdTf = 0.f;
    int my_last = 0;
    if (inside) {
        float gb[8];
        const float* gp = a.gbuf + (int64_t)v * 8 * plane + (int64_t)y * a.W + x;
#pragma unroll
        for (int c = 0; c < 8; c++) gb[c] = gp[c * plane];
        Tf = a.t_final[pix];
        my_last = a.n_contrib[pix];
        float4 dC = a.d_rgba[pix];
        float3 dray = pixel_ray(a.cams[v], X, Y);
        float dT;
        if (kInd) {
            float li[3];
            const float* gi = a.gind + (int64_t)v * 3 * plane + (int64_t)y * a.W + x;
            li[0] = gi[0]; li[1] = gi[plane]; li[2] = gi[2 * plane];
            float vis = a.vis ? a.vis[pix] : 1.0f;
            dT = shade_pixel_bwd<true>(a.env, a.sc, gb, Tf, dray, make_float3(dC.x, dC.y, dC.z),
                                       gx, li, vis, gli);
        } else {
            dT = shade_pixel_bwd(a.env, a.sc, gb, Tf, dray, make_float3(dC.x, dC.y, dC.z), gx);
        }
        dLdTf = dT - dC.w;   // A = 1 - T_final
    } else {
#pragma unroll
        for (int c = 0; c < 8; c++) gx[c] = 0.f;
    }
    int wmax = wave_max_dpp(my_last);
    if (lane == 0) smax[w] = wmax;
    __syncthreads();
    int tile_max = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
    float Tr = Tf;
    float accum = 0.f;
    unsigned long long ccur = 0, cend = 0;   // this wave's chunk of the partial buffer

    for (int bend = tile_max; bend > 0; bend -= kBwdBatch) {
        int bstart = max(0, bend - kBwdBatch);
        int nb = bend - bstart;
        __syncthreads();
        uint32_t qmask = 0;
        if (tid < nb) {
            int id = a.pair_ids[range.x + bstart + tid];
            // splat-major slot row of this (splat, tile): k = row-major index of the tile
            // inside the splat's rectangle (the list holds only splats covering the tile)
            int4 rr = a.rect[(int64_t)v * a.n + id];
            int64_t si = a.start[(int64_t)v * a.n + id] + (int64_t)(ty - rr.y) * (rr.z - rr.x) +
                         (tx - rr.x);
            sslot[tid] = si < a.cap ? (int32_t)si : -1;
            const float4* src = a.rec + ((int64_t)v * a.n + id) * kRec4;
            float4 r0 = src[0], r1 = src[1], r2 = src[2], r3 = src[3];
            srec[tid * kRec4 + 0] = r0;
            srec[tid * kRec4 + 1] = r1;
            srec[tid * kRec4 + 2] = r2;
            srec[tid * kRec4 + 3] = r3;
#pragma unroll
            for (int q = 4; q < kRec4; q++) srec[tid * kRec4 + q] = src[q];
            if (kInd) slind[tid] = a.lind[(int64_t)v * a.n + id];
            qmask = quad_mask_uv(r0, r1, r2, r3, tx * kTile, ty * kTile, a.S, a.amin);
        }
        if (tid < kBwdBatch) smask[tid] = qmask;
        __syncthreads();
        int jtop = min(nb, wmax - bstart);
        // candidates of this wave's 8x8 block below jtop, visited back to front
        for (int rr = kBwdBatch / kWave - 1; rr >= 0; rr--) {
          int jb = rr * kWave + lane;
          uint64_t cand = __ballot(jb < jtop && ((smask[jb] >> w) & 1u));
          while (cand) {
            int j = rr * kWave + 63 - __builtin_clzll(cand);
            cand &= ~(1ull << (j - rr * kWave));
            const float4* r = srec + j * kRec4;
            int pos = bstart + j;
            SplatEval ev = eval_splat(r, X, Y, a.S, a.amin, a.amax);
            float u = ev.u, vv = ev.v, alpha = ev.alpha, oG = ev.oG, G = ev.G, inv = ev.inv;
            bool bl = inside && pos < my_last && ev.hit;
            uint64_t blm = __ballot(bl);
            if (blm == 0) continue;
            float geo[kGeoN];
            int i0 = 0x7fffffff, i1 = -1, j0 = 0x7fffffff, j1 = -1;   // texel taps (blended)
            unsigned wmx = 0u, wmy = 0u;   // variants: level-0 columns and rows touched
            bool lblend = false;           // trilinear: this lane blends two levels
#pragma unroll
            for (int k = 0; k < kGeoN; k++) geo[k] = 0.f;
            if (bl && kVar != 0) {
                float4 c1 = r[1], c2 = r[2], c3 = r[3], c4 = r[4], c5 = r[5], c6 = r[6];
                int chart = __builtin_amdgcn_readfirstlane(__float_as_int(c6.y));
                float dx = ev.dx - c6.z, dy = ev.dy - c6.w;
                // the chart's entry (the same for the wave), its level(s) and taps as the
                // forward takes them
                const int2 ce = chart_entry<kVar == 2>(a.tex, chart);
                const bool cok = ce.y >= 0;
                const int Lc = cok ? ce.y : 0;
                const int Tc = 1 << Lc;
                constexpr unsigned tb = kFmt ? 28u : 32u;
                const unsigned n_tex =
                    cok ? (kVar == 2 ? chain_texels(Tc) : (unsigned)(Tc * Tc)) : 0u;
                __amdgpu_buffer_rsrc_t tr = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(a.tex.atlas + (int64_t)(unsigned)ce.x * tb), (short)0,
                    (int)(n_tex * tb), 0x00020000);
                Footprint fp = {};
                Levels lv = {0, 0, 0.f, false};
                if (kVar == 2) {
                    fp = footprint(c1, c2, c3, u, vv, inv, a.S);
                    lv = mip_levels(Lc, fp.lr);
                    lblend = lv.blend;
                }
                const Taps ka = bilinear_taps(Tc >> lv.la, u, vv, a.S);
                float sa[8], sax[8], say[8], sb[8];
                if (kVar == 2) {
                    level_value<kFmt>(tr, level_offset(Tc, lv.la), Tc >> lv.la, ka, sa);
                } else {
                    level_sample<kFmt>(tr, 0u, Tc, ka, sa, sax, say);
                }
                Taps kb = ka;
                if (lv.blend) {
                    kb = bilinear_taps(Tc >> lv.lb, u, vv, a.S);
                    level_value<kFmt>(tr, level_offset(Tc, lv.lb), Tc >> lv.lb, kb, sb);
                }
                float tv[8];
                if (lv.blend) {
#pragma unroll
                    for (int c = 0; c < 8; c++) tv[c] = fmaf(lv.f, sb[c] - sa[c], sa[c]);
                } else {
#pragma unroll
                    for (int c = 0; c < 8; c++) tv[c] = sa[c];
                }
                if (kFmt == 1) tv[6] = sqrtf(fmaxf(0.f, 1.f - tv[4] * tv[4] - tv[5] * tv[5]));
                float nl = tv[4] * tv[4] + tv[5] * tv[5] + tv[6] * tv[6];
                float nh[3], il = 0.f;
                bool hasn = nl > 0.f;
                if (hasn) {
                    il = rsqrtf(nl);
                    nh[0] = tv[4] * il; nh[1] = tv[5] * il; nh[2] = tv[6] * il;
                } else {
                    nh[0] = 0.f; nh[1] = 0.f; nh[2] = 1.f;
                }
                float sR[9] = {c4.x, c4.y, c4.z, c4.w, c5.x, c5.y, c5.z, c5.w, c6.x};
                float nw[3];
                for (int i = 0; i < 3; i++) nw[i] = sR[3 * i] * nh[0] + sR[3 * i + 1] * nh[1] + sR[3 * i + 2] * nh[2];
                float r1m = 1.0f / (1.0f - alpha);
                float Tb = Tr * r1m;
                float wgt = alpha * Tb;
                float cdot = gx[0] * tv[0] + gx[1] * tv[1] + gx[2] * tv[2] + gx[3] * tv[7] +
                             gx[4] * tv[3] + gx[5] * nw[0] + gx[6] * nw[1] + gx[7] * nw[2];
                if (kInd) {
                    float4 l4 = slind[j];
                    cdot += gli[0] * l4.x + gli[1] * l4.y + gli[2] * l4.z;
                }
                float dalpha = Tb * cdot - (accum + dLdTf * Tf) * r1m;
                accum = fmaf(wgt, cdot, accum);
                Tr = Tb;
                float q[8];
                q[0] = wgt * gx[0]; q[1] = wgt * gx[1]; q[2] = wgt * gx[2];
                q[3] = wgt * gx[4];
                q[7] = wgt * gx[3];
                float dnw[3] = {wgt * gx[5], wgt * gx[6], wgt * gx[7]};
                float dnh[3];
                for (int k = 0; k < 3; k++) dnh[k] = sR[k] * dnw[0] + sR[3 + k] * dnw[1] + sR[6 + k] * dnw[2];
                if (hasn) {
                    float pp = nh[0] * dnh[0] + nh[1] * dnh[1] + nh[2] * dnh[2];
                    q[4] = (dnh[0] - nh[0] * pp) * il;
                    q[5] = (dnh[1] - nh[1] * pp) * il;
                    q[6] = (dnh[2] - nh[2] * pp) * il;
                } else {
                    q[4] = q[5] = q[6] = 0.f;
                }
                if (kFmt == 1) {
                    if (tv[6] > 0.f) {
                        float r6 = q[6] / tv[6];
                        q[4] -= r6 * tv[4];
                        q[5] -= r6 * tv[5];
                    }
                    q[6] = 0.f;
                }
                for (int i = 0; i < 3; i++)
                    for (int k = 0; k < 3; k++) geo[10 + 3 * i + k] = dnw[i] * nh[k];
                float gu = 0.f, gv = 0.f, go = 0.f;
                if (ev.oG < a.amax) {
                    go = dalpha * ev.G;
                    gu = -dalpha * ev.oG * u;
                    gv = -dalpha * ev.oG * vv;
                }
                // through each level's bilinear weights (texel coordinate = u T_l/(2S) + ...)
                const float wa = lv.blend ? 1.f - lv.f : 1.f;
                float qsa = 0.f;   // q . s_a (trilinear)
                {
                    float gX = 0.f, gY = 0.f;
                    if (kVar == 2) {
                        level_dots<kFmt>(tr, level_offset(Tc, lv.la), Tc >> lv.la, ka, q, gX, gY,
                                         qsa);
                    } else {
#pragma unroll
                        for (int c = 0; c < 8; c++) {
                            gX = fmaf(q[c], sax[c], gX);
                            gY = fmaf(q[c], say[c], gY);
                        }
                    }
                    const float sca = (float)(Tc >> lv.la) / (2.0f * a.S);
                    gu = fmaf(wa * gX, sca, gu);
                    gv = fmaf(wa * gY, sca, gv);
                }
                float g_ux = 0.f, g_uy = 0.f, g_vx = 0.f, g_vy = 0.f, g_wx = 0.f, g_wy = 0.f;
                float g_w0 = 0.f, g_px = 0.f, g_py = 0.f;
                if (lv.blend) {
                    float gX, gY, qsb;
                    level_dots<kFmt>(tr, level_offset(Tc, lv.lb), Tc >> lv.lb, kb, q, gX, gY, qsb);
                    const float scb = (float)(Tc >> lv.lb) / (2.0f * a.S);
                    gu = fmaf(lv.f * gX, scb, gu);
                    gv = fmaf(lv.f * gY, scb, gv);
                    // the blend fraction f = lambda - floor(lambda): dL/dlambda = q . (s_b - s_a),
                    // lambda = L_c + 0.5 log2 max(ax, ay) - log2(2S)
                    const float glam = qsb - qsa;
                    const float m = fmaxf(fp.ax, fp.ay);
                    const float gm = glam * (0.5f * 1.44269504088896341f) / m;
                    float gdux = 0.f, gduy = 0.f, gdvx = 0.f, gdvy = 0.f;
                    if (fp.ax >= fp.ay) {
                        gdux = 2.f * fp.dux * gm;
                        gdvx = 2.f * fp.dvx * gm;
                    } else {
                        gduy = 2.f * fp.duy * gm;
                        gdvy = 2.f * fp.dvy * gm;
                    }
                    // du/dX = (ux - u wx) inv, du/dY = (uy - u wy) inv, dv/dX, dv/dY likewise
                    g_ux = gdux * inv;
                    g_uy = gduy * inv;
                    g_vx = gdvx * inv;
                    g_vy = gdvy * inv;
                    g_wx = -(gdux * u + gdvx * vv) * inv;
                    g_wy = -(gduy * u + gdvy * vv) * inv;
                    gu -= (gdux * c3.x + gduy * c3.y) * inv;
                    gv -= (gdvx * c3.x + gdvy * c3.y) * inv;
                    // inv = 1/den, den = wx dx + wy dy + w0
                    const float gden = -(gdux * fp.dux + gduy * fp.duy + gdvx * fp.dvx +
                                         gdvy * fp.dvy) * inv;
                    g_wx = fmaf(gden, dx, g_wx);
                    g_wy = fmaf(gden, dy, g_wy);
                    g_w0 = gden;
                    g_px = -gden * c3.x;
                    g_py = -gden * c3.y;
                }
                float e = -(gu * u + gv * vv) * inv;
                geo[2] = fmaf(gu * dx, inv, g_ux);
                geo[3] = fmaf(gu * dy, inv, g_uy);
                geo[4] = fmaf(gv * dx, inv, g_vx);
                geo[5] = fmaf(gv * dy, inv, g_vy);
                geo[6] = fmaf(e, dx, g_wx);
                geo[7] = fmaf(e, dy, g_wy);
                geo[8] = e + g_w0;
                geo[0] = -(gu * c1.z + gv * c2.y) * inv - e * c3.x + g_px;
                geo[1] = -(gu * c1.w + gv * c2.z) * inv - e * c3.y + g_py;
                geo[9] = go;
                if (kInd) {
                    geo[kGeo + 0] = wgt * gli[0];
                    geo[kGeo + 1] = wgt * gli[1];
                    geo[kGeo + 2] = wgt * gli[2];
                }
                // level-0 texels under the taps of each level (a level-l texel is the mean of
                // a 2^l x 2^l block of level 0)
                wmx = bit_range(ka.i0 << lv.la, ((ka.i1 + 1) << lv.la) - 1);
                wmy = bit_range(ka.j0 << lv.la, ((ka.j1 + 1) << lv.la) - 1);
                if (lv.blend) {
                    wmx |= bit_range(kb.i0 << lv.lb, ((kb.i1 + 1) << lv.lb) - 1);
                    wmy |= bit_range(kb.j0 << lv.lb, ((kb.j1 + 1) << lv.lb) - 1);
                }
                float* me = E + (int)lanes_below(blm) * kEntN;
                me[0] = __int_as_float(ka.i0); me[1] = __int_as_float(ka.i1);
                me[2] = __int_as_float(ka.j0); me[3] = __int_as_float(ka.j1);
                me[4] = ka.fx; me[5] = ka.fy;
                me[6] = __int_as_float(kb.i0); me[7] = __int_as_float(kb.i1);
                me[8] = __int_as_float(kb.j0); me[9] = __int_as_float(kb.j1);
                me[10] = kb.fx; me[11] = kb.fy;
                me[12] = ldexpf(wa, -2 * lv.la);
                me[13] = lv.blend ? ldexpf(lv.f, -2 * lv.lb) : 0.f;
                me[14] = __int_as_float(lv.la); me[15] = __int_as_float(lv.lb);
#pragma unroll
                for (int c = 0; c < 8; c++) me[16 + c] = q[c];
            }
            if (bl && kVar == 0) {
                float4 c1 = r[1], c2 = r[2], c3 = r[3], c4 = r[4], c5 = r[5], c6 = r[6];
                int chart = __builtin_amdgcn_readfirstlane(__float_as_int(c6.y));
                // offsets from the exact projected centre (head + low part)
                float dx = ev.dx - c6.z, dy = ev.dy - c6.w;
                float sx = fmaf(u, tscale, toff), sy = fmaf(vv, tscale, toff);
                float fx0 = floorf(sx), fy0 = floorf(sy);
                float fx = sx - fx0, fy = sy - fy0;
                i0 = (int)fx0;
                j0 = (int)fy0;
                i1 = min(max(i0 + 1, 0), T - 1);
                j1 = min(max(j0 + 1, 0), T - 1);
                i0 = min(max(i0, 0), T - 1);
                j0 = min(max(j0, 0), T - 1);
                float4 p00, q00, p10, q10, p01, q01, p11, q11;
                if (kFmt == 0) {
                    __amdgpu_buffer_rsrc_t tr = chart_rsrc(
                        a.atlas + (size_t)(unsigned)chart * chart4, (unsigned)chart4 * 16u);
                    load_texel8(tr, (unsigned)(j0 * T + i0), p00, q00);
                    load_texel8(tr, (unsigned)(j0 * T + i1), p10, q10);
                    load_texel8(tr, (unsigned)(j1 * T + i0), p01, q01);
                    load_texel8(tr, (unsigned)(j1 * T + i1), p11, q11);
                } else {
                    // 28-byte texels, channel 6 (n_z) read as 0
                    const unsigned cb = (unsigned)(T * T) * 28u;
                    __amdgpu_buffer_rsrc_t tr = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)((const char*)a.atlas + (size_t)(unsigned)chart * cb), (short)0,
                        (int)cb, 0x00020000);
                    fetch_texel(tr, 1, (unsigned)(j0 * T + i0), p00, q00);
                    fetch_texel(tr, 1, (unsigned)(j0 * T + i1), p10, q10);
                    fetch_texel(tr, 1, (unsigned)(j1 * T + i0), p01, q01);
                    fetch_texel(tr, 1, (unsigned)(j1 * T + i1), p11, q11);
                }
                float v00[8] = {p00.x, p00.y, p00.z, p00.w, q00.x, q00.y, q00.z, q00.w};
                float v10[8] = {p10.x, p10.y, p10.z, p10.w, q10.x, q10.y, q10.z, q10.w};
                float v01[8] = {p01.x, p01.y, p01.z, p01.w, q01.x, q01.y, q01.z, q01.w};
                float v11[8] = {p11.x, p11.y, p11.z, p11.w, q11.x, q11.y, q11.z, q11.w};
                float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy);
                float w01 = (1.f - fx) * fy, w11 = fx * fy;
                float tv[8];
#pragma unroll
                for (int c = 0; c < 8; c++)
                    tv[c] = w00 * v00[c] + w10 * v10[c] + w01 * v01[c] + w11 * v11[c];
                if (kFmt == 1) tv[6] = sqrtf(fmaxf(0.f, 1.f - tv[4] * tv[4] - tv[5] * tv[5]));
                float nl = tv[4] * tv[4] + tv[5] * tv[5] + tv[6] * tv[6];
                float nh[3], il = 0.f;
                bool hasn = nl > 0.f;
                if (hasn) {
                    il = rsqrtf(nl);
                    nh[0] = tv[4] * il; nh[1] = tv[5] * il; nh[2] = tv[6] * il;
                } else {
                    nh[0] = 0.f; nh[1] = 0.f; nh[2] = 1.f;
                }
                float sR[9] = {c4.x, c4.y, c4.z, c4.w, c5.x, c5.y, c5.z, c5.w, c6.x};
                float nw[3];
                for (int i = 0; i < 3; i++) nw[i] = sR[3 * i] * nh[0] + sR[3 * i + 1] * nh[1] + sR[3 * i + 2] * nh[2];
                // transmittance before this splat and dL/dalpha
                float r1m = 1.0f / (1.0f - alpha);
                float Tb = Tr * r1m;
                float wgt = alpha * Tb;
                float cdot = gx[0] * tv[0] + gx[1] * tv[1] + gx[2] * tv[2] + gx[3] * tv[7] +
                             gx[4] * tv[3] + gx[5] * nw[0] + gx[6] * nw[1] + gx[7] * nw[2];
                if (kInd) {
                    float4 l4 = slind[j];
                    cdot += gli[0] * l4.x + gli[1] * l4.y + gli[2] * l4.z;
                }
                float dalpha = Tb * cdot - (accum + dLdTf * Tf) * r1m;
                accum = fmaf(wgt, cdot, accum);
                Tr = Tb;
                // texture-sample gradients q[8] (channel order of the texels)
                float q[8];
                q[0] = wgt * gx[0]; q[1] = wgt * gx[1]; q[2] = wgt * gx[2];
                q[3] = wgt * gx[4];                     // roughness
                q[7] = wgt * gx[3];                     // metallic
                float dnw[3] = {wgt * gx[5], wgt * gx[6], wgt * gx[7]};
                float dnh[3];
                for (int k = 0; k < 3; k++) dnh[k] = sR[k] * dnw[0] + sR[3 + k] * dnw[1] + sR[6 + k] * dnw[2];
                if (hasn) {
                    float pp = nh[0] * dnh[0] + nh[1] * dnh[1] + nh[2] * dnh[2];
                    q[4] = (dnh[0] - nh[0] * pp) * il;
                    q[5] = (dnh[1] - nh[1] * pp) * il;
                    q[6] = (dnh[2] - nh[2] * pp) * il;
                } else {
                    q[4] = q[5] = q[6] = 0.f;
                }
                if (kFmt == 1) {   // n_z = sqrt(1 - n_x^2 - n_y^2) of the filtered sample
                    if (tv[6] > 0.f) {
                        float r6 = q[6] / tv[6];
                        q[4] -= r6 * tv[4];
                        q[5] -= r6 * tv[5];
                    }
                    q[6] = 0.f;
                }
                // d(sigma R): outer(dnw, nh)
                for (int i = 0; i < 3; i++)
                    for (int k = 0; k < 3; k++) geo[10 + 3 * i + k] = dnw[i] * nh[k];
                // (u,v) through alpha and through the texture coordinates
                float gu = 0.f, gv = 0.f, go = 0.f;
                if (oG < a.amax) {
                    go = dalpha * G;
                    gu = -dalpha * oG * u;
                    gv = -dalpha * oG * vv;
                }
                // through the bilinear weights: with D_ab = q . v_ab (the four taps),
                // dL/dfx = (1-fy)(D10 - D00) + fy (D11 - D01), dL/dfy likewise
                float D00 = 0.f, D10 = 0.f, D01 = 0.f, D11 = 0.f;
#pragma unroll
                for (int c = 0; c < 8; c++) {
                    D00 = fmaf(q[c], v00[c], D00);
                    D10 = fmaf(q[c], v10[c], D10);
                    D01 = fmaf(q[c], v01[c], D01);
                    D11 = fmaf(q[c], v11[c], D11);
                }
                float gX = (1.f - fy) * (D10 - D00) + fy * (D11 - D01);
                float gY = (1.f - fx) * (D01 - D00) + fx * (D11 - D10);
                gu = fmaf(gX, tscale, gu);
                gv = fmaf(gY, tscale, gv);
                // (u,v) = (ux dx + uy dy, vx dx + vy dy) / (wx dx + wy dy + w0), dx = X - px
                float e = -(gu * u + gv * vv) * inv;
                geo[2] = gu * dx * inv;                 // ux
                geo[3] = gu * dy * inv;                 // uy
                geo[4] = gv * dx * inv;                 // vx
                geo[5] = gv * dy * inv;                 // vy
                geo[6] = e * dx;                        // wx
                geo[7] = e * dy;                        // wy
                geo[8] = e;                             // w0
                geo[0] = -(gu * c1.z + gv * c2.y) * inv - e * c3.x;   // px
                geo[1] = -(gu * c1.w + gv * c2.z) * inv - e * c3.y;   // py
                geo[9] = go;                            // opacity
                if (kInd) {                             // dL/dl_ind of this splat
                    geo[kGeo + 0] = wgt * gli[0];
                    geo[kGeo + 1] = wgt * gli[1];
                    geo[kGeo + 2] = wgt * gli[2];
                }
                // lane entry, at the lane's rank among the blended lanes
                float* me = E + (int)lanes_below(blm) * kEntN;
                me[0] = __int_as_float(i0); me[1] = __int_as_float(i1);
                me[2] = __int_as_float(j0); me[3] = __int_as_float(j1);
                me[4] = fx; me[5] = fy;
#pragma unroll
                for (int c = 0; c < 8; c++) me[6 + c] = q[c];
            }
            // window of texels touched by this wave: OR over the blended lanes of bit masks of
            // their tap columns and rows (at least one lane is blended here; i1 >= i0, j1 >= j0)
            int wi0, wj0, wi1, wj1;
            if (kVar != 0) {
                unsigned mx = wave_or_dpp(wmx), my = wave_or_dpp(wmy);
                wi0 = __builtin_ctz(mx);
                wi1 = 31 - __builtin_clz(mx);
                wj0 = __builtin_ctz(my);
                wj1 = 31 - __builtin_clz(my);
            } else if (T <= 16) {
                unsigned mk = bl ? (1u << i0) | (1u << i1) | (0x10000u << j0) | (0x10000u << j1) : 0u;
                unsigned m = wave_or_dpp(mk);
                wi0 = __builtin_ctz(m & 0xFFFFu);
                wi1 = 31 - __builtin_clz(m & 0xFFFFu);
                wj0 = __builtin_ctz(m >> 16);
                wj1 = 31 - __builtin_clz(m >> 16);
            } else {
                unsigned mx = wave_or_dpp(bl ? (1u << i0) | (1u << i1) : 0u);
                unsigned my = wave_or_dpp(bl ? (1u << j0) | (1u << j1) : 0u);
                wi0 = __builtin_ctz(mx);
                wi1 = 31 - __builtin_clz(mx);
                wj0 = __builtin_ctz(my);
                wj1 = 31 - __builtin_clz(my);
            }
            int wi = wi1 - wi0 + 1, wj = wj1 - wj0 + 1, wt = wi * wj;
            int64_t need = kHdrN + (int64_t)wt * 8;
            // space from this wave's current chunk; a new chunk (one integer atomic) when
            // it is used up
            if (ccur + (unsigned long long)need > cend) {
                unsigned long long take = (unsigned long long)max(need, (int64_t)kChunk);
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(a.part_top, take);
                base = __shfl(base, 0);
                ccur = base;
                cend = base + take;
            }
            unsigned long long off = ccur;
            ccur += (unsigned long long)need;
            bool fits = (int64_t)off + need <= a.part_cap;
            const int srow = sslot[j];
            const int64_t slot_idx = (int64_t)srow * 4 + w;
            if (!fits) {
                if (lane == 0) {
                    a.status[0] = 2;
                    if (srow >= 0) a.slots[slot_idx] = -1;
                }
                continue;
            }
            float* dst = a.part + off;
            // geometric sums over the wave (zeros from the other lanes) by transposing
            // reductions in a fixed order
            {
                // the first 16 sums in lanes 0-15 (value bitrev4(lane)), the other 3 (6 with
                // the indirect term) in lanes 16-19 (16-23)
                constexpr int kRest = kGeoN - 16 <= 4 ? 4 : 8;
                static_assert(kGeoN > 16 && kGeoN - 16 <= 8, "16 + at most 8 sums");
                float xa[16], xb[kRest];
#pragma unroll
                for (int k = 0; k < 16; k++) xa[k] = geo[k];
#pragma unroll
                for (int k = 0; k < kRest; k++) xb[k] = 16 + k < kGeoN ? geo[16 + k] : 0.f;
                float ta = wave_transpose_sum<16>(xa, lane);
                float tb = wave_transpose_sum<kRest>(xb, lane);
                const int l4 = lane & 15;
                const int va = ((l4 & 1) << 3) | ((l4 & 2) << 1) | ((l4 & 4) >> 1) | ((l4 & 8) >> 3);
                const int lr = lane & (kRest - 1);
                const int vb = 16 + (kRest == 4 ? (((lr & 1) << 1) | ((lr & 2) >> 1))
                                                : (((lr & 1) << 2) | (lr & 2) | ((lr & 4) >> 2)));
                if (lane < 16) dst[va] = ta;
                else if (lane < 16 + kRest && vb < kGeoN) dst[vb] = tb;
                if (lane == kWave - 1) {
                    dst[kGeoN + 0] = __int_as_float(wi0);
                    dst[kGeoN + 1] = __int_as_float(wj0);
                    dst[kGeoN + 2] = __int_as_float(wi);
                    dst[kGeoN + 3] = __int_as_float(wj);
                    dst[kGeoN + 4] = 0.f;
                }
            }
            // texel window: lanes form groups of L = pow2 >= wt lanes (texel = lane mod L);
            // the blended pixels' entries sit at their ranks 0..nbw-1 among the blended lanes;
            // group g sums entries g, g + 64/L, ... in order, then the groups are combined by
            // a fixed butterfly
            const int nbw = __builtin_popcountll(blm);
            // the second level's weights are zero unless a lane of the wave blends two levels
            const int nlev = (kVar == 2 && __ballot(lblend) != 0) ? 2 : 1;
            int L = 1;
            while (L < wt && L < kWave) L <<= 1;
            const int ngrp = kWave / L;
            const int tl = lane & (L - 1), grp = lane / L;
            for (int t0 = 0; t0 < wt; t0 += kWave) {
                int tt = t0 + tl;
                int ti = wi0 + (tt % wi), tj = wj0 + (tt / wi);
                float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                for (int p = grp; p < nbw; p += ngrp) {
                    const float* pe = E + p * kEntN;
                    if (kVar == 0) {
                        int pi0 = __float_as_int(pe[0]), pi1 = __float_as_int(pe[1]);
                        int pj0 = __float_as_int(pe[2]), pj1 = __float_as_int(pe[3]);
                        float pfx = pe[4], pfy = pe[5];
                        float wxp = (ti == pi0 ? 1.f - pfx : 0.f) + (ti == pi1 ? pfx : 0.f);
                        float wyp = (tj == pj0 ? 1.f - pfy : 0.f) + (tj == pj1 ? pfy : 0.f);
                        float wq = wxp * wyp;
#pragma unroll
                        for (int c = 0; c < 8; c++) acc[c] = fmaf(wq, pe[6 + c], acc[c]);
                    } else {
                        // level-0 texel (ti, tj) lies under level-l texel (ti >> l, tj >> l)
                        float wq = 0.f;
#pragma unroll
                        for (int b = 0; b < nlev; b++) {
                            const float* pb = pe + 6 * b;
                            int l = __float_as_int(pe[14 + b]);
                            int si = ti >> l, sj = tj >> l;
                            float pfx = pb[4], pfy = pb[5];
                            float wxp = (si == __float_as_int(pb[0]) ? 1.f - pfx : 0.f) +
                                        (si == __float_as_int(pb[1]) ? pfx : 0.f);
                            float wyp = (sj == __float_as_int(pb[2]) ? 1.f - pfy : 0.f) +
                                        (sj == __float_as_int(pb[3]) ? pfy : 0.f);
                            wq = fmaf(pe[12 + b], wxp * wyp, wq);
                        }
#pragma unroll
                        for (int c = 0; c < 8; c++) acc[c] = fmaf(wq, pe[16 + c], acc[c]);
                    }
                }
                for (int sft = L; sft < kWave; sft <<= 1) {
#pragma unroll
                    for (int c = 0; c < 8; c++) acc[c] += __shfl_xor(acc[c], sft);
                }
                if (grp == 0 && tt < wt) {
                    float4* d4 = (float4*)(dst + kHdrN + (int64_t)tt * 8);
                    d4[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
                    d4[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
                }
            }
            if (lane == 0 && srow >= 0) a.slots[slot_idx] = (int32_t)(off / 8);
          }
        }
    }
}

// Every (entry, 8x8 block) slot starts empty: rows [0, min(pairs, cap)) of the splat-major
// slot array, pairs = end of the last tile list.
__global__ __launch_bounds__(256) void k_clear_slots(const int32_t* __restrict__ ranges,
                                                     int64_t last, int64_t cap,
                                                     int32_t* __restrict__ slots) {
    int64_t rows = min((int64_t)ranges[2 * last + 1], cap);
    int4* s4 = (int4*)slots;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        s4[i] = make_int4(-1, -1, -1, -1);
}

// Exclusive scan of rect areas over (view, splat) -> int64 start offsets, in three passes:
// per-block totals (1024 entries per block, 4 per thread), a scan of the block totals, and the
// in-block scan plus the block's offset.
constexpr int kAreaPer = 4;
constexpr int kAreaBlock = 256 * kAreaPer;

__device__ inline int64_t rect_area(int4 r) {
    return (int64_t)max(r.z - r.x, 0) * max(r.w - r.y, 0);
}

__device__ inline int64_t block_excl_scan_256(int64_t x, int64_t* sh, int64_t* total) {
    int tid = threadIdx.x;
    sh[tid] = x;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int64_t y = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += y;
        __syncthreads();
    }
    int64_t incl = sh[tid];
    if (total) *total = sh[255];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(256) void k_area_sums(const int4* __restrict__ rect, int64_t m,
                                                   int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[256];
    int64_t i0 = (int64_t)blockIdx.x * kAreaBlock + threadIdx.x * kAreaPer;
    int64_t s = 0;
    for (int k = 0; k < kAreaPer; k++)
        if (i0 + k < m) s += rect_area(rect[i0 + k]);
    int64_t tot;
    block_excl_scan_256(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block totals in place.
__global__ __launch_bounds__(256) void k_area_scan_sums(int64_t* __restrict__ bsum, int nb) {
    __shared__ int64_t sh[256];
    int per = (nb + 255) / 256;
    int a0 = threadIdx.x * per, a1 = min(nb, a0 + per);
    int64_t s = 0;
    for (int i = a0; i < a1; i++) s += bsum[i];
    int64_t run = block_excl_scan_256(s, sh, nullptr);
    for (int i = a0; i < a1; i++) {
        int64_t x = bsum[i];
        bsum[i] = run;
        run += x;
    }
}

__global__ __launch_bounds__(256) void k_area_apply(const int4* __restrict__ rect, int64_t m,
                                                    const int64_t* __restrict__ bsum,
                                                    int64_t* __restrict__ start) {
    __shared__ int64_t sh[256];
    int64_t i0 = (int64_t)blockIdx.x * kAreaBlock + threadIdx.x * kAreaPer;
    int64_t ar[kAreaPer];
    int64_t s = 0;
    for (int k = 0; k < kAreaPer; k++) {
        ar[k] = i0 + k < m ? rect_area(rect[i0 + k]) : 0;
        s += ar[k];
    }
    int64_t run = block_excl_scan_256(s, sh, nullptr) + bsum[blockIdx.x];
    for (int k = 0; k < kAreaPer; k++)
        if (i0 + k < m) {
            start[i0 + k] = run;
            run += ar[k];
        }
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }
__global__ void k_copy_u64(const unsigned long long* src, int64_t* dst) { *dst = (int64_t)*src; }

// One wave per splat: views in order, tiles of rect(s) in row-major order, quadrants 0..3.
// Lane l owns texels l, l+64, ... of the splat's chart; one pass over the partials per group
// of 64 texels. The entries are taken 64 at a time: lane e looks up entry e's slot and window
// (so those dependent loads overlap), then the entries are summed one after another in order,
// their slot and window read from the owning lane.
template <bool kInd, int kFmt, int kVar>
__global__ __launch_bounds__(64) void k_bwd_gather(int V, int n, int T, TexArgs tex,
                                                   const int4* __restrict__ rect,
                                                   const int64_t* __restrict__ start,
                                                   int64_t cap,
                                                   const int32_t* __restrict__ slots,
                                                   const float* __restrict__ part,
                                                   const int32_t* __restrict__ chart_of,
                                                   const int32_t* __restrict__ status,
                                                   float beta, float* __restrict__ rec_grad,
                                                   float* __restrict__ d_atlas,
                                                   float* __restrict__ d_lind) {
    constexpr int kGeoN = geo_n<kInd>();
    constexpr int kHdrN = hdr_n<kInd>();
    if (status[0] != 0) return;   // incomplete partials: leave the outputs untouched
    int s = blockIdx.x, lane = threadIdx.x;
    constexpr int C = kFmt ? 7 : 8;
    // the splat's chart: level-0 texel offset and side (a chart outside the atlas samples as 0
    // and takes no texel gradient)
    int Tg = T;
    int64_t cbase = (int64_t)chart_of[s] * T * T;
    bool cok = true;
    if (kVar != 0) {
        int2 ce = chart_entry<kVar == 2>(tex, chart_of[s]);
        cok = ce.y >= 0;
        Tg = cok ? 1 << ce.y : 1;
        cbase = (unsigned)ce.x;
    }
    int TT = Tg * Tg;
    float* dch = d_atlas + cbase * C;
    for (int t0 = 0; t0 < TT; t0 += kWave) {
        int tt = t0 + lane;
        int ti = tt % Tg, tj = tt / Tg;
        bool own = cok && tt < TT;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int v = 0; v < V; v++) {
            int4 r = rect[(int64_t)v * n + s];
            int cnt = max(r.z - r.x, 0) * max(r.w - r.y, 0);
            if (cnt == 0) {
                if (t0 == 0 && lane < kGeo) rec_grad[((int64_t)v * n + s) * kGeo + lane] = 0.f;
                if (kInd && t0 == 0 && lane >= kGeo && lane < kGeo + 4)
                    d_lind[((int64_t)v * n + s) * 4 + lane - kGeo] = 0.f;
                continue;
            }
            int64_t st = start[(int64_t)v * n + s];
            float gs = 0.f;
            int ne = cnt * 4;
            for (int e0 = 0; e0 < ne; e0 += kWave) {
                int e = e0 + lane;
                int sl = -1;
                int win = 0;   // packed i0 | j0 << 8 | wi << 16 | wj << 24 (all < 256)
                if (e < ne && st + (e >> 2) < cap) {
                    sl = slots[(st + (e >> 2)) * 4 + (e & 3)];
                    if (sl >= 0) {
                        const float* h = part + (int64_t)sl * 8 + kGeoN;
                        win = __float_as_int(h[0]) | (__float_as_int(h[1]) << 8) |
                              (__float_as_int(h[2]) << 16) | (__float_as_int(h[3]) << 24);
                    }
                }
                // entries with a partial, in order, four at a time: the loads of the four
                // are issued together, then added in entry order
                uint64_t vm = __ballot(sl >= 0);
                while (vm) {
                    int js[4];
                    int nj = 0;
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        js[u] = 0;
                        if (vm) {
                            js[u] = __builtin_ctzll(vm);
                            vm &= vm - 1;
                            nj = u + 1;
                        }
                    }
                    float g[4];
                    float4 lo[4], hi[4];
                    bool in[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        g[u] = 0.f;
                        in[u] = false;
                        lo[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                        hi[u] = lo[u];
                        if (u < nj) {
                            int slj = __builtin_amdgcn_readlane(sl, js[u]);
                            int wj = __builtin_amdgcn_readlane(win, js[u]);
                            const float* src = part + (int64_t)slj * 8;
                            if (t0 == 0 && lane < kGeoN) g[u] = src[lane];
                            int li = ti - (wj & 255), lj = tj - ((wj >> 8) & 255);
                            int wi = (wj >> 16) & 255, wh = (wj >> 24) & 255;
                            in[u] = own && li >= 0 && lj >= 0 && li < wi && lj < wh;
                            if (in[u]) {
                                const float4* s4 =
                                    (const float4*)(src + kHdrN + (int64_t)(lj * wi + li) * 8);
                                lo[u] = s4[0];
                                hi[u] = s4[1];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        if (u < nj && t0 == 0 && lane < kGeoN) gs += g[u];
                        if (in[u]) {
                            acc[0] += lo[u].x; acc[1] += lo[u].y; acc[2] += lo[u].z; acc[3] += lo[u].w;
                            acc[4] += hi[u].x; acc[5] += hi[u].y; acc[6] += hi[u].z; acc[7] += hi[u].w;
                        }
                    }
                }
            }
            if (t0 == 0 && lane < kGeo) rec_grad[((int64_t)v * n + s) * kGeo + lane] = gs;
            if (kInd && t0 == 0 && lane >= kGeo && lane < kGeo + 4)
                d_lind[((int64_t)v * n + s) * 4 + lane - kGeo] = gs;   // lane kGeo + 3: 0
        }
        if (own) {
            float4 lo = make_float4(acc[0], acc[1], acc[2], acc[3]);
            float4 hi = make_float4(acc[4], acc[5], acc[6], acc[7]);
            if (kFmt == 0) {
                float4* dst = (float4*)dch;
                if (beta != 0.f) {
                    float4 o0 = dst[tt * 2], o1 = dst[tt * 2 + 1];
                    lo.x += beta * o0.x; lo.y += beta * o0.y; lo.z += beta * o0.z; lo.w += beta * o0.w;
                    hi.x += beta * o1.x; hi.y += beta * o1.y; hi.z += beta * o1.z; hi.w += beta * o1.w;
                }
                dst[tt * 2] = lo;
                dst[tt * 2 + 1] = hi;
            } else {
                // 7-float texels: albedo rgb, roughness, n_x, n_y, metallic
                float* d7 = dch + (int64_t)tt * 7;
                float v7[7] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.w};
#pragma unroll
                for (int c = 0; c < 7; c++) d7[c] = beta != 0.f ? v7[c] + beta * d7[c] : v7[c];
            }
        }
    }
    // the chain's coarser levels are derived from level 0: no gradient of their own
    if (kVar == 2 && cok) {
        const int64_t end = (int64_t)chain_texels(Tg) * C;
        for (int64_t i = (int64_t)TT * C + lane; i < end; i += kWave)
            dch[i] = beta != 0.f ? beta * dch[i] : 0.f;
    }
}

// Chain rule of the projection set-up (see k_preprocess), double precision, views in order.
__global__ __launch_bounds__(256) void k_bwd_params(int V, int n, const ts_camera* __restrict__ cams,
                                                    const float* __restrict__ means,
                                                    const float* __restrict__ quats,
                                                    const float* __restrict__ scales,
                                                    const int4* __restrict__ rect,
                                                    const float* __restrict__ rec_grad,
                                                    const int32_t* __restrict__ status, float beta,
                                                    float* d_means, float* d_quats, float* d_scales,
                                                    float* d_opac) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || status[0] != 0) return;
    double mu[3] = {means[3 * s], means[3 * s + 1], means[3 * s + 2]};
    double q[4] = {quats[4 * s], quats[4 * s + 1], quats[4 * s + 2], quats[4 * s + 3]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                   2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    double su = scales[2 * s], sv = scales[2 * s + 1];
    double dmu[3] = {0, 0, 0}, dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dsu = 0, dsv = 0, dop = 0;
    for (int v = 0; v < V; v++) {
        int4 rr = rect[(int64_t)v * n + s];
        if (rr.z <= rr.x || rr.w <= rr.y) continue;
        const float* gr = rec_grad + ((int64_t)v * n + s) * kGeo;
        const ts_camera& cam = cams[v];
        double Wr[9], t[3];
        for (int i = 0; i < 3; i++) {
            for (int j = 0; j < 3; j++) Wr[i * 3 + j] = cam.w2c[i * 4 + j];
            t[i] = cam.w2c[i * 4 + 3];
        }
        // the set-up of ts_preprocess: camera-frame points by A = W^{-T}, covectors by W
        double A[9];
        {
            const double* M = Wr;
            double C[9] = {M[4] * M[8] - M[5] * M[7], M[5] * M[6] - M[3] * M[8], M[3] * M[7] - M[4] * M[6],
                           M[2] * M[7] - M[1] * M[8], M[0] * M[8] - M[2] * M[6], M[1] * M[6] - M[0] * M[7],
                           M[1] * M[5] - M[2] * M[4], M[2] * M[3] - M[0] * M[5], M[0] * M[4] - M[1] * M[3]};
            double id = 1.0 / (M[0] * C[0] + M[1] * C[1] + M[2] * C[2]);
            for (int i = 0; i < 9; i++) A[i] = C[i] * id;
        }
        double mc[3], gu[3], gv[3], nc[3];
        for (int i = 0; i < 3; i++) {
            mc[i] = A[i * 3] * mu[0] + A[i * 3 + 1] * mu[1] + A[i * 3 + 2] * mu[2] + t[i];
            gu[i] = Wr[i * 3] * R[0] + Wr[i * 3 + 1] * R[3] + Wr[i * 3 + 2] * R[6];
            gv[i] = Wr[i * 3] * R[1] + Wr[i * 3 + 1] * R[4] + Wr[i * 3 + 2] * R[7];
            nc[i] = Wr[i * 3] * R[2] + Wr[i * 3 + 1] * R[5] + Wr[i * 3 + 2] * R[8];
        }
        double fx = cam.fx, fy = cam.fy;
        double nmu = nc[0] * mc[0] + nc[1] * mc[1] + nc[2] * mc[2];
        double sg = nmu > 0 ? 1.0 : -1.0;
        double mgu = mc[0] * gu[0] + mc[1] * gu[1] + mc[2] * gu[2];
        double mgv = mc[0] * gv[0] + mc[1] * gv[1] + mc[2] * gv[2];
        double Au[3], Bv[3];
        for (int i = 0; i < 3; i++) {
            Au[i] = nmu * gu[i] - mgu * nc[i];
            Bv[i] = nmu * gv[i] - mgv * nc[i];
        }
        double iz = 1.0 / mc[2];
        double g_px = gr[0], g_py = gr[1], g_ux = gr[2], g_uy = gr[3], g_vx = gr[4], g_vy = gr[5];
        double g_wx = gr[6], g_wy = gr[7], g_w0 = gr[8];
        dop += gr[9];
        // sigma R -> R (sigma = facing sign, constant)
        double o[3];
        for (int i = 0; i < 3; i++) o[i] = -(Wr[0 * 3 + i] * t[0] + Wr[1 * 3 + i] * t[1] + Wr[2 * 3 + i] * t[2]);
        double nwd = R[2] * (o[0] - mu[0]) + R[5] * (o[1] - mu[1]) + R[8] * (o[2] - mu[2]);
        double sigma = nwd >= 0.0 ? 1.0 : -1.0;
        for (int k = 0; k < 9; k++) dR[k] += sigma * gr[10 + k];
        double dmc[3] = {0, 0, 0}, dgu[3] = {0, 0, 0}, dgv[3] = {0, 0, 0}, dnc[3] = {0, 0, 0};
        double dnmu = 0.0;
        // px = fx mc0/mc2 + cx, py = fy mc1/mc2 + cy
        dmc[0] += g_px * fx * iz;
        dmc[1] += g_py * fy * iz;
        dmc[2] += -(g_px * fx * mc[0] + g_py * fy * mc[1]) * iz * iz;
        // ux = sg Au0/(su fx), uy = sg Au1/(su fy); vx = sg Bv0/(sv fx), vy = sg Bv1/(sv fy)
        double dA[3] = {sg * g_ux / (su * fx), sg * g_uy / (su * fy), 0.0};
        double dB[3] = {sg * g_vx / (sv * fx), sg * g_vy / (sv * fy), 0.0};
        dsu += -(g_ux * sg * Au[0] / (su * fx) + g_uy * sg * Au[1] / (su * fy)) / su;
        dsv += -(g_vx * sg * Bv[0] / (sv * fx) + g_vy * sg * Bv[1] / (sv * fy)) / sv;
        // Au = nmu gu - (mc.gu) nc, Bv = nmu gv - (mc.gv) nc
        {
            double dAg = dA[0] * gu[0] + dA[1] * gu[1] + dA[2] * gu[2];
            double dBg = dB[0] * gv[0] + dB[1] * gv[1] + dB[2] * gv[2];
            double dAn = dA[0] * nc[0] + dA[1] * nc[1] + dA[2] * nc[2];
            double dBn = dB[0] * nc[0] + dB[1] * nc[1] + dB[2] * nc[2];
            dnmu += dAg + dBg;
            for (int i = 0; i < 3; i++) {
                dgu[i] += nmu * dA[i] - dAn * mc[i];
                dgv[i] += nmu * dB[i] - dBn * mc[i];
                dmc[i] += -dAn * gu[i] - dBn * gv[i];
                dnc[i] += -mgu * dA[i] - mgv * dB[i];
            }
        }
        // wx = sg nc0/fx, wy = sg nc1/fy, w0 = sg nmu/mc2
        dnc[0] += sg * g_wx / fx;
        dnc[1] += sg * g_wy / fy;
        dnmu += sg * g_w0 * iz;
        dmc[2] += -sg * g_w0 * nmu * iz * iz;
        // nmu = nc.mc
        for (int i = 0; i < 3; i++) {
            dnc[i] += dnmu * mc[i];
            dmc[i] += dnmu * nc[i];
        }
        // camera frame -> world: gu = W R[:,0], gv = W R[:,1], nc = W R[:,2]; mc = A mu + t
        for (int j = 0; j < 3; j++) {
            double wtu = 0, wtv = 0, wnc = 0, wmc = 0;
            for (int i = 0; i < 3; i++) {
                wtu += Wr[i * 3 + j] * dgu[i];
                wtv += Wr[i * 3 + j] * dgv[i];
                wnc += Wr[i * 3 + j] * dnc[i];
                wmc += A[i * 3 + j] * dmc[i];
            }
            dR[j * 3 + 0] += wtu;
            dR[j * 3 + 1] += wtv;
            dR[j * 3 + 2] += wnc;
            dmu[j] += wmc;
        }
    }
    // rotation matrix of the unit quaternion -> quaternion
    double dw = -2 * z * dR[1] + 2 * y * dR[2] + 2 * z * dR[3] - 2 * x * dR[5] - 2 * y * dR[6] + 2 * x * dR[7];
    double dx = 2 * y * dR[1] + 2 * z * dR[2] + 2 * y * dR[3] - 4 * x * dR[4] - 2 * w * dR[5] + 2 * z * dR[6] + 2 * w * dR[7] - 4 * x * dR[8];
    double dy = -4 * y * dR[0] + 2 * x * dR[1] + 2 * w * dR[2] + 2 * x * dR[3] + 2 * z * dR[5] - 2 * w * dR[6] + 2 * z * dR[7] - 4 * y * dR[8];
    double dz = -4 * z * dR[0] - 2 * w * dR[1] + 2 * x * dR[2] + 2 * w * dR[3] - 4 * z * dR[4] + 2 * y * dR[5] + 2 * x * dR[6] + 2 * y * dR[7];
    double dot = w * dw + x * dx + y * dy + z * dz;
    double dq[4] = {(dw - w * dot) / qn, (dx - x * dot) / qn, (dy - y * dot) / qn, (dz - z * dot) / qn};
    float b = beta;
    for (int i = 0; i < 3; i++) d_means[3 * s + i] = (float)dmu[i] + (b != 0.f ? b * d_means[3 * s + i] : 0.f);
    for (int i = 0; i < 4; i++) d_quats[4 * s + i] = (float)dq[i] + (b != 0.f ? b * d_quats[4 * s + i] : 0.f);
    d_scales[2 * s] = (float)dsu + (b != 0.f ? b * d_scales[2 * s] : 0.f);
    d_scales[2 * s + 1] = (float)dsv + (b != 0.f ? b * d_scales[2 * s + 1] : 0.f);
    d_opac[s] = (float)dop + (b != 0.f ? b * d_opac[s] : 0.f);
}

struct BwdLayout {
    size_t off_start, off_slots, off_recgrad, off_top, off_bsum, total;
    int area_blocks;
};

inline BwdLayout bwd_layout(int V, int n, int64_t cap) {
    BwdLayout L;
    size_t vn = (size_t)V * (size_t)(n > 0 ? n : 1);
    size_t c = (size_t)(cap > 0 ? cap : 1);
    size_t off = 0;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.off_start = off; off = al(off + vn * 8);
    L.off_slots = off; off = al(off + c * 16);
    L.off_recgrad = off; off = al(off + vn * kGeo * 4);
    L.off_top = off; off = al(off + 8);
    L.area_blocks = (int)((vn + kAreaBlock - 1) / kAreaBlock);
    L.off_bsum = off; off = al(off + (size_t)L.area_blocks * 8);
    L.total = off;
    return L;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_raster_bwd_workspace(int32_t n_views, int32_t n, int64_t pair_capacity,
                                       size_t* bytes) {
    if (!bytes || n_views < 1 || n < 0 || pair_capacity < 0) {
        set_error("ts_raster_bwd_workspace: bad argument");
        return TS_E_ARG;
    }
    *bytes = bwd_layout(n_views, n, pair_capacity).total;
    return TS_OK;
}

template <bool kInd, int kFmt, int kVar>
static void launch_bwd(const BwdArgs& a, int n_views, int n_tiles, int n, int T, const int32_t* rect,
                       const int64_t* start, int64_t pair_capacity, const int32_t* slots,
                       const float* partials, const int32_t* chart_of, const int32_t* status,
                       float beta, float* rec_grad, float* d_atlas, float* d_lind,
                       hipStream_t stream) {
    hipLaunchKernelGGL((k_raster_bwd<kInd, kFmt, kVar>), dim3(n_views * n_tiles), dim3(256), 0,
                       stream, a);
    hipLaunchKernelGGL((k_bwd_gather<kInd, kFmt, kVar>), dim3(n), dim3(64), 0, stream, n_views, n,
                       T, a.tex, (const int4*)rect, start, pair_capacity, slots, partials, chart_of,
                       status, beta, rec_grad, d_atlas, d_lind);
}

template <bool kInd, int kFmt>
static void launch_bwd_var(int var, const BwdArgs& a, int n_views, int n_tiles, int n, int T,
                           const int32_t* rect, const int64_t* start, int64_t pair_capacity,
                           const int32_t* slots, const float* partials, const int32_t* chart_of,
                           const int32_t* status, float beta, float* rec_grad, float* d_atlas,
                           float* d_lind, hipStream_t stream) {
    if (var == 2)
        launch_bwd<kInd, kFmt, 2>(a, n_views, n_tiles, n, T, rect, start, pair_capacity, slots,
                                  partials, chart_of, status, beta, rec_grad, d_atlas, d_lind,
                                  stream);
    else if (var == 1)
        launch_bwd<kInd, kFmt, 1>(a, n_views, n_tiles, n, T, rect, start, pair_capacity, slots,
                                  partials, chart_of, status, beta, rec_grad, d_atlas, d_lind,
                                  stream);
    else
        launch_bwd<kInd, kFmt, 0>(a, n_views, n_tiles, n, T, rect, start, pair_capacity, slots,
                                  partials, chart_of, status, beta, rec_grad, d_atlas, d_lind,
                                  stream);
}

extern "C" int ts_raster_bwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                             const ts_params* params, int32_t n, const float* means,
                             const float* quats, const float* scales, const int32_t* chart_of,
                             const float* rec, const int32_t* rect, const int32_t* tile_ranges,
                             const int32_t* pair_ids, int64_t pair_capacity, const float* atlas,
                             const ts_env* env, const float* gbuf, const float* t_final,
                             const int32_t* n_contrib, const float* d_rgba, void* ws,
                             size_t ws_bytes, float* partials, int64_t partial_capacity,
                             int32_t* status, int64_t* partial_used, float beta, float* d_means, float* d_quats,
                             float* d_scales, float* d_opac, float* d_atlas, const float* lind,
                             const float* vis, const float* gbuf_ind, float* d_lind,
                             hipStream_t stream) {
    if (n_views < 1 || width < 1 || height < 1 || n < 0 || !params || !cams || !env ||
        !tile_ranges || !gbuf || !t_final || !n_contrib || !d_rgba || !status ||
        (n > 0 && (!means || !quats || !scales || !chart_of || !rec || !rect || !pair_ids ||
                   !atlas || !d_means || !d_quats || !d_scales || !d_opac || !d_atlas ||
                   !partials))) {
        set_error("ts_raster_bwd: bad argument");
        return TS_E_ARG;
    }
    if (params->tex_res < 1 || params->tex_res > 32) {
        set_error("ts_raster_bwd: tex_res %d outside 1..32", params->tex_res);
        return TS_E_ARG;
    }
    if (params->sampler != TS_SAMPLER_BILINEAR && params->sampler != TS_SAMPLER_TRILINEAR) {
        set_error("ts_raster_bwd: the bilinear and trilinear samplers are differentiated (T = 1 "
                  "textures give the untextured primitive)");
        return params->sampler == TS_SAMPLER_HARDWARE ? TS_E_UNSUPPORTED : TS_E_ARG;
    }
    if (params->tex_format != TS_TEX_RGBN3 && params->tex_format != TS_TEX_RGBN2) {
        set_error("ts_raster_bwd: unknown tex_format %d", params->tex_format);
        return TS_E_ARG;
    }
    const bool tri = params->sampler == TS_SAMPLER_TRILINEAR;
    if (tri && !params->chart_table && (params->tex_res & (params->tex_res - 1)) != 0) {
        set_error("ts_raster_bwd: trilinear sampling needs a power-of-two tex_res (got %d)",
                  params->tex_res);
        return TS_E_ARG;
    }
    if (params->chart_table && params->atlas_texels <= 0) {
        set_error("ts_raster_bwd: chart_table needs atlas_texels");
        return TS_E_ARG;
    }
    if (lind && (!gbuf_ind || !d_lind)) {
        set_error("ts_raster_bwd: the indirect term needs gbuf_ind and d_lind");
        return TS_E_ARG;
    }
    if (!lind && (vis || gbuf_ind || d_lind)) {
        set_error("ts_raster_bwd: vis, gbuf_ind and d_lind need lind (the indirect term)");
        return TS_E_ARG;
    }
    if (partial_capacity < 0 || partial_capacity > (int64_t)INT32_MAX * 8) {
        set_error("ts_raster_bwd: partial_capacity %lld outside 0..2^34 floats",
                  (long long)partial_capacity);
        return TS_E_ARG;
    }
    BwdLayout L = bwd_layout(n_views, n, pair_capacity);
    if (!ws || ws_bytes < L.total) {
        set_error("ts_raster_bwd: workspace %zu < %zu bytes", ws_bytes, L.total);
        return TS_E_WORKSPACE;
    }
    if (n == 0) return TS_OK;
    char* wsc = (char*)ws;
    int64_t* start = (int64_t*)(wsc + L.off_start);
    int32_t* slots = (int32_t*)(wsc + L.off_slots);
    float* rec_grad = (float*)(wsc + L.off_recgrad);
    unsigned long long* top = (unsigned long long*)(wsc + L.off_top);
    int ntx = tiles_x(width), n_tiles = ntx * tiles_y(height);
    int64_t vn = (int64_t)n_views * n;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, top);
    int64_t* bsum = (int64_t*)(wsc + L.off_bsum);
    hipLaunchKernelGGL(k_area_sums, dim3(L.area_blocks), dim3(256), 0, stream, (const int4*)rect,
                       vn, bsum);
    hipLaunchKernelGGL(k_area_scan_sums, dim3(1), dim3(256), 0, stream, bsum, L.area_blocks);
    hipLaunchKernelGGL(k_area_apply, dim3(L.area_blocks), dim3(256), 0, stream,
                       (const int4*)rect, vn, (const int64_t*)bsum, start);
    if (pair_capacity > 0)
        hipLaunchKernelGGL(k_clear_slots, dim3(2048), dim3(256), 0, stream, tile_ranges,
                           (int64_t)n_views * n_tiles - 1, pair_capacity, slots);
    BwdArgs a = {};
    a.V = n_views; a.W = width; a.H = height; a.ntx = ntx; a.n_tiles = n_tiles;
    a.T = params->tex_res; a.n = n; a.cams = cams;
    a.S = params->s_sigma; a.amin = params->alpha_min; a.amax = params->alpha_max;
    a.tmin = params->t_min;
    for (int c = 0; c < 3; c++) a.sc.bg[c] = params->bg[c];
    if (!env->spec || !env->irr || !env->lut) {
        set_error("ts_raster_bwd: bad ts_env");
        return TS_E_ARG;
    }
    a.env.spec = (const float4*)env->spec; a.env.irr = (const float4*)env->irr;
    a.env.lut = (const float2*)env->lut; a.env.spec_res = env->spec_res;
    a.env.levels = env->spec_levels; a.env.irr_res = env->irr_res; a.env.lut_res = env->lut_res;
    a.rec = (const float4*)rec; a.ranges = (const int2*)tile_ranges; a.pair_ids = pair_ids;
    a.cap = pair_capacity; a.atlas = (const float4*)atlas; a.gbuf = gbuf; a.t_final = t_final;
    a.n_contrib = n_contrib; a.d_rgba = (const float4*)d_rgba; a.slots = slots;
    a.rect = (const int4*)rect; a.start = (const int64_t*)start;
    a.part = partials; a.part_cap = partial_capacity; a.part_top = top; a.status = status;
    a.lind = (const float4*)lind; a.gind = gbuf_ind; a.vis = vis;
    a.tex.atlas = (const char*)atlas;
    a.tex.table = (const int2*)params->chart_table;
    a.tex.atlas_texels = params->atlas_texels;
    a.tex.T = params->tex_res;
    a.tex.L = ilog2(params->tex_res);
    a.tex.chart_texels = tri ? chain_texels(params->tex_res)
                             : (unsigned)(params->tex_res * params->tex_res);
    a.tex.fmt = params->tex_format;
    const int var = tri ? 2 : params->chart_table ? 1 : 0;
    const bool xy = params->tex_format == TS_TEX_RGBN2;
    if (lind && xy)
        launch_bwd_var<true, 1>(var, a, n_views, n_tiles, n, params->tex_res, rect, start,
                                pair_capacity, slots, partials, chart_of, status, beta, rec_grad,
                                d_atlas, d_lind, stream);
    else if (lind)
        launch_bwd_var<true, 0>(var, a, n_views, n_tiles, n, params->tex_res, rect, start,
                                pair_capacity, slots, partials, chart_of, status, beta, rec_grad,
                                d_atlas, d_lind, stream);
    else if (xy)
        launch_bwd_var<false, 1>(var, a, n_views, n_tiles, n, params->tex_res, rect, start,
                                 pair_capacity, slots, partials, chart_of, status, beta, rec_grad,
                                 d_atlas, nullptr, stream);
    else
        launch_bwd_var<false, 0>(var, a, n_views, n_tiles, n, params->tex_res, rect, start,
                                 pair_capacity, slots, partials, chart_of, status, beta, rec_grad,
                                 d_atlas, nullptr, stream);
    hipLaunchKernelGGL(k_bwd_params, dim3((n + 255) / 256), dim3(256), 0, stream, n_views, n, cams,
                       means, quats, scales, (const int4*)rect, (const float*)rec_grad,
                       (const int32_t*)status, beta, d_means, d_quats, d_scales, d_opac);
    if (partial_used) hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(1), 0, stream, top, partial_used);
    return launch_check("ts_raster_bwd");
}

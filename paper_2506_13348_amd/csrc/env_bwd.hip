// ts_env_bwd: gradients of a loss on the shaded RGBA with respect to the texels of the
// environment's shading tables — the diffuse irradiance cube and every prefiltered specular
// level — taken as learnable parameters (the environment is optimised end to end with the
// splats, Sec. 3.5-3.6; Eq. 11-12 read the tables through bilinear cube lookups).
//
// The shaded colour is linear in each table texel: per pixel, dL/dE = dL/dC * albedo (1-M)/pi
// at the irradiance lookup of N, and dL/dL_pref = dL/dC * V (F0 A + B) split between the two
// levels around R (L-1) at the lookup of the reflected direction (V the pixel's visibility:
// with the indirect term the specular radiance is V L_pref + (1 - V) L_ind, Eq. 12). Each lookup spreads its
// gradient over 4 texels with the bilinear weights.
//
// Deterministic without floating-point atomics:
//  1. k_env_records: per pixel, 12 (texel, gradient) records (3 lookups x 4 taps; unused ones
//     carry the key 0xFFFFFFFF).
//  2. a stable radix sort of the record keys: the records of one texel end up together, in
//     pixel order.
//  3. k_env_block_sums: per block of 256 sorted records, each texel's run inside the block is
//     summed by a segmented scan of fixed shape.
//  4. k_env_texel_sums: per texel run, its block pieces added in block order, written to the
//     gradient tables (overwrite or accumulate).
#include "shade.h"
#include "sort_kernels.h"
#include "ts_internal.h"

namespace ts {

constexpr int kEnvRec = 12;          // records per pixel
constexpr int kEnvBlock = 256;       // sorted records per reduction block
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

struct EnvBwdArgs {
    int V, W, H;
    const ts_camera* cams;
    EnvDev env;
    const float* gbuf;       // [V][8][H][W]
    const float* t_final;    // [V][H][W]
    const float4* d_rgba;    // [V][H][W]
    const float* vis;        // [V][H][W] visibility or null (V = 1)
    uint32_t* keys;          // [P * 12]
    float4* vals;            // [P * 12]
    int n_irr;               // texels of the irradiance cube (6 r^2)
};

// Texel keys and weights of one bilinear cube lookup (as face_bilinear takes them).
__device__ inline void cube_taps(int r, int face, float X, float Y, uint32_t base, uint32_t* k,
                                 float* w) {
    float x0 = floorf(X), y0 = floorf(Y);
    float fx = X - x0, fy = Y - y0;
    int i0 = (int)x0, j0 = (int)y0;
    int i1 = min(max(i0 + 1, 0), r - 1), j1 = min(max(j0 + 1, 0), r - 1);
    i0 = min(max(i0, 0), r - 1);
    j0 = min(max(j0, 0), r - 1);
    uint32_t f0 = base + (uint32_t)face * r * r;
    k[0] = f0 + j0 * r + i0; w[0] = (1.f - fx) * (1.f - fy);
    k[1] = f0 + j0 * r + i1; w[1] = fx * (1.f - fy);
    k[2] = f0 + j1 * r + i0; w[2] = (1.f - fx) * fy;
    k[3] = f0 + j1 * r + i1; w[3] = fx * fy;
}

__global__ __launch_bounds__(256) void k_env_records(EnvBwdArgs a) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t P = (int64_t)a.V * a.H * a.W;
    if (gid >= P) return;
    int64_t plane = (int64_t)a.H * a.W;
    int v = (int)(gid / plane);
    int64_t pix = gid - (int64_t)v * plane;
    int y = (int)(pix / a.W), x = (int)(pix - (int64_t)y * a.W);
    uint32_t* ko = a.keys + gid * kEnvRec;
    float4* vo = a.vals + gid * kEnvRec;
    float Tf = a.t_final[gid];
    if (!(Tf < 1.0f)) {   // empty pixel: background only, no table read
        for (int q = 0; q < kEnvRec; q++) { ko[q] = kNoKey; vo[q] = make_float4(0.f, 0.f, 0.f, 0.f); }
        return;
    }
    float g[8];
    const float* gp = a.gbuf + (int64_t)v * 8 * plane + pix;
    for (int c = 0; c < 8; c++) g[c] = gp[c * plane];
    float4 dC = a.d_rgba[gid];
    float3 dray = pixel_ray(a.cams[v], (float)x + 0.5f, (float)y + 0.5f);
    // the forward's lookups (shade_pixel / shade_pixel_bwd)
    float il = rsqrtf(dray.x * dray.x + dray.y * dray.y + dray.z * dray.z);
    float wo[3] = {-dray.x * il, -dray.y * il, -dray.z * il};
    float nn = g[5] * g[5] + g[6] * g[6] + g[7] * g[7];
    float Nh[3];
    if (nn > 0.f) {
        float inv = rsqrtf(nn);
        Nh[0] = g[5] * inv; Nh[1] = g[6] * inv; Nh[2] = g[7] * inv;
    } else {
        Nh[0] = wo[0]; Nh[1] = wo[1]; Nh[2] = wo[2];
    }
    float ndv = Nh[0] * wo[0] + Nh[1] * wo[1] + Nh[2] * wo[2];
    float wr[3] = {2.f * ndv * Nh[0] - wo[0], 2.f * ndv * Nh[1] - wo[1], 2.f * ndv * Nh[2] - wo[2]};
    const EnvDev& env = a.env;
    float M = g[3], R = g[4];
    float rc = fminf(fmaxf(R, 0.f), 1.f);
    float lev = rc * (float)(env.levels - 1);
    int l0 = min((int)floorf(lev), env.levels - 1);
    int l1 = min(l0 + 1, env.levels - 1);
    float fl = lev - (float)l0;
    uint32_t off0 = 0, off1 = 0;
    int r0 = env.spec_res, r1 = env.spec_res;
    {
        uint32_t off = 0;
        for (int l = 0; l < env.levels; l++) {
            int rl = max(env.spec_res >> l, 1);
            if (l == l0) { off0 = off; r0 = rl; }
            if (l == l1) { off1 = off; r1 = rl; }
            off += 6u * rl * rl;
        }
    }
    float xl = fminf(fmaxf(ndv, 0.f), 1.f);
    float2 ab = lut_sample(env.lut, env.lut_res, xl, rc);
    const float ipi = 1.0f / 3.14159265358979323846f;
    float kd = (1.f - M) * ipi;
    float dE[3], dP0[3], dP1[3];
    float dCv[3] = {dC.x, dC.y, dC.z};
    const float vis = a.vis ? a.vis[gid] : 1.0f;
    for (int c = 0; c < 3; c++) {
        float F0 = 0.04f * (1.f - M) + g[c] * M;
        float dLp = dCv[c] * vis * (F0 * ab.x + ab.y);
        dE[c] = dCv[c] * g[c] * kd;
        dP0[c] = dLp * (1.f - fl);
        dP1[c] = dLp * fl;
    }
    uint32_t k[4];
    float w[4];
    float X, Y;
    int face = cube_coords(Nh[0], Nh[1], Nh[2], env.irr_res, X, Y);
    cube_taps(env.irr_res, face, X, Y, 0u, k, w);
    for (int q = 0; q < 4; q++) {
        ko[q] = k[q];
        vo[q] = make_float4(w[q] * dE[0], w[q] * dE[1], w[q] * dE[2], 0.f);
    }
    uint32_t sbase = (uint32_t)a.n_irr;
    face = cube_coords(wr[0], wr[1], wr[2], r0, X, Y);
    cube_taps(r0, face, X, Y, sbase + off0, k, w);
    for (int q = 0; q < 4; q++) {
        ko[4 + q] = k[q];
        vo[4 + q] = make_float4(w[q] * dP0[0], w[q] * dP0[1], w[q] * dP0[2], 0.f);
    }
    face = cube_coords(wr[0], wr[1], wr[2], r1, X, Y);
    cube_taps(r1, face, X, Y, sbase + off1, k, w);
    for (int q = 0; q < 4; q++) {
        ko[8 + q] = k[q];
        vo[8 + q] = make_float4(w[q] * dP1[0], w[q] * dP1[1], w[q] * dP1[2], 0.f);
    }
}

// Per block of 256 sorted records: a segmented inclusive scan (Hillis-Steele, fixed shape)
// leaves at the last record of each run the run's sum inside the block, stored as piece
// first + (run id - run id of the block's first record). run_id[i] = run of sorted record i.
__global__ __launch_bounds__(kEnvBlock) void k_env_block_sums(const uint32_t* __restrict__ keys,
                                                              const int32_t* __restrict__ order,
                                                              const float4* __restrict__ vals,
                                                              const int32_t* __restrict__ run_id,
                                                              int64_t m, float4* __restrict__ pieces) {
    __shared__ float4 sv[kEnvBlock];
    __shared__ uint32_t sk[kEnvBlock];
    int t = threadIdx.x;
    int64_t first = (int64_t)blockIdx.x * kEnvBlock;
    int64_t i = first + t;
    uint32_t key = i < m ? keys[i] : kNoKey;
    float4 x = i < m ? vals[order[i]] : make_float4(0.f, 0.f, 0.f, 0.f);
    sk[t] = key;
    sv[t] = x;
    __syncthreads();
    for (int o = 1; o < kEnvBlock; o <<= 1) {
        float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
        bool take = t >= o && sk[t - o] == key;
        if (take) y = sv[t - o];
        __syncthreads();
        if (take) { x.x = y.x + x.x; x.y = y.y + x.y; x.z = y.z + x.z; }
        sv[t] = x;
        __syncthreads();
    }
    bool last = i < m && (t == kEnvBlock - 1 || i + 1 >= m || sk[t + 1] != key);
    if (last) pieces[first + (run_id[i] - run_id[first])] = x;
}

// A sorted record starts a run when its key differs from the one before it; an inclusive scan
// of these flags minus one is the run id of every record.
__device__ inline int run_start(const uint32_t* __restrict__ keys, int64_t i) {
    return (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// Inclusive scan of the run-start flags, taken from the sorted keys (1024 per block: block
// totals, a one-block scan of those, then each block's scan plus its offset), minus one: run
// ids.
constexpr int kEnvScanPer = 4;
constexpr int kEnvScanBlock = 256 * kEnvScanPer;

__device__ inline int block_excl_scan_i32(int x, int* sh, int* total) {
    int tid = threadIdx.x;
    sh[tid] = x;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int y = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += y;
        __syncthreads();
    }
    int incl = sh[tid];
    if (total) *total = sh[255];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(256) void k_env_scan_sums(const uint32_t* __restrict__ keys,
                                                       int64_t m, int32_t* __restrict__ bsum) {
    __shared__ int sh[256];
    int64_t i0 = (int64_t)blockIdx.x * kEnvScanBlock + threadIdx.x * kEnvScanPer;
    int s = 0;
    for (int k = 0; k < kEnvScanPer; k++)
        if (i0 + k < m) s += run_start(keys, i0 + k);
    int tot;
    block_excl_scan_i32(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the nb block totals in place by one block, in tiles of kEnvScanBlock
// (4 consecutive totals per thread, so each tile's loads coalesce) with a running carry; the
// next tile is loaded before the current one is scanned.
__global__ __launch_bounds__(256) void k_env_scan_bsums(int32_t* __restrict__ bsum, int nb) {
    __shared__ int sh[256];
    int carry = 0;
    int i0 = threadIdx.x * kEnvScanPer;
    int x[kEnvScanPer];
    for (int k = 0; k < kEnvScanPer; k++) x[k] = i0 + k < nb ? bsum[i0 + k] : 0;
    for (int base = 0; base < nb; base += kEnvScanBlock) {
        int j0 = i0 + kEnvScanBlock, nx[kEnvScanPer], s = 0;
        for (int k = 0; k < kEnvScanPer; k++) {
            nx[k] = j0 + k < nb ? bsum[j0 + k] : 0;
            s += x[k];
        }
        int tot;
        int run = carry + block_excl_scan_i32(s, sh, &tot);
        for (int k = 0; k < kEnvScanPer; k++)
            if (i0 + k < nb) {
                bsum[i0 + k] = run;
                run += x[k];
            }
        carry += tot;
        i0 = j0;
        for (int k = 0; k < kEnvScanPer; k++) x[k] = nx[k];
    }
}

__global__ __launch_bounds__(256) void k_env_scan_apply(const uint32_t* __restrict__ keys,
                                                        int32_t* __restrict__ f, int64_t m,
                                                        const int32_t* __restrict__ bsum) {
    __shared__ int sh[256];
    int64_t i0 = (int64_t)blockIdx.x * kEnvScanBlock + threadIdx.x * kEnvScanPer;
    int x[kEnvScanPer];
    int s = 0;
    for (int k = 0; k < kEnvScanPer; k++) {
        x[k] = i0 + k < m ? run_start(keys, i0 + k) : 0;
        s += x[k];
    }
    int run = block_excl_scan_i32(s, sh, nullptr) + bsum[blockIdx.x];
    for (int k = 0; k < kEnvScanPer; k++)
        if (i0 + k < m) {
            run += x[k];
            f[i0 + k] = run - 1;   // inclusive count minus one = run id
        }
}

// One thread per sorted record; the run's first record adds the run's pieces in block order
// and writes the texel's gradient.
__global__ __launch_bounds__(256) void k_env_texel_sums(const uint32_t* __restrict__ keys,
                                                        const int32_t* __restrict__ run_id,
                                                        const float4* __restrict__ pieces,
                                                        int64_t m, uint32_t n_irr, uint32_t n_spec,
                                                        float beta, float4* __restrict__ d_irr,
                                                        float4* __restrict__ d_spec) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    uint32_t key = keys[s];
    if (key == kNoKey) return;
    if (s > 0 && keys[s - 1] == key) return;          // not the first record of its run
    int g = run_id[s];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t first = (s / kEnvBlock) * kEnvBlock;; first += kEnvBlock) {
        float4 p = pieces[first + (g - run_id[first])];
        acc.x += p.x; acc.y += p.y; acc.z += p.z;
        int64_t next = first + kEnvBlock;              // does the run reach the next block?
        if (next >= m || keys[next] != key) break;
    }
    float4* dst;
    if (key < n_irr) dst = d_irr + key;
    else if (key - n_irr < n_spec) dst = d_spec + (key - n_irr);
    else return;
    if (beta != 0.f) {
        float4 o = *dst;
        acc.x += beta * o.x; acc.y += beta * o.y; acc.z += beta * o.z;
    }
    *dst = make_float4(acc.x, acc.y, acc.z, 0.f);
}

__global__ __launch_bounds__(256) void k_env_clear(float4* __restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

struct EnvBwdLayout {
    int64_t m;               // records
    int nblk_sort, nb_scan;
    size_t off_keys, off_vals, off_ka, off_kb, off_va, off_order, off_hist, off_stmp, off_run,
        off_bsum, off_pieces, total;
};

inline EnvBwdLayout env_bwd_layout(int V, int W, int H) {
    EnvBwdLayout L;
    L.m = (int64_t)V * W * H * kEnvRec;
    size_t m = (size_t)(L.m > 0 ? L.m : 1);
    L.nblk_sort = (int)((m + kSortItems - 1) / kSortItems);
    L.nb_scan = (int)((m + kEnvScanBlock - 1) / kEnvScanBlock);
    size_t off = 0;
    L.off_keys = off; off = align256(off + m * 4);
    L.off_vals = off; off = align256(off + m * 16);
    L.off_ka = off; off = align256(off + m * 4);
    L.off_kb = off; off = align256(off + m * 4);
    L.off_va = off; off = align256(off + m * 4);
    L.off_order = off; off = align256(off + m * 4);
    L.off_hist = off; off = align256(off + (size_t)kSortBuckets * L.nblk_sort * 4);
    L.off_stmp = off;
    off = align256(off + (size_t)sort_scan_tmp_entries((int)(m < 0x7FFFFFFF ? m : 0x7FFFFFFF)) * 4);
    L.off_run = off; off = align256(off + m * 4);
    L.off_bsum = off; off = align256(off + (size_t)(L.nb_scan + 1) * 4);
    L.off_pieces = off; off = align256(off + m * 16);
    L.total = off;
    return L;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_env_bwd_workspace(int32_t n_views, int32_t width, int32_t height,
                                    size_t* bytes) {
    if (!bytes || n_views < 1 || width < 1 || height < 1) {
        set_error("ts_env_bwd_workspace: bad argument");
        return TS_E_ARG;
    }
    *bytes = env_bwd_layout(n_views, width, height).total;
    return TS_OK;
}

extern "C" int ts_env_bwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                          const ts_env* env, const float* gbuf, const float* t_final,
                          const float* d_rgba, const float* vis, void* ws, size_t ws_bytes,
                          float beta, float* d_irr, float* d_spec, hipStream_t stream) {
    // texels no record reaches are left as they are, so only these two modes are exact
    if (beta != 0.f && beta != 1.f) {
        set_error("ts_env_bwd: beta must be 0 (overwrite) or 1 (accumulate), got %g", (double)beta);
        return TS_E_ARG;
    }
    if (n_views < 1 || width < 1 || height < 1 || !cams || !env || !gbuf || !t_final ||
        !d_rgba || !d_irr || !d_spec || !env->spec || !env->irr || !env->lut ||
        env->spec_levels < 1 || env->spec_res < 1 || env->irr_res < 1 || env->lut_res < 1) {
        set_error("ts_env_bwd: bad argument");
        return TS_E_ARG;
    }
    EnvBwdLayout L = env_bwd_layout(n_views, width, height);
    if (L.m > 0x7FFFFFFFLL) {
        set_error("ts_env_bwd: %lld records exceed 2^31-1", (long long)L.m);
        return TS_E_ARG;
    }
    if (!ws || ws_bytes < L.total) {
        set_error("ts_env_bwd: workspace %zu < %zu bytes", ws_bytes, L.total);
        return TS_E_WORKSPACE;
    }
    int64_t n_irr = 6LL * env->irr_res * env->irr_res, n_spec = 0;
    for (int l = 0; l < env->spec_levels; l++) {
        int64_t rl = max(env->spec_res >> l, 1);
        n_spec += 6 * rl * rl;
    }
    if (n_irr + n_spec >= (int64_t)kNoKey) {
        set_error("ts_env_bwd: tables too large");
        return TS_E_ARG;
    }
    char* w = (char*)ws;
    uint32_t* keys = (uint32_t*)(w + L.off_keys);
    float4* vals = (float4*)(w + L.off_vals);
    uint32_t* ka = (uint32_t*)(w + L.off_ka);
    uint32_t* kb = (uint32_t*)(w + L.off_kb);
    int32_t* va = (int32_t*)(w + L.off_va);
    int32_t* order = (int32_t*)(w + L.off_order);
    uint32_t* hist = (uint32_t*)(w + L.off_hist);
    int32_t* run = (int32_t*)(w + L.off_run);
    int32_t* bsum = (int32_t*)(w + L.off_bsum);
    float4* pieces = (float4*)(w + L.off_pieces);
    if (beta == 0.f) {
        hipLaunchKernelGGL(k_env_clear, dim3((unsigned)((n_irr + 255) / 256)), dim3(256), 0,
                           stream, (float4*)d_irr, n_irr);
        hipLaunchKernelGGL(k_env_clear, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0,
                           stream, (float4*)d_spec, n_spec);
    }
    EnvBwdArgs a;
    a.V = n_views; a.W = width; a.H = height; a.cams = cams;
    a.env.spec = (const float4*)env->spec; a.env.irr = (const float4*)env->irr;
    a.env.lut = (const float2*)env->lut; a.env.spec_res = env->spec_res;
    a.env.levels = env->spec_levels; a.env.irr_res = env->irr_res; a.env.lut_res = env->lut_res;
    a.gbuf = gbuf; a.t_final = t_final; a.d_rgba = (const float4*)d_rgba; a.vis = vis;
    a.keys = keys; a.vals = vals; a.n_irr = (int)n_irr;
    int64_t P = (int64_t)n_views * width * height;
    hipLaunchKernelGGL(k_env_records, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, a);
    int m = (int)L.m;
    // Texel keys are below n_irr + n_spec, so only the digits that span that range are sorted;
    // the unused records' key (all ones) is above every texel key in those low bits too, so
    // they still sort last. Sorted keys land in kb, the record order in `order`.
    int passes = 1;
    while (passes < kSortPasses && (n_irr + n_spec) >= (1LL << (kSortRadixBits * passes))) passes++;
    radix_sort_indices(keys, m, 1, ka, kb, va, hist, order, stream,
                       (uint32_t*)(w + L.off_stmp), passes);
    unsigned g256 = (unsigned)((L.m + 255) / 256);
    hipLaunchKernelGGL(k_env_scan_sums, dim3(L.nb_scan), dim3(256), 0, stream, kb, L.m, bsum);
    hipLaunchKernelGGL(k_env_scan_bsums, dim3(1), dim3(256), 0, stream, bsum, L.nb_scan);
    hipLaunchKernelGGL(k_env_scan_apply, dim3(L.nb_scan), dim3(256), 0, stream, kb, run, L.m,
                       bsum);
    hipLaunchKernelGGL(k_env_block_sums, dim3((unsigned)((L.m + kEnvBlock - 1) / kEnvBlock)),
                       dim3(kEnvBlock), 0, stream, kb, order, vals, run, L.m, pieces);
    hipLaunchKernelGGL(k_env_texel_sums, dim3(g256), dim3(256), 0, stream, kb, run, pieces, L.m,
                       (uint32_t)n_irr, (uint32_t)n_spec, beta, (float4*)d_irr, (float4*)d_spec);
    return launch_check("ts_env_bwd");
}

// ts_env_bwd: gradients of a loss on the shaded RGBA with respect to the texels of the
// environment's shading tables — the diffuse irradiance cube and every prefiltered specular
// level — taken as learnable parameters (the environment is optimised end to end with the
// splats, Sec. 3.5-3.6; Eq. 11-12 read the tables through bilinear cube lookups).
//
// The shaded colour is linear in each table texel: per pixel, dL/dE = dL/dC * albedo (1-M)/pi
// at the irradiance lookup of N, and dL/dL_pref = dL/dC * V (F0 A + B) split between the two
// levels around R (L-1) at the lookup of the reflected direction (V the pixel's visibility:
// with the indirect term the specular radiance is V L_pref + (1 - V) L_ind, Eq. 12). Each lookup spreads its
// gradient over 4 texels with the bilinear weights: 12 (texel, rgb) contributions per pixel.
//
// Summed in 64-bit fixed point, so the result does not depend on the order of the additions
// and integer atomics can do them:
//  1. k_env_max: the largest |contribution| M of the call (an integer max over float bits).
//  2. k_env_accum: one workgroup per 16x16 pixels; each contribution x becomes
//     q = round(x 2^(61-b-e)), e = the exponent with M < 2^e and b = the bits of the record
//     count, so that every partial sum stays below 2^61 in magnitude; the workgroup adds its q
//     per texel in an LDS hash table (integer atomics; a texel that finds no slot within a few
//     probes goes straight to the global table) and then adds the table into one of up to 16
//     copies of the global accumulators.
//  3. k_env_finish: per texel, the copies' sum x 2^-(61-b-e) in double, rounded to float.
// A contribution is rounded by at most 2^(e+b-62), M 2^(b-61) relative to the largest one.
#include "shade.h"
#include "ts_internal.h"

namespace ts {

constexpr int kEnvRec = 12;           // contributions per pixel
constexpr int kEnvTile = 16;          // pixels a side of one k_env_accum workgroup
constexpr int kEnvSlots = 1024;       // LDS hash slots per workgroup
constexpr int kEnvProbes = 8;         // slots tried before a texel goes to the global table
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
// copies of the global accumulators, workgroup g adding into copy g % copies: the integer
// atomics on a texel that most workgroups reach (the irradiance cube's) are spread over up to
// 16 addresses instead of queueing on one; as many copies as fit 64 MB (at least one), so
// large tables do not pay for clearing and reading back copies they hardly need
constexpr int kEnvCopies = 16;
constexpr int64_t kEnvCopyBudget = 64ll << 20;
inline int env_copies(int64_t n_tex) {
    const int64_t per = n_tex * 3 * (int64_t)sizeof(unsigned long long);
    return (int)max((int64_t)1, min((int64_t)kEnvCopies, kEnvCopyBudget / max(per, (int64_t)1)));
}

struct EnvBwdArgs {
    int V, W, H, tiles_x, tiles_per_view;
    const ts_camera* cams;
    EnvDev env;
    const float* gbuf;       // [V][8][H][W]
    const float* t_final;    // [V][H][W]
    const float4* d_rgba;    // [V][H][W]
    const float* vis;        // [V][H][W] visibility or null (V = 1)
    uint32_t n_irr;          // texels of the irradiance cube (6 r^2)
    int bits;                // b: contributions of the call < 2^b
    unsigned long long* acc; // [copies][n_irr + n_spec][3] fixed-point sums
    int64_t n_acc;           // (n_irr + n_spec) * 3: the stride between copies
    int copies;              // env_copies(n_irr + n_spec)
    uint32_t* words;         // [0] bits of M, [1] non-finite contribution seen
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

// The pixel of thread `tid` in workgroup `blk` (16x16 pixels of one view): false outside the
// frame.
__device__ inline bool env_pixel(const EnvBwdArgs& a, int blk, int tid, int& v, int& x, int& y) {
    v = blk / a.tiles_per_view;
    int t = blk - v * a.tiles_per_view;
    int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    x = tx * kEnvTile + (tid % kEnvTile);
    y = ty * kEnvTile + (tid / kEnvTile);
    return x < a.W && y < a.H;
}

// The 12 (texel key, rgb) contributions of pixel (v, x, y) to the tables; false for an empty
// pixel (background only: no table read).
__device__ inline bool env_contributions(const EnvBwdArgs& a, int v, int x, int y, uint32_t* ko,
                                         float (*vo)[3]) {
    int64_t plane = (int64_t)a.H * a.W;
    int64_t pix = (int64_t)y * a.W + x;
    int64_t gid = (int64_t)v * plane + pix;
    float Tf = a.t_final[gid];
    if (!(Tf < 1.0f)) return false;
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
        for (int c = 0; c < 3; c++) vo[q][c] = w[q] * dE[c];
    }
    uint32_t sbase = a.n_irr;
    face = cube_coords(wr[0], wr[1], wr[2], r0, X, Y);
    cube_taps(r0, face, X, Y, sbase + off0, k, w);
    for (int q = 0; q < 4; q++) {
        ko[4 + q] = k[q];
        for (int c = 0; c < 3; c++) vo[4 + q][c] = w[q] * dP0[c];
    }
    face = cube_coords(wr[0], wr[1], wr[2], r1, X, Y);
    cube_taps(r1, face, X, Y, sbase + off1, k, w);
    for (int q = 0; q < 4; q++) {
        ko[8 + q] = k[q];
        for (int c = 0; c < 3; c++) vo[8 + q][c] = w[q] * dP1[c];
    }
    return true;
}

// The fixed-point scale 2^(61-b-e) of the call (e: M < 2^e), from the bits of M.
__device__ inline double env_scale(const EnvBwdArgs& a) {
    const float M = __uint_as_float(a.words[0]);
    const int e = M > 0.f ? ilogbf(M) + 1 : 0;
    return ldexp(1.0, 61 - a.bits - e);
}

__global__ __launch_bounds__(256) void k_env_clear_acc(unsigned long long* __restrict__ acc,
                                                       int64_t n, uint32_t* __restrict__ words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) acc[i] = 0ull;
    if (i < 2) words[i] = 0u;
}

// Pass 1: M = max |contribution| (float bits of non-negative values order like the values), and
// whether any contribution is not finite.
__global__ __launch_bounds__(256) void k_env_max(EnvBwdArgs a) {
    int v, x, y;
    float m = 0.f;
    bool bad = false;
    if (env_pixel(a, blockIdx.x, threadIdx.x, v, x, y)) {
        uint32_t ko[kEnvRec];
        float vo[kEnvRec][3];
        if (env_contributions(a, v, x, y, ko, vo)) {
            for (int q = 0; q < kEnvRec; q++)
                for (int c = 0; c < 3; c++) {
                    float t = fabsf(vo[q][c]);
                    bad |= !(t <= 3.402823466e38f);
                    m = fmaxf(m, t);
                }
        }
    }
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float wm[4];
    __shared__ int wb[4];
    const int w = threadIdx.x >> 6;
    const bool anybad = __ballot(bad) != 0;
    if ((threadIdx.x & 63) == 0) {
        wm[w] = m;
        wb[w] = anybad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float bm = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        // one atomic per workgroup, and only while it can raise the maximum (a stale read
        // costs an atomic, never a wrong result)
        const uint32_t cur = *(volatile uint32_t*)&a.words[0];
        if (bm > 0.f && __float_as_uint(bm) > cur) atomicMax(&a.words[0], __float_as_uint(bm));
        if (wb[0] | wb[1] | wb[2] | wb[3]) atomicOr(&a.words[1], 1u);
    }
}

// Pass 2: the fixed-point contributions of 16x16 pixels summed per texel in LDS, then added to
// the global accumulators.
__global__ __launch_bounds__(256) void k_env_accum(EnvBwdArgs a) {
    __shared__ uint32_t skey[kEnvSlots];
    __shared__ unsigned long long sacc[kEnvSlots][3];
    const int tid = threadIdx.x;
    for (int i = tid; i < kEnvSlots; i += 256) {
        skey[i] = kNoKey;
        sacc[i][0] = 0ull; sacc[i][1] = 0ull; sacc[i][2] = 0ull;
    }
    __syncthreads();
    unsigned long long* const gacc = a.acc + (int64_t)(blockIdx.x % a.copies) * a.n_acc;
    int v, x, y;
    if (a.words[1] == 0u && env_pixel(a, blockIdx.x, tid, v, x, y)) {
        uint32_t ko[kEnvRec];
        float vo[kEnvRec][3];
        if (env_contributions(a, v, x, y, ko, vo)) {
            const double sc = env_scale(a);
            for (int q = 0; q < kEnvRec; q++) {
                long long qi[3];
                for (int c = 0; c < 3; c++) qi[c] = llrint((double)vo[q][c] * sc);
                if ((qi[0] | qi[1] | qi[2]) == 0) continue;
                const uint32_t key = ko[q];
                uint32_t h = (key * 2654435761u) >> 22;   // 10 bits: kEnvSlots = 1024
                bool placed = false;
                for (int p = 0; p < kEnvProbes; p++) {
                    uint32_t old = atomicCAS(&skey[h], kNoKey, key);
                    if (old == kNoKey || old == key) {
                        for (int c = 0; c < 3; c++)
                            if (qi[c]) atomicAdd(&sacc[h][c], (unsigned long long)qi[c]);
                        placed = true;
                        break;
                    }
                    h = (h + 1) & (kEnvSlots - 1);
                }
                if (!placed) {
                    unsigned long long* g = gacc + (int64_t)key * 3;
                    for (int c = 0; c < 3; c++)
                        if (qi[c]) atomicAdd(g + c, (unsigned long long)qi[c]);
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < kEnvSlots; i += 256) {
        const uint32_t key = skey[i];
        if (key == kNoKey) continue;
        unsigned long long* g = gacc + (int64_t)key * 3;
        for (int c = 0; c < 3; c++)
            if (sacc[i][c]) atomicAdd(g + c, sacc[i][c]);
    }
}

// Pass 3: per texel, the fixed-point sums back to float (overwrite or accumulate); NaN
// everywhere if a contribution was not finite.
__global__ __launch_bounds__(256) void k_env_finish(EnvBwdArgs a, int64_t n_tex, float beta,
                                                    float4* __restrict__ d_irr,
                                                    float4* __restrict__ d_spec) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tex) return;
    float r[3];
    if (a.words[1] != 0u) {
        r[0] = r[1] = r[2] = __builtin_nanf("");
    } else {
        const double inv = 1.0 / env_scale(a);   // a power of two: exact
        for (int c = 0; c < 3; c++) {
            unsigned long long sum = 0ull;
            for (int k = 0; k < a.copies; k++) sum += a.acc[(int64_t)k * a.n_acc + t * 3 + c];
            r[c] = (float)((double)(long long)sum * inv);
        }
    }
    float4* dst = t < (int64_t)a.n_irr ? d_irr + t : d_spec + (t - (int64_t)a.n_irr);
    if (beta != 0.f) {
        float4 o = *dst;
        r[0] += o.x; r[1] += o.y; r[2] += o.z;
    }
    *dst = make_float4(r[0], r[1], r[2], 0.f);
}

// Texels of the environment's tables: the irradiance cube then every specular level.
inline int64_t env_texels(const ts_env& e, int64_t* n_irr_out) {
    int64_t n_irr = 6LL * e.irr_res * e.irr_res, n_spec = 0;
    for (int l = 0; l < e.spec_levels; l++) {
        int64_t rl = max(e.spec_res >> l, 1);
        n_spec += 6 * rl * rl;
    }
    if (n_irr_out) *n_irr_out = n_irr;
    return n_irr + n_spec;
}

// Accumulators (env_copies x 24 bytes per texel, rounded up to 256 bytes) then the two status
// words.
inline size_t env_acc_bytes(int64_t n_tex) {
    return ((size_t)env_copies(n_tex) * n_tex * 3 * sizeof(unsigned long long) + 255) &
           ~(size_t)255;
}
size_t env_bwd_bytes(int64_t n_tex) { return env_acc_bytes(n_tex) + 256; }

}  // namespace ts

using namespace ts;

extern "C" int ts_env_bwd_workspace(const ts_env* env, size_t* bytes) {
    if (!bytes || !env || env->spec_levels < 1 || env->spec_res < 1 || env->irr_res < 1) {
        set_error("ts_env_bwd_workspace: bad argument");
        return TS_E_ARG;
    }
    *bytes = env_bwd_bytes(env_texels(*env, nullptr));
    return TS_OK;
}

extern "C" int ts_env_bwd(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                          const ts_env* env, const float* gbuf, const float* t_final,
                          const float* d_rgba, const float* vis, void* ws, size_t ws_bytes,
                          float beta, float* d_irr, float* d_spec, hipStream_t stream) {
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
    int64_t n_irr = 0;
    const int64_t n_tex = env_texels(*env, &n_irr);
    if (n_tex >= (int64_t)kNoKey) {
        set_error("ts_env_bwd: tables too large");
        return TS_E_ARG;
    }
    const int64_t m = (int64_t)n_views * width * height * kEnvRec;
    if (m > (1LL << 40)) {
        set_error("ts_env_bwd: %lld contributions exceed 2^40", (long long)m);
        return TS_E_ARG;
    }
    const size_t need = env_bwd_bytes(n_tex);
    if (!ws || ws_bytes < need) {
        set_error("ts_env_bwd: workspace %zu < %zu bytes", ws_bytes, need);
        return TS_E_WORKSPACE;
    }
    EnvBwdArgs a;
    a.V = n_views; a.W = width; a.H = height; a.cams = cams;
    a.tiles_x = (width + kEnvTile - 1) / kEnvTile;
    a.tiles_per_view = a.tiles_x * ((height + kEnvTile - 1) / kEnvTile);
    a.env.spec = (const float4*)env->spec; a.env.irr = (const float4*)env->irr;
    a.env.lut = (const float2*)env->lut; a.env.spec_res = env->spec_res;
    a.env.levels = env->spec_levels; a.env.irr_res = env->irr_res; a.env.lut_res = env->lut_res;
    a.gbuf = gbuf; a.t_final = t_final; a.d_rgba = (const float4*)d_rgba; a.vis = vis;
    a.n_irr = (uint32_t)n_irr;
    a.bits = 1;
    while ((1LL << a.bits) <= m) a.bits++;
    a.acc = (unsigned long long*)ws;
    a.words = (uint32_t*)((char*)ws + env_acc_bytes(n_tex));
    a.n_acc = n_tex * 3;
    a.copies = env_copies(n_tex);
    const int64_t n_all = a.n_acc * a.copies;
    hipLaunchKernelGGL(k_env_clear_acc, dim3((unsigned)((n_all + 255) / 256)), dim3(256), 0,
                       stream, a.acc, n_all, a.words);
    const unsigned blocks = (unsigned)((int64_t)a.tiles_per_view * n_views);
    hipLaunchKernelGGL(k_env_max, dim3(blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_env_accum, dim3(blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_env_finish, dim3((unsigned)((n_tex + 255) / 256)), dim3(256), 0, stream,
                       a, n_tex, beta, (float4*)d_irr, (float4*)d_spec);
    return launch_check("ts_env_bwd");
}

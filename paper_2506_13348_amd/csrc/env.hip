// Shading tables, built once per environment (Sec. 3.5.4): the split-sum BRDF lookup, the
// diffuse irradiance cube and the roughness-prefiltered specular levels.
#include <math.h>

#include "ts_internal.h"

namespace ts {

__device__ inline uint32_t bit_reverse32(uint32_t b) { return __builtin_bitreverse32(b); }

// One thread per LUT texel, in double precision: near N.V = 0 the visibility term divides
// by N.V and float32 loses ~1e-4 there, while the table feeds radiances of order 10.
__global__ __launch_bounds__(256) void k_brdf_lut(int n, int samples, float2* __restrict__ lut) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int i = idx % n, j = idx / n;
    double rough = ((double)j + 0.5) / (double)n;
    double nv = ((double)i + 0.5) / (double)n;
    double a = rough * rough;
    double a2 = a * a;
    double kk = 0.5 * a;
    double Vx = sqrt(fmax(0.0, 1.0 - nv * nv)), Vz = nv;
    double g1v = nv / (nv * (1.0 - kk) + kk);
    double A = 0.0, B = 0.0;
    for (int s = 0; s < samples; s++) {
        double xi1 = (double)s / (double)samples;
        double xi2 = (double)bit_reverse32((uint32_t)s) * 2.3283064365386963e-10;
        double phi = 2.0 * 3.14159265358979323846 * xi1;
        double ct = sqrt((1.0 - xi2) / (1.0 + (a2 - 1.0) * xi2));
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double Hx = st * cos(phi), Hz = ct;
        double vh = Vx * Hx + Vz * Hz;
        double Lz = 2.0 * vh * Hz - Vz;
        double nl = fmax(Lz, 0.0), nh = fmax(Hz, 0.0);
        vh = fmax(vh, 0.0);
        if (nl > 0.0) {
            double g1l = nl / (nl * (1.0 - kk) + kk);
            double gvis = g1v * g1l * vh / (nh * nv);
            double om = 1.0 - vh;
            double om2 = om * om;
            double fc = om2 * om2 * om;
            A += (1.0 - fc) * gvis;
            B += fc * gvis;
        }
    }
    lut[idx] = make_float2((float)(A / samples), (float)(B / samples));
}

// Texel-centre directions and exact solid angles of a cube resolution, in double.
__device__ inline double area_elem(double x, double y) { return atan2(x * y, sqrt(x * x + y * y + 1.0)); }

__device__ inline void texel_dir(int f, int i, int j, int r, double* d) {
    double sc = 2.0 * ((double)i + 0.5) / (double)r - 1.0, tc = 2.0 * ((double)j + 0.5) / (double)r - 1.0;
    double x, y, z;
    switch (f) {
        case 0: x = 1.0; y = -tc; z = -sc; break;
        case 1: x = -1.0; y = -tc; z = sc; break;
        case 2: x = sc; y = 1.0; z = tc; break;
        case 3: x = sc; y = -1.0; z = -tc; break;
        case 4: x = sc; y = -tc; z = 1.0; break;
        default: x = -sc; y = -tc; z = -1.0; break;
    }
    double il = 1.0 / sqrt(x * x + y * y + z * z);
    d[0] = x * il; d[1] = y * il; d[2] = z * il;
}

__global__ __launch_bounds__(256) void k_texel_table(int r, double4* __restrict__ out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 6 * r * r) return;
    int f = idx / (r * r), rem = idx % (r * r);
    int j = rem / r, i = rem % r;
    double d[3];
    texel_dir(f, i, j, r, d);
    double x0 = 2.0 * i / r - 1.0, x1 = 2.0 * (i + 1) / r - 1.0;
    double y0 = 2.0 * j / r - 1.0, y1 = 2.0 * (j + 1) / r - 1.0;
    double sa = area_elem(x1, y1) - area_elem(x0, y1) - area_elem(x1, y0) + area_elem(x0, y0);
    out[idx] = make_double4(d[0], d[1], d[2], sa);
}

__global__ __launch_bounds__(256) void k_env_copy(const float* __restrict__ env, int m,
                                                  float4* __restrict__ out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m) return;
    out[idx] = make_float4(env[3 * idx], env[3 * idx + 1], env[3 * idx + 2], 0.f);
}

// One workgroup per output texel: weighted sums over all source texels in double precision,
// then a tree reduction in LDS.
//   mode 0: irradiance, weight (n.w)^+ dOmega, no normalisation
//   mode 1: GGX prefilter with N = V = R, weight (r.w)^+ D(h) dOmega, normalised
template <int kMode>
__global__ __launch_bounds__(256) void k_cube_filter(const double4* __restrict__ texels,
                                                     const float4* __restrict__ src, int nsrc,
                                                     int out_res, double alpha,
                                                     float4* __restrict__ out) {
    __shared__ double red[4][256];
    int o = blockIdx.x, tid = threadIdx.x;
    int f = o / (out_res * out_res), rem = o % (out_res * out_res);
    int j = rem / out_res, i = rem % out_res;
    double n[3];
    texel_dir(f, i, j, out_res, n);
    double a2 = alpha * alpha;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < nsrc; k += 256) {
        double4 tw = texels[k];
        double cs = n[0] * tw.x + n[1] * tw.y + n[2] * tw.z;
        if (cs <= 0.0) continue;
        double wt;
        if (kMode == 0) {
            wt = cs * tw.w;
        } else {
            double hx = n[0] + tw.x, hy = n[1] + tw.y, hz = n[2] + tw.z;
            double hl = sqrt(hx * hx + hy * hy + hz * hz);
            double ndh = (n[0] * hx + n[1] * hy + n[2] * hz) / hl;
            double d = ndh * ndh * (a2 - 1.0) + 1.0;
            wt = cs * (a2 / (3.14159265358979323846 * d * d)) * tw.w;
        }
        float4 L = src[k];
        s[0] += wt * (double)L.x;
        s[1] += wt * (double)L.y;
        s[2] += wt * (double)L.z;
        s[3] += wt;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) red[q][tid] = s[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
#pragma unroll
            for (int q = 0; q < 4; q++) red[q][tid] += red[q][tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (kMode == 0) out[o] = make_float4((float)red[0][0], (float)red[1][0], (float)red[2][0], 0.f);
        else {
            double iw = 1.0 / red[3][0];
            out[o] = make_float4((float)(red[0][0] * iw), (float)(red[1][0] * iw),
                                 (float)(red[2][0] * iw), 0.f);
        }
    }
}

}  // namespace ts

using namespace ts;

extern "C" int ts_brdf_lut(int32_t n, int32_t samples, float* lut, hipStream_t stream) {
    if (n < 1 || samples < 1 || !lut) {
        set_error("ts_brdf_lut: bad argument");
        return TS_E_ARG;
    }
    int m = n * n;
    hipLaunchKernelGGL(k_brdf_lut, dim3((m + 255) / 256), dim3(256), 0, stream, n, samples,
                       (float2*)lut);
    return launch_check("ts_brdf_lut");
}

extern "C" int ts_env_tables(const float* env, int32_t r, int32_t levels, int32_t irr_res,
                             float* spec, float* irr, void* texel_ws, hipStream_t stream) {
    if (!env || !spec || !irr || !texel_ws || r < 1 || levels < 1 || irr_res < 1) {
        set_error("ts_env_tables: bad argument");
        return TS_E_ARG;
    }
    int nsrc = 6 * r * r;
    double4* tex = (double4*)texel_ws;
    float4* s0 = (float4*)spec;
    hipLaunchKernelGGL(k_texel_table, dim3((nsrc + 255) / 256), dim3(256), 0, stream, r, tex);
    hipLaunchKernelGGL(k_env_copy, dim3((nsrc + 255) / 256), dim3(256), 0, stream, env, nsrc, s0);
    size_t off = (size_t)nsrc;
    for (int l = 1; l < levels; l++) {
        int rl = r >> l;
        if (rl < 1) rl = 1;
        double rough = (double)l / (double)(levels - 1);
        hipLaunchKernelGGL(k_cube_filter<1>, dim3(6 * rl * rl), dim3(256), 0, stream, (const double4*)tex,
                           (const float4*)s0, nsrc, rl, rough * rough, s0 + off);
        off += (size_t)6 * rl * rl;
    }
    hipLaunchKernelGGL(k_cube_filter<0>, dim3(6 * irr_res * irr_res), dim3(256), 0, stream,
                       (const double4*)tex, (const float4*)s0, nsrc, irr_res, 0.0, (float4*)irr);
    return launch_check("ts_env_tables");
}

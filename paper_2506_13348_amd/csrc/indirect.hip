// ts_indirect_eval: per (view, splat) indirect radiance l_ind from per-splat spherical
// harmonics (Sec. 3.5-3.6: the indirect light of Eq. 12 is encoded per primitive with SH and
// blended as a G-buffer map by Eq. 9).
//
// For splat k and camera c: d = unit direction from the camera centre to the splat centre,
// n = splat normal (third column of R(q)), w_r = d - 2 (d.n) n the mirror reflection of the
// view ray about the splat plane (unchanged when n flips), and per colour channel
//   l_ind = max(0, sum_j c_kj Y_j(w_r)),
// Y_j the real orthonormal SH basis (no Condon-Shortley phase, index l*l + l + m, degree <= 3)
// written out as polynomials of the unit vector. A workgroup takes 64 splats (one per lane)
// and 16 views (4 per wave): the 64 splats' coefficients are staged in LDS with coalesced
// loads, each lane keeps its splat's coefficients in registers and evaluates its views; the
// output rows [view][splat] are written 64 splats at a time. The arithmetic is float32 (unit
// vectors and O(1) coefficients: the result is within a few ulp of the sum of |c_j Y_j|;
// double precision took 1.7x as long).
#include <math.h>

#include "ts_internal.h"

namespace ts {

struct IndArgs {
    int V, n;
    const ts_camera* cams;
    const float* means;
    const float* quats;
    const float* sh;     // [n][K][3]
    float4* lind;        // [V][n]
};

// Real SH basis up to degree D at the unit vector (x, y, z).
template <int D>
__device__ inline void sh_basis_f(float x, float y, float z, float* Y) {
    Y[0] = 0.28209479177387814f;                      // 1 / (2 sqrt(pi))
    if (D < 1) return;
    const float c1 = 0.48860251190291992f;            // sqrt(3 / (4 pi))
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    if (D < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * x * y;               // sqrt(15/pi) / 2
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);  // sqrt(5/pi) / 4
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.54627421529603959f * (xx - yy);          // sqrt(15/pi) / 4
    if (D < 3) return;
    Y[9] = 0.59004358992664352f * y * (3.0f * xx - yy);   // sqrt(35/(2 pi)) / 4
    Y[10] = 2.8906114426405538f * x * y * z;              // sqrt(105/pi) / 2
    Y[11] = 0.45704579946446572f * y * (5.0f * zz - 1.0f);  // sqrt(21/(2 pi)) / 4
    Y[12] = 0.37317633259011540f * z * (5.0f * zz - 3.0f);  // sqrt(7/pi) / 4
    Y[13] = 0.45704579946446572f * x * (5.0f * zz - 1.0f);
    Y[14] = 1.4453057213202769f * z * (xx - yy);          // sqrt(105/pi) / 4
    Y[15] = 0.59004358992664352f * x * (xx - 3.0f * yy);
}

constexpr int kIndSplats = 64;          // splats per workgroup (one per lane)
constexpr int kIndViewsPerWave = 4;
constexpr int kIndViews = 4 * kIndViewsPerWave;   // views per workgroup (4 waves)

template <int D>
__global__ __launch_bounds__(256) void k_indirect_eval(IndArgs a) {
    constexpr int K = (D + 1) * (D + 1);
    constexpr int kStride = 3 * K + 1;
    __shared__ float sc[kIndSplats * kStride];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k0 = blockIdx.x * kIndSplats;
    const int nk = min(kIndSplats, a.n - k0);
    const float* src = a.sh + (int64_t)k0 * K * 3;
    for (int i = threadIdx.x; i < nk * 3 * K; i += blockDim.x) {
        int s = i / (3 * K), j = i - s * (3 * K);
        sc[s * kStride + j] = src[i];
    }
    __syncthreads();
    const int k = k0 + lane;
    const int v0 = blockIdx.y * kIndViews + wv;
    if (lane >= nk || v0 >= a.V) return;
    float c[K * 3];
#pragma unroll
    for (int j = 0; j < K * 3; j++) c[j] = sc[lane * kStride + j];
    float q0 = a.quats[4 * k + 0], q1 = a.quats[4 * k + 1], q2 = a.quats[4 * k + 2], q3 = a.quats[4 * k + 3];
    float qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    float s = qq > 0.f ? 2.f / qq : 0.f;
    float nx = s * (q1 * q3 + q0 * q2), ny = s * (q2 * q3 - q0 * q1), nz = 1.f - s * (q1 * q1 + q2 * q2);
    const float mx = a.means[3 * k + 0], my = a.means[3 * k + 1], mz = a.means[3 * k + 2];
    for (int i = 0; i < kIndViewsPerWave; i++) {
        const int v = v0 + 4 * i;
        if (v >= a.V) break;
        const float* w = a.cams[v].w2c;
        float ox = -(w[0] * w[3] + w[4] * w[7] + w[8] * w[11]);
        float oy = -(w[1] * w[3] + w[5] * w[7] + w[9] * w[11]);
        float oz = -(w[2] * w[3] + w[6] * w[7] + w[10] * w[11]);
        float dx = mx - ox, dy = my - oy, dz = mz - oz;
        float dd = dx * dx + dy * dy + dz * dz;
        float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
        if (qq > 0.f && dd > 0.f) {
            float idl = rsqrtf(dd);
            dx *= idl; dy *= idl; dz *= idl;
            float dn = dx * nx + dy * ny + dz * nz;
            float rx = dx - 2.f * dn * nx, ry = dy - 2.f * dn * ny, rz = dz - 2.f * dn * nz;
            float irl = rsqrtf(rx * rx + ry * ry + rz * rz);
            rx *= irl; ry *= irl; rz *= irl;
            float Y[K];
            sh_basis_f<D>(rx, ry, rz, Y);
            float r = 0.f, g = 0.f, b = 0.f;
#pragma unroll
            for (int j = 0; j < K; j++) {
                r = fmaf(c[3 * j + 0], Y[j], r);
                g = fmaf(c[3 * j + 1], Y[j], g);
                b = fmaf(c[3 * j + 2], Y[j], b);
            }
            out = make_float4(fmaxf(r, 0.f), fmaxf(g, 0.f), fmaxf(b, 0.f), 0.f);
        }
        a.lind[(int64_t)v * a.n + k] = out;
    }
}

}  // namespace ts

using namespace ts;

extern "C" int ts_indirect_eval(int32_t n_views, const ts_camera* cams, int32_t n,
                                const float* means, const float* quats, const float* sh,
                                int32_t sh_degree, float* lind, hipStream_t stream) {
    if (n_views < 1 || n < 0 || !cams || sh_degree < 0 || sh_degree > 3) {
        set_error("ts_indirect_eval: bad argument (views=%d n=%d degree=%d)", n_views, n,
                  sh_degree);
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    if (!means || !quats || !sh || !lind) {
        set_error("ts_indirect_eval: null array");
        return TS_E_ARG;
    }
    if ((int64_t)n_views * n > 0x7FFFFFFFLL) {
        set_error("ts_indirect_eval: n_views * n above 2^31-1");
        return TS_E_ARG;
    }
    IndArgs a;
    a.V = n_views; a.n = n; a.cams = cams; a.means = means; a.quats = quats; a.sh = sh;
    a.lind = (float4*)lind;
    dim3 grid((unsigned)((n + kIndSplats - 1) / kIndSplats),
              (unsigned)((n_views + kIndViews - 1) / kIndViews)),
        block(256);
    switch (sh_degree) {
        case 0: hipLaunchKernelGGL(k_indirect_eval<0>, grid, block, 0, stream, a); break;
        case 1: hipLaunchKernelGGL(k_indirect_eval<1>, grid, block, 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_indirect_eval<2>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_indirect_eval<3>, grid, block, 0, stream, a); break;
    }
    return launch_check("ts_indirect_eval");
}

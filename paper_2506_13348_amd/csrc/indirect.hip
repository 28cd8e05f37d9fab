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
// and 64 views (16 per wave): the 64 splats' coefficients are staged in LDS with coalesced
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
// 16 views per wave: the staged coefficients and the per-splat set-up serve 64 views (measured
// back to back on 64 views x 100k splats at degree 3: 29 us, against 37 us with 4 views per
// wave and 82 us with 1)
constexpr int kIndViewsPerWave = 16;
constexpr int kIndViews = 4 * kIndViewsPerWave;   // views per workgroup (4 waves)

template <int D>
__global__ __launch_bounds__(256) void k_indirect_eval(IndArgs a) {
    constexpr int K = (D + 1) * (D + 1);
    // a splat's 3K coefficients as whole float4 rows; an odd number of float4 per splat keeps
    // the lanes' 16-byte reads on distinct banks
    constexpr int kC4 = (3 * K + 3) / 4;
    constexpr int kStride = 4 * (kC4 % 2 ? kC4 : kC4 + 1);
    __shared__ __align__(16) float sc[kIndSplats * kStride];
    __shared__ float so[kIndViews * 3];   // camera centres of the workgroup's views
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k0 = blockIdx.x * kIndSplats;
    const int nk = min(kIndSplats, a.n - k0);
    const float* src = a.sh + (int64_t)k0 * K * 3;
    for (int i = threadIdx.x; i < nk * 3 * K; i += blockDim.x) {
        int s = i / (3 * K), j = i - s * (3 * K);
        sc[s * kStride + j] = src[i];
    }
    if (threadIdx.x < kIndViews && (int)(blockIdx.y * kIndViews + threadIdx.x) < a.V) {
        // o = -R^T t of the world-to-camera transform [R | t]
        const float* w = a.cams[blockIdx.y * kIndViews + threadIdx.x].w2c;
        so[3 * threadIdx.x + 0] = -(w[0] * w[3] + w[4] * w[7] + w[8] * w[11]);
        so[3 * threadIdx.x + 1] = -(w[1] * w[3] + w[5] * w[7] + w[9] * w[11]);
        so[3 * threadIdx.x + 2] = -(w[2] * w[3] + w[6] * w[7] + w[10] * w[11]);
    }
    __syncthreads();
    const int k = k0 + lane;
    const int v0 = blockIdx.y * kIndViews + wv;
    if (lane >= nk || v0 >= a.V) return;
    float c[kC4 * 4];
#pragma unroll
    for (int j = 0; j < kC4; j++) {
        float4 q = *(const float4*)(sc + lane * kStride + 4 * j);
        c[4 * j] = q.x; c[4 * j + 1] = q.y; c[4 * j + 2] = q.z; c[4 * j + 3] = q.w;
    }
    float q0 = a.quats[4 * k + 0], q1 = a.quats[4 * k + 1], q2 = a.quats[4 * k + 2], q3 = a.quats[4 * k + 3];
    float qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    float s = qq > 0.f ? 2.f / qq : 0.f;
    float nx = s * (q1 * q3 + q0 * q2), ny = s * (q2 * q3 - q0 * q1), nz = 1.f - s * (q1 * q1 + q2 * q2);
    const float mx = a.means[3 * k + 0], my = a.means[3 * k + 1], mz = a.means[3 * k + 2];
    for (int i = 0; i < kIndViewsPerWave; i++) {
        const int v = v0 + 4 * i;
        if (v >= a.V) break;
        const float* o = so + 3 * (wv + 4 * i);
        float dx = mx - o[0], dy = my - o[1], dz = mz - o[2];
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

// dL/dw at the unit vector w = (x, y, z) of L = sum_j dY[j] Y_j(w), from the Cartesian
// gradients of the basis polynomials (the normalisation of w projects out the radial part).
template <int D>
__device__ inline void sh_basis_grad_f(float x, float y, float z, const float* dY, float* dw) {
    dw[0] = 0.f; dw[1] = 0.f; dw[2] = 0.f;
    if (D < 1) return;
    const float c1 = 0.48860251190291992f;
    dw[1] += c1 * dY[1];
    dw[2] += c1 * dY[2];
    dw[0] += c1 * dY[3];
    if (D < 2) return;
    const float a2 = 1.0925484305920792f, b2 = 0.31539156525252005f, e2 = 0.54627421529603959f;
    dw[0] += a2 * (y * dY[4] + z * dY[7]) + 2.f * e2 * x * dY[8];
    dw[1] += a2 * (x * dY[4] + z * dY[5]) - 2.f * e2 * y * dY[8];
    dw[2] += a2 * (y * dY[5] + x * dY[7]) + 6.f * b2 * z * dY[6];
    if (D < 3) return;
    const float e3 = 0.59004358992664352f, f3 = 2.8906114426405538f;
    const float g3 = 0.45704579946446572f, h3 = 0.37317633259011540f, k3 = 1.4453057213202769f;
    const float xx = x * x, yy = y * y, zz = z * z;
    dw[0] += 6.f * e3 * x * y * dY[9] + f3 * y * z * dY[10] + g3 * (5.f * zz - 1.f) * dY[13] +
             2.f * k3 * x * z * dY[14] + e3 * (3.f * xx - 3.f * yy) * dY[15];
    dw[1] += e3 * (3.f * xx - 3.f * yy) * dY[9] + f3 * x * z * dY[10] +
             g3 * (5.f * zz - 1.f) * dY[11] - 2.f * k3 * y * z * dY[14] - 6.f * e3 * x * y * dY[15];
    dw[2] += f3 * x * y * dY[10] + 10.f * g3 * y * z * dY[11] + h3 * (15.f * zz - 3.f) * dY[12] +
             10.f * g3 * x * z * dY[13] + k3 * (xx - yy) * dY[14];
}

struct IndBwdArgs {
    int V, n;
    const ts_camera* cams;
    const float* means;
    const float* quats;
    const float* sh;
    const float4* lind;
    const float4* d_lind;
    float beta;
    float* d_sh;
    float* d_means;
    float* d_quats;
};

// One thread per splat, views in order: coefficient gradients Y_j(w_r) dL/dl_ind, and the
// chain through w_r = normalize(d - 2 (d.n) n), d = normalize(mu - o), n = R(q/|q|) e_z.
template <int D>
__global__ __launch_bounds__(256) void k_indirect_bwd(IndBwdArgs a) {
    constexpr int K = (D + 1) * (D + 1);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    float c[K * 3], ds[K * 3];
#pragma unroll
    for (int j = 0; j < K * 3; j++) {
        c[j] = a.sh[(int64_t)k * K * 3 + j];
        ds[j] = 0.f;
    }
    float q0 = a.quats[4 * k + 0], q1 = a.quats[4 * k + 1], q2 = a.quats[4 * k + 2],
          q3 = a.quats[4 * k + 3];
    float qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    float qn = sqrtf(qq), iq = qq > 0.f ? 1.f / qn : 0.f;
    float w_ = q0 * iq, x_ = q1 * iq, y_ = q2 * iq, z_ = q3 * iq;    // unit quaternion
    float nx = 2.f * (x_ * z_ + w_ * y_), ny = 2.f * (y_ * z_ - w_ * x_),
          nz = 1.f - 2.f * (x_ * x_ + y_ * y_);
    const float mx = a.means[3 * k + 0], my = a.means[3 * k + 1], mz = a.means[3 * k + 2];
    float dmu[3] = {0.f, 0.f, 0.f}, dnv[3] = {0.f, 0.f, 0.f};
    for (int v = 0; v < a.V && qq > 0.f; v++) {
        const float4 lv = a.lind[(int64_t)v * a.n + k];
        const float4 gv = a.d_lind[(int64_t)v * a.n + k];
        // a channel clamped at zero passes no gradient
        const float g[3] = {lv.x > 0.f ? gv.x : 0.f, lv.y > 0.f ? gv.y : 0.f,
                            lv.z > 0.f ? gv.z : 0.f};
        if (g[0] == 0.f && g[1] == 0.f && g[2] == 0.f) continue;
        const float* cw = a.cams[v].w2c;
        float ox = -(cw[0] * cw[3] + cw[4] * cw[7] + cw[8] * cw[11]);
        float oy = -(cw[1] * cw[3] + cw[5] * cw[7] + cw[9] * cw[11]);
        float oz = -(cw[2] * cw[3] + cw[6] * cw[7] + cw[10] * cw[11]);
        float dx = mx - ox, dy = my - oy, dz = mz - oz;
        float dd = dx * dx + dy * dy + dz * dz;
        if (!(dd > 0.f)) continue;
        float idl = rsqrtf(dd);
        dx *= idl; dy *= idl; dz *= idl;
        float dn = dx * nx + dy * ny + dz * nz;
        float ux = dx - 2.f * dn * nx, uy = dy - 2.f * dn * ny, uz = dz - 2.f * dn * nz;
        float irl = rsqrtf(ux * ux + uy * uy + uz * uz);
        float rx = ux * irl, ry = uy * irl, rz = uz * irl;
        float Y[K], dY[K];
        sh_basis_f<D>(rx, ry, rz, Y);
#pragma unroll
        for (int j = 0; j < K; j++) {
            ds[3 * j + 0] = fmaf(Y[j], g[0], ds[3 * j + 0]);
            ds[3 * j + 1] = fmaf(Y[j], g[1], ds[3 * j + 1]);
            ds[3 * j + 2] = fmaf(Y[j], g[2], ds[3 * j + 2]);
            dY[j] = c[3 * j] * g[0] + c[3 * j + 1] * g[1] + c[3 * j + 2] * g[2];
        }
        float dw[3];
        sh_basis_grad_f<D>(rx, ry, rz, dY, dw);
        // w = u / |u|
        float wd = rx * dw[0] + ry * dw[1] + rz * dw[2];
        float du[3] = {(dw[0] - rx * wd) * irl, (dw[1] - ry * wd) * irl, (dw[2] - rz * wd) * irl};
        // u = d - 2 (d.n) n
        float ndu = nx * du[0] + ny * du[1] + nz * du[2];
        float ddv[3] = {du[0] - 2.f * ndu * nx, du[1] - 2.f * ndu * ny, du[2] - 2.f * ndu * nz};
        dnv[0] -= 2.f * (dn * du[0] + dx * ndu);
        dnv[1] -= 2.f * (dn * du[1] + dy * ndu);
        dnv[2] -= 2.f * (dn * du[2] + dz * ndu);
        // d = (mu - o) / |mu - o|
        float dpd = dx * ddv[0] + dy * ddv[1] + dz * ddv[2];
        dmu[0] += (ddv[0] - dx * dpd) * idl;
        dmu[1] += (ddv[1] - dy * dpd) * idl;
        dmu[2] += (ddv[2] - dz * dpd) * idl;
    }
    float* out = a.d_sh + (int64_t)k * K * 3;
#pragma unroll
    for (int j = 0; j < K * 3; j++) out[j] = a.beta != 0.f ? ds[j] + a.beta * out[j] : ds[j];
    a.d_means[3 * k + 0] += dmu[0];
    a.d_means[3 * k + 1] += dmu[1];
    a.d_means[3 * k + 2] += dmu[2];
    // n = (2(xz + wy), 2(yz - wx), 1 - 2(x^2 + y^2)) of the unit quaternion, then q / |q|
    float gw = 2.f * (y_ * dnv[0] - x_ * dnv[1]);
    float gx = 2.f * (z_ * dnv[0] - w_ * dnv[1]) - 4.f * x_ * dnv[2];
    float gy = 2.f * (w_ * dnv[0] + z_ * dnv[1]) - 4.f * y_ * dnv[2];
    float gz = 2.f * (x_ * dnv[0] + y_ * dnv[1]);
    float pq = w_ * gw + x_ * gx + y_ * gy + z_ * gz;
    a.d_quats[4 * k + 0] += (gw - w_ * pq) * iq;
    a.d_quats[4 * k + 1] += (gx - x_ * pq) * iq;
    a.d_quats[4 * k + 2] += (gy - y_ * pq) * iq;
    a.d_quats[4 * k + 3] += (gz - z_ * pq) * iq;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_indirect_bwd(int32_t n_views, const ts_camera* cams, int32_t n,
                               const float* means, const float* quats, const float* sh,
                               int32_t sh_degree, const float* lind, const float* d_lind,
                               float beta, float* d_sh, float* d_means, float* d_quats,
                               hipStream_t stream) {
    if (n_views < 1 || n < 0 || !cams || sh_degree < 0 || sh_degree > 3) {
        set_error("ts_indirect_bwd: bad argument (views=%d n=%d degree=%d)", n_views, n,
                  sh_degree);
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    if (!means || !quats || !sh || !lind || !d_lind || !d_sh || !d_means || !d_quats) {
        set_error("ts_indirect_bwd: null array");
        return TS_E_ARG;
    }
    if ((int64_t)n_views * n > 0x7FFFFFFFLL) {
        set_error("ts_indirect_bwd: n_views * n above 2^31-1");
        return TS_E_ARG;
    }
    IndBwdArgs a;
    a.V = n_views; a.n = n; a.cams = cams; a.means = means; a.quats = quats; a.sh = sh;
    a.lind = (const float4*)lind; a.d_lind = (const float4*)d_lind; a.beta = beta;
    a.d_sh = d_sh; a.d_means = d_means; a.d_quats = d_quats;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (sh_degree) {
        case 0: hipLaunchKernelGGL(k_indirect_bwd<0>, grid, block, 0, stream, a); break;
        case 1: hipLaunchKernelGGL(k_indirect_bwd<1>, grid, block, 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_indirect_bwd<2>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_indirect_bwd<3>, grid, block, 0, stream, a); break;
    }
    return launch_check("ts_indirect_bwd");
}

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

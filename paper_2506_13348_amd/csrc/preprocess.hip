// ts_preprocess: per (view, splat) projection, depth key and conservative screen bound.
//
// Geometry (Sec. 3.1, Eq. 1): P(u,v) = p + s_u t_u u + s_v t_v v. In camera space, with
// mu the centre, a pixel ray d = ((X-cx)/fx, (Y-cy)/fy, 1) meets the plane where
//   u = ((t_v x mu) . d) / (s_u (n . d)),   v = ((mu x t_u) . d) / (s_v (n . d)),
// since (t_v x mu).mu = (mu x t_u).mu = 0 these numerators only see d - mu/mu_z, i.e. the
// pixel offset from the projected centre (px, py), which keeps the float32 per-pixel
// evaluation well conditioned. The hit is in front of the camera iff n.mu and n.d share a
// sign; all coefficients are multiplied by sign(n.mu) so that the test becomes den > 0.
// The per-splat set-up runs in double precision; records are stored as float32.
//
// The camera's rotation W arrives in float32 and is orthogonal only to rounding (~1e-7),
// while a pixel's ray is defined in the world as W^T d (with origin o = -W^T t). The camera
// frame is therefore taken as the one in which those rays are d: points map by A = W^{-T}
// (p_cam = A (p - o) = A p + t) and the vectors that enter dot products with rays (the
// normal and the in-plane axes, as covectors) by W. With g_u = W t_u, g_v = W t_v, n = W n_w
// the numerators take the general form a_u = (n.mu) g_u - (mu.g_u) n (and likewise a_v),
// equal to the cross products above for an orthonormal frame. (Mapping points by W instead
// shifts (u,v) by about 1e-7 / |cos| of the ray-normal angle, visible on near edge-on splats.)
#include <math.h>

#include "ts_internal.h"

namespace ts {

struct PreArgs {
    int V, W, H, n;
    const ts_camera* cams;
    float S, amin, near_z;
    const float* means;
    const float* quats;
    const float* scales;
    const float* opac;
    const int32_t* chart_of;
    float* rec;
    int4* rect;
    uint32_t* depth_key;
};

__device__ inline double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ void preprocess_one(const PreArgs& a, int64_t gid, float4* r4);

// A = W^{-T} of a 3x3 row-major matrix: its cofactor matrix over its determinant.
__device__ inline void cam_points_map(const double* W, double* A) {
    double C[9] = {W[4] * W[8] - W[5] * W[7], W[5] * W[6] - W[3] * W[8], W[3] * W[7] - W[4] * W[6],
                   W[2] * W[7] - W[1] * W[8], W[0] * W[8] - W[2] * W[6], W[1] * W[6] - W[0] * W[7],
                   W[1] * W[5] - W[2] * W[4], W[2] * W[3] - W[0] * W[5], W[0] * W[4] - W[1] * W[3]};
    double id = 1.0 / (W[0] * C[0] + W[1] * C[1] + W[2] * C[2]);
    for (int i = 0; i < 9; i++) A[i] = C[i] * id;
}

// a_u = (n.mu) g_u - (mu.g_u) n and a_v = (n.mu) g_v - (mu.g_v) n: with a pixel ray d,
// u = a_u.d / (s_u n.d) and v = a_v.d / (s_v n.d) (a_u.mu = a_v.mu = 0).
__device__ inline void plane_numerators(const double* nc, const double* mc, double nmu,
                                        const double* gu, const double* gv, double* au,
                                        double* av) {
    double mgu = dot3(mc, gu), mgv = dot3(mc, gv);
    for (int i = 0; i < 3; i++) {
        au[i] = nmu * gu[i] - mgu * nc[i];
        av[i] = nmu * gv[i] - mgv * nc[i];
    }
}

// Records leave through LDS: each thread builds its 7 float4 there, then the workgroup
// writes its 256 consecutive records (28 KB) with consecutive lanes on consecutive float4s
// (a thread writing its own 112-byte record would touch 7 lines per lane and store).
// Records of dropped splats are written too (zeros); no list refers to them.
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
    __shared__ float4 srec[256 * kRec4];
    const int64_t block0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t total = (int64_t)a.V * a.n;
    const int nrec = (int)min((int64_t)blockDim.x, total - block0);
#pragma unroll
    for (int q = 0; q < kRec4; q++) srec[threadIdx.x * kRec4 + q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (threadIdx.x < nrec) preprocess_one(a, block0 + threadIdx.x, srec + threadIdx.x * kRec4);
    __syncthreads();
    float4* dst = (float4*)a.rec + block0 * kRec4;
    for (int i = threadIdx.x; i < nrec * kRec4; i += blockDim.x) dst[i] = srec[i];
}

// One (view, splat): rect, depth key, and the record into r4 (left untouched when dropped).
__device__ void preprocess_one(const PreArgs& a, int64_t gid, float4* r4) {
    int v = (int)(gid / a.n);
    int k = (int)(gid - (int64_t)v * a.n);
    const ts_camera& cam = a.cams[v];

    double Wr[9], t[3];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) Wr[i * 3 + j] = cam.w2c[i * 4 + j];
        t[i] = cam.w2c[i * 4 + 3];
    }
    double mu[3] = {a.means[3 * k + 0], a.means[3 * k + 1], a.means[3 * k + 2]};
    // camera depth, evaluated left to right without contraction so that its float32
    // rounding (the sort key) is reproducible
    double z = __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn(Wr[6], mu[0]), __dmul_rn(Wr[7], mu[1])),
                                   __dmul_rn(Wr[8], mu[2])), t[2]);
    int4 rect_out = make_int4(0, 0, 0, 0);
    uint32_t key = 0xFFFFFFFFu;
    float op = a.opac[k];
    bool keep = z > (double)a.near_z && op >= a.amin;

    // A = W^{-T} (cofactor matrix over the determinant): camera-frame points
    double A[9];
    cam_points_map(Wr, A);
    double mc[3];
    for (int i = 0; i < 3; i++) mc[i] = A[i * 3 + 0] * mu[0] + A[i * 3 + 1] * mu[1] + A[i * 3 + 2] * mu[2] + t[i];

    // rotation of the normalised quaternion; columns t_u, t_v, n
    double q[4] = {a.quats[4 * k + 0], a.quats[4 * k + 1], a.quats[4 * k + 2], a.quats[4 * k + 3]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0)) keep = false;
    double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, zq = q[3] / qn;
    double R[9] = {1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y),
                   2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x),
                   2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)};
    // covectors g_u, g_v, n (map by W) and in-plane point displacements t_u, t_v (map by A)
    double gu[3], gv[3], nc[3], tu[3], tv[3];
    for (int i = 0; i < 3; i++) {
        gu[i] = Wr[i * 3 + 0] * R[0] + Wr[i * 3 + 1] * R[3] + Wr[i * 3 + 2] * R[6];
        gv[i] = Wr[i * 3 + 0] * R[1] + Wr[i * 3 + 1] * R[4] + Wr[i * 3 + 2] * R[7];
        nc[i] = Wr[i * 3 + 0] * R[2] + Wr[i * 3 + 1] * R[5] + Wr[i * 3 + 2] * R[8];
        tu[i] = A[i * 3 + 0] * R[0] + A[i * 3 + 1] * R[3] + A[i * 3 + 2] * R[6];
        tv[i] = A[i * 3 + 0] * R[1] + A[i * 3 + 1] * R[4] + A[i * 3 + 2] * R[7];
    }
    // facing sign in world space: +1 if n.(o - mu) >= 0, o = -W^T t
    double o[3];
    for (int i = 0; i < 3; i++) o[i] = -(Wr[0 * 3 + i] * t[0] + Wr[1 * 3 + i] * t[1] + Wr[2 * 3 + i] * t[2]);
    double nw[3] = {R[2], R[5], R[8]};
    double om[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    double sigma = dot3(nw, om) >= 0.0 ? 1.0 : -1.0;

    double nmu = dot3(nc, mc);
    if (nmu == 0.0) keep = false;   // the camera lies in the splat's plane: no ray hits it
    double su = a.scales[2 * k + 0], sv = a.scales[2 * k + 1];
    if (!(su > 0) || !(sv > 0)) keep = false;

    if (keep) {
        key = __float_as_uint((float)z);
        double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
        double iz = 1.0 / mc[2];
        double px = fx * mc[0] * iz + cx, py = fy * mc[1] * iz + cy;
        double Au[3], Bv[3];
        plane_numerators(nc, mc, nmu, gu, gv, Au, Bv);
        double sg = nmu > 0 ? 1.0 : -1.0;
        double ux = sg * Au[0] / (su * fx), uy = sg * Au[1] / (su * fy);
        double vx = sg * Bv[0] / (sv * fx), vy = sg * Bv[1] / (sv * fy);
        double wx = sg * nc[0] / fx, wy = sg * nc[1] / fy, w0 = sg * nmu * iz;
        float px_hi = (float)px, py_hi = (float)py;
        double px_lo = px - (double)px_hi, py_lo = py - (double)py_hi;
        double u0 = -(ux * px_lo + uy * py_lo);
        double v0 = -(vx * px_lo + vy * py_lo);
        w0 -= wx * px_lo + wy * py_lo;

        // Conservative screen bound of the region that can blend: the support square
        // max(|u|,|v|) <= S intersected with the disk u^2+v^2 <= 2 ln(o/alpha_min), both
        // slightly enlarged so float32 per-pixel tests never fall outside it.
        double Sx = (double)a.S * (1.0 + 1e-3) + 1e-4;
        double ra2 = 2.0 * log((double)op / (double)a.amin);
        double ra = sqrt(ra2 > 0 ? ra2 : 0.0) * (1.0 + 1e-3) + 1e-3;
        double xlo = 0, xhi = a.W - 1e-9, ylo = 0, yhi = a.H - 1e-9;   // in pixel coordinates
        bool full = false;
        double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
        for (int c = 0; c < 4; c++) {
            double cu = (c & 1) ? Sx : -Sx, cv = (c & 2) ? Sx : -Sx;
            double P[3];
            for (int i = 0; i < 3; i++) P[i] = mc[i] + su * cu * tu[i] + sv * cv * tv[i];
            if (P[2] <= 1e-7 * (fabs(mc[2]) + su * Sx + sv * Sx)) { full = true; break; }
            double X = fx * P[0] / P[2] + cx, Y = fy * P[1] / P[2] + cy;
            bx0 = fmin(bx0, X); bx1 = fmax(bx1, X);
            by0 = fmin(by0, Y); by1 = fmax(by1, Y);
        }
        if (full) { bx0 = xlo; bx1 = xhi + 1; by0 = ylo; by1 = yhi + 1; }
        if (ra < Sx * 1.4142135623730951) {
            // image of the disk: a conic; dual conic C* = M diag(r^2, r^2, -1) M^T with
            // M = K [s_u t_u | s_v t_v | mu]; vertical/horizontal tangents bound it
            double c1[3] = {fx * su * tu[0] + cx * su * tu[2], fy * su * tu[1] + cy * su * tu[2], su * tu[2]};
            double c2[3] = {fx * sv * tv[0] + cx * sv * tv[2], fy * sv * tv[1] + cy * sv * tv[2], sv * tv[2]};
            double c3[3] = {fx * mc[0] + cx * mc[2], fy * mc[1] + cy * mc[2], mc[2]};
            double r2 = ra * ra;
            double C33 = r2 * (c1[2] * c1[2] + c2[2] * c2[2]) - c3[2] * c3[2];
            if (C33 < -1e-12 * c3[2] * c3[2]) {
                double C11 = r2 * (c1[0] * c1[0] + c2[0] * c2[0]) - c3[0] * c3[0];
                double C22 = r2 * (c1[1] * c1[1] + c2[1] * c2[1]) - c3[1] * c3[1];
                double C13 = r2 * (c1[0] * c1[2] + c2[0] * c2[2]) - c3[0] * c3[2];
                double C23 = r2 * (c1[1] * c1[2] + c2[1] * c2[2]) - c3[1] * c3[2];
                double dx = sqrt(fmax(C13 * C13 - C11 * C33, 0.0));
                double dy = sqrt(fmax(C23 * C23 - C22 * C33, 0.0));
                double ex0 = (C13 + dx) / C33, ex1 = (C13 - dx) / C33;
                double ey0 = (C23 + dy) / C33, ey1 = (C23 - dy) / C33;
                bx0 = fmax(bx0, fmin(ex0, ex1)); bx1 = fmin(bx1, fmax(ex0, ex1));
                by0 = fmax(by0, fmin(ey0, ey1)); by1 = fmin(by1, fmax(ey0, ey1));
            }
        }
        // pixels whose centre x+1/2 lies in [bx0, bx1], with a small safety margin
        double mg = 0.02 + 1e-4 * fmax(bx1 - bx0, by1 - by0);
        double fx0 = ceil(fmax(bx0 - mg - 0.5, -1.0)), fx1 = floor(fmin(bx1 + mg - 0.5, (double)a.W));
        double fy0 = ceil(fmax(by0 - mg - 0.5, -1.0)), fy1 = floor(fmin(by1 + mg - 0.5, (double)a.H));
        int ix0 = (int)fmax(fx0, 0.0), ix1 = (int)fmin(fx1, (double)(a.W - 1));
        int iy0 = (int)fmax(fy0, 0.0), iy1 = (int)fmin(fy1, (double)(a.H - 1));
        if (ix0 <= ix1 && iy0 <= iy1 && bx0 <= bx1 && by0 <= by1) {
            rect_out = make_int4(ix0 / kTile, iy0 / kTile, ix1 / kTile + 1, iy1 / kTile + 1);
            r4[0] = make_float4((float)ix0, (float)iy0, (float)ix1, (float)iy1);
            r4[1] = make_float4(px_hi, py_hi, (float)ux, (float)uy);
            r4[2] = make_float4((float)u0, (float)vx, (float)vy, (float)v0);
            r4[3] = make_float4((float)wx, (float)wy, (float)w0, op);
            float sR[9];
            for (int i = 0; i < 9; i++) sR[i] = (float)(sigma * R[i]);
            r4[4] = make_float4(sR[0], sR[1], sR[2], sR[3]);
            r4[5] = make_float4(sR[4], sR[5], sR[6], sR[7]);
            r4[6] = make_float4(sR[8], __int_as_float(a.chart_of[k]), (float)px_lo, (float)py_lo);
        }
    }
    a.rect[(int64_t)v * a.n + k] = rect_out;
    a.depth_key[(int64_t)v * a.n + k] = key;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_preprocess(int32_t n_views, int32_t width, int32_t height, const ts_camera* cams,
                             const ts_params* params, int32_t n, const float* means,
                             const float* quats, const float* scales, const float* opac,
                             const int32_t* chart_of, float* rec, int32_t* rect,
                             uint32_t* depth_key, hipStream_t stream) {
    if (!params || !cams || n < 0 || n_views < 1 || width < 1 || height < 1) {
        set_error("ts_preprocess: bad argument (n=%d views=%d %dx%d)", n, n_views, width, height);
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    if (!means || !quats || !scales || !opac || !chart_of || !rec || !rect || !depth_key) {
        set_error("ts_preprocess: null array");
        return TS_E_ARG;
    }
    PreArgs a;
    a.V = n_views; a.W = width; a.H = height; a.n = n; a.cams = cams;
    a.S = params->s_sigma; a.amin = params->alpha_min; a.near_z = params->near_z;
    a.means = means; a.quats = quats; a.scales = scales; a.opac = opac; a.chart_of = chart_of;
    a.rec = rec; a.rect = (int4*)rect; a.depth_key = depth_key;
    int64_t total = (int64_t)n_views * n;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(256), 0, stream, a);
    return launch_check("ts_preprocess");
}

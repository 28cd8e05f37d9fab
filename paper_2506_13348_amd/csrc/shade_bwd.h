// Adjoint of the split-sum shading (Eq. 10-12): given dL/dC for one pixel, the gradient with
// respect to the eight blended G-buffer channels and the transmittance (tables are constant).
#pragma once
#include "shade.h"

namespace ts {

// Face geometry: sc = s_sign d[s_ax], tc = t_sign d[t_ax], |ma| = m_sign d[m_ax].
__device__ inline void face_axes(int face, int& m_ax, float& m_sign, int& s_ax, float& s_sign,
                                 int& t_ax, float& t_sign) {
    switch (face) {
        case 0: m_ax = 0; m_sign = 1.f; s_ax = 2; s_sign = -1.f; t_ax = 1; t_sign = -1.f; break;
        case 1: m_ax = 0; m_sign = -1.f; s_ax = 2; s_sign = 1.f; t_ax = 1; t_sign = -1.f; break;
        case 2: m_ax = 1; m_sign = 1.f; s_ax = 0; s_sign = 1.f; t_ax = 2; t_sign = 1.f; break;
        case 3: m_ax = 1; m_sign = -1.f; s_ax = 0; s_sign = 1.f; t_ax = 2; t_sign = -1.f; break;
        case 4: m_ax = 2; m_sign = 1.f; s_ax = 0; s_sign = 1.f; t_ax = 1; t_sign = -1.f; break;
        default: m_ax = 2; m_sign = -1.f; s_ax = 0; s_sign = -1.f; t_ax = 1; t_sign = -1.f; break;
    }
}

// Cube sample with its adjoint: value at direction d, and dL/dd += J^T dv.
struct CubeTap {
    int face;
    float X, Y;
};

__device__ inline float3 cube_sample_tap(const float4* __restrict__ cube, int r, const float* d,
                                         CubeTap& tap) {
    tap.face = cube_coords(d[0], d[1], d[2], r, tap.X, tap.Y);
    return face_bilinear(cube, r, tap.face, tap.X, tap.Y);
}

__device__ inline void cube_sample_bwd(const float4* __restrict__ cube, int r, const float* d,
                                       const CubeTap& tap, float3 dv, float* gd) {
    float x0 = floorf(tap.X), y0 = floorf(tap.Y);
    float fx = tap.X - x0, fy = tap.Y - y0;
    int i0 = (int)x0, j0 = (int)y0;
    int i1 = min(max(i0 + 1, 0), r - 1), j1 = min(max(j0 + 1, 0), r - 1);
    i0 = min(max(i0, 0), r - 1);
    j0 = min(max(j0, 0), r - 1);
    const float4* F = cube + (size_t)tap.face * r * r;
    float4 a = F[j0 * r + i0], b = F[j0 * r + i1], c = F[j1 * r + i0], e = F[j1 * r + i1];
    float dX = dv.x * ((1.f - fy) * (b.x - a.x) + fy * (e.x - c.x)) +
               dv.y * ((1.f - fy) * (b.y - a.y) + fy * (e.y - c.y)) +
               dv.z * ((1.f - fy) * (b.z - a.z) + fy * (e.z - c.z));
    float dY = dv.x * ((1.f - fx) * (c.x - a.x) + fx * (e.x - b.x)) +
               dv.y * ((1.f - fx) * (c.y - a.y) + fx * (e.y - b.y)) +
               dv.z * ((1.f - fx) * (c.z - a.z) + fx * (e.z - b.z));
    int m_ax, s_ax, t_ax;
    float m_sign, s_sign, t_sign;
    face_axes(tap.face, m_ax, m_sign, s_ax, s_sign, t_ax, t_sign);
    // axis selects instead of indexing by a run-time axis (keeps d and gd in registers)
    auto pick = [&](int ax) {
        return (float)(ax == 0) * d[0] + (float)(ax == 1) * d[1] + (float)(ax == 2) * d[2];
    };
    float ma = m_sign * pick(m_ax);
    float sc = s_sign * pick(s_ax), tc = t_sign * pick(t_ax);
    float hr = 0.5f * (float)r;
    float ima = 1.0f / ma;
    // X = hr (sc/ma + 1) - 1/2
    float gs = dX * hr * ima * s_sign;
    float gt = dY * hr * ima * t_sign;
    float gm = -(dX * sc + dY * tc) * hr * ima * ima * m_sign;
#pragma unroll
    for (int k = 0; k < 3; k++)
        gd[k] += (float)(s_ax == k) * gs + (float)(t_ax == k) * gt + (float)(m_ax == k) * gm;
}

// LUT sample with derivatives in x and y.
__device__ inline float2 lut_sample_d(const float2* __restrict__ lut, int n, float x, float y,
                                      float2& ddx, float2& ddy) {
    float X = fmaf(x, (float)n, -0.5f), Y = fmaf(y, (float)n, -0.5f);
    float x0 = floorf(X), y0 = floorf(Y);
    float fx = X - x0, fy = Y - y0;
    int i0 = (int)x0, j0 = (int)y0;
    int i1 = min(max(i0 + 1, 0), n - 1), j1 = min(max(j0 + 1, 0), n - 1);
    i0 = min(max(i0, 0), n - 1);
    j0 = min(max(j0, 0), n - 1);
    float2 a = lut[j0 * n + i0], b = lut[j0 * n + i1], c = lut[j1 * n + i0], d = lut[j1 * n + i1];
    float fn = (float)n;
    ddx = make_float2(fn * ((1.f - fy) * (b.x - a.x) + fy * (d.x - c.x)),
                      fn * ((1.f - fy) * (b.y - a.y) + fy * (d.y - c.y)));
    ddy = make_float2(fn * ((1.f - fx) * (c.x - a.x) + fx * (d.x - b.x)),
                      fn * ((1.f - fx) * (c.y - a.y) + fx * (d.y - b.y)));
    float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy), w01 = (1.f - fx) * fy, w11 = fx * fy;
    return make_float2(w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x,
                       w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y);
}

// dC = dL/d(rgb). Writes dg[8] = dL/dg and returns dL/dT (through the (1-A) bg term). With
// the indirect term (kInd) the specular radiance is V L_dir + (1 - V) L_ind: li = the blended
// L_ind, vis = V, and dli[3] = dL/dL_ind is written too.
template <bool kInd = false>
__device__ inline float shade_pixel_bwd(const EnvDev& env, const ShadeConst& sc, const float* g,
                                        float T, float3 dray, float3 dC, float* dg,
                                        const float* li = nullptr, float vis = 1.0f,
                                        float* dli = nullptr) {
#pragma unroll
    for (int c = 0; c < 8; c++) dg[c] = 0.f;
    if (kInd) {
        dli[0] = 0.f; dli[1] = 0.f; dli[2] = 0.f;
    }
    if (T >= 1.0f) return 0.f;
    float il = rsqrtf(dray.x * dray.x + dray.y * dray.y + dray.z * dray.z);
    float wo[3] = {-dray.x * il, -dray.y * il, -dray.z * il};
    float N[3] = {g[5], g[6], g[7]};
    float nn = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
    float Nh[3], inv = 0.f;
    bool has_n = nn > 0.f;
    if (has_n) {
        inv = rsqrtf(nn);
        Nh[0] = N[0] * inv; Nh[1] = N[1] * inv; Nh[2] = N[2] * inv;
    } else {
        Nh[0] = wo[0]; Nh[1] = wo[1]; Nh[2] = wo[2];
    }
    float ndv = Nh[0] * wo[0] + Nh[1] * wo[1] + Nh[2] * wo[2];
    float wr[3] = {2.f * ndv * Nh[0] - wo[0], 2.f * ndv * Nh[1] - wo[1], 2.f * ndv * Nh[2] - wo[2]};
    float M = g[3], R = g[4];
    CubeTap tE, t0, t1;
    float3 E = cube_sample_tap(env.irr, env.irr_res, Nh, tE);
    float rc = fminf(fmaxf(R, 0.f), 1.f);
    float lev = rc * (float)(env.levels - 1);
    int l0 = min((int)floorf(lev), env.levels - 1);
    int l1 = min(l0 + 1, env.levels - 1);
    float fl = lev - (float)l0;
    const float4* s0 = env.spec;
    const float4* s1 = env.spec;
    int r0 = env.spec_res, r1 = env.spec_res;
    {
        size_t off = 0;
        for (int l = 0; l < env.levels; l++) {
            int rl = max(env.spec_res >> l, 1);
            if (l == l0) { s0 = env.spec + off; r0 = rl; }
            if (l == l1) { s1 = env.spec + off; r1 = rl; }
            off += (size_t)6 * rl * rl;
        }
    }
    float3 P0 = cube_sample_tap(s0, r0, wr, t0);
    float3 P1 = (l1 != l0) ? cube_sample_tap(s1, r1, wr, t1) : P0;
    float2 ddx, ddy;
    float xl = fminf(fmaxf(ndv, 0.f), 1.f);
    float2 ab = lut_sample_d(env.lut, env.lut_res, xl, rc, ddx, ddy);
    float oneM = 1.f - M;
    const float ipi = 1.0f / 3.14159265358979323846f;
    float kd = oneM * ipi;
    float dCv[3] = {dC.x, dC.y, dC.z};
    float Ev[3] = {E.x, E.y, E.z}, P0v[3] = {P0.x, P0.y, P0.z}, P1v[3] = {P1.x, P1.y, P1.z};
    float dM = 0.f, dfl = 0.f, da = 0.f, db = 0.f;
    float dE[3], dP0[3], dP1[3];
    for (int c = 0; c < 3; c++) {
        float Lp = P0v[c] + fl * (P1v[c] - P0v[c]);
        if (kInd) Lp = vis * Lp + (1.f - vis) * li[c];   // the mixed specular radiance
        float F0 = 0.04f * oneM + g[c] * M;
        dg[c] = dCv[c] * (kd * Ev[c] + Lp * ab.x * M);
        dM += dCv[c] * (-g[c] * Ev[c] * ipi + Lp * ab.x * (g[c] - 0.04f));
        float dLp = dCv[c] * (F0 * ab.x + ab.y);
        if (kInd) {
            dli[c] = dLp * (1.f - vis);
            dLp *= vis;
        }
        dE[c] = dCv[c] * g[c] * kd;
        da += dCv[c] * Lp * F0;
        db += dCv[c] * Lp;
        dfl += dLp * (P1v[c] - P0v[c]);
        dP0[c] = dLp * (1.f - fl);
        dP1[c] = dLp * fl;
    }
    dg[3] = dM;
    float drc = dfl * (float)(env.levels - 1) + da * ddy.x + db * ddy.y;
    dg[4] = (R >= 0.f && R <= 1.f) ? drc : 0.f;
    float dndv = (ndv >= 0.f && ndv <= 1.f) ? (da * ddx.x + db * ddx.y) : 0.f;
    float dwr[3] = {0.f, 0.f, 0.f};
    if (l1 != l0) {
        cube_sample_bwd(s0, r0, wr, t0, make_float3(dP0[0], dP0[1], dP0[2]), dwr);
        cube_sample_bwd(s1, r1, wr, t1, make_float3(dP1[0], dP1[1], dP1[2]), dwr);
    } else {
        cube_sample_bwd(s0, r0, wr, t0, make_float3(dP0[0] + dP1[0], dP0[1] + dP1[1],
                                                    dP0[2] + dP1[2]), dwr);
    }
    float dNh[3] = {0.f, 0.f, 0.f};
    cube_sample_bwd(env.irr, env.irr_res, Nh, tE, make_float3(dE[0], dE[1], dE[2]), dNh);
    float ndw = Nh[0] * dwr[0] + Nh[1] * dwr[1] + Nh[2] * dwr[2];
    for (int k = 0; k < 3; k++) dNh[k] += 2.f * (ndv * dwr[k] + ndw * wo[k]) + dndv * wo[k];
    if (has_n) {
        float p = Nh[0] * dNh[0] + Nh[1] * dNh[1] + Nh[2] * dNh[2];
        for (int k = 0; k < 3; k++) dg[5 + k] = (dNh[k] - Nh[k] * p) * inv;
    }
    return dCv[0] * sc.bg[0] + dCv[1] * sc.bg[1] + dCv[2] * sc.bg[2];
}

}  // namespace ts

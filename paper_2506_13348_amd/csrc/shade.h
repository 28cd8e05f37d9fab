// Deferred split-sum shading of one pixel (Eq. 10-12), used by the fused raster epilogue
// and by ts_shade. With the indirect term the specular radiance is V L_dir + (1 - V) L_ind
// (Eq. 12), V the pixel's visibility and L_ind the blended indirect map; without it V = 1.
#pragma once
#include "ts_internal.h"

namespace ts {

struct EnvDev {
    const float4* spec;   // levels back to back
    const float4* irr;
    const float2* lut;
    int spec_res, levels, irr_res, lut_res;
};

struct ShadeConst {
    float bg[3];
};

// Cube face and in-face texel coordinates (texel units, centres at integers) of direction d:
// OpenGL major-axis rule, ties going X, then Y, then Z.
__device__ inline int cube_coords(float dx, float dy, float dz, int r, float& X, float& Y) {
    float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int face;
    float sc, tc, ma;
    if (ax >= ay && ax >= az) {
        ma = ax;
        if (dx >= 0.f) { face = 0; sc = -dz; tc = -dy; } else { face = 1; sc = dz; tc = -dy; }
    } else if (ay >= az) {
        ma = ay;
        if (dy >= 0.f) { face = 2; sc = dx; tc = dz; } else { face = 3; sc = dx; tc = -dz; }
    } else {
        ma = az;
        if (dz >= 0.f) { face = 4; sc = dx; tc = -dy; } else { face = 5; sc = -dx; tc = -dy; }
    }
    float inv = 1.0f / ma;
    float hr = 0.5f * (float)r;
    X = fmaf(sc * inv, hr, hr - 0.5f);
    Y = fmaf(tc * inv, hr, hr - 0.5f);
    return face;
}

// bilinear inside one face at texel coordinates (X,Y), clamp-to-edge
__device__ inline float3 face_bilinear(const float4* __restrict__ cube, int r, int face, float X,
                                       float Y) {
    float x0 = floorf(X), y0 = floorf(Y);
    float fx = X - x0, fy = Y - y0;
    int i0 = (int)x0, j0 = (int)y0;
    int i1 = min(max(i0 + 1, 0), r - 1), j1 = min(max(j0 + 1, 0), r - 1);
    i0 = min(max(i0, 0), r - 1);
    j0 = min(max(j0, 0), r - 1);
    const float4* F = cube + (size_t)face * r * r;
    float4 a = F[j0 * r + i0], b = F[j0 * r + i1], c = F[j1 * r + i0], d = F[j1 * r + i1];
    float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy), w01 = (1.f - fx) * fy, w11 = fx * fy;
    return make_float3(w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x,
                       w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y,
                       w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z);
}

__device__ inline float3 cube_sample(const float4* __restrict__ cube, int r, float dx, float dy,
                                     float dz) {
    float X, Y;
    int f = cube_coords(dx, dy, dz, r, X, Y);
    return face_bilinear(cube, r, f, X, Y);
}

__device__ inline float2 lut_sample(const float2* __restrict__ lut, int n, float x, float y) {
    float X = fmaf(x, (float)n, -0.5f), Y = fmaf(y, (float)n, -0.5f);
    float x0 = floorf(X), y0 = floorf(Y);
    float fx = X - x0, fy = Y - y0;
    int i0 = (int)x0, j0 = (int)y0;
    int i1 = min(max(i0 + 1, 0), n - 1), j1 = min(max(j0 + 1, 0), n - 1);
    i0 = min(max(i0, 0), n - 1);
    j0 = min(max(j0, 0), n - 1);
    float2 a = lut[j0 * n + i0], b = lut[j0 * n + i1], c = lut[j1 * n + i0], d = lut[j1 * n + i1];
    float w00 = (1.f - fx) * (1.f - fy), w10 = fx * (1.f - fy), w01 = (1.f - fx) * fy, w11 = fx * fy;
    return make_float2(w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x,
                       w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y);
}

// World direction of the ray through pixel centre (X,Y) (not normalised).
__device__ inline float3 pixel_ray(const ts_camera& cam, float X, float Y) {
    float cx = (X - cam.cx) / cam.fx, cy = (Y - cam.cy) / cam.fy;
    const float* w = cam.w2c;   // rows of the world->camera rotation = camera axes in world
    return make_float3(w[0] * cx + w[4] * cy + w[8], w[1] * cx + w[5] * cy + w[9],
                       w[2] * cx + w[6] * cy + w[10]);
}

// g = blended (albedo r,g,b, metallic, roughness, normal x,y,z); T = transmittance;
// li = blended indirect radiance and vis = visibility (read only when kInd).
template <bool kInd = false>
__device__ inline float3 shade_pixel(const EnvDev& env, const ShadeConst& sc, const float* g,
                                     float T, float3 d, const float* li = nullptr,
                                     float vis = 1.0f) {
    if (T >= 1.0f) return make_float3(sc.bg[0], sc.bg[1], sc.bg[2]);
    float A = 1.0f - T;
    float il = rsqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
    float ox = -d.x * il, oy = -d.y * il, oz = -d.z * il;
    float nx = g[5], ny = g[6], nz = g[7];
    float nn = nx * nx + ny * ny + nz * nz;
    if (nn > 0.f) {
        float in = rsqrtf(nn);
        nx *= in; ny *= in; nz *= in;
    } else {
        nx = ox; ny = oy; nz = oz;
    }
    float ndv = nx * ox + ny * oy + nz * oz;
    float rx = 2.f * ndv * nx - ox, ry = 2.f * ndv * ny - oy, rz = 2.f * ndv * nz - oz;
    float M = g[3], R = g[4];
    float3 E = cube_sample(env.irr, env.irr_res, nx, ny, nz);
    float rc = fminf(fmaxf(R, 0.f), 1.f);
    float lev = rc * (float)(env.levels - 1);
    int l0 = min((int)floorf(lev), env.levels - 1);
    int l1 = min(l0 + 1, env.levels - 1);
    float fl = lev - (float)l0;
    // level offsets (texels) and resolutions
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
    float3 P0 = cube_sample(s0, r0, rx, ry, rz);
    float3 P1 = (l1 != l0) ? cube_sample(s1, r1, rx, ry, rz) : P0;
    float2 ab = lut_sample(env.lut, env.lut_res, fminf(fmaxf(ndv, 0.f), 1.f), rc);
    float oneM = 1.f - M;
    float kd = oneM * (1.0f / 3.14159265358979323846f);
    float3 C;
    float Lp, F0;
    Lp = P0.x + fl * (P1.x - P0.x); F0 = 0.04f * oneM + g[0] * M;
    if (kInd) Lp = vis * Lp + (1.f - vis) * li[0];
    C.x = g[0] * kd * E.x + Lp * (F0 * ab.x + ab.y) + (1.f - A) * sc.bg[0];
    Lp = P0.y + fl * (P1.y - P0.y); F0 = 0.04f * oneM + g[1] * M;
    if (kInd) Lp = vis * Lp + (1.f - vis) * li[1];
    C.y = g[1] * kd * E.y + Lp * (F0 * ab.x + ab.y) + (1.f - A) * sc.bg[1];
    Lp = P0.z + fl * (P1.z - P0.z); F0 = 0.04f * oneM + g[2] * M;
    if (kInd) Lp = vis * Lp + (1.f - vis) * li[2];
    C.z = g[2] * kd * E.z + Lp * (F0 * ab.x + ab.y) + (1.f - A) * sc.bg[2];
    return C;
}

}  // namespace ts

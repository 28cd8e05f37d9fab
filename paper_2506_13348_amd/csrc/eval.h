// Per-pixel evaluation of one projected splat record, shared by the forward and backward
// rasterisers so both take the same float32 decisions.
#pragma once
#include "ts_internal.h"

namespace ts {

struct SplatEval {
    float dx, dy;      // pixel centre minus projected centre (float head)
    float den, inv;    // ray-plane denominator and its reciprocal
    float u, v;        // local coordinates (Sec. 3.1)
    float G, oG, alpha;
    bool hit;          // in front, inside the square support, alpha >= alpha_min
};

// Quadrant mask of a record for a 16x16 tile at (tx0, ty0): bit q set when the record's pixel
// bounds overlap the 8x8 block (tx0 + 8 (q&1), ty0 + 8 (q>>1)).
__device__ inline uint32_t quad_mask(float4 bb, int tx0, int ty0) {
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        float x0 = (float)(tx0 + (q & 1) * 8), y0 = (float)(ty0 + (q >> 1) * 8);
        bool hit = !(bb.z < x0 || bb.x > x0 + 7.f || bb.w < y0 || bb.y > y0 + 7.f);
        m |= hit ? (1u << q) : 0u;
    }
    return m;
}

// r: record (7 float4). (X,Y): pixel centre.
__device__ inline SplatEval eval_splat(const float4* r, float X, float Y, float S, float amin,
                                       float amax) {
    SplatEval e;
    float4 c1 = r[1], c2 = r[2], c3 = r[3];
    e.dx = X - c1.x;
    e.dy = Y - c1.y;
    float nu = fmaf(c1.z, e.dx, fmaf(c1.w, e.dy, c2.x));
    float nv = fmaf(c2.y, e.dx, fmaf(c2.z, e.dy, c2.w));
    e.den = fmaf(c3.x, e.dx, fmaf(c3.y, e.dy, c3.z));
    e.inv = __builtin_amdgcn_rcpf(e.den);     // v_rcp_f32, 1 ulp
    e.u = nu * e.inv;
    e.v = nv * e.inv;
    float m = fmaxf(fabsf(e.u), fabsf(e.v));
    // G = exp(-(u^2+v^2)/2) = exp2(-(log2 e)/2 (u^2+v^2))
    e.G = __builtin_amdgcn_exp2f(-0.72134752044448170368f * fmaf(e.u, e.u, e.v * e.v));
    e.oG = c3.w * e.G;
    e.alpha = fminf(amax, e.oG);
    e.hit = e.den > 0.f && m <= S && e.alpha >= amin;
    return e;
}

}  // namespace ts

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

// quad_mask refined through the (u,v) image of each 8x8 block. With a positive ray-plane
// denominator over the block, the block's pixel-centre rectangle maps to a convex
// quadrilateral whose corners are the images of the rectangle's corners, so the bounding box
// of those four (u,v) must reach the disk u^2+v^2 <= 2 ln(o/alpha_min) (where alpha >=
// alpha_min) and the square |u|,|v| <= S for any pixel of the block to pass eval_splat's hit
// test. Blocks whose denominator sign is uncertain are kept; the box is widened by a bound on
// the float32 rounding of both this test and eval_splat, and the disk and square are
// enlarged, so a block holding a hit is never dropped.
__device__ inline uint32_t quad_mask_uv(float4 bb, float4 c1, float4 c2, float4 c3, int tx0,
                                        int ty0, float S, float amin) {
    uint32_t m = quad_mask(bb, tx0, ty0);
    if (!m) return 0u;
    // 2 ln(o / alpha_min) = 2 ln2 (log2 o - log2 alpha_min)
    float r2 = 1.38629436f * (__builtin_amdgcn_logf(c3.w) - __builtin_amdgcn_logf(amin));
    r2 = fmaf(r2, 1.002f, 1e-3f);
    float Sx = fmaf(S, 1.001f, 1e-4f);
    uint32_t out = 0u;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (!((m >> q) & 1u)) continue;
        float xa = (float)(tx0 + (q & 1) * 8) + 0.5f - c1.x;
        float ya = (float)(ty0 + (q >> 1) * 8) + 0.5f - c1.y;
        float ul = 3.0e38f, uh = -3.0e38f, vl = 3.0e38f, vh = -3.0e38f;
        int npos = 0, nneg = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            float dx = xa + (float)((k & 1) * 7), dy = ya + (float)((k >> 1) * 7);
            float tu0 = c1.z * dx, tu1 = c1.w * dy;
            float tv0 = c2.y * dx, tv1 = c2.z * dy;
            float td0 = c3.x * dx, td1 = c3.y * dy;
            float nu = fmaf(c1.z, dx, fmaf(c1.w, dy, c2.x));
            float nv = fmaf(c2.y, dx, fmaf(c2.z, dy, c2.w));
            float den = fmaf(c3.x, dx, fmaf(c3.y, dy, c3.z));
            float dmag = fabsf(td0) + fabsf(td1) + fabsf(c3.z);
            if (den > 1e-4f * dmag) npos++;
            else if (den < -1e-4f * dmag) nneg++;
            float id = 1.0f / den;
            float u = nu * id, v = nv * id;
            // rounding bound (about 16 ulp of every term), for this test and eval_splat
            float eu = 2e-6f * ((fabsf(tu0) + fabsf(tu1) + fabsf(c2.x)) * fabsf(id) + fabsf(u) * dmag * fabsf(id));
            float ev = 2e-6f * ((fabsf(tv0) + fabsf(tv1) + fabsf(c2.w)) * fabsf(id) + fabsf(v) * dmag * fabsf(id));
            ul = fminf(ul, u - eu); uh = fmaxf(uh, u + eu);
            vl = fminf(vl, v - ev); vh = fmaxf(vh, v + ev);
        }
        bool keep;
        if (nneg == 4) keep = false;            // den <= 0 on the whole block: no hit
        else if (npos < 4) keep = true;         // the horizon may cross the block
        else {
            float cu = fminf(fmaxf(0.f, ul), uh), cv = fminf(fmaxf(0.f, vl), vh);
            keep = fmaf(cu, cu, cv * cv) <= r2 && ul <= Sx && uh >= -Sx && vl <= Sx && vh >= -Sx;
        }
        out |= keep ? (1u << q) : 0u;
    }
    return out;
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

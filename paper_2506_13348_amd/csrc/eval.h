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
    e.inv = 1.0f / e.den;
    e.u = nu * e.inv;
    e.v = nv * e.inv;
    float m = fmaxf(fabsf(e.u), fabsf(e.v));
    e.G = __expf(-0.5f * fmaf(e.u, e.u, e.v * e.v));
    e.oG = c3.w * e.G;
    e.alpha = fminf(amax, e.oG);
    e.hit = e.den > 0.f && m <= S && e.alpha >= amin;
    return e;
}

}  // namespace ts

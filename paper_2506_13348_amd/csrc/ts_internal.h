// Internal declarations shared by the texsplat HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "texsplat.h"

namespace ts {

constexpr int kTile = TS_TILE;           // 16x16 pixel tiles, one 256-thread workgroup each
constexpr int kRec = TS_REC_FLOATS;      // floats per projected record (7 float4)
constexpr int kRec4 = kRec / 4;
constexpr int kWave = 64;
constexpr int kXcd = 8;                  // MI355X: 8 XCDs, workgroups dealt round-robin

// record layout (float offsets)
//  0..3   pixel bounds ix0, iy0, ix1, iy1 (inclusive, pixel indices, as floats)
//  4..7   px, py (projected centre, float32 head of the double value), ux, uy
//  8..11  u0, vx, vy, v0
//  12..15 wx, wy, w0, opacity
//  16..24 sigma * R (row-major 3x3, world frame), 25 chart id (int bits),
//  26..27 px - px_head, py - py_head (float low parts of the projected centre)
// per pixel (X,Y) = pixel centre:   dx = X - px, dy = Y - py
//   num_u = ux dx + uy dy + u0,  num_v = vx dx + vy dy + v0,  den = wx dx + wy dy + w0
//   (u,v) = (num_u, num_v) / den, the ray meets the front of the plane iff den > 0

void set_error(const char* fmt, ...);
int launch_check(const char* what);

inline int tiles_x(int w) { return (w + kTile - 1) / kTile; }
inline int tiles_y(int h) { return (h + kTile - 1) / kTile; }

// Logical workgroup index such that each XCD receives a contiguous range (spatially adjacent
// tiles of one view then share that XCD's L2).
__device__ inline int xcd_remap(int i, int g) {
    int q = g / kXcd, r = g % kXcd;
    int x = i % kXcd, k = i / kXcd;
    return x * q + (x < r ? x : r) + k;
}

// Wave64 reductions with DPP lane moves (quad permutes, row mirrors, row broadcasts 15 and
// 31). The combination order is the same on every call, so the result is deterministic; the
// total ends in lanes 48..63 (read it from lane 63). `ident` fills lanes a move leaves unset.
template <typename Op>
__device__ inline int dpp_reduce_i(int x, int ident, Op op) {
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0x141, 0xF, 0xF, false));  // row half-mirror
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0x140, 0xF, 0xF, false));  // row mirror
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0x142, 0xA, 0xF, false));  // row bcast 15
    x = op(x, __builtin_amdgcn_update_dpp(ident, x, 0x143, 0xC, 0xF, false));  // row bcast 31
    return x;
}

__device__ inline float dpp_sum_f(float x) {
    auto add = [](int a, int b) { return __float_as_int(__int_as_float(a) + __int_as_float(b)); };
    return __int_as_float(dpp_reduce_i(__float_as_int(x), 0, add));
}

// Wave-uniform min / max of an int (from lane 63 of the DPP reduction).
__device__ inline int wave_min_dpp(int x) {
    int r = dpp_reduce_i(x, 0x7fffffff, [](int a, int b) { return min(a, b); });
    return __builtin_amdgcn_readlane(r, 63);
}
__device__ inline int wave_max_dpp(int x) {
    int r = dpp_reduce_i(x, (int)0x80000000, [](int a, int b) { return max(a, b); });
    return __builtin_amdgcn_readlane(r, 63);
}

// Buffer descriptor over one chart of the atlas (SGPR base, bounded to the chart's bytes: an
// out-of-range offset reads 0 instead of faulting). Word 3 = raw 32-bit data, gfx9 layout.
__device__ inline __amdgpu_buffer_rsrc_t chart_rsrc(const float4* chart_base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)chart_base, (short)0, (int)bytes, 0x00020000);
}

// The 8 channels of texel t of a chart: two 16-byte loads at byte offset 32 t.
__device__ inline void load_texel8(__amdgpu_buffer_rsrc_t r, unsigned t, float4& lo, float4& hi) {
    lo = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, t * 32u, 0, 0));
    hi = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, t * 32u + 16u, 0, 0));
}

__device__ inline unsigned lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace ts

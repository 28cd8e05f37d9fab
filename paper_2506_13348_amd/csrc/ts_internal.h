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

template <int kCtrl>
__device__ inline float dpp_f(float x) {
    return __builtin_amdgcn_update_dpp(-0.0f, x, kCtrl, 0xF, 0xF, false);
}
// Transposing wave sum of M = 4, 8, 16 or 32 values per lane: at each of log2 M levels a lane
// keeps half of its values and adds its partner's copy of that half (partners differ in one
// lane bit: quad permutes for bits 0-1, row shifts for bits 2-3, lane shuffles for bit 4), so
// each lane ends with one value summed over M lanes; plain butterfly sums over the remaining
// lane bits (up to bit 5) complete the totals. Lane l returns the total of value index
// bitrev_{log2 M}(l mod M) (M = 32: 16 b0 + 8 b1 + 4 b2 + 2 b3 + b4, b_k = bit k of the lane).
// The combination order is fixed, so the result is deterministic.
template <int M>
__device__ inline float wave_transpose_sum(float (&x)[M], int lane) {
    static_assert(M == 4 || M == 8 || M == 16 || M == 32, "4, 8, 16 or 32 values");
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    const bool b4 = (lane >> 4) & 1;
    constexpr int H1 = M / 2, H2 = M / 4, H3 = M / 8, H4 = M / 16;
#pragma unroll
    for (int j = 0; j < H1; j++) {   // partner lane ^ 1
        float lo = x[j], hi = x[H1 + j];
        float send = b0 ? lo : hi, keep = b0 ? hi : lo;
        x[j] = keep + dpp_f<0xB1>(send);
    }
#pragma unroll
    for (int j = 0; j < H2; j++) {   // partner lane ^ 2
        float lo = x[j], hi = x[H2 + j];
        float send = b1 ? lo : hi, keep = b1 ? hi : lo;
        x[j] = keep + dpp_f<0x4E>(send);
    }
    if constexpr (M >= 8) {
#pragma unroll
        for (int j = 0; j < H3; j++) {   // partner lane ^ 4
            float lo = x[j], hi = x[H3 + j];
            float send = b2 ? lo : hi, keep = b2 ? hi : lo;
            float from_up = dpp_f<0x104>(send), from_down = dpp_f<0x114>(send);
            x[j] = keep + (b2 ? from_down : from_up);
        }
    } else {
        float from_up = dpp_f<0x104>(x[0]), from_down = dpp_f<0x114>(x[0]);
        x[0] = b2 ? from_down + x[0] : x[0] + from_up;
    }
    if constexpr (M >= 16) {
#pragma unroll
        for (int j = 0; j < H4; j++) {   // partner lane ^ 8
            float lo = x[j], hi = x[H4 + j];
            float send = b3 ? lo : hi, keep = b3 ? hi : lo;
            float from_up = dpp_f<0x108>(send), from_down = dpp_f<0x118>(send);
            x[j] = keep + (b3 ? from_down : from_up);
        }
    } else {
        float from_up = dpp_f<0x108>(x[0]), from_down = dpp_f<0x118>(x[0]);
        x[0] = b3 ? from_down + x[0] : x[0] + from_up;
    }
    if constexpr (M == 32) {         // partner lane ^ 16
        float send = b4 ? x[0] : x[1], keep = b4 ? x[1] : x[0];
        x[0] = keep + __shfl_xor(send, 16);
    } else {
        float o = __shfl_xor(x[0], 16);
        x[0] = b4 ? o + x[0] : x[0] + o;
    }
    float o = __shfl_xor(x[0], 32);
    return lane & 32 ? o + x[0] : x[0] + o;
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
__device__ inline unsigned wave_or_dpp(unsigned x) {
    int r = dpp_reduce_i((int)x, 0, [](int a, int b) { return a | b; });
    return (unsigned)__builtin_amdgcn_readlane(r, 63);
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

// Error reporting, workspace sizing and atlas packing for the texsplat C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "ts_internal.h"
#include "binsort_layout.h"
#include "sort_kernels.h"

namespace ts {

static thread_local char g_err[512] = "no error";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return TS_E_LAUNCH;
    }
    return TS_OK;
}

// Packs per-primitive textures into charts: chart perm[k] <- primitive k (Supp. Sec. 1:
// the atlas holds every primitive's T x T texels, found through the indirection buffer).
__global__ void k_atlas_pack(const float4* __restrict__ tex, int n, int per_prim4,
                             const int32_t* __restrict__ perm, float4* __restrict__ atlas,
                             int32_t* __restrict__ chart_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)n * per_prim4;
    if (i >= total) return;
    int k = (int)(i / per_prim4);
    int o = (int)(i % per_prim4);
    int c = perm ? perm[k] : k;
    atlas[(int64_t)c * per_prim4 + o] = tex[i];
    if (o == 0) chart_of[k] = c;
}

// Bounding box of the centres: one block, strided min/max then a tree in LDS.
__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ means, int n,
                                              float* __restrict__ box) {
    __shared__ float lo[3][256], hi[3][256];
    int tid = threadIdx.x;
    float l[3] = {3.4e38f, 3.4e38f, 3.4e38f}, h[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
    for (int i = tid; i < n; i += 256)
        for (int c = 0; c < 3; c++) {
            float x = means[3 * i + c];
            l[c] = fminf(l[c], x);
            h[c] = fmaxf(h[c], x);
        }
    for (int c = 0; c < 3; c++) { lo[c][tid] = l[c]; hi[c][tid] = h[c]; }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o)
            for (int c = 0; c < 3; c++) {
                lo[c][tid] = fminf(lo[c][tid], lo[c][tid + o]);
                hi[c][tid] = fmaxf(hi[c][tid], hi[c][tid + o]);
            }
        __syncthreads();
    }
    if (tid < 3) { box[tid] = lo[tid][0]; box[3 + tid] = hi[tid][0]; }
}

__device__ inline uint32_t spread10(uint32_t x) {
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x030000ff;
    x = (x | (x << 8)) & 0x0300f00f;
    x = (x | (x << 4)) & 0x030c30c3;
    x = (x | (x << 2)) & 0x09249249;
    return x;
}

// 30-bit Morton code of each centre on a 1024^3 grid over the bounding box.
__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ means, int n,
                                                const float* __restrict__ box,
                                                uint32_t* __restrict__ code) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    for (int c = 0; c < 3; c++) {
        float ext = fmaxf(box[3 + c] - box[c], 1e-30f);
        float f = (means[3 * i + c] - box[c]) / ext;
        q[c] = (uint32_t)fminf(fmaxf(f * 1024.f, 0.f), 1023.f);
    }
    code[i] = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
}

__global__ __launch_bounds__(256) void k_rank(const int32_t* __restrict__ order, int n,
                                              int32_t* __restrict__ perm) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) perm[order[r]] = r;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_locality_perm_workspace(int32_t n, size_t* bytes) {
    if (!bytes || n < 0) {
        set_error("ts_locality_perm_workspace: bad argument");
        return TS_E_ARG;
    }
    size_t m = (size_t)(n > 0 ? n : 1);
    int nblk = n > 0 ? (n + kSortItems - 1) / kSortItems : 1;
    *bytes = align256(32) + 4 * align256(m * 4) + align256((size_t)kSortBuckets * nblk * 4);
    return TS_OK;
}

extern "C" int ts_locality_perm(const float* means, int32_t n, void* ws, size_t ws_bytes,
                                int32_t* perm, hipStream_t stream) {
    size_t need = 0;
    if (ts_locality_perm_workspace(n, &need) != TS_OK) return TS_E_ARG;
    if (n > 0 && (!means || !perm)) {
        set_error("ts_locality_perm: null array");
        return TS_E_ARG;
    }
    if (!ws || ws_bytes < need) {
        set_error("ts_locality_perm: workspace %zu < %zu bytes", ws_bytes, need);
        return TS_E_WORKSPACE;
    }
    if (n == 0) return TS_OK;
    char* w = (char*)ws;
    size_t m4 = align256((size_t)n * 4);
    float* box = (float*)w;
    uint32_t* code = (uint32_t*)(w + align256(32));
    uint32_t* ka = (uint32_t*)(w + align256(32) + m4);
    uint32_t* kb = (uint32_t*)(w + align256(32) + 2 * m4);
    int32_t* va = (int32_t*)(w + align256(32) + 3 * m4);
    uint32_t* hist = (uint32_t*)(w + align256(32) + 4 * m4);
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, stream, means, n, box);
    hipLaunchKernelGGL(k_morton, dim3((n + 255) / 256), dim3(256), 0, stream, means, n, box, code);
    // the codes are read by the first pass only, so the sorted order can land in their buffer
    int32_t* order = (int32_t*)code;
    radix_sort_indices(code, n, 1, ka, kb, va, hist, order, stream);
    hipLaunchKernelGGL(k_rank, dim3((n + 255) / 256), dim3(256), 0, stream, order, n, perm);
    return launch_check("ts_locality_perm");
}

extern "C" const char* ts_last_error(void) { return g_err; }

extern "C" int ts_raster_bwd_workspace(int32_t n_views, int32_t n, int64_t pair_capacity,
                                       size_t* bytes);
namespace ts { size_t env_bwd_bytes(int64_t n_tex); }
extern "C" int ts_atlas_charts_workspace(int32_t n, size_t* bytes);

extern "C" int ts_workspace_size(int32_t op, int32_t n_views, int32_t n, int32_t width,
                                 int32_t height, int64_t pair_capacity, size_t* bytes) {
    if (!bytes || n < 0) {
        set_error("ts_workspace_size: bad argument");
        return TS_E_ARG;
    }
    switch (op) {
        case TS_OP_BIN_SORT: {
            if (n_views < 1 || width < 1 || height < 1) {
                set_error("ts_workspace_size: bad argument");
                return TS_E_ARG;
            }
            *bytes = binsort_layout(n_views, n, width, height).total;
            return TS_OK;
        }
        case TS_OP_RASTER_BWD: return ts_raster_bwd_workspace(n_views, n, pair_capacity, bytes);
        case TS_OP_ENV_BWD:
            if (n < 1) {
                set_error("ts_workspace_size: the environment's table texels n must be >= 1");
                return TS_E_ARG;
            }
            *bytes = ts::env_bwd_bytes(n);
            return TS_OK;
        case TS_OP_LOCALITY_PERM: return ts_locality_perm_workspace(n, bytes);
        case TS_OP_ATLAS_CHARTS: return ts_atlas_charts_workspace(n, bytes);
        default:
            set_error("ts_workspace_size: unknown op %d", op);
            return TS_E_ARG;
    }
}

extern "C" int ts_atlas_pack(const float* textures, int32_t n, int32_t tex_res,
                             const int32_t* perm, float* atlas, int32_t* chart_of,
                             hipStream_t stream) {
    if (!textures || !atlas || !chart_of || n < 0 || tex_res < 1 || tex_res > 32) {
        set_error("ts_atlas_pack: bad argument");
        return TS_E_ARG;
    }
    if (n == 0) return TS_OK;
    int per4 = tex_res * tex_res * 2;
    int64_t total = (int64_t)n * per4;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_atlas_pack, dim3(blocks), dim3(256), 0, stream,
                       (const float4*)textures, n, per4, perm, (float4*)atlas, chart_of);
    return launch_check("ts_atlas_pack");
}

// Error reporting, workspace sizing and atlas packing for the texsplat C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "ts_internal.h"
#include "binsort_layout.h"

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

}  // namespace ts

using namespace ts;

extern "C" const char* ts_last_error(void) { return g_err; }

extern "C" int ts_workspace_size(int32_t op, int32_t n_views, int32_t n, int32_t width,
                                 int32_t height, size_t* bytes) {
    if (!bytes || n_views < 1 || n < 0 || width < 1 || height < 1) {
        set_error("ts_workspace_size: bad argument");
        return TS_E_ARG;
    }
    if (op != TS_OP_BIN_SORT) {
        set_error("ts_workspace_size: unknown op %d", op);
        return TS_E_ARG;
    }
    BinSortLayout L = binsort_layout(n_views, n, width, height);
    *bytes = L.total;
    return TS_OK;
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

// ts_bin_sort: per-view depth order (LSD radix sort of the float32 depth bits, 8 bits per
// pass, stable) and per-tile splat lists in that order (the global sort of the 2DGS-style
// rasteriser the paper builds on, Supp. Sec. 3).
//
// Tile lists without sorting (tile, depth) pairs: the depth-sorted splats of a view are cut
// into chunks; one wavefront per chunk counts, in LDS, how many of its splats cover each
// tile; the sum over chunks and a scan over tiles give every tile's list range; then one
// workgroup per (view, super-tile of 8x8 tiles) streams the view's rectangles in depth order
// and writes the lists of its 64 tiles, 256 splats at a time, each tile's entries of a batch
// at consecutive addresses. Each pair is written once (4 bytes) and the order inside every
// list is the depth order by construction.
#include <mutex>

#include "binsort_layout.h"
#include "sort_kernels.h"
#include "ts_internal.h"

namespace ts {

// ---------------------------------------------------------------------------------------
// radix sort (segmented by view)
// ---------------------------------------------------------------------------------------

// Per-block digit histogram, written digit-major per view: hist[v][d][b].
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ keys,
                                                            int n, int nblk, int shift,
                                                            uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kSortBuckets];
    int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t* kv = keys + (int64_t)v * n;
    int base = b * kSortItems;
    for (int r = 0; r < kSortItemsPerThread; r++) {
        int i = base + r * kSortThreads + tid;
        if (i < n) atomicAdd(&h[(kv[i] >> shift) & (kSortBuckets - 1)], 1u);
    }
    __syncthreads();
    hist[((int64_t)v * kSortBuckets + tid) * nblk + b] = h[tid];
}

// Exclusive scan of one view's hist (digit-major, block-minor), in place.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t part[1024];
    int v = blockIdx.x, tid = threadIdx.x;
    uint32_t* hv = hist + (int64_t)v * kSortBuckets * nblk;
    int m = kSortBuckets * nblk;
    int per = (m + 1023) / 1024;
    int s0 = tid * per, s1 = min(m, s0 + per);
    uint32_t sum = 0;
    for (int i = s0; i < s1; i++) sum += hv[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t x = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    uint32_t run = part[tid] - sum;
    for (int i = s0; i < s1; i++) {
        uint32_t x = hv[i];
        hv[i] = run;
        run += x;
    }
}

// Multi-block form of the same exclusive scan, for histograms too long for one block:
// per 1024-entry block totals, a one-block scan of those per segment, then each block's own
// scan plus its offset.
__device__ inline uint32_t block_excl_scan_u32(uint32_t x, uint32_t* sh, uint32_t* total) {
    int tid = threadIdx.x;
    sh[tid] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t y = tid >= o ? sh[tid - o] : 0u;
        __syncthreads();
        sh[tid] += y;
        __syncthreads();
    }
    uint32_t incl = sh[tid];
    if (total) *total = sh[1023];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(1024) void k_sort_scan_sums(const uint32_t* __restrict__ hist,
                                                         int nblk, int nbs,
                                                         uint32_t* __restrict__ tmp) {
    __shared__ uint32_t sh[1024];
    int b = blockIdx.x, v = blockIdx.y;
    int64_t m = (int64_t)kSortBuckets * nblk;
    int64_t i = (int64_t)b * 1024 + threadIdx.x;
    uint32_t x = i < m ? hist[(int64_t)v * m + i] : 0u;
    uint32_t tot;
    block_excl_scan_u32(x, sh, &tot);
    if (threadIdx.x == 0) tmp[(int64_t)v * nbs + b] = tot;
}

__global__ __launch_bounds__(1024) void k_sort_scan_tmp(uint32_t* __restrict__ tmp, int nbs) {
    __shared__ uint32_t sh[1024];
    int v = blockIdx.x;
    uint32_t* t = tmp + (int64_t)v * nbs;
    int per = (nbs + 1023) / 1024;
    int a0 = threadIdx.x * per, a1 = min(nbs, a0 + per);
    uint32_t s = 0;
    for (int i = a0; i < a1; i++) s += t[i];
    uint32_t run = block_excl_scan_u32(s, sh, nullptr);
    for (int i = a0; i < a1; i++) {
        uint32_t x = t[i];
        t[i] = run;
        run += x;
    }
}

__global__ __launch_bounds__(1024) void k_sort_scan_apply(uint32_t* __restrict__ hist, int nblk,
                                                          int nbs,
                                                          const uint32_t* __restrict__ tmp) {
    __shared__ uint32_t sh[1024];
    int b = blockIdx.x, v = blockIdx.y;
    int64_t m = (int64_t)kSortBuckets * nblk;
    int64_t i = (int64_t)b * 1024 + threadIdx.x;
    uint32_t x = i < m ? hist[(int64_t)v * m + i] : 0u;
    uint32_t ex = block_excl_scan_u32(x, sh, nullptr) + tmp[(int64_t)v * nbs + b];
    if (i < m) hist[(int64_t)v * m + i] = ex;
}

// Stable scatter. Wave w of the block owns items [w*1024, (w+1)*1024) of the block's range,
// taken 64 at a time in order; lanes with equal digits are ranked with ballots, and a
// per-wave running count per digit (LDS) carries ranks across rounds.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int n, int nblk,
    int shift, const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
    int32_t* __restrict__ vals_out) {
    __shared__ uint32_t cnt[kSortThreads / kWave][kSortBuckets];
    int b = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
    int w = tid / kWave, lane = tid % kWave;
    for (int i = tid; i < (kSortThreads / kWave) * kSortBuckets; i += kSortThreads)
        (&cnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t* kv = keys_in + (int64_t)v * n;
    const int32_t* vv = vals_in ? vals_in + (int64_t)v * n : nullptr;
    int base = b * kSortItems + w * (kSortItemsPerThread * kWave);
    uint32_t key[kSortItemsPerThread];
    int32_t val[kSortItemsPerThread];
    uint32_t loc[kSortItemsPerThread];
#pragma unroll
    for (int r = 0; r < kSortItemsPerThread; r++) {
        int i = base + r * kWave + lane;
        bool ok = i < n;
        uint32_t k = ok ? kv[i] : 0u;
        key[r] = k;
        val[r] = ok ? (vv ? vv[i] : i) : 0;
        uint32_t d = (k >> shift) & (kSortBuckets - 1);
        // lanes holding the same digit (invalid lanes excluded from every peer set)
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < kSortRadixBits; bit++) {
            uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        uint32_t old = ok ? cnt[w][d] : 0u;
        loc[r] = old + lanes_below(peers);
        bool leader = ok && ((peers >> lane) == 1ull);
        if (leader) cnt[w][d] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // wave offsets inside the block plus the block's global offset per digit
    {
        int d = tid;  // kSortThreads == kSortBuckets
        uint32_t g = offsets[((int64_t)v * kSortBuckets + d) * nblk + b];
        uint32_t run = g;
        for (int ww = 0; ww < kSortThreads / kWave; ww++) {
            uint32_t c = cnt[ww][d];
            cnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
    uint32_t* ko = keys_out + (int64_t)v * n;
    int32_t* vo = vals_out + (int64_t)v * n;
#pragma unroll
    for (int r = 0; r < kSortItemsPerThread; r++) {
        int i = base + r * kWave + lane;
        if (i < n) {
            uint32_t d = (key[r] >> shift) & (kSortBuckets - 1);
            uint32_t pos = cnt[w][d] + loc[r];
            ko[pos] = key[r];
            vo[pos] = val[r];
        }
    }
}

// Views of at most kSortItems splats: all four passes in one workgroup per view. The items
// stay in LDS between passes; each pass ranks them exactly as k_sort_scatter does (per-wave
// ballot ranking in item order, wave prefixes per digit), with the block's own exclusive scan
// of the 256 digit totals as the offsets, so the order is the same stable LSD sort.
static_assert(kSortThreads == kSortBuckets, "one thread per digit in the digit scans");
__global__ __launch_bounds__(kSortThreads) void k_sort_small(const uint32_t* __restrict__ keys,
                                                             int n,
                                                             int32_t* __restrict__ vals_out) {
    __shared__ uint32_t sk[kSortItems];
    __shared__ int32_t sv[kSortItems];
    __shared__ uint32_t cnt[kSortThreads / kWave][kSortBuckets];
    __shared__ uint32_t tot[kSortBuckets];
    const int v = blockIdx.x, tid = threadIdx.x;
    const int w = tid / kWave, lane = tid % kWave;
    const int base = w * (kSortItemsPerThread * kWave);
    const uint32_t* kv = keys + (int64_t)v * n;
    for (int i = tid; i < n; i += kSortThreads) {
        sk[i] = kv[i];
        sv[i] = i;
    }
    __syncthreads();
    for (int p = 0; p < kSortPasses; p++) {
        const int shift = p * kSortRadixBits;
        for (int i = tid; i < (kSortThreads / kWave) * kSortBuckets; i += kSortThreads)
            (&cnt[0][0])[i] = 0;
        __syncthreads();
        uint32_t key[kSortItemsPerThread];
        int32_t val[kSortItemsPerThread];
        uint32_t loc[kSortItemsPerThread];
#pragma unroll
        for (int r = 0; r < kSortItemsPerThread; r++) {
            int i = base + r * kWave + lane;
            bool ok = i < n;
            uint32_t k = ok ? sk[i] : 0u;
            key[r] = k;
            val[r] = ok ? sv[i] : 0;
            uint32_t d = (k >> shift) & (kSortBuckets - 1);
            uint64_t peers = __ballot(ok);
#pragma unroll
            for (int bit = 0; bit < kSortRadixBits; bit++) {
                uint64_t m = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? m : ~m;
            }
            uint32_t old = ok ? cnt[w][d] : 0u;
            loc[r] = old + lanes_below(peers);
            bool leader = ok && ((peers >> lane) == 1ull);
            if (leader) cnt[w][d] = old + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        {
            // digit d = tid: its count over the waves, then the exclusive scan over digits
            int d = tid;   // kSortThreads == kSortBuckets
            uint32_t t = 0;
            for (int ww = 0; ww < kSortThreads / kWave; ww++) t += cnt[ww][d];
            tot[d] = t;
            __syncthreads();
            for (int o = 1; o < kSortBuckets; o <<= 1) {
                uint32_t y = d >= o ? tot[d - o] : 0u;
                __syncthreads();
                tot[d] += y;
                __syncthreads();
            }
            uint32_t run = tot[d] - t;   // exclusive prefix of digit d
            for (int ww = 0; ww < kSortThreads / kWave; ww++) {
                uint32_t c = cnt[ww][d];
                cnt[ww][d] = run;
                run += c;
            }
        }
        __syncthreads();   // every item is in registers: the LDS rows can be overwritten
#pragma unroll
        for (int r = 0; r < kSortItemsPerThread; r++) {
            int i = base + r * kWave + lane;
            if (i < n) {
                uint32_t d = (key[r] >> shift) & (kSortBuckets - 1);
                uint32_t pos = cnt[w][d] + loc[r];
                sk[pos] = key[r];
                sv[pos] = val[r];
            }
        }
        __syncthreads();
    }
    int32_t* vo = vals_out + (int64_t)v * n;
    for (int i = tid; i < n; i += kSortThreads) vo[i] = sv[i];
}

// ---------------------------------------------------------------------------------------
// tile lists
// ---------------------------------------------------------------------------------------

struct BinArgs {
    int n, n_chunks, chunk, ntx, n_tiles;
    const int32_t* sorted;   // [V][n]
    const int4* rect;        // [V][n]
    uint32_t* counts;        // [V][n_chunks][n_tiles]
};

// LDS words the count kernel may use (64 KB); grids taller than that are counted in bands of
// tile rows, each a pass over the chunk's splats.
constexpr int kBinLdsWords = 16384;

__host__ __device__ inline int count_band_rows(int ntx) { return max(1, kBinLdsWords / (ntx + 1) - 1); }

// Counts per (view, chunk, tile): one wavefront per chunk adds each splat's rectangle into an
// LDS difference grid ((ntx+1) x (rows+1): +1 at (x0,y0) and (x1,y1), -1 at (x1,y0) and
// (x0,y1); integer adds, so the order does not matter), then a 2D prefix sum turns it into
// coverage counts. Rectangles are clipped to the band of tile rows in LDS.
__global__ __launch_bounds__(kWave) void k_bin_count(BinArgs a, int nty) {
    extern __shared__ uint32_t cnt[];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int v = bid / a.n_chunks, c = bid - v * a.n_chunks, lane = threadIdx.x;
    const int gw = a.ntx + 1, band = count_band_rows(a.ntx);
    int i0 = c * a.chunk, i1 = min(a.n, i0 + a.chunk);
    const int32_t* sv = a.sorted + (int64_t)v * a.n;
    const int4* rv = a.rect + (int64_t)v * a.n;
    uint32_t* row = a.counts + ((int64_t)v * a.n_chunks + c) * a.n_tiles;
    for (int y0 = 0; y0 < nty; y0 += band) {
        const int y1 = min(nty, y0 + band), gh = y1 - y0 + 1;
        for (int t = lane; t < gw * gh; t += kWave) cnt[t] = 0u;
        __syncthreads();
        for (int b = i0 + lane; b < i1; b += kWave) {
            int4 r = rv[sv[b]];
            int ya = max(r.y, y0) - y0, yb = min(r.w, y1) - y0;
            if (r.z <= r.x || yb <= ya) continue;
            atomicAdd(&cnt[ya * gw + r.x], 1u);
            atomicAdd(&cnt[yb * gw + r.z], 1u);
            atomicSub(&cnt[ya * gw + r.z], 1u);
            atomicSub(&cnt[yb * gw + r.x], 1u);
        }
        __syncthreads();
        // prefix along rows, then along columns (wrap-around arithmetic is exact)
        for (int y = lane; y < gh; y += kWave) {
            uint32_t run = 0;
            for (int x = 0; x < gw; x++) { run += cnt[y * gw + x]; cnt[y * gw + x] = run; }
        }
        __syncthreads();
        for (int x = lane; x < gw; x += kWave) {
            uint32_t run = 0;
            for (int y = 0; y < gh; y++) { run += cnt[y * gw + x]; cnt[y * gw + x] = run; }
        }
        __syncthreads();
        for (int t = y0 * a.ntx + lane; t < y1 * a.ntx; t += kWave) {
            int ty = t / a.ntx, tx = t - ty * a.ntx;
            row[t] = cnt[(ty - y0) * gw + tx];
        }
        __syncthreads();
    }
}

// Ordered fill by super-tiles of 8x8 tiles. One workgroup per (view, super-tile, group of
// chunks) streams the group's splats in depth order (their rectangles, packed and gathered
// once by k_bin_gather_rects, and ids; 1024 per step with the next step's loads in flight),
// keeps those touching its 64 tiles (appended in order to an LDS ring with a 64-bit tile mask
// each) and, 256 at a time, ranks them per tile with one ballot per (wave, tile): a splat's
// slot in tile b's list is the tile's cursor plus the earlier waves' counts plus the lanes
// below it in the ballot; the cursor starts at the tile's list start plus the chunk prefix of
// the group's first chunk. A tile's entries of a batch land at consecutive addresses (whole
// cache lines from one workgroup) instead of one 4-byte write per (chunk, tile) run; every
// list comes out in depth order, the same lists as a per-splat append. Views with few
// super-tiles are split into several chunk groups so that the grid still fills the chip.
constexpr int kSt = 8;                      // super-tile side in tiles (64 tiles: one mask bit each)
constexpr int kFillThreads = 256;
constexpr int kFillWaves = kFillThreads / kWave;
constexpr int kFillUnroll = 4;              // splats per thread and step
constexpr int kFillSpan = kFillThreads * kFillUnroll;
constexpr int kFillRing = 2048;             // >= 255 waiting + kFillSpan appended, power of two
constexpr int kFillTargetGroups = 4096;     // workgroups the grid aims at
static_assert(kFillRing >= kFillThreads - 1 + kFillSpan && (kFillRing & (kFillRing - 1)) == 0,
              "the ring holds the entries of a step plus an unprocessed remainder");

__global__ __launch_bounds__(256) void k_bin_gather_rects(const int32_t* __restrict__ sorted,
                                                          const int4* __restrict__ rect,
                                                          int64_t vn, int n,
                                                          uint2* __restrict__ srect) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= vn) return;
    int64_t v = i / n;
    int4 r = rect[v * n + sorted[i]];
    // tile coordinates are below 8192 (rows of more tiles are refused): 16 bits each
    bool empty = r.z <= r.x || r.w <= r.y;
    srect[i] = empty ? make_uint2(0u, 0u)
                     : make_uint2((uint32_t)r.x | ((uint32_t)r.z << 16),
                                  (uint32_t)r.y | ((uint32_t)r.w << 16));
}

// Tile mask of a packed rectangle within the super-tile at (tx0, ty0) of tw x th tiles
// (bit 8 y + x for tile (x, y) of the super-tile); 0 if they do not meet.
__device__ inline uint64_t super_tile_mask(uint2 r, int tx0, int ty0, int tw, int th) {
    const int x0 = max((int)(r.x & 0xFFFFu) - tx0, 0), x1 = min((int)(r.x >> 16) - tx0, tw);
    const int y0 = max((int)(r.y & 0xFFFFu) - ty0, 0), y1 = min((int)(r.y >> 16) - ty0, th);
    if (x1 <= x0 || y1 <= y0) return 0ull;
    const uint64_t row = ((1ull << (x1 - x0)) - 1ull) << x0;            // 1..8 bits
    const uint64_t rows = (0x0101010101010101ull >> (8 * (kSt - (y1 - y0)))) << (8 * y0);
    return row * rows;   // the row pattern in each selected byte (no carries: row < 256)
}

// Ranks and writes ring entries [head, head + count) (count <= kFillThreads).
__device__ inline void fill_st_batch(int head, int count, const int32_t* cid,
                                     const uint64_t* cmask, uint64_t (*wball)[64],
                                     uint32_t (*wbase)[64], uint32_t* cursor,
                                     int32_t* __restrict__ pair_ids, int64_t cap) {
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int e = (head + tid) & (kFillRing - 1);
    const uint64_t m = tid < count ? cmask[e] : 0ull;
    const int id = tid < count ? cid[e] : 0;
    // the wave's 64 per-tile ballots are the transpose of the 64 x 64 bit matrix whose row l is
    // lane l's tile mask: six stages, stage j swapping bit j of the row and column indices
    // between lanes l and l ^ j (lane b ends with the ballot of tile b; 64 ballots took about
    // five times the instructions)
    uint64_t t = m;
#pragma unroll
    for (int j = 32; j >= 1; j >>= 1) {
        const uint64_t lo = j == 32 ? 0x00000000FFFFFFFFull : j == 16 ? 0x0000FFFF0000FFFFull
                          : j == 8 ? 0x00FF00FF00FF00FFull : j == 4 ? 0x0F0F0F0F0F0F0F0Full
                          : j == 2 ? 0x3333333333333333ull : 0x5555555555555555ull;
        const uint64_t p = __shfl_xor(t, j);
        t = (lane & j) ? ((t & ~lo) | ((p >> j) & lo)) : ((t & lo) | ((p & lo) << j));
    }
    wball[w][lane] = t;
    __syncthreads();
    if (tid < 64) {
        uint32_t p = cursor[tid];
        for (int k = 0; k < kFillWaves; k++) {
            wbase[k][tid] = p;
            p += (uint32_t)__popcll(wball[k][tid]);
        }
        cursor[tid] = p;
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t mm = m;
    while (mm) {
        int b = __builtin_ctzll(mm);
        mm &= mm - 1;
        uint32_t pos = wbase[w][b] + (uint32_t)__popcll(wball[w][b] & below);
        if ((int64_t)pos < cap) pair_ids[pos] = id;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kFillThreads) void k_bin_fill_st(
    int n, int chunk, int n_chunks, int groups, int ntx, int nty, int nsx, int n_st,
    const int32_t* __restrict__ sorted, const uint2* __restrict__ srect,
    const uint32_t* __restrict__ prefix, const int32_t* __restrict__ ranges,
    int32_t* __restrict__ pair_ids, int64_t cap) {
    __shared__ uint32_t cursor[64];
    __shared__ int32_t cid[kFillRing];
    __shared__ uint64_t cmask[kFillRing];
    __shared__ uint64_t wball[kFillWaves][64];
    __shared__ uint32_t wbase[kFillWaves][64];
    __shared__ uint32_t wtot[kFillUnroll][kFillWaves];
    // the workgroups of a view on the same XCD: they stream the same rectangles
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int per_view = n_st * groups;
    const int v = bid / per_view, rem = bid - v * per_view;
    const int st = rem / groups, g = rem - st * groups;
    const int sy = st / nsx, sx = st - sy * nsx;
    const int tx0 = sx * kSt, ty0 = sy * kSt;
    const int tw = min(kSt, ntx - tx0), th = min(kSt, nty - ty0);
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int cpg = (n_chunks + groups - 1) / groups;
    const int c0 = min(n_chunks, g * cpg), c1 = min(n_chunks, c0 + cpg);
    const int i0 = min(n, c0 * chunk), i1 = min(n, c1 * chunk);
    if (i0 >= i1) return;   // the whole workgroup leaves together
    const int64_t n_tiles = (int64_t)ntx * nty;
    if (tid < 64) {
        const int lx = tid % kSt, ly = tid / kSt;
        uint32_t c = 0u;
        if (lx < tw && ly < th) {
            const int64_t t = (int64_t)(ty0 + ly) * ntx + tx0 + lx;
            c = (uint32_t)ranges[2 * ((int64_t)v * n_tiles + t)] +
                prefix[((int64_t)v * n_chunks + c0) * n_tiles + t];
        }
        cursor[tid] = c;
    }
    const uint2* sr = srect + (int64_t)v * n;
    const int32_t* sv = sorted + (int64_t)v * n;
    // head and count of the waiting entries (the same values in every thread)
    int head = 0, nc = 0;
    uint2 nr[kFillUnroll];
    int nid[kFillUnroll];
#pragma unroll
    for (int u = 0; u < kFillUnroll; u++) {
        const int i = i0 + u * kFillThreads + tid;
        nr[u] = i < i1 ? sr[i] : make_uint2(0u, 0u);
        nid[u] = i < i1 ? sv[i] : 0;
    }
    for (int b0 = i0; b0 < i1; b0 += kFillSpan) {
        uint64_t m[kFillUnroll];
        int id[kFillUnroll];
#pragma unroll
        for (int u = 0; u < kFillUnroll; u++) {
            m[u] = super_tile_mask(nr[u], tx0, ty0, tw, th);
            id[u] = nid[u];
        }
        // the next step's rectangles and ids in flight while this step is ranked and written
#pragma unroll
        for (int u = 0; u < kFillUnroll; u++) {
            const int i = b0 + kFillSpan + u * kFillThreads + tid;
            nr[u] = i < i1 ? sr[i] : make_uint2(0u, 0u);
            nid[u] = i < i1 ? sv[i] : 0;
        }
        // append the hits in list order: sub-step u, then wave, then lane
        uint64_t hit[kFillUnroll];
#pragma unroll
        for (int u = 0; u < kFillUnroll; u++) {
            hit[u] = __ballot(m[u] != 0ull);
            if (lane == 0) wtot[u][w] = (uint32_t)__popcll(hit[u]);
        }
        __syncthreads();
        int base = head + nc;
#pragma unroll
        for (int u = 0; u < kFillUnroll; u++) {
            int mine = base;
            for (int k = 0; k < kFillWaves; k++) {
                mine += k < w ? (int)wtot[u][k] : 0;
                base += (int)wtot[u][k];
            }
            if (m[u]) {
                const int pos = (mine + (int)lanes_below(hit[u])) & (kFillRing - 1);
                cid[pos] = id[u];
                cmask[pos] = m[u];
            }
        }
        nc = base - head;   // fewer than 256 waited, at most kFillSpan were added
        __syncthreads();
        while (nc >= kFillThreads) {
            fill_st_batch(head, kFillThreads, cid, cmask, wball, wbase, cursor, pair_ids, cap);
            head = (head + kFillThreads) & (kFillRing - 1);
            nc -= kFillThreads;
        }
    }
    if (nc > 0) fill_st_batch(head, nc, cid, cmask, wball, wbase, cursor, pair_ids, cap);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t m, uint32_t x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = x;
}

// Column scan over chunks per (view, tile): counts become exclusive prefixes. A workgroup
// takes 64 (view, tile) columns (lane = column, coalesced rows) and cuts the chunks into 16
// segments, one per wave: segment sums, their prefix across the waves in LDS, then each wave
// rewrites its segment. One column per thread walking every chunk would serialise thousands
// of dependent steps when one view is cut into many chunks.
constexpr int kScanSegs = 16;

__global__ __launch_bounds__(kScanSegs * kWave) void k_bin_scan_chunks(
    uint32_t* __restrict__ counts, int V, int n_chunks, int n_tiles, uint32_t* __restrict__ totals) {
    __shared__ uint32_t seg[kScanSegs][kWave];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t i = (int64_t)blockIdx.x * kWave + lane;
    const bool valid = i < (int64_t)V * n_tiles;
    const int v = valid ? (int)(i / n_tiles) : 0, t = valid ? (int)(i % n_tiles) : 0;
    uint32_t* col = counts + (int64_t)v * n_chunks * n_tiles + t;
    const int per = (n_chunks + kScanSegs - 1) / kScanSegs;
    const int c0 = min(n_chunks, wv * per), c1 = min(n_chunks, c0 + per);
    uint32_t s = 0;
    if (valid) {
#pragma unroll 8
        for (int c = c0; c < c1; c++) s += col[(int64_t)c * n_tiles];
    }
    seg[wv][lane] = s;
    __syncthreads();
    uint32_t run = 0;
    for (int k = 0; k < wv; k++) run += seg[k][lane];
    if (valid) {
#pragma unroll 8
        for (int c = c0; c < c1; c++) {
            uint32_t x = col[(int64_t)c * n_tiles];
            col[(int64_t)c * n_tiles] = run;
            run += x;
        }
        // the last segment ends at n_chunks: its running sum is the column total
        if (wv == kScanSegs - 1) totals[i] = run;
    }
}

// Exclusive scan of all (view, tile) totals in three steps: block sums, a scan of the block
// sums, then each block's own scan plus its offset -> ranges, total count, overflow status.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_scan_block_sums(const uint32_t* __restrict__ x,
                                                                int64_t m,
                                                                int64_t* __restrict__ sums) {
    __shared__ int64_t red[kScanBlock];
    int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    red[threadIdx.x] = i < m ? (int64_t)x[i] : 0;
    __syncthreads();
    for (int o = kScanBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh) {
    int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
        int64_t y = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += y;
        __syncthreads();
    }
    int64_t incl = sh[tid];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int64_t* __restrict__ sums, int nb,
                                                          int64_t cap,
                                                          int64_t* __restrict__ n_pairs,
                                                          int32_t* __restrict__ status) {
    __shared__ int64_t sh[kScanBlock];
    int64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanBlock) {
        int i = b0 + threadIdx.x;
        int64_t v = i < nb ? sums[i] : 0;
        int64_t ex = block_exclusive_scan(v, sh);
        if (i < nb) sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) sh[0] = ex + v;
        __syncthreads();
        carry += sh[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        n_pairs[0] = carry;
        status[0] = carry > cap ? 1 : 0;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_ranges(const uint32_t* __restrict__ x,
                                                            int64_t m,
                                                            const int64_t* __restrict__ sums,
                                                            int32_t* __restrict__ ranges) {
    __shared__ int64_t sh[kScanBlock];
    int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    int64_t v = i < m ? (int64_t)x[i] : 0;
    int64_t ex = block_exclusive_scan(v, sh) + sums[blockIdx.x];
    if (i < m) {
        ranges[2 * i] = (int32_t)min(ex, (int64_t)0x7FFFFFFF);
        ranges[2 * i + 1] = (int32_t)min(ex + v, (int64_t)0x7FFFFFFF);
    }
}

}  // namespace ts

using namespace ts;

namespace ts {

// Argument checks of ts_bin_sort and its scratch-array variant (no workspace involved).
static int bin_sort_check(const char* who, int32_t n_views, int32_t width, int32_t height,
                          int32_t n, const int32_t* rect, const uint32_t* depth_key,
                          int64_t pair_capacity, const int32_t* sorted_ids,
                          const int32_t* tile_ranges, const int32_t* pair_ids,
                          const int64_t* n_pairs, const int32_t* status) {
    if (n_views < 1 || width < 1 || height < 1 || n < 0 || pair_capacity < 0 || !tile_ranges ||
        !n_pairs || !status || (n > 0 && (!rect || !depth_key || !sorted_ids)) ||
        (pair_capacity > 0 && !pair_ids)) {
        set_error("%s: bad argument", who);
        return TS_E_ARG;
    }
    if (pair_capacity > 0x7FFFFFFFLL) {
        set_error("%s: pair_capacity above 2^31-1", who);
        return TS_E_ARG;
    }
    if (tiles_x(width) + 1 > kBinLdsWords / 2) {
        set_error("%s: %d tiles per row exceed the per-view limit", who, tiles_x(width));
        return TS_E_ARG;
    }
    return TS_OK;
}

// The kernels of ts_bin_sort on a checked argument set and a workspace of at least
// binsort_layout(...).total bytes. Every workspace word the kernels read is written by an
// earlier kernel of the same call, so the workspace needs no clearing.
static int bin_sort_enqueue(int32_t n_views, int32_t width, int32_t height, int32_t n,
                            const int32_t* rect, const uint32_t* depth_key, char* w,
                            int64_t pair_capacity, int32_t* sorted_ids, int32_t* tile_ranges,
                            int32_t* pair_ids, int64_t* n_pairs, int32_t* status,
                            hipStream_t stream) {
    BinSortLayout L = binsort_layout(n_views, n, width, height);
    uint32_t* keys_a = (uint32_t*)(w + L.off_keys_a);
    uint32_t* keys_b = (uint32_t*)(w + L.off_keys_b);
    int32_t* vals_a = (int32_t*)(w + L.off_vals_a);
    uint32_t* hist = (uint32_t*)(w + L.off_hist);
    uint32_t* counts = (uint32_t*)(w + L.off_counts);
    uint32_t* totals = (uint32_t*)(w + L.off_totals);
    int64_t* block_sums = (int64_t*)(w + L.off_blocksums);
    int rc;
    if (n > 0) {
        // pass p reads (keys_in, vals_in) and writes (keys_out, vals_out); the final pass
        // writes the splat ids to sorted_ids (also used as the ping-pong value buffer)
        if (n <= kSortItems)
            hipLaunchKernelGGL(k_sort_small, dim3(n_views), dim3(kSortThreads), 0, stream,
                               depth_key, n, sorted_ids);
        else
            radix_sort_indices(depth_key, n, n_views, keys_a, keys_b, vals_a, hist, sorted_ids,
                               stream);
        static_assert(kSortPasses % 2 == 0, "the last pass must land in sorted_ids");
        if ((rc = launch_check("ts_bin_sort(sort)")) != TS_OK) return rc;
    }
    BinArgs a;
    a.n = n; a.n_chunks = L.n_chunks; a.chunk = L.chunk; a.ntx = L.ntx; a.n_tiles = L.n_tiles;
    a.sorted = sorted_ids; a.rect = (const int4*)rect; a.counts = counts;
    size_t lds_count = (size_t)(L.ntx + 1) * (min(L.nty, count_band_rows(L.ntx)) + 1) * 4;
    if (n > 0) {
        hipLaunchKernelGGL(k_bin_count, dim3(L.n_chunks * n_views), dim3(kWave), lds_count,
                           stream, a, L.nty);
    } else {
        // a kernel, not a memset: the call may be captured into a graph
        int64_t mc = (int64_t)n_views * L.n_chunks * L.n_tiles;
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((mc + 255) / 256)), dim3(256), 0, stream,
                           counts, mc, 0u);
    }
    int64_t m = (int64_t)n_views * L.n_tiles;
    int nsb = (int)((m + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_bin_scan_chunks, dim3((unsigned)((m + kWave - 1) / kWave)),
                       dim3(kScanSegs * kWave), 0, stream, counts, n_views, L.n_chunks, L.n_tiles,
                       totals);
    hipLaunchKernelGGL(k_scan_block_sums, dim3(nsb), dim3(kScanBlock), 0, stream, totals, m,
                       block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, stream, block_sums, nsb,
                       pair_capacity, n_pairs, status);
    hipLaunchKernelGGL(k_scan_ranges, dim3(nsb), dim3(kScanBlock), 0, stream, totals, m,
                       block_sums, tile_ranges);
    if (n > 0) {
        // the sort's key buffers are free now: the packed rectangles in depth order go there
        uint2* srect = (uint2*)keys_a;
        const int64_t vn = (int64_t)n_views * n;
        hipLaunchKernelGGL(k_bin_gather_rects, dim3((unsigned)((vn + 255) / 256)), dim3(256), 0,
                           stream, sorted_ids, (const int4*)rect, vn, n, srect);
        const int nsx = (L.ntx + kSt - 1) / kSt, nsy = (L.nty + kSt - 1) / kSt;
        const int64_t units = (int64_t)n_views * nsx * nsy;
        const int groups = (int)max((int64_t)1, min((int64_t)L.n_chunks, kFillTargetGroups / units));
        hipLaunchKernelGGL(k_bin_fill_st, dim3((unsigned)(units * groups)), dim3(kFillThreads), 0,
                           stream, n, L.chunk, L.n_chunks, groups, L.ntx, L.nty, nsx, nsx * nsy,
                           sorted_ids, srect, counts, tile_ranges, pair_ids, pair_capacity);
    }
    return launch_check("ts_bin_sort(bin)");
}

}  // namespace ts

extern "C" int ts_bin_sort(int32_t n_views, int32_t width, int32_t height, int32_t n,
                           const int32_t* rect, const uint32_t* depth_key, void* ws,
                           size_t ws_bytes, int64_t pair_capacity, int32_t* sorted_ids,
                           int32_t* tile_ranges, int32_t* pair_ids, int64_t* n_pairs,
                           int32_t* status, hipStream_t stream) {
    int rc = bin_sort_check("ts_bin_sort", n_views, width, height, n, rect, depth_key,
                            pair_capacity, sorted_ids, tile_ranges, pair_ids, n_pairs, status);
    if (rc != TS_OK) return rc;
    const size_t need = binsort_layout(n_views, n, width, height).total;
    if (!ws || ws_bytes < need) {
        set_error("ts_bin_sort: workspace %zu < %zu bytes", ws_bytes, need);
        return TS_E_WORKSPACE;
    }
    return bin_sort_enqueue(n_views, width, height, n, rect, depth_key, (char*)ws, pair_capacity,
                            sorted_ids, tile_ranges, pair_ids, n_pairs, status, stream);
}

// ---- ts_bin_sort_noalloc: the same kernels on a library-owned scratch array ----------------
// A file-scope device array replaces the caller's workspace. In host code `scratch` is only a
// host-side stand-in for the symbol, so its device address (one per GPU: each device holds its
// own copy of the array) is taken once per device with hipGetSymbolAddress and only that
// address is passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace ts {

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, or null

// Device address of the scratch array on the current device (looked up on the first call per
// device, under a lock); null with the error set on failure.
static char* scratch_on_current_device(const char* who) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("%s: no current device (or device index above %d)", who, kMaxDevices - 1);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("%s: hipGetSymbolAddress(scratch) failed: %s", who, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = (char*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace ts

extern "C" size_t ts_bin_sort_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

extern "C" int ts_bin_sort_noalloc(int32_t n_views, int32_t width, int32_t height, int32_t n,
                                   const int32_t* rect, const uint32_t* depth_key,
                                   int64_t pair_capacity, int32_t* sorted_ids,
                                   int32_t* tile_ranges, int32_t* pair_ids, int64_t* n_pairs,
                                   int32_t* status, hipStream_t stream) {
    int rc = bin_sort_check("ts_bin_sort_noalloc", n_views, width, height, n, rect, depth_key,
                            pair_capacity, sorted_ids, tile_ranges, pair_ids, n_pairs, status);
    if (rc != TS_OK) return rc;
    const size_t need = binsort_layout(n_views, n, width, height).total;
    if (need > kNoAllocScratchBytes) {
        set_error("ts_bin_sort_noalloc: this call needs %zu bytes of scratch, above the %zu-byte "
                  "static array (use ts_bin_sort with a workspace)", need, kNoAllocScratchBytes);
        return TS_E_WORKSPACE;
    }
    char* w = scratch_on_current_device("ts_bin_sort_noalloc");
    if (!w) return TS_E_LAUNCH;
    // every scratch word the kernels read is written earlier in the same call, so the
    // contents left by a previous call need no clearing
    return bin_sort_enqueue(n_views, width, height, n, rect, depth_key, w, pair_capacity,
                            sorted_ids, tile_ranges, pair_ids, n_pairs, status, stream);
}

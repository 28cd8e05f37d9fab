// ts_bin_sort: per-view depth order (LSD radix sort of the float32 depth bits, 8 bits per
// pass, stable) and per-tile splat lists in that order (the global sort of the 2DGS-style
// rasteriser the paper builds on, Supp. Sec. 3).
//
// Tile lists without sorting (tile, depth) pairs: the depth-sorted splats of a view are cut
// into chunks; one wavefront per chunk counts, in LDS, how many of its splats cover each
// tile; a column scan over chunks plus a scan over tiles gives every (chunk, tile) its write
// offset; a second pass over each chunk, in order, writes the splat ids. Each pair is written
// once (4 bytes) and the order inside every list is the depth order by construction.
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
    const int32_t* ranges;   // [V][n_tiles][2] (fill)
    int32_t* pair_ids;
    int64_t cap;
};

// LDS words the count and fill kernels may use (64 KB); grids taller than that are done in
// bands of tile rows, each a pass over the chunk's splats.
constexpr int kBinLdsWords = 16384;
// The fill asks for at least 16 KB of LDS, so at most 10 chunk waves share a CU (160 KB):
// fewer tile lists are written at once and more of the partially written 128-byte lines are
// completed in the L2 before they leave it (measured on the 64-view sq100k step: 2.36 ms for
// ts_bin_sort at 16 waves per CU, 2.27 at 6, 2.14 at 8, 2.09 at 10, 2.16 at 12).
constexpr size_t kFillMinLds = 16 * 1024;

__host__ __device__ inline int count_band_rows(int ntx) { return max(1, kBinLdsWords / (ntx + 1) - 1); }
__host__ __device__ inline int fill_band_rows(int ntx) { return max(1, kBinLdsWords / ntx); }

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

// Ordered fill: one wavefront per (view, chunk) walks its splats in depth order; the lanes
// cover the splat's rectangle in 8x8 tile blocks; LDS cursors per tile give each entry its slot.
// Grids with more tiles than LDS words are filled in bands of tile rows (a pass each).
__global__ __launch_bounds__(kWave) void k_bin_fill(BinArgs a, int nty) {
    extern __shared__ uint32_t cur[];
    // every chunk of a view on the same XCD: the chunks write interleaved short runs of the
    // same tile lists, whose cache lines are then completed in one L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int v = bid / a.n_chunks, c = bid - v * a.n_chunks, lane = threadIdx.x;
    const uint32_t* row = a.counts + ((int64_t)v * a.n_chunks + c) * a.n_tiles;
    const int32_t* rg = a.ranges + (int64_t)v * a.n_tiles * 2;
    int i0 = c * a.chunk, i1 = min(a.n, i0 + a.chunk);
    const int32_t* sv = a.sorted + (int64_t)v * a.n;
    const int4* rv = a.rect + (int64_t)v * a.n;
    const int lx = lane & 7, ly = lane >> 3;
    const int band = fill_band_rows(a.ntx);
    for (int ya = 0; ya < nty; ya += band) {
        const int yb = min(nty, ya + band);
        const int t0 = ya * a.ntx;
        for (int t = t0 + lane; t < yb * a.ntx; t += kWave) cur[t - t0] = (uint32_t)rg[2 * t] + row[t];
        __syncthreads();
        for (int b = i0; b < i1; b += kWave) {
            int m = min(kWave, i1 - b);
            int id = lane < m ? sv[b + lane] : 0;
            int4 r = lane < m ? rv[id] : make_int4(0, 0, 0, 0);
            for (int j = 0; j < m; j++) {
                int x0 = __builtin_amdgcn_readlane(r.x, j), y0 = __builtin_amdgcn_readlane(r.y, j);
                int x1 = __builtin_amdgcn_readlane(r.z, j), y1 = __builtin_amdgcn_readlane(r.w, j);
                y0 = max(y0, ya);
                y1 = min(y1, yb);
                if (x1 <= x0 || y1 <= y0) continue;
                int sid = __builtin_amdgcn_readlane(id, j);
                for (int by = y0; by < y1; by += 8) {
                    for (int bx = x0; bx < x1; bx += 8) {
                        int tx = bx + lx, ty = by + ly;
                        if (tx < x1 && ty < y1) {
                            int t = ty * a.ntx + tx - t0;
                            uint32_t p = cur[t];
                            cur[t] = p + 1;
                            if ((int64_t)p < a.cap) a.pair_ids[p] = sid;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
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
    a.sorted = sorted_ids; a.rect = (const int4*)rect; a.counts = counts; a.ranges = tile_ranges;
    a.pair_ids = pair_ids; a.cap = pair_capacity;
    size_t lds_count = (size_t)(L.ntx + 1) * (min(L.nty, count_band_rows(L.ntx)) + 1) * 4;
    size_t lds_fill = (size_t)L.ntx * min(L.nty, fill_band_rows(L.ntx)) * 4;
    if (lds_fill < kFillMinLds) lds_fill = kFillMinLds;
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
    if (n > 0)
        hipLaunchKernelGGL(k_bin_fill, dim3(L.n_chunks * n_views), dim3(kWave), lds_fill, stream,
                           a, L.nty);
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

// Workspace layout of ts_bin_sort (host side).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "ts_internal.h"

namespace ts {

constexpr int kSortThreads = 256;
constexpr int kSortItemsPerThread = 16;
constexpr int kSortItems = kSortThreads * kSortItemsPerThread;   // keys per sort block
constexpr int kSortRadixBits = 8;
constexpr int kSortBuckets = 1 << kSortRadixBits;
constexpr int kSortPasses = 32 / kSortRadixBits;
constexpr int kBinTargetWaves = 4096;                             // chunks over all views

struct BinSortLayout {
    int n_tiles, ntx, nty;
    int sort_blocks;      // sort blocks per view
    int n_chunks;         // depth-ordered chunks per view for the tile-list build
    int chunk;            // splats per chunk
    size_t off_keys_a, off_keys_b, off_vals_a, off_hist, off_counts, off_totals, off_blocksums;
    size_t total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline BinSortLayout binsort_layout(int V, int n, int W, int H) {
    BinSortLayout L;
    L.ntx = tiles_x(W);
    L.nty = tiles_y(H);
    L.n_tiles = L.ntx * L.nty;
    L.sort_blocks = n > 0 ? (n + kSortItems - 1) / kSortItems : 1;
    int nch = (kBinTargetWaves + V - 1) / V;
    int max_ch = n > 0 ? (n + 31) / 32 : 1;
    if (nch > max_ch) nch = max_ch;
    if (nch < 1) nch = 1;
    L.chunk = n > 0 ? (n + nch - 1) / nch : 1;
    L.n_chunks = n > 0 ? (n + L.chunk - 1) / L.chunk : 1;
    size_t vn = (size_t)V * (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    L.off_keys_a = off; off = align256(off + vn * 4);
    L.off_keys_b = off; off = align256(off + vn * 4);
    L.off_vals_a = off; off = align256(off + vn * 4);
    L.off_hist = off;   off = align256(off + (size_t)V * kSortBuckets * L.sort_blocks * 4);
    L.off_counts = off; off = align256(off + (size_t)V * L.n_chunks * L.n_tiles * 4);
    L.off_totals = off; off = align256(off + (size_t)V * L.n_tiles * 4);
    L.off_blocksums = off; off = align256(off + (((size_t)V * L.n_tiles + 1023) / 1024 + 1) * 8);
    L.total = off;
    return L;
}

}  // namespace ts

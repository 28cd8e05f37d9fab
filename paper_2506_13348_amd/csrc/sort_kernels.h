// Radix-sort kernels of binsort.hip, shared with other entry points of the library.
#pragma once
#include "binsort_layout.h"

namespace ts {
__global__ void k_sort_hist(const uint32_t* __restrict__ keys, int n, int nblk, int shift,
                            uint32_t* __restrict__ hist);
__global__ void k_sort_scan(uint32_t* __restrict__ hist, int nblk);
__global__ void k_sort_scan_sums(const uint32_t* __restrict__ hist, int nblk, int nbs,
                                 uint32_t* __restrict__ tmp);
__global__ void k_sort_scan_tmp(uint32_t* __restrict__ tmp, int nbs);
__global__ void k_sort_scan_apply(uint32_t* __restrict__ hist, int nblk, int nbs,
                                  const uint32_t* __restrict__ tmp);

// Entries of the scratch the multi-block histogram scan needs per segment.
inline int sort_scan_tmp_entries(int n) {
    int nblk = n > 0 ? (n + kSortItems - 1) / kSortItems : 1;
    return (kSortBuckets * nblk + 1023) / 1024;
}
__global__ void k_sort_scatter(const uint32_t* __restrict__ keys_in,
                               const int32_t* __restrict__ vals_in, int n, int nblk, int shift,
                               const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
                               int32_t* __restrict__ vals_out);

// Stable LSD sort of n 32-bit keys per segment (grid.y segments of n keys each):
// vals_out[s][i] = index of the i-th smallest key of segment s, the keys themselves in that
// order in keys_b. `passes` digits of 8 bits from the lowest: with fewer than four the order
// is that of the low 8 * passes bits of each key. Scratch: keys_a, keys_b,
// vals_a of n * segs each and hist of segs * 256 * nblk words; scan_tmp (segs *
// sort_scan_tmp_entries(n) words) or null: the digit histograms are then scanned by one block
// per segment, which suits short histograms only.
inline void radix_sort_indices(const uint32_t* keys, int n, int segs, uint32_t* keys_a,
                               uint32_t* keys_b, int32_t* vals_a, uint32_t* hist,
                               int32_t* vals_out, hipStream_t stream,
                               uint32_t* scan_tmp = nullptr, int passes = kSortPasses) {
    int nblk = n > 0 ? (n + kSortItems - 1) / kSortItems : 1;
    int nbs = sort_scan_tmp_entries(n);
    const uint32_t* kin = keys;
    const int32_t* vin = nullptr;
    for (int p = 0; p < passes; p++) {
        // the last pass writes keys_b / vals_out, earlier ones alternate back from there
        bool last_parity = ((passes - 1 - p) & 1) == 0;
        uint32_t* kout = last_parity ? keys_b : keys_a;
        int32_t* vout = last_parity ? vals_out : vals_a;
        int shift = p * kSortRadixBits;
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk, segs), dim3(kSortThreads), 0, stream, kin, n,
                           nblk, shift, hist);
        if (scan_tmp) {
            hipLaunchKernelGGL(k_sort_scan_sums, dim3(nbs, segs), dim3(1024), 0, stream, hist,
                               nblk, nbs, scan_tmp);
            hipLaunchKernelGGL(k_sort_scan_tmp, dim3(segs), dim3(1024), 0, stream, scan_tmp, nbs);
            hipLaunchKernelGGL(k_sort_scan_apply, dim3(nbs, segs), dim3(1024), 0, stream, hist,
                               nblk, nbs, scan_tmp);
        } else {
            hipLaunchKernelGGL(k_sort_scan, dim3(segs), dim3(1024), 0, stream, hist, nblk);
        }
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk, segs), dim3(kSortThreads), 0, stream, kin,
                           vin, n, nblk, shift, hist, kout, vout);
        kin = kout;
        vin = vout;
    }
}
}  // namespace ts

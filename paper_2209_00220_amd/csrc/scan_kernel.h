// Single-column scans of the slice layouts (PP-VBS, ByteSlice): one wave per
// 2048-row tile, grid-stride over tiles, the next tiles' loads in flight.
#pragma once

#include "slice_scan.h"

namespace bst {
namespace dev {

template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(scan_waves<MODE, SHORT, DENSE>(), 8))) void k_scan_slices(
    const DevCol c, const ScanLit lit, const uint64_t* __restrict__ in_mask, uint64_t* __restrict__ out,
    unsigned long long* __restrict__ counters) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[kWavesPerBlock][kWaveLds];
    uint8_t* lds = stage[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Stats st;
    scan_slices_range<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, in_mask, out, wave, c.ntiles, nwaves, lane, lds, st);
    if (COUNT) flush_stats(counters, st, lane);
}

template <int MODE, int SHORT, bool COUNT>
static void launch_slices_s(uint32_t grid, hipStream_t st, const DevCol& c, const ScanLit& lit,
                            const uint64_t* in, uint64_t* out, unsigned long long* counters) {
    const bool dense = c.layout == BST_BYTESLICE;
#define BST_GO(D, I)                                                                                           \
    hipLaunchKernelGGL((k_scan_slices<MODE, SHORT, D, I, COUNT>), dim3(grid), dim3(kBlock), 0, st, c, lit, in, \
                       out, counters)
    if (dense) {
        if (in) BST_GO(true, true); else BST_GO(true, false);
    } else {
        if (in) BST_GO(false, true); else BST_GO(false, false);
    }
#undef BST_GO
}

// Launch one slice-layout scan whose literal mode is MODE.
template <int MODE>
int launch_slices_mode(const DevCol& c, const ScanLit& lit, const uint64_t* in, uint64_t* out,
                       unsigned long long* counters, hipStream_t st) {
    // Workgroups per CU: 3 where the literal is settled by byte 1 (fewer
    // concurrent streams read faster) and for ByteSlice '<', '>' and '='; 4 for
    // PP-VBS literals of several bytes and ByteSlice BETWEEN, whose gathers and
    // compares need more waves to keep HBM busy (measured on the 500M-row
    // benchmark column: 5 % less time for the PP-VBS scans concerned, 1 % for
    // the ByteSlice step).
    const bool byte1 = lit.llo == 1 && (MODE != kModeBetween || lit.lhi == 1);
    const uint32_t per_cu = (!byte1 && (c.layout == BST_PPVBS || MODE == kModeBetween)) ? 4u : 3u;
    const uint32_t grid = tile_grid(c.ntiles, g_tune[BST_TUNE_SCAN_GRID], per_cu);
    if (counters) {
        launch_slices_s<MODE, -1, true>(grid, st, c, lit, in, out, counters);
    } else {
        const int sh = (lit.llo == 1 ? 1 : 0) | (MODE == kModeBetween && lit.lhi == 1 ? 2 : 0);
        if constexpr (MODE == kModeBetween) {
            switch (sh) {
                case 0: launch_slices_s<MODE, 0, false>(grid, st, c, lit, in, out, nullptr); break;
                case 1: launch_slices_s<MODE, 1, false>(grid, st, c, lit, in, out, nullptr); break;
                case 2: launch_slices_s<MODE, 2, false>(grid, st, c, lit, in, out, nullptr); break;
                default: launch_slices_s<MODE, 3, false>(grid, st, c, lit, in, out, nullptr); break;
            }
        } else {
            if (sh & 1) launch_slices_s<MODE, 1, false>(grid, st, c, lit, in, out, nullptr);
            else launch_slices_s<MODE, 0, false>(grid, st, c, lit, in, out, nullptr);
        }
    }
    return hip_check(hipGetLastError(), "scan_slices launch");
}

extern template int launch_slices_mode<kModeLT>(const DevCol&, const ScanLit&, const uint64_t*, uint64_t*,
                                                unsigned long long*, hipStream_t);
extern template int launch_slices_mode<kModeGT>(const DevCol&, const ScanLit&, const uint64_t*, uint64_t*,
                                                unsigned long long*, hipStream_t);
extern template int launch_slices_mode<kModeEQ>(const DevCol&, const ScanLit&, const uint64_t*, uint64_t*,
                                                unsigned long long*, hipStream_t);
extern template int launch_slices_mode<kModeBetween>(const DevCol&, const ScanLit&, const uint64_t*, uint64_t*,
                                                     unsigned long long*, hipStream_t);

}  // namespace dev
}  // namespace bst

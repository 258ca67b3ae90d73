// Single-column scans of the slice layouts (PP-VBS, ByteSlice): one wave per
// 2048-row tile, grid-stride over tiles.
#include "device_common.h"

namespace bst {
namespace dev {

template <int MODE, bool DENSE, bool HAS_IN, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_scan_slices(const DevCol c, const ScanLit lit,
                                                        const uint64_t* __restrict__ in_mask,
                                                        uint64_t* __restrict__ out,
                                                        unsigned long long* __restrict__ counters) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Stats st;
    for (uint64_t t = wave; t < c.ntiles; t += nwaves)
        scan_slices_tile<MODE, DENSE, HAS_IN, COUNT>(c, lit, in_mask, out, t, lane, st);
    if (COUNT) flush_stats(counters, st, lane);
}

template <int MODE, bool DENSE, bool COUNT>
static void launch_slices_m(uint32_t grid, hipStream_t st, const DevCol& c, const ScanLit& lit, const uint64_t* in,
                            uint64_t* out, unsigned long long* counters) {
    if (in)
        hipLaunchKernelGGL((k_scan_slices<MODE, DENSE, true, COUNT>), dim3(grid), dim3(kBlock), 0, st, c, lit, in, out,
                           counters);
    else
        hipLaunchKernelGGL((k_scan_slices<MODE, DENSE, false, COUNT>), dim3(grid), dim3(kBlock), 0, st, c, lit, in,
                           out, counters);
}

template <bool COUNT>
static int launch_slices_t(const DevCol& c, const ScanLit& lit, const uint64_t* in, uint64_t* out,
                           unsigned long long* counters, hipStream_t st) {
    const uint32_t grid = tile_grid(c.ntiles, g_tune[BST_TUNE_SCAN_GRID]);
    const bool dense = c.layout == BST_BYTESLICE;
#define BST_LS(MODE)                                                                     \
    if (dense) launch_slices_m<MODE, true, COUNT>(grid, st, c, lit, in, out, counters); \
    else launch_slices_m<MODE, false, COUNT>(grid, st, c, lit, in, out, counters);
    switch (lit.mode) {
        case kModeLT: BST_LS(kModeLT) break;
        case kModeGT: BST_LS(kModeGT) break;
        case kModeEQ: BST_LS(kModeEQ) break;
        case kModeBetween: BST_LS(kModeBetween) break;
        default: return set_error(BST_EINVAL, "bad literal mode");
    }
#undef BST_LS
    return hip_check(hipGetLastError(), "scan_slices launch");
}

int launch_slices(const DevCol& c, const ScanLit& lit, const uint64_t* in, uint64_t* out,
                  unsigned long long* counters, hipStream_t st) {
    if (counters) return launch_slices_t<true>(c, lit, in, out, counters, st);
    return launch_slices_t<false>(c, lit, in, out, nullptr, st);
}

}  // namespace dev
}  // namespace bst

// Single-column Bit-Packed scans, code widths 1..16.
#include "device_common.h"

namespace bst {
namespace dev {

template <int W, bool HAS_IN>
__global__ __launch_bounds__(kBlock) void k_scan_packed(const DevCol c, const PackedLit pl,
                                                        const uint64_t* __restrict__ in_mask,
                                                        uint64_t* __restrict__ out,
                                                        unsigned long long* __restrict__ counters) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    uint64_t alg = 0;
    scan_packed_range<W, HAS_IN>(c, pl, in_mask, out, wave, c.ntiles, nwaves, lane, alg);
    if (counters) {
        Stats st;
        st.alg = alg;
        st.full = alg;
        st.lines = alg / 128;   // whole words of whole tiles: every byte's line is read in full
        flush_stats(counters, st, lane);
    }
}

template <int W>
static void launch_packed_w(uint32_t grid, hipStream_t st, const DevCol& c, const PackedLit& pl, const uint64_t* in,
                            uint64_t* out, unsigned long long* counters) {
    if (in) hipLaunchKernelGGL((k_scan_packed<W, true>), dim3(grid), dim3(kBlock), 0, st, c, pl, in, out, counters);
    else hipLaunchKernelGGL((k_scan_packed<W, false>), dim3(grid), dim3(kBlock), 0, st, c, pl, in, out, counters);
}

int launch_packed_1_16(const DevCol& c, const PackedLit& pl, const uint64_t* in, uint64_t* out,
                      unsigned long long* counters, hipStream_t st) {
    const uint32_t grid = tile_grid(c.ntiles, g_tune[BST_TUNE_SCAN_GRID], 2);
    switch (c.width) {
#define BST_LW(W) \
    case W: launch_packed_w<W>(grid, st, c, pl, in, out, counters); break;
        BST_LW(1) BST_LW(2) BST_LW(3) BST_LW(4) BST_LW(5) BST_LW(6) BST_LW(7) BST_LW(8) BST_LW(9) BST_LW(10) BST_LW(11) BST_LW(12) BST_LW(13) BST_LW(14) BST_LW(15) BST_LW(16)
#undef BST_LW
        default:
            return set_error(BST_EINVAL, "bad Bit-Packed width");
    }
    return hip_check(hipGetLastError(), "scan_packed launch");
}

}  // namespace dev
}  // namespace bst

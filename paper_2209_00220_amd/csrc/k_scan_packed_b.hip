// Single-column Bit-Packed scans, code widths 17..32.
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

int launch_packed_17_32(const DevCol& c, const PackedLit& pl, const uint64_t* in, uint64_t* out,
                      unsigned long long* counters, hipStream_t st) {
    const uint32_t grid = tile_grid(c.ntiles, g_tune[BST_TUNE_SCAN_GRID], 2);
    switch (c.width) {
#define BST_LW(W) \
    case W: launch_packed_w<W>(grid, st, c, pl, in, out, counters); break;
        BST_LW(17) BST_LW(18) BST_LW(19) BST_LW(20) BST_LW(21) BST_LW(22) BST_LW(23) BST_LW(24) BST_LW(25) BST_LW(26) BST_LW(27) BST_LW(28) BST_LW(29) BST_LW(30) BST_LW(31) BST_LW(32)
#undef BST_LW
        default:
            return set_error(BST_EINVAL, "bad Bit-Packed width");
    }
    return hip_check(hipGetLastError(), "scan_packed launch");
}

int launch_packed_1_16(const DevCol&, const PackedLit&, const uint64_t*, uint64_t*, unsigned long long*, hipStream_t);

int launch_packed(const DevCol& c, const PackedLit& pl, const uint64_t* in, uint64_t* out,
                  unsigned long long* counters, hipStream_t st) {
    if (c.width >= 1 && c.width <= 16) return launch_packed_1_16(c, pl, in, out, counters, st);
    return launch_packed_17_32(c, pl, in, out, counters, st);
}

}  // namespace dev
}  // namespace bst

// Persistent batch kernel of the slice layouts (PP-VBS, ByteSlice), shared by
// the translation units that instantiate its variants.
#pragma once

#include "slice_scan.h"

namespace bst {
namespace dev {

// Tiles are handed out in takes of `grab` consecutive tiles of the group's
// concatenated tile list.  A wave's first take is fixed by its index; later
// takes come from the group's counter and lie past the region of first takes
// (waves * grab tiles).  So a group that the first takes cover costs no atomic,
// and a large one costs one atomic per later take: atomics on one address
// serialise, and thousands of them would cost more than a small group's scan.
__device__ __forceinline__ uint64_t batch_first_take(uint32_t grab) {
    return (uint64_t)uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)) * grab;
}

__device__ __forceinline__ uint64_t batch_next_take(unsigned long long* counter, uint32_t grab, uint64_t total,
                                                    uint32_t lane) {
    const uint64_t fixed = (uint64_t)gridDim.x * kWavesPerBlock * grab;
    if (fixed >= total) return total;
    uint64_t s = 0;
    if (lane == 0) s = atomicAdd(counter, (unsigned long long)grab);
    s = ((uint64_t)uniform((uint32_t)(s >> 32)) << 32) | uniform((uint32_t)s);
    return fixed + s;
}

// Waves scan their takes item by item (a take may straddle items); the
// per-tile work is the single-column scan's, inlined.
template <int MODE, int SHORT, bool DENSE, bool HAS_IN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kMinWaves, 8))) void k_batch_slices(
    const BatchHeader* __restrict__ hdr, const BatchItem* __restrict__ items, unsigned long long* __restrict__ counter,
    uint32_t grab) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[kWavesPerBlock][kWaveLds];
    uint8_t* lds = stage[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t total = hdr->total_tiles;
    const uint32_t n_items = hdr->n_items;
    Stats st;
    for (uint64_t start = batch_first_take(grab); start < total;
         start = batch_next_take(counter, grab, total, lane)) {
        const uint64_t stop = std::min<uint64_t>(total, start + grab);
        for (uint32_t cur = batch_find(items, n_items, start); cur < n_items && items[cur].tile0 < stop; ++cur) {
            const BatchItem& it = items[cur];
            const uint64_t b0 = std::max<uint64_t>(start, it.tile0) - it.tile0;
            const uint64_t b1 = std::min<uint64_t>(stop, it.tile0 + it.c.ntiles) - it.tile0;
            scan_slices_range<MODE, SHORT, DENSE, HAS_IN, false>(it.c, it.lit, it.in_mask, it.out, b0, b1, 1, lane,
                                                                  lds, st);
        }
    }
}

}  // namespace dev
}  // namespace bst

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

// The segments (item, first tile, end tile, stride) a wave scans, one at a
// time, so that a kernel inlines its tile scan once for both assignments:
//  * takes (grab > 0): consecutive tiles of the group's concatenated tile list,
//    item by item (a take may straddle items), stride 1;
//  * round robin (grab == 0): the group's tile g goes to wave g mod W of the W
//    waves in the launch, so each item is scanned as a single-column launch
//    scans it (a wave takes every W-th tile, neighbouring waves neighbouring
//    tiles), the waves get equal tile counts within one, and no counter is
//    touched.
struct BatchSegments {
    const BatchItem* __restrict__ items;
    unsigned long long* __restrict__ counter;
    uint64_t total, start, stop, waves, wave;
    uint32_t n_items, grab, lane, cur;

    __device__ __forceinline__ BatchSegments(const BatchHeader* __restrict__ hdr, const BatchItem* __restrict__ it,
                                             unsigned long long* __restrict__ ctr, uint32_t g, uint32_t ln)
        : items(it), counter(ctr), total(hdr->total_tiles), start(0), stop(0),
          waves((uint64_t)gridDim.x * kWavesPerBlock), wave(uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6))),
          n_items(hdr->n_items), grab(g), lane(ln), cur(0) {
        if (grab) {
            start = batch_first_take(grab);
            stop = std::min<uint64_t>(total, start + grab);
            cur = start < total ? batch_find(items, n_items, start) : n_items;
        }
    }

    __device__ __forceinline__ bool next(uint32_t& item, uint64_t& b0, uint64_t& b1, uint64_t& stride) {
        if (!grab) {
            for (; cur < n_items; ++cur) {
                const uint64_t first = (wave + waves - items[cur].tile0 % waves) % waves;
                if (first < items[cur].c.ntiles) {
                    item = cur++;
                    b0 = first;
                    b1 = items[item].c.ntiles;
                    stride = waves;
                    return true;
                }
            }
            return false;
        }
        while (start < total) {
            if (cur < n_items && items[cur].tile0 < stop) {
                const BatchItem& it = items[cur];
                b0 = std::max<uint64_t>(start, it.tile0) - it.tile0;
                b1 = std::min<uint64_t>(stop, it.tile0 + it.c.ntiles) - it.tile0;
                stride = 1;
                item = cur++;
                return true;
            }
            start = batch_next_take(counter, grab, total, lane);
            if (start >= total) return false;
            stop = std::min<uint64_t>(total, start + grab);
            cur = batch_find(items, n_items, start);
        }
        return false;
    }
};

// Waves per SIMD a batch variant is built for: the single-column variant's
// where a tile ends with its byte-1 pass; kMinWaves where later levels are read,
// since the item loop around the tile state needs the registers.
template <int MODE, int SHORT, bool DENSE>
constexpr int batch_waves() {
    return (SliceScan<MODE, SHORT, DENSE, false, false>::kByte1Only || SHORT == 0) ? scan_waves<MODE, SHORT, DENSE>()
                                                                                    : kMinWaves;
}

// Waves scan their segments (BatchSegments); the per-tile work is the
// single-column scan's, inlined.
template <int MODE, int SHORT, bool DENSE, bool HAS_IN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(batch_waves<MODE, SHORT, DENSE>(), 8))) void k_batch_slices(
    const BatchHeader* __restrict__ hdr, const BatchItem* __restrict__ items, unsigned long long* __restrict__ counter,
    uint32_t grab) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[kWavesPerBlock][kWaveLds];
    uint8_t* lds = stage[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63;
    Stats st;
    BatchSegments seg(hdr, items, counter, grab, lane);
    uint32_t i;
    uint64_t b0, b1, stride;
    while (seg.next(i, b0, b1, stride)) {
        const BatchItem& it = items[uniform(i)];
        scan_slices_range<MODE, SHORT, DENSE, HAS_IN, false>(it.c, it.lit, it.in_mask, it.out, b0, b1, stride, lane,
                                                              lds, st);
    }
}

}  // namespace dev
}  // namespace bst

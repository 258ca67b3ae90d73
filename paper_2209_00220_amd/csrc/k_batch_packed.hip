// Batched Bit-Packed scans: one persistent kernel per code width (own
// translation unit, compiled alongside the slice-layout batch kernels).
#include "batch_kernel.h"

namespace bst {
namespace dev {

template <int W, bool HAS_IN>
__global__ __launch_bounds__(kBlock) void k_batch_packed(const BatchHeader* __restrict__ hdr,
                                                         const BatchItem* __restrict__ items,
                                                         unsigned long long* __restrict__ counter, uint32_t grab) {
    const uint32_t lane = threadIdx.x & 63;
    uint64_t alg = 0;
    BatchSegments seg(hdr, items, counter, grab, lane);
    uint32_t i;
    uint64_t b0, b1, stride;
    while (seg.next(i, b0, b1, stride)) {
        const BatchItem& it = items[uniform(i)];
        scan_packed_range<W, HAS_IN>(it.c, it.pl, it.in_mask, it.out, b0, b1, stride, lane, alg);
    }
}

BatchKernel batch_packed_kernel(uint32_t w, bool has_in) {
    switch (w) {
#define BST_W(W) \
    case W: return has_in ? k_batch_packed<W, true> : k_batch_packed<W, false>;
        BST_W(1) BST_W(2) BST_W(3) BST_W(4) BST_W(5) BST_W(6) BST_W(7) BST_W(8)
        BST_W(9) BST_W(10) BST_W(11) BST_W(12) BST_W(13) BST_W(14) BST_W(15) BST_W(16)
        BST_W(17) BST_W(18) BST_W(19) BST_W(20) BST_W(21) BST_W(22) BST_W(23) BST_W(24)
        BST_W(25) BST_W(26) BST_W(27) BST_W(28) BST_W(29) BST_W(30) BST_W(31) BST_W(32)
#undef BST_W
        default: return nullptr;
    }
}

}  // namespace dev
}  // namespace bst

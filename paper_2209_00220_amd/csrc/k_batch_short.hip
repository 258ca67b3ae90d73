// Batched slice-layout scans whose literals are one byte long (settled by byte 1
// and the presence of byte 2), compiled in their own translation unit.
#include "batch_kernel.h"

namespace bst {
namespace dev {

BatchKernel batch_short_kernel(int mi, bool dense, bool has_in) {
#define BST_K(MODE, SH)                                                                                    \
    return dense ? (has_in ? k_batch_slices<MODE, SH, true, true> : k_batch_slices<MODE, SH, true, false>) \
                 : (has_in ? k_batch_slices<MODE, SH, false, true> : k_batch_slices<MODE, SH, false, false>)
    switch (mi) {
        case 0: BST_K(kModeLT, 1);
        case 1: BST_K(kModeGT, 1);
        case 2: BST_K(kModeEQ, 1);
        default: BST_K(kModeBetween, 3);
    }
#undef BST_K
}

}  // namespace dev
}  // namespace bst

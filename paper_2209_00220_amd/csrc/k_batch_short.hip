// Batched slice-layout scans whose literals are one byte long (settled by byte 1
// and the presence of byte 2), compiled in their own translation unit.
#include "batch_kernel.h"

namespace bst {
namespace dev {

BatchKernel batch_short_kernel(int mi, bool dense, bool has_in, bool rr) {
#define BST_KR(MODE, SH, RR)                                                                           \
    (dense ? (has_in ? k_batch_slices<MODE, SH, true, true, RR> : k_batch_slices<MODE, SH, true, false, RR>) \
           : (has_in ? k_batch_slices<MODE, SH, false, true, RR> : k_batch_slices<MODE, SH, false, false, RR>))
#define BST_K(MODE, SH) return rr ? BST_KR(MODE, SH, true) : BST_KR(MODE, SH, false)
    switch (mi) {
        case 0: BST_K(kModeLT, 1);
        case 1: BST_K(kModeGT, 1);
        case 2: BST_K(kModeEQ, 1);
        default: BST_K(kModeBetween, 3);
    }
#undef BST_K
#undef BST_KR
}

}  // namespace dev
}  // namespace bst

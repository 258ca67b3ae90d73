// Dispatch of single-column slice-layout scans by literal mode.
#include "scan_kernel.h"

namespace bst {
namespace dev {

int launch_slices(const DevCol& c, const ScanLit& lit, const uint64_t* in, uint64_t* out,
                  unsigned long long* counters, hipStream_t st) {
    switch (lit.mode) {
        case kModeLT: return launch_slices_mode<kModeLT>(c, lit, in, out, counters, st);
        case kModeGT: return launch_slices_mode<kModeGT>(c, lit, in, out, counters, st);
        case kModeEQ: return launch_slices_mode<kModeEQ>(c, lit, in, out, counters, st);
        case kModeBetween: return launch_slices_mode<kModeBetween>(c, lit, in, out, counters, st);
        default: return set_error(BST_EINVAL, "bad literal mode");
    }
}

}  // namespace dev
}  // namespace bst

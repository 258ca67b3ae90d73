// Slice-layout scan kernels for literal mode kModeBetween.
#include "scan_kernel.h"

namespace bst {
namespace dev {
template int launch_slices_mode<kModeBetween>(const DevCol&, const ScanLit&, const uint64_t*, uint64_t*, unsigned long long*,
                                    hipStream_t);
}  // namespace dev
}  // namespace bst

// Instantiations of the F-COO tile kernel: bfloat16 factors in 4-column lane chunks (SpMTTKRP).
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_bf16_half(const SegLaunch &L, hipStream_t s) { return seg_dispatch_half<dev::bf16raw>(L, s); }
}  // namespace fcoo

// Instantiations of the F-COO tile kernel: dev::bf16raw factors, fused residual = false.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_bf16(const SegLaunch &L, hipStream_t s) { return seg_dispatch<dev::bf16raw, false>(L, s); }
}  // namespace fcoo

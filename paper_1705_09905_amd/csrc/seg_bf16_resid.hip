// Instantiations of the F-COO tile kernel: dev::bf16raw factors, fused residual = true.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_bf16_resid(const SegLaunch &L, hipStream_t s) { return seg_dispatch<dev::bf16raw, true>(L, s); }
}  // namespace fcoo

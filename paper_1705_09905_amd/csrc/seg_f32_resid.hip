// Instantiations of the F-COO tile kernel: float factors, fused residual = true.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_f32_resid(const SegLaunch &L, hipStream_t s) { return seg_dispatch<float, true>(L, s); }
}  // namespace fcoo

// Instantiations of the F-COO tile kernel: float factors, fused residual = false.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_f32(const SegLaunch &L, hipStream_t s) { return seg_dispatch<float, false>(L, s); }
}  // namespace fcoo

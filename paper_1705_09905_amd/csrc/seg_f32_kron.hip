// Instantiations of the F-COO tile kernel for SpTTMc (Kronecker rows), float32 factors.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_f32_kron(const SegLaunch &L, hipStream_t s) { return seg_dispatch_kron<float>(L, s); }
}  // namespace fcoo

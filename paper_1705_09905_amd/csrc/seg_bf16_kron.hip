// Instantiations of the F-COO tile kernel for SpTTMc (Kronecker rows), bfloat16 factors.
#include "fcoo_seg_dispatch.h"

namespace fcoo {
hipError_t seg_launch_bf16_kron(const SegLaunch &L, hipStream_t s) { return seg_dispatch_kron<dev::bf16raw>(L, s); }
}  // namespace fcoo

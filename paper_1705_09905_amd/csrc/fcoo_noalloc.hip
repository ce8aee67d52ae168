// SpMTTKRP for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// fcoo_spmttkrp keeps its scratch (the tile carries of the segmented scan
// and, for an XCD-blocked build, the per-block partial rows) in buffers the
// build grows on demand.  This entry point runs the same kernels with that
// scratch in one fixed array of device memory, `scratch`, instead: a
// file-scope __device__ array, so each GPU the library runs on holds its own
// copy until the process ends, and the call itself allocates nothing.
//
// In host code the array's name stands for a host-side shadow, not a device
// address.  Its device address is looked up once per device, with that
// device current, by hipGetSymbolAddress on the first call there, and only
// that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fcoo_internal.h"

static __device__ __align__(256) float scratch[FCOO_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace fcoo {

namespace {

constexpr int64_t kScratchFloats = (int64_t)FCOO_NOALLOC_SCRATCH_BYTES / (int64_t)sizeof(float);
constexpr int kMaxDevices = 64;

std::mutex g_mu;
float *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// The device address of this device's `scratch`, looked up on the first call
// with the device current.
int scratch_ptr(float **out)
{
    int dev = 0;
    FCOO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FCOO_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        FCOO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FCOO_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch[dev] = static_cast<float *>(p);
    }
    *out = g_scratch[dev];
    return FCOO_OK;
}

constexpr int64_t align64(int64_t n) { return (n + 63) & ~(int64_t)63; }   // 256-byte steps of floats

}  // namespace

}  // namespace fcoo

using namespace fcoo;

extern "C" int fcoo_spmttkrp_noalloc(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R,
                                     float *M, void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_MTTKRP, true, &rc);
    if (!b) return rc;
    if ((rc = check_factors(t, mode, factors, dtype, R))) return rc;
    if (!M) return fail(FCOO_EINVAL, "M is NULL");
    // scratch layout: carries (2 x ntiles x R), then the blocked build's partial rows
    const int64_t ncarry = align64(2 * b->ntiles * (int64_t)R);
    const int64_t npart = b->nblk > 1 ? (int64_t)b->nblk * b->rows * R : 0;
    if (ncarry + npart > kScratchFloats)
        return fail(FCOO_ERANGE,
                    "no-alloc SpMTTKRP needs %lld bytes of scratch (tile carries%s), above its fixed %lld bytes",
                    (long long)((ncarry + npart) * 4), npart ? " and XCD-block partial rows" : "",
                    (long long)FCOO_NOALLOC_SCRATCH_BYTES);
    float *base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    hipStream_t s = (hipStream_t)stream;
    TileProblem p{};
    p.b = b;
    for (size_t q = 0; q < b->pmodes.size(); ++q) p.fac[q] = factors[b->pmodes[q]];
    p.vals = b->d_val;
    p.dtype = dtype;
    p.R = R;
    p.out = M;
    p.carry = base;
    p.bpart = npart ? base + ncarry : nullptr;
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    return launch_segmented(p, s, false);
}

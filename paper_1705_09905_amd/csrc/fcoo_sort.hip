// Device primitives of the GPU F-COO build: a stable least-significant-digit
// radix sort of (64-bit key, 32-bit value) pairs and a prefix sum of int32.
//
// Radix sort, 8-bit digits, one pass per digit below end_bit.  The input is
// cut into tiles of 4096 pairs (one workgroup of 256 lanes, 16 pairs each):
//   1. histogram: per tile, the count of every digit (LDS atomics), stored
//      digit-major (digit * ntiles + tile);
//   2. exclusive prefix sum of those counts: the output position of each
//      (digit, tile) run -- stability across tiles comes from this order;
//   3. scatter: the tile's pairs are ranked in input order, 256 at a time --
//      within a wave by matching digits with 8 ballots, across the 4 waves and
//      the earlier rounds through per-digit counters in LDS -- and placed in
//      LDS at their tile-local sorted position; then written out in that
//      order, so the pairs of one digit leave as a contiguous run.
// Prefix sum: per-tile sums, an exclusive scan of the tile sums by one
// workgroup, then each tile's own scan plus its offset.
#include <hip/hip_runtime.h>

#include "fcoo_internal.h"

namespace fcoo {
namespace dev {

constexpr int kSortItems = 16;
constexpr int kSortTile = 256 * kSortItems;
constexpr int kScanItems = 16;
constexpr int kScanTile = 256 * kScanItems;

// Exclusive prefix sum over the 256 lanes of a workgroup; also returns the total.
__device__ __forceinline__ int block_exclusive(int v, int *s_w, int &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    int off = 0;
    for (int i = 0; i < w; ++i) off += s_w[i];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return off + inc - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const int32_t *__restrict__ in, int64_t n,
                                                          int32_t *__restrict__ sums)
{
    __shared__ int s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) v += in[base + i];
    int total;
    (void)block_exclusive(v, s_w, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the nb tile sums, in place.
__global__ __launch_bounds__(256) void scan_top_kernel(int32_t *__restrict__ sums, int64_t nb)
{
    __shared__ int s_w[4];
    int carry = 0;
    for (int64_t start = 0; start < nb; start += kScanTile) {
        const int64_t base = start + (int64_t)threadIdx.x * kScanItems;
        int x[kScanItems];
        int v = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            x[i] = base + i < nb ? sums[base + i] : 0;
            v += x[i];
        }
        int total;
        int run = carry + block_exclusive(v, s_w, total);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < nb) sums[base + i] = run;
            run += x[i];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(256) void scan_down_kernel(const int32_t *__restrict__ in, int64_t n,
                                                        const int32_t *__restrict__ offs,
                                                        int32_t *__restrict__ out, int inclusive)
{
    __shared__ int s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int x[kScanItems];
    int v = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        x[i] = base + i < n ? in[base + i] : 0;
        v += x[i];
    }
    int total;
    int run = offs[blockIdx.x] + block_exclusive(v, s_w, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (inclusive) run += x[i];
        if (base + i < n) out[base + i] = run;
        if (!inclusive) run += x[i];
    }
}

__global__ __launch_bounds__(256) void radix_hist_kernel(const uint64_t *__restrict__ key, int64_t n, int shift,
                                                         int64_t ntiles, int32_t *__restrict__ hist)
{
    __shared__ int s_cnt[256];
    s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t e = base + (int64_t)r * 256 + threadIdx.x;
        if (e < n) atomicAdd(&s_cnt[(int)((key[e] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = s_cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void radix_scatter_kernel(const uint64_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin, int64_t n,
                                                            int shift, int64_t ntiles,
                                                            const int32_t *__restrict__ hist,
                                                            const int32_t *__restrict__ offs,
                                                            uint64_t *__restrict__ kout,
                                                            uint32_t *__restrict__ vout)
{
    __shared__ uint64_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ int s_toff[256];      // tile-local start of each digit
    __shared__ int s_glob[256];      // output start of this tile's run of each digit
    __shared__ int s_run[256];       // pairs of each digit placed by the earlier rounds
    __shared__ int s_wcnt[4][256];   // pairs of each digit in each wave, this round
    __shared__ int s_wpre[4][256];   // tile-local rank of a wave's first pair of each digit
    __shared__ int s_w[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int tn = (int)(n - base < kSortTile ? n - base : kSortTile);

    // the tile's pairs, all in flight at once (pair r * 256 + tid of the tile)
    uint64_t kr[kSortItems];
    uint32_t vr[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = r * 256 + tid;
        kr[r] = i < tn ? kin[base + i] : 0ull;
        vr[r] = i < tn ? vin[base + i] : 0u;
    }
    const int64_t hi = (int64_t)tid * ntiles + blockIdx.x;
    int total;
    s_toff[tid] = block_exclusive(hist[hi], s_w, total);
    s_glob[tid] = offs[hi];
    s_run[tid] = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = r * 256 + tid;
        const bool valid = i < tn;
        const uint64_t k = kr[r];
        const uint32_t v = vr[r];
        const int d = (int)((k >> shift) & 255u);
#pragma unroll
        for (int q = 0; q < 4; ++q) s_wcnt[q][tid] = 0;
        __syncthreads();
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) s_wcnt[w][d] = __popcll(peers);
        __syncthreads();
        {
            int c = s_run[tid];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s_wpre[q][tid] = c;
                c += s_wcnt[q][tid];
            }
            s_run[tid] = c;
        }
        __syncthreads();
        if (valid) {
            const int lp = s_toff[d] + s_wpre[w][d] + rank;
            if (lp < tn) {
                s_key[lp] = k;
                s_val[lp] = v;
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < tn; i += 256) {
        const uint64_t k = s_key[i];
        const int d = (int)((k >> shift) & 255u);
        const int64_t dst = (int64_t)s_glob[d] + (i - s_toff[d]);
        if (dst >= 0 && dst < n) {
            kout[dst] = k;
            vout[dst] = s_val[i];
        }
    }
}

}  // namespace dev

int64_t scan_work_ints(int64_t n) { return (n + dev::kScanTile - 1) / dev::kScanTile + 1; }

int64_t sort_work_ints(int64_t n)
{
    const int64_t nh = 256 * ((n + dev::kSortTile - 1) / dev::kSortTile);
    return 2 * nh + scan_work_ints(nh);
}

int scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, int32_t *work, hipStream_t s)
{
    if (n <= 0) return FCOO_OK;
    const int64_t nb = (n + dev::kScanTile - 1) / dev::kScanTile;
    if (nb > 0x7fffffffll) return fail(FCOO_EUNSUPPORTED, "prefix sum of %lld elements", (long long)n);
    hipLaunchKernelGGL(dev::scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, work);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::scan_top_kernel, dim3(1), dim3(256), 0, s, work, nb);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::scan_down_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, work, out,
                       inclusive ? 1 : 0);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}

int sort_pairs_u64(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int end_bit,
                   int32_t *work, hipStream_t s, int *passes)
{
    *passes = 0;
    if (n <= 0) return FCOO_OK;
    const int64_t ntiles = (n + dev::kSortTile - 1) / dev::kSortTile;
    if (n > 0x7fffffffll) return fail(FCOO_EUNSUPPORTED, "sort of %lld pairs", (long long)n);
    int32_t *hist = work, *offs = work + 256 * ntiles, *sw = offs + 256 * ntiles;
    for (int shift = 0; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(dev::radix_hist_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, k0, n, shift, ntiles,
                           hist);
        FCOO_HIP(hipGetLastError());
        int rc = scan_i32(hist, offs, 256 * ntiles, false, sw, s);
        if (rc) return rc;
        hipLaunchKernelGGL(dev::radix_scatter_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, k0, v0, n, shift,
                           ntiles, hist, offs, k1, v1);
        FCOO_HIP(hipGetLastError());
        uint64_t *tk = k0; k0 = k1; k1 = tk;
        uint32_t *tv = v0; v0 = v1; v1 = tv;
        ++*passes;
    }
    return FCOO_OK;
}

}  // namespace fcoo

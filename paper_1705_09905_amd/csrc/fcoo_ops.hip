// Launch plans of the segmented F-COO operations, the carry fix-up, empty
// rows, value permutation, deterministic float64 reductions and the CP
// model at the nonzeros.
#include "fcoo_internal.h"
#include "fcoo_seg_dispatch.h"

namespace fcoo {

namespace dev {

// Carry fix-up: entry (b, a, row) finishes the segment that tile a starts
// (its last open partial) and tile b closes (its first partial; b = ntiles
// is the end of the tensor), with tiles a+1 .. b-1 lying wholly inside it.
__global__ __launch_bounds__(256) void fixup_kernel(const int32_t *__restrict__ fix,
                                                    const float *__restrict__ ca,
                                                    const float *__restrict__ cb, int64_t ntiles,
                                                    int R, float *__restrict__ out)
{
    __shared__ float red[256];
    const int64_t e = blockIdx.x;
    const int tb = fix[3 * e], ta = fix[3 * e + 1], row = fix[3 * e + 2];
    const int tid = threadIdx.x;
    if (R > 256) {
        // wide rows (SpTTMc): one column per thread, the chain summed in order
        for (int c = tid; c < R; c += 256) {
            float v = cb[(int64_t)ta * R + c];
            int64_t t = (int64_t)ta + 1;
            for (; t + 7 < tb; t += 8) {
                float x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = ca[(t + u) * R + c];
#pragma unroll
                for (int u = 0; u < 8; ++u) v += x[u];
            }
            for (; t < tb; ++t) v += ca[t * R + c];
            if (tb < ntiles) v += ca[(int64_t)tb * R + c];
            out[(int64_t)row * R + c] = v;
        }
        return;
    }
    const int slots = 256 / R;
    const int slot = tid / R, c = tid - (tid / R) * R;
    float s = 0.f;
    if (slot < slots) {
        // long chains (a slice over hundreds of tiles): 8 loads in flight,
        // then the adds in tile order
        int64_t t = (int64_t)ta + 1 + slot;
        for (; t + 7 * slots < tb; t += 8 * slots) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = ca[(t + u * slots) * R + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; t < tb; t += slots) s += ca[t * R + c];
    }
    red[tid] = s;
    __syncthreads();
    if (tid < R) {
        float v = cb[(int64_t)ta * R + tid];
        for (int k = 0; k < slots; ++k) v += red[k * R + tid];
        if (tb < ntiles) v += ca[(int64_t)tb * R + tid];
        out[(int64_t)row * R + tid] = v;
    }
}

// XCD blocks: out[i][c] = sum over blocks b of part[b][i][c], in block order.
__global__ __launch_bounds__(256) void reduce_blocks_kernel(const float *__restrict__ part, int nblk,
                                                            int64_t n, float *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        float v = part[e];
        for (int k = 1; k < nblk; ++k) v += part[(int64_t)k * n + e];
        out[e] = v;
    }
}

// Rows of an MTTKRP result that no nonzero touches are zero.
__global__ __launch_bounds__(256) void zero_rows_kernel(const int32_t *__restrict__ rows, int64_t nrows,
                                                        int R, float *__restrict__ out)
{
    const int64_t n = nrows * R;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / R;
        out[(int64_t)rows[r] * R + (i - r * R)] = 0.f;
    }
}

__global__ __launch_bounds__(256) void permute_kernel(const int32_t *__restrict__ perm,
                                                      const float *__restrict__ g, int64_t n,
                                                      float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = g[perm[i]];
}

// One workgroup: fixed-order strided sums, then a tree; bitwise repeatable.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ p, int64_t n,
                                                              double scale, double *__restrict__ out)
{
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s += p[i];
    sh[tid] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    if (tid == 0) out[0] = sh[0] * scale;
}

struct ModelArgs {
    const int32_t *idx[kMaxOrder];
    const void *fac[kMaxOrder];
    float *xhat;
    int64_t nnz;
    int order;
    int R;
};

// xhat[e] = sum_r prod_m A_m[i_m(e), r]: a lane group of LPN lanes per
// nonzero, VW columns per lane, rank tiles looped inside (R <= 256).
template <typename FT, int VW, int LPN>
__global__ __launch_bounds__(256) void model_kernel(ModelArgs A)
{
    constexpr int Q = 64 / LPN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane / LPN, j = lane % LPN;
    const int64_t stride = (int64_t)gridDim.x * 4 * Q;
    for (int64_t e = ((int64_t)blockIdx.x * 4 + w) * Q + q; e < A.nnz; e += stride) {
        int ix[kMaxOrder];
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) ix[m] = m < A.order ? __builtin_nontemporal_load(A.idx[m] + e) : 0;
        float s = 0.f;
        for (int c0 = 0; c0 < A.R; c0 += LPN * VW) {
            const int col = c0 + j * VW;
            if (col < A.R) {
                Raw<FT, VW> raw[kMaxOrder];
#pragma unroll
                for (int m = 0; m < kMaxOrder; ++m)
                    if (m < A.order) load_raw<FT, VW>(reinterpret_cast<const FT *>(A.fac[m]) + (int64_t)ix[m] * A.R + col, raw[m]);
                float p[VW];
                to_float<FT, VW>(raw[0], p);
#pragma unroll
                for (int m = 1; m < kMaxOrder; ++m) {
                    if (m < A.order) {
                        float x[VW];
                        to_float<FT, VW>(raw[m], x);
#pragma unroll
                        for (int k = 0; k < VW; ++k) p[k] *= x[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < VW; ++k) s += p[k];
            }
        }
        s = group_sum<LPN>(s);
        if (j == 0) A.xhat[e] = s;
    }
}

}  // namespace dev

static int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

static int grid_for(int64_t work, int64_t per_block, int cap = 65535 * 8)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

int launch_segmented(const TileProblem &p, hipStream_t s, bool resid)
{
    const Built &b = *p.b;
    const int R = p.R;
    if (b.nnz > 0) {
        SegLaunch L{};
        dev::SegArgs &a = L.args;
        const int np = (int)b.pmodes.size();
        for (int q = 0; q < np; ++q) {
            a.pidx[q] = b.d_pidx[q];
            a.fac[q] = p.fac[q];
        }
        a.vals = p.vals;
        a.bf = b.d_bf;
        a.tile_seg0 = b.d_tile_seg0;
        a.seg_row = b.op == FCOO_OP_MTTKRP ? b.d_seg_row : nullptr;
        a.out = b.nblk > 1 ? p.bpart : p.out;
        a.carry_a = p.carry;
        a.carry_b = p.carry + b.ntiles * (int64_t)R;
        a.own = p.own;
        a.partial = p.partial;
        a.nnz = b.nnz;
        a.ntiles = b.ntiles;
        a.R = R;
        a.np = np;
        a.tile_nnz = b.tile_nnz;
        a.nseg = (int)b.nseg;
        a.inv_nnz = p.inv_nnz;
        // bfloat16 in 4-column (8-byte) lane chunks: twice the rows per gather
        // batch at 4 waves per SIMD, against 8-column chunks at 3 waves.  The
        // build's lane_cols picks (fcoo_autotune times both); by default 4
        // columns with exactly two product modes (with three, the batch per mode
        // gets short and 8-column chunks won on the order-4 Zipf tensor)
        const bool half_ok = p.dtype == FCOO_BF16 && !resid && !p.kron && np <= 3 && R % 4 == 0 && R <= 64;
        L.half = half_ok && (b.lane_cols == 4 || (b.lane_cols == 0 && np == 2 && b.op == FCOO_OP_MTTKRP));
        const int V = (p.dtype == FCOO_F32 || L.half) ? 4 : 8;
        // a lane's VW columns must lie in one row piece of the (last) factor
        L.vec = ((p.kron ? p.kr[np - 1] : R) % V) == 0;
        const int VW = L.vec ? V : 1;
        // SpTTMc: KB columns of the second-to-last mode per lane when they divide it
        const int KBv = p.dtype == FCOO_F32 ? 4 : 2;
        L.kb = (p.kron && L.vec && np >= 2 && p.kr[np - 2] % KBv == 0) ? KBv : 1;
        const int AW = VW * L.kb;
        const int lanes = (R + AW - 1) / AW;          // lanes per nonzero over the whole row
        int lpn = next_pow2(lanes);
        if (p.kron) {
            for (int q = 0; q < np; ++q) a.kr[q] = p.kr[q];
            if (lpn < 4) lpn = 4;
            if (lpn > 64) lpn = 64;
        } else if (L.vec && lpn > 16) {
            lpn = 16;
        }
        if (!L.vec) lpn = 64;
        L.lpn = lpn;
        const int rt = lpn * AW;
        const int nrt = (lanes + lpn - 1) / lpn;
        if (resid && nrt > 1)
            return fail(FCOO_EUNSUPPORTED, "fused residual needs R <= %d for this dtype (R = %d)", rt, R);
        L.npt = np <= 3 ? np : 0;
        L.rowmap = b.op == FCOO_OP_MTTKRP;
        a.nblk = b.nblk;
        a.rows_own = (int)b.rows;
        if (p.sp_words) {
            a.sp_words = p.sp_words;
            a.sp_from = b.d_sp_from;
            a.sp_ticket = b.d_sp_ticket;
            a.sp_err = b.d_sp_err;
            a.sp_base = b.sp_tickets;
            a.sp_epoch = p.sp_epoch;
            a.sp_tail_from = b.sp_tail_from;
        }
        int64_t gx = b.ntiles;
        if (b.nblk > 1) {
            for (int k = 0; k <= b.nblk; ++k) a.blk_ts[k] = b.blk_ts[k];
            gx = (int64_t)kXcds * b.max_block_tiles();   // workgroup w: XCD w % 8, its block's tiles
            if (gx < 1) gx = 1;
        }
        L.grid = dim3((unsigned)gx, (unsigned)nrt, 1);
        hipError_t e;
        if (p.ev_before) FCOO_HIP(hipEventRecord(p.ev_before, s));
        if (p.kron) e = p.dtype == FCOO_F32 ? seg_launch_f32_kron(L, s) : seg_launch_bf16_kron(L, s);
        else if (p.dtype == FCOO_F32) e = resid ? seg_launch_f32_resid(L, s) : seg_launch_f32(L, s);
        else if (L.half) e = seg_launch_bf16_half(L, s);
        else e = resid ? seg_launch_bf16_resid(L, s) : seg_launch_bf16(L, s);
        if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
        if (p.sp_words)   // every workgroup of the launch takes one ticket
            const_cast<Built &>(b).sp_tickets += (unsigned long long)L.grid.x * L.grid.y;
        if (p.ev_after) FCOO_HIP(hipEventRecord(p.ev_after, s));
        const int64_t nfix = p.sp_words ? 0 : b.nfix();
        if (nfix > 0) {
            hipLaunchKernelGGL(dev::fixup_kernel, dim3((unsigned)nfix), dim3(256), 0, s, b.d_fix,
                               a.carry_a, a.carry_b, b.ntiles, R, a.out);
            FCOO_HIP(hipGetLastError());
        }
    }
    float *outp = b.nblk > 1 ? p.bpart : p.out;
    const int64_t nempty = (int64_t)b.empty_rows.size();
    if (nempty > 0) {
        hipLaunchKernelGGL(dev::zero_rows_kernel, dim3(grid_for(nempty * R, 256)), dim3(256), 0, s,
                           b.d_empty, nempty, R, outp);
        FCOO_HIP(hipGetLastError());
    }
    if (b.nblk > 1) {
        const int64_t n = b.rows * (int64_t)R;
        hipLaunchKernelGGL(dev::reduce_blocks_kernel, dim3(grid_for(n, 256 * 4)), dim3(256), 0, s, p.bpart,
                           b.nblk, n, p.out);
        FCOO_HIP(hipGetLastError());
    }
    return FCOO_OK;
}

int launch_permute_values(const Built &b, const float *g, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(dev::permute_kernel, dim3(grid_for(b.nnz, 256 * 8)), dim3(256), 0, s, b.d_perm, g,
                       b.nnz, out);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}

int launch_reduce_partials(const double *partial, int64_t n, double scale, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(dev::reduce_partials_kernel, dim3(1), dim3(256), 0, s, partial, n, scale, out);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}

template <typename FT>
static hipError_t model_go(const dev::ModelArgs &a, bool vec, int lpn, hipStream_t s)
{
    constexpr int V = dev::Elem<FT>::VEC;
    auto grid = [&](int L) { return dim3(grid_for(a.nnz, 4 * (64 / L) * 4, 65535 * 4)); };
    if (!vec) {
        hipLaunchKernelGGL((dev::model_kernel<FT, 1, 64>), grid(64), dim3(256), 0, s, a);
    } else {
        switch (lpn) {
            case 1: hipLaunchKernelGGL((dev::model_kernel<FT, V, 1>), grid(1), dim3(256), 0, s, a); break;
            case 2: hipLaunchKernelGGL((dev::model_kernel<FT, V, 2>), grid(2), dim3(256), 0, s, a); break;
            case 4: hipLaunchKernelGGL((dev::model_kernel<FT, V, 4>), grid(4), dim3(256), 0, s, a); break;
            case 8: hipLaunchKernelGGL((dev::model_kernel<FT, V, 8>), grid(8), dim3(256), 0, s, a); break;
            default: hipLaunchKernelGGL((dev::model_kernel<FT, V, 16>), grid(16), dim3(256), 0, s, a); break;
        }
    }
    return hipGetLastError();
}

int launch_model(const fcoo_tensor *t, const void *const *factors, int dtype, int R, float *xhat,
                 hipStream_t s)
{
    if (t->nnz == 0) return FCOO_OK;
    dev::ModelArgs a{};
    for (int m = 0; m < t->order; ++m) {
        a.idx[m] = t->d_coo[m];
        a.fac[m] = factors[m];
    }
    a.xhat = xhat;
    a.nnz = t->nnz;
    a.order = t->order;
    a.R = R;
    const int V = dtype == FCOO_F32 ? 4 : 8;
    const bool vec = R % V == 0;
    int lpn = next_pow2((R + V - 1) / V);
    if (lpn > 16) lpn = 16;
    hipError_t e = dtype == FCOO_F32 ? model_go<float>(a, vec, lpn, s) : model_go<dev::bf16raw>(a, vec, lpn, s);
    if (e != hipSuccess) return hip_fail(e, "model kernel launch");
    return FCOO_OK;
}

}  // namespace fcoo

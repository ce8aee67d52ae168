// The one-shot F-COO tile kernel (SpMTTKRP, SpTTM, value-replaced
// SpMTTKRP, fused MSE residual SpMTTKRP) and the carry fix-up pass.
//
// Method (Sec. IV-C, IV-D): every nonzero gathers the rows of its product
// modes, multiplies them (Hadamard product, or a single row for SpTTM),
// scales by its value and is summed into its segment (slice for SpMTTKRP,
// fibre for SpTTM).  Work is split by nonzeros, not by segments, so load
// balance does not depend on the sparsity pattern, and the sums are formed
// by a segmented scan driven by the bf / sf flags instead of atomics.
//
// MI355X layout (the paper's Titan X design is one thread per partition of
// threadlen nonzeros and one grid row per rank column; here):
//   * a workgroup (4 wave64s) owns a tile of tile_nnz consecutive nonzeros
//     and a rank tile of LPN * VW columns (grid.y counts rank tiles);
//   * a lane group of LPN lanes owns a contiguous run of the tile and walks
//     it in order; each lane holds VW columns, so one gather instruction
//     fetches 64 / LPN whole rows (16 bytes per lane);
//   * the stream (product indices, values) is read coalesced, one element
//     per lane, non-temporally, and broadcast inside the group by
//     ds_swizzle; the bf word of a 64-nonzero window gives the heads;
//   * a segment that starts and ends inside a run is written directly;
//     the partial sums at run boundaries go through a wave-level segmented
//     scan (cross-lane moves), then through LDS across the 4 waves; a
//     segment crossing a tile boundary is finished by the fix-up kernel,
//     which sums the tiles' boundary partials along a host-precomputed chain.
//   No atomics are used, so results are bitwise repeatable.
//
// The segmented-scan element of a range is (f, a, b): f = the range holds a
// segment start, a = sum before the first start (the whole sum if f = 0),
// b = sum from the last start to the end (= a if f = 0).  Combining X then Y:
//   f = fX | fY,  a = fX ? aX : aX + aY,  b = fY ? bY : bX + aY,
// and the segment closed at Y's first start is complete (started inside the
// combined range) iff fX, with value bX + aY.
#pragma once

#include "fcoo_device.h"

namespace fcoo {
namespace dev {

constexpr int kMaxNP = 7;

struct SegArgs {
    const int32_t *pidx[kMaxNP];     // product-mode index streams (stored order)
    const void *fac[kMaxNP];         // factor matrix of each product mode
    const float *vals;               // values in stored order
    const uint32_t *bf;              // bit stream, padded
    const int32_t *tile_seg0;        // per tile: segment ordinal of its first nonzero
    const int32_t *seg_row;          // per segment output row (NULL: row = ordinal)
    float *out;                      // output rows, leading dimension R
    float *carry_a;                  // ntiles x R
    float *carry_b;                  // ntiles x R
    const void *own;                 // RESID: factor of the index mode
    double *partial;                 // RESID: per-tile partial sum of squared residuals
    int64_t nnz;
    int64_t ntiles;
    int R;
    int np;                          // number of product modes (runtime, for NP == 0)
    int tile_nnz;
    float inv_nnz;                   // RESID: 1 / Z
};

template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

template <int VW>
__device__ __forceinline__ void zero(float (&v)[VW])
{
#pragma unroll
    for (int k = 0; k < VW; ++k) v[k] = 0.f;
}

// Inclusive segmented scan across the Q lane groups of a wave (each group's
// LPN lanes hold the same f and their own columns of a, b).
template <int LPN, int VW>
__device__ __forceinline__ void wave_segscan(int &f, float (&a)[VW], float (&b)[VW], int q)
{
    constexpr int Q = 64 / LPN;
#pragma unroll
    for (int d = 1; d < Q; d <<= 1) {
        const int fu = __shfl_up(f, d * LPN, 64);
        float au[VW], bu[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            au[k] = __shfl_up(a[k], d * LPN, 64);
            bu[k] = __shfl_up(b[k], d * LPN, 64);
        }
        if (q >= d) {
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const float na = fu ? au[k] : au[k] + a[k];
                const float nb = f ? b[k] : bu[k] + a[k];
                a[k] = na;
                b[k] = nb;
            }
            f = f | fu;
        }
    }
}

template <typename FT, int VW, int LPN, int NP, bool RESID>
__global__ __launch_bounds__(256) void seg_tile_kernel(SegArgs A)
{
    constexpr int Q = 64 / LPN;                       // lane groups per wave
    constexpr int NPM = NP > 0 ? NP : kMaxNP;         // product modes held per step
    constexpr int CH = NP > 0 ? (LPN < 8 ? LPN : 8) : (LPN < 2 ? LPN : 2);  // steps per gather batch
    constexpr int RT = LPN * VW;                      // columns of this rank tile

    __shared__ int s_cnt[4];
    __shared__ int s_f[4];
    __shared__ float s_a[4][RT];
    __shared__ float s_b[4][RT];
    __shared__ double s_loss[4];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int q = lane / LPN, j = lane % LPN;
    const int64_t tile = blockIdx.x;
    const int T = A.tile_nnz;
    const int S = T / (4 * Q);                        // run length of one lane group
    const int64_t t0 = tile * (int64_t)T;
    const int64_t rs = t0 + (int64_t)(w * Q + q) * S;
    const int64_t re = rs + S < A.nnz ? rs + S : A.nnz;
    const int col = (int)blockIdx.y * RT + j * VW;
    const bool cval = col < A.R;
    const int R = A.R;
    const int np = NP > 0 ? NP : A.np;

    // ---- 1. heads before each run: tile prefix from tile_seg0, then counts
    int cnt = 0;
    for (int64_t base = rs; base < re; base += 64) {
        const int n = (int)(re - base < 64 ? re - base : 64);
        cnt += __popcll(head_window(A.bf, base, n));
    }
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < Q; d <<= 1) {
        const int u = __shfl_up(inc, d * LPN, 64);
        if (q >= d) inc += u;
    }
    if (lane == 63) s_cnt[w] = inc;
    __syncthreads();
    int wave_before = 0;
    for (int i = 0; i < w; ++i) wave_before += s_cnt[i];
    // heads strictly before the tile: ordinal of its first nonzero + 1, less
    // one if that nonzero is itself a head
    const int H_tile = A.tile_seg0[tile] + 1 - (int)head_at(A.bf, t0);
    const int H_wave = H_tile + wave_before;
    const int H_run = H_wave + inc - cnt;

    // ---- 2. walk the run
    float acc[VW], pre[VW];
    zero(acc);
    zero(pre);
    int have = 0;
    int g = H_run - 1;                                // segment open before the run
    float own[VW];
    float lsum = 0.f;
    if constexpr (RESID) {
        zero(own);
        if (g >= 0 && rs < re && cval)
            load_row<FT, VW>(reinterpret_cast<const FT *>(A.own) + (int64_t)A.seg_row[g] * R + col, own);
    }

    for (int64_t base = rs; base < re; base += 64) {
        const int n = (int)(re - base < 64 ? re - base : 64);
        const uint64_t hm = head_window(A.bf, base, n);
        for (int c = 0; c < n; c += LPN) {
            const int el = c + j;
            const bool ev = el < n;
            const int64_t e = base + el;
            int my_idx[NPM];
#pragma unroll
            for (int qq = 0; qq < NPM; ++qq)
                my_idx[qq] = (ev && qq < np) ? __builtin_nontemporal_load(A.pidx[qq] + e) : 0;
            const float my_v = ev ? __builtin_nontemporal_load(A.vals + e) : 0.f;

            static_for<LPN / CH>([&](auto c2c) {
                constexpr int C2 = decltype(c2c)::value * CH;
                Raw<FT, VW> rows[CH][NPM];
                static_for<CH>([&](auto jjc) {
                    constexpr int JJ = decltype(jjc)::value;
#pragma unroll
                    for (int qq = 0; qq < NPM; ++qq) {
                        const int idx = bcast_imm<LPN, C2 + JJ>(my_idx[qq]);
                        if (cval && qq < np)
                            load_raw<FT, VW>(reinterpret_cast<const FT *>(A.fac[qq]) + (int64_t)idx * R + col,
                                             rows[JJ][qq]);
                        else
                            set_one<FT, VW>(rows[JJ][qq]);
                    }
                });
                static_for<CH>([&](auto jjc) {
                    constexpr int JJ = decltype(jjc)::value;
                    const int st = c + C2 + JJ;
                    const float v = bcast_imm_f<LPN, C2 + JJ>(my_v);
                    float h[VW];
                    to_float<FT, VW>(rows[JJ][0], h);
#pragma unroll
                    for (int qq = 1; qq < NPM; ++qq) {
                        float x[VW];
                        to_float<FT, VW>(rows[JJ][qq], x);
#pragma unroll
                        for (int k = 0; k < VW; ++k) h[k] *= x[k];
                    }
                    if ((hm >> st) & 1ull) {
                        if (!have) {
#pragma unroll
                            for (int k = 0; k < VW; ++k) pre[k] = acc[k];
                            have = 1;
                        } else if (cval) {
                            const int64_t row = A.seg_row ? (int64_t)A.seg_row[g] : (int64_t)g;
                            store_row<VW>(A.out + row * R + col, acc);
                        }
                        zero(acc);
                        ++g;
                        if constexpr (RESID) {
                            if (cval)
                                load_row<FT, VW>(reinterpret_cast<const FT *>(A.own) + (int64_t)A.seg_row[g] * R + col, own);
                        }
                    }
                    if (st < n) {
                        if constexpr (RESID) {
                            float d = 0.f;
#pragma unroll
                            for (int k = 0; k < VW; ++k) d += own[k] * h[k];
                            d = group_sum<LPN>(d);
                            const float r = d - v;
                            const float sc = r * A.inv_nnz;
#pragma unroll
                            for (int k = 0; k < VW; ++k) acc[k] += sc * h[k];
                            if (j == 0) lsum += r * r;
                        } else {
#pragma unroll
                            for (int k = 0; k < VW; ++k) acc[k] += v * h[k];
                        }
                    }
                });
            });
        }
    }

    // ---- 3. wave-level segmented scan of the runs' (f, a, b)
    const int fo = have;
    float ao[VW];
    int f = have;
    float a[VW], b[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        ao[k] = have ? pre[k] : acc[k];
        a[k] = ao[k];
        b[k] = acc[k];
    }
    wave_segscan<LPN, VW>(f, a, b, q);
    {   // exclusive prefix of this group: the inclusive value of group q - 1
        const int fp = __shfl_up(f, LPN, 64);
        float bp[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) bp[k] = __shfl_up(b[k], LPN, 64);
        if (q >= 1 && fo && fp && cval) {
            float v[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) v[k] = bp[k] + ao[k];
            const int gc = H_run - 1;
            const int64_t row = A.seg_row ? (int64_t)A.seg_row[gc] : (int64_t)gc;
            store_row<VW>(A.out + row * R + col, v);
        }
    }
    if (q == Q - 1) {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            s_a[w][j * VW + k] = a[k];
            s_b[w][j * VW + k] = b[k];
        }
        if (j == 0) s_f[w] = f;
    }
    if constexpr (RESID) {
        float l = lsum;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
        if (lane == 0) s_loss[w] = (double)l;
    }
    // H_wave of every wave, for the cross-wave closings below
    __shared__ int s_hw[4];
    if (lane == 0) s_hw[w] = H_wave;
    __syncthreads();

    // ---- 4. tile level: a wave's first closing whose segment started in an
    //         earlier wave of the tile; then the tile's carries
    if (q == 0 && w >= 1 && s_f[w] && cval) {
        int fx = s_f[0];
        float bx[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) bx[k] = s_b[0][j * VW + k];
        for (int i = 1; i < w; ++i) {
#pragma unroll
            for (int k = 0; k < VW; ++k) bx[k] = s_f[i] ? s_b[i][j * VW + k] : bx[k] + s_a[i][j * VW + k];
            fx |= s_f[i];
        }
        if (fx) {
            float v[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) v[k] = bx[k] + s_a[w][j * VW + k];
            const int gc = s_hw[w] - 1;
            const int64_t row = A.seg_row ? (int64_t)A.seg_row[gc] : (int64_t)gc;
            store_row<VW>(A.out + row * R + col, v);
        }
    }
    if (w == 0 && q == 0 && cval) {
        int ft = s_f[0];
        float at[VW], bt[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) { at[k] = s_a[0][j * VW + k]; bt[k] = s_b[0][j * VW + k]; }
        for (int i = 1; i < 4; ++i) {
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const float ai = s_a[i][j * VW + k], bi = s_b[i][j * VW + k];
                const float na = ft ? at[k] : at[k] + ai;
                const float nb = s_f[i] ? bi : bt[k] + ai;
                at[k] = na;
                bt[k] = nb;
            }
            ft |= s_f[i];
        }
        store_row<VW>(A.carry_a + tile * R + col, at);
        store_row<VW>(A.carry_b + tile * R + col, bt);
    }
    if constexpr (RESID) {
        if (tid == 0 && blockIdx.y == 0 && A.partial)
            A.partial[tile] = ((s_loss[0] + s_loss[1]) + s_loss[2]) + s_loss[3];
    }
}

}  // namespace dev
}  // namespace fcoo

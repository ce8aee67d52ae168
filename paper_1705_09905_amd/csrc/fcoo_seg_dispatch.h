// Picks the tile-kernel instantiation for a (storage type, lane layout,
// number of product modes) and launches it.  Included by the four
// instantiation units (float32 / bfloat16, plain / fused residual), which
// are compiled separately to keep build times short.
#pragma once

#include "fcoo_segscan.h"

namespace fcoo {

struct SegLaunch {
    dev::SegArgs args;
    bool vec;        // 16-byte row chunks per lane (R a multiple of the vector width)
    int lpn;         // lanes per nonzero: 1, 2, 4, 8, 16 (vector; SpTTMc up to 64) or 64 (scalar)
    int npt;         // product modes as a template value: 1, 2, 3, or 0 (runtime count)
    bool rowmap;     // output row = seg_row[segment] (SpMTTKRP) or the segment ordinal (SpTTM)
    int kb;          // SpTTMc: column blocks per lane (1, or KronBlock<FT>::KB)
    bool half;       // bfloat16 in 4-column (8-byte) lane chunks
    dim3 grid;
};

template <typename FT, int VW, int LPN, int NP, bool RESID, bool ROWMAP>
static hipError_t seg_go(const SegLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL((dev::seg_tile_kernel<FT, VW, LPN, NP, RESID, ROWMAP>), L.grid, dim3(256), 0, s,
                       L.args);
    return hipGetLastError();
}

template <typename FT, int VW, int LPN, int NP, int KB = 1>
static hipError_t seg_go_k(const SegLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL((dev::seg_tile_kernel<FT, VW, LPN, NP, false, true, true, KB>), L.grid, dim3(256), 0, s,
                       L.args);
    return hipGetLastError();
}

// SpTTM has one product mode and identity row map; SpMTTKRP maps rows.
template <typename FT, int VW, int LPN, bool RESID>
static hipError_t seg_np(const SegLaunch &L, hipStream_t s)
{
    if constexpr (!RESID) {
        if (!L.rowmap) return seg_go<FT, VW, LPN, 1, false, false>(L, s);
    }
    switch (L.npt) {
        case 1: return seg_go<FT, VW, LPN, 1, RESID, true>(L, s);
        case 2: return seg_go<FT, VW, LPN, 2, RESID, true>(L, s);
        case 3: return seg_go<FT, VW, LPN, 3, RESID, true>(L, s);
        default: return seg_go<FT, VW, LPN, 0, RESID, true>(L, s);
    }
}

template <typename FT, bool RESID>
static hipError_t seg_dispatch(const SegLaunch &L, hipStream_t s)
{
    constexpr int V = dev::Elem<FT>::VEC;
    if (!L.vec) {
        if constexpr (!RESID) {
            if (!L.rowmap) return seg_go<FT, 1, 64, 0, false, false>(L, s);
        }
        return seg_go<FT, 1, 64, 0, RESID, true>(L, s);
    }
    switch (L.lpn) {
        case 1: return seg_np<FT, V, 1, RESID>(L, s);
        case 2: return seg_np<FT, V, 2, RESID>(L, s);
        case 4: return seg_np<FT, V, 4, RESID>(L, s);
        case 8: return seg_np<FT, V, 8, RESID>(L, s);
        default: return seg_np<FT, V, 16, RESID>(L, s);
    }
}

// bfloat16 in 4-column lane chunks (SpMTTKRP with 1-3 product modes, or
// SpTTM): half the row bytes per lane, so twice the rows per gather batch.
template <typename FT, int LPN>
static hipError_t seg_np_half(const SegLaunch &L, hipStream_t s)
{
    if (!L.rowmap) return seg_go<FT, 4, LPN, 1, false, false>(L, s);
    switch (L.npt) {
        case 1: return seg_go<FT, 4, LPN, 1, false, true>(L, s);
        case 2: return seg_go<FT, 4, LPN, 2, false, true>(L, s);
        default: return seg_go<FT, 4, LPN, 3, false, true>(L, s);
    }
}

template <typename FT>
static hipError_t seg_dispatch_half(const SegLaunch &L, hipStream_t s)
{
    switch (L.lpn) {
        case 1: return seg_np_half<FT, 1>(L, s);
        case 2: return seg_np_half<FT, 2>(L, s);
        case 4: return seg_np_half<FT, 4>(L, s);
        case 8: return seg_np_half<FT, 8>(L, s);
        default: return seg_np_half<FT, 16>(L, s);
    }
}

// SpTTMc: Kronecker rows (generic path), output row = seg_row[segment].
// Lanes per nonzero: 4 .. 64 (vector) or 64 (scalar); product modes 2, 3 or
// a runtime count.
template <typename FT, int VW, int LPN, int KB>
static hipError_t seg_np_kron(const SegLaunch &L, hipStream_t s)
{
    switch (L.npt) {
        case 2: return seg_go_k<FT, VW, LPN, 2, KB>(L, s);
        case 3: return seg_go_k<FT, VW, LPN, 3, KB>(L, s);
        default: return seg_go_k<FT, VW, LPN, 0, KB>(L, s);
    }
}

// column blocks per lane with SpTTMc: 4 (float32) / 2 (bfloat16) elements of
// the second-to-last product mode, or 1
template <typename FT> struct KronBlock { static constexpr int KB = sizeof(FT) == 4 ? 4 : 2; };

template <typename FT, int KB>
static hipError_t seg_lpn_kron(const SegLaunch &L, hipStream_t s)
{
    constexpr int V = dev::Elem<FT>::VEC;
    switch (L.lpn) {
        case 4: return seg_np_kron<FT, V, 4, KB>(L, s);
        case 8: return seg_np_kron<FT, V, 8, KB>(L, s);
        case 16: return seg_np_kron<FT, V, 16, KB>(L, s);
        case 32: return seg_np_kron<FT, V, 32, KB>(L, s);
        default: return seg_np_kron<FT, V, 64, KB>(L, s);
    }
}

template <typename FT>
static hipError_t seg_dispatch_kron(const SegLaunch &L, hipStream_t s)
{
    if (!L.vec) return seg_go_k<FT, 1, 64, 0>(L, s);
    if (L.kb > 1) return seg_lpn_kron<FT, KronBlock<FT>::KB>(L, s);
    return seg_lpn_kron<FT, 1>(L, s);
}

hipError_t seg_launch_f32(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_bf16(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_bf16_half(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_f32_resid(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_bf16_resid(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_f32_kron(const SegLaunch &L, hipStream_t s);
hipError_t seg_launch_bf16_kron(const SegLaunch &L, hipStream_t s);

}  // namespace fcoo

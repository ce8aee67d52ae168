// Device-side building blocks for gfx950 (CDNA4, wave64): F-COO flag
// decoding, cross-lane moves inside a lane group, row loads of float32 /
// bfloat16 factor matrices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcoo {
namespace dev {

// ----- F-COO flags ----------------------------------------------------------
// bf is one bit per nonzero (a parity bit toggled at each segment start,
// Sec. IV-B), stored as uint32 words with two zero words of padding, so any
// 64-bit window that starts below Z can be read.

__device__ __forceinline__ uint64_t fetch64(const uint32_t *__restrict__ bf, int64_t pos)
{
    const int64_t w0 = pos >> 5;
    const int sh = (int)(pos & 31);
    const uint64_t lo = (uint64_t)bf[w0] | ((uint64_t)bf[w0 + 1] << 32);
    if (sh == 0) return lo;
    const uint64_t hi = (uint64_t)bf[w0 + 2];
    return (lo >> sh) | (hi << (64 - sh));
}

__device__ __forceinline__ uint32_t bit_at(const uint32_t *__restrict__ bf, int64_t pos)
{
    return pos < 0 ? 0u : (bf[pos >> 5] >> (pos & 31)) & 1u;
}

// Segment heads of nonzeros [pos, pos + n), n <= 64: bit k set iff nonzero
// pos + k starts a segment, i.e. its bf bit differs from the previous one
// (the bit before nonzero 0 counts as 0, so nonzero 0 is always a head).
__device__ __forceinline__ uint64_t head_window(const uint32_t *__restrict__ bf, int64_t pos, int n)
{
    const uint64_t cur = fetch64(bf, pos);
    const uint64_t hm = cur ^ ((cur << 1) | (uint64_t)bit_at(bf, pos - 1));
    return n >= 64 ? hm : (hm & ((1ull << n) - 1ull));
}

__device__ __forceinline__ uint32_t head_at(const uint32_t *__restrict__ bf, int64_t pos)
{
    return bit_at(bf, pos) ^ bit_at(bf, pos - 1);
}

// ----- lane-group moves -------------------------------------------------------
// A lane group is LPN consecutive lanes (LPN a power of two) working on one
// nonzero; ds_swizzle in bit-mask mode moves data inside 32-lane halves
// without touching LDS memory.

template <int LPN>
__device__ __forceinline__ int bcast_i(int x, int src)
{
    if constexpr (LPN == 1) {
        return x;
    } else if constexpr (LPN <= 32) {
        // and_mask keeps the group bits, or_mask selects the source lane
        // (the pattern must be an immediate: callers pass compile-time src)
        return __builtin_amdgcn_ds_bpermute(
            (int)(((__lane_id() & ~(LPN - 1)) | src) << 2), x);
    } else {
        return __builtin_amdgcn_readlane(x, src);
    }
}

// Broadcast with a compile-time source lane: ds_swizzle, bit-mask mode.
template <int LPN, int SRC>
__device__ __forceinline__ int bcast_imm(int x)
{
    if constexpr (LPN == 1) {
        return x;
    } else if constexpr (LPN <= 32) {
        constexpr int pattern = ((0x1F & ~(LPN - 1)) | (SRC << 5));
        return __builtin_amdgcn_ds_swizzle(x, pattern);
    } else {
        return __builtin_amdgcn_readlane(x, SRC);
    }
}

template <int LPN, int SRC>
__device__ __forceinline__ float bcast_imm_f(float x)
{
    return __int_as_float(bcast_imm<LPN, SRC>(__float_as_int(x)));
}

// Butterfly sum over the LPN lanes of a group.
template <int LPN>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (LPN >= 2) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (1 << 10)));
    if constexpr (LPN >= 4) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (2 << 10)));
    if constexpr (LPN >= 8) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (4 << 10)));
    if constexpr (LPN >= 16) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (8 << 10)));
    if constexpr (LPN >= 32) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (16 << 10)));
    if constexpr (LPN >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// ----- factor rows ------------------------------------------------------------
// Factor storage: float32, or bfloat16 kept as its raw 16 bits (the upper
// half of a float32).  VW elements per lane: 16-byte vector loads when the
// row length allows it, one element otherwise.

struct bf16raw { uint16_t x; };

template <typename FT> struct Elem;
template <> struct Elem<float> { static constexpr int VEC = 4; };
template <> struct Elem<bf16raw> { static constexpr int VEC = 8; };

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// A row chunk as loaded (raw registers), converted to float32 when used.
template <typename FT, int VW> struct Raw;
template <> struct Raw<float, 4> { float4 v; };
template <> struct Raw<bf16raw, 8> { uint4 v; };
template <> struct Raw<float, 1> { float v; };
template <> struct Raw<bf16raw, 1> { uint32_t v; };
template <> struct Raw<bf16raw, 2> { uint32_t v; };   // two consecutive bfloat16
template <> struct Raw<bf16raw, 4> { uint2 v; };      // four consecutive bfloat16 (8-byte loads)

template <typename FT, int VW>
__device__ __forceinline__ void load_raw(const FT *__restrict__ p, Raw<FT, VW> &r)
{
    if constexpr (sizeof(FT) == 4 && VW == 4) r.v = *reinterpret_cast<const float4 *>(p);
    else if constexpr (sizeof(FT) == 2 && VW == 8) r.v = *reinterpret_cast<const uint4 *>(p);
    else if constexpr (sizeof(FT) == 4 && VW == 1) r.v = *reinterpret_cast<const float *>(p);
    else if constexpr (sizeof(FT) == 2 && VW == 2) r.v = *reinterpret_cast<const uint32_t *>(p);
    else if constexpr (sizeof(FT) == 2 && VW == 4) r.v = *reinterpret_cast<const uint2 *>(p);
    else r.v = (uint32_t)(*reinterpret_cast<const uint16_t *>(p));
}

template <typename FT, int VW>
__device__ __forceinline__ void set_one(Raw<FT, VW> &r)
{
    if constexpr (sizeof(FT) == 4 && VW == 4) r.v = make_float4(1.f, 1.f, 1.f, 1.f);
    else if constexpr (sizeof(FT) == 2 && VW == 8) r.v = make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u);
    else if constexpr (sizeof(FT) == 4 && VW == 1) r.v = 1.f;
    else if constexpr (sizeof(FT) == 2 && VW == 2) r.v = 0x3F803F80u;
    else if constexpr (sizeof(FT) == 2 && VW == 4) r.v = make_uint2(0x3F803F80u, 0x3F803F80u);
    else r.v = 0x3F80u;
}

template <typename FT, int VW>
__device__ __forceinline__ void to_float(const Raw<FT, VW> &r, float (&out)[VW])
{
    if constexpr (sizeof(FT) == 4 && VW == 4) {
        out[0] = r.v.x; out[1] = r.v.y; out[2] = r.v.z; out[3] = r.v.w;
    } else if constexpr (sizeof(FT) == 2 && VW == 8) {
        out[0] = bf16_to_f32(r.v.x & 0xFFFFu); out[1] = bf16_to_f32(r.v.x >> 16);
        out[2] = bf16_to_f32(r.v.y & 0xFFFFu); out[3] = bf16_to_f32(r.v.y >> 16);
        out[4] = bf16_to_f32(r.v.z & 0xFFFFu); out[5] = bf16_to_f32(r.v.z >> 16);
        out[6] = bf16_to_f32(r.v.w & 0xFFFFu); out[7] = bf16_to_f32(r.v.w >> 16);
    } else if constexpr (sizeof(FT) == 4 && VW == 1) {
        out[0] = r.v;
    } else if constexpr (sizeof(FT) == 2 && VW == 2) {
        out[0] = bf16_to_f32(r.v & 0xFFFFu);
        out[1] = bf16_to_f32(r.v >> 16);
    } else if constexpr (sizeof(FT) == 2 && VW == 4) {
        out[0] = bf16_to_f32(r.v.x & 0xFFFFu); out[1] = bf16_to_f32(r.v.x >> 16);
        out[2] = bf16_to_f32(r.v.y & 0xFFFFu); out[3] = bf16_to_f32(r.v.y >> 16);
    } else {
        out[0] = bf16_to_f32(r.v);
    }
}

template <typename FT, int VW>
__device__ __forceinline__ void load_row(const FT *__restrict__ p, float (&out)[VW])
{
    Raw<FT, VW> r;
    load_raw<FT, VW>(p, r);
    to_float<FT, VW>(r, out);
}

template <int VW>
__device__ __forceinline__ void store_row(float *__restrict__ p, const float (&v)[VW])
{
    if constexpr (VW % 4 == 0) {
#pragma unroll
        for (int k = 0; k < VW; k += 4)
            *reinterpret_cast<float4 *>(p + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) p[k] = v[k];
    }
}

// The same, as streaming stores (bypass the cache's reuse policy): for
// outputs written once and not read back by the kernel.
template <int VW>
__device__ __forceinline__ void store_row_stream(float *__restrict__ p, const float (&v)[VW])
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    if constexpr (VW % 4 == 0) {
#pragma unroll
        for (int k = 0; k < VW; k += 4) {
            const f4 x = {v[k], v[k + 1], v[k + 2], v[k + 3]};
            __builtin_nontemporal_store(x, reinterpret_cast<f4 *>(p + k));
        }
    } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) __builtin_nontemporal_store(v[k], p + k);
    }
}

template <int VW>
__device__ __forceinline__ void load_out(const float *__restrict__ p, float (&v)[VW])
{
    if constexpr (VW % 4 == 0) {
#pragma unroll
        for (int k = 0; k < VW; k += 4) {
            const float4 x = *reinterpret_cast<const float4 *>(p + k);
            v[k] = x.x; v[k + 1] = x.y; v[k + 2] = x.z; v[k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = p[k];
    }
}

}  // namespace dev
}  // namespace fcoo

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
//
// SpTTMc (Eq. 4, Table I third row) uses the SpMTTKRP encoding of its mode
// and the same scan; only the per-nonzero product changes: output column c
// of a row is a digit tuple (p_1, .., p_k) over the product modes (the last
// runs fastest) and takes val * U_1(i_1, p_1) * .. * U_k(i_k, p_k).  A lane
// owns VW consecutive columns inside one block of the last mode, so it
// gathers one element of every other mode's row and VW of the last one.
#pragma once

#include "fcoo_device.h"

namespace fcoo {
namespace dev {

constexpr int kMaxNP = 7;
constexpr int kXcdBlocks = 8;        // XCDs of an MI355X: workgroup w runs on XCD w % 8

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
    int nseg;                        // number of segments
    float inv_nnz;                   // RESID: 1 / Z
    int kr[kMaxNP];                  // KRON: columns of each product mode's factor (R = their product)
    // XCD blocks: workgroup w runs tile blk_ts[w % 8] + w / 8 of block w % 8
    // (none past blk_ts[w % 8 + 1]); output rows are block * rows_own + row
    int64_t blk_ts[kXcdBlocks + 1];
    int nblk;                        // 1: plain tile order
    int rows_own;                    // RESID with blocks: rows of the index mode
    // single pass (plain tile order): segments that cross tiles are finished
    // inside this launch.  Each tile publishes its two boundary partials as
    // words (float bits | epoch << 32); the tile holding a segment's closing
    // head (or the last tile, for the segment open at the end) waits for the
    // words of the chain's earlier tiles and writes the row.  Workgroups take
    // their tile from a ticket counter, so every tile waited on has started.
    uint64_t *sp_words;              // null: carries + fix-up pass; else ntiles x 2 x R words
    const int32_t *sp_from;          // per tile: start tile of the chain its first head closes, or -1
    unsigned long long *sp_ticket;   // ticket counter (never reset; sp_base is this launch's first)
    int *sp_err;                     // the tag of the last launch whose bounded wait gave up (0: none)
    unsigned long long sp_base;
    uint32_t sp_epoch;               // this launch's tag (never 0)
    int sp_tail_from;                // start tile of the segment open at the end of the tensor
};

constexpr int kSpinMax = 1 << 20;    // polls of one word before a wait gives up

// Publish a boundary partial of the single-pass variant.
__device__ __forceinline__ void sp_put(uint64_t *p, float v, uint32_t epoch)
{
    const uint64_t w = ((uint64_t)epoch << 32) | (uint64_t)__float_as_uint(v);
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (bounded) for a published partial of this launch and return it.  A
// wait that gives up writes the launch's tag to the error word, and every
// other wait of the launch returns soon after it sees it there, so a launch
// whose partials never arrive still ends in about one wait's bound.
__device__ __forceinline__ float sp_get(const uint64_t *p, uint32_t epoch, int *err)
{
    uint64_t w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int it = 0; (uint32_t)(w >> 32) != epoch; ++it) {
        if (it >= kSpinMax) {
            __hip_atomic_store(err, (int)epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0.f;
        }
        if ((it & 63) == 63 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)epoch)
            return 0.f;
        __builtin_amdgcn_s_sleep(2);
        w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return __uint_as_float((uint32_t)w);
}

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

constexpr int pow2_floor(int x)
{
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// The stream of one chunk as held by one lane: U entries per array (entry
// u of lane j is step u * LPN + j of the chunk), the three bf words that
// cover nonzeros [base - 1, base + 63] (decoded only when the chunk is
// used, so that loading the next chunk never waits), and the chunk length.
template <int U, int NPM>
struct Chunk {
    int idx[U][NPM];
    float v[U];
    uint32_t w0, w1, w2;
    int sh;                      // bit of nonzero base - 1 in w0; -1 when base == 0
    int n;
};

template <int LPN, int CL, int U, int NPM>
__device__ __forceinline__ void load_chunk(const SegArgs &A, int np, int j, int64_t base, int64_t re,
                                           Chunk<U, NPM> &c)
{
    const int64_t rem = re - base;
    c.n = rem < CL ? (int)rem : CL;
    const int64_t p1 = base - 1;
    const int64_t wi = p1 < 0 ? 0 : (p1 >> 5);
    c.sh = p1 < 0 ? -1 : (int)(p1 & 31);
    c.w0 = A.bf[wi];
    c.w1 = A.bf[wi + 1];
    c.w2 = A.bf[wi + 2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int el = u * LPN + j;
        const bool ev = el < c.n;
        const int64_t e = base + el;
#pragma unroll
        for (int qq = 0; qq < NPM; ++qq)
            c.idx[u][qq] = (ev && qq < np) ? __builtin_nontemporal_load(A.pidx[qq] + e) : 0;
        c.v[u] = ev ? __builtin_nontemporal_load(A.vals + e) : 0.f;
    }
}

// Segment heads of the chunk's n steps (bit s: step s starts a segment).
template <int U, int NPM>
__device__ __forceinline__ uint64_t chunk_heads(const Chunk<U, NPM> &c)
{
    const uint64_t lo = (uint64_t)c.w0 | ((uint64_t)c.w1 << 32);
    const int sh = c.sh < 0 ? 0 : c.sh;
    const uint64_t x = sh ? ((lo >> sh) | ((uint64_t)c.w2 << (64 - sh))) : lo;  // from nonzero base - 1
    const uint64_t top = (c.w2 >> sh) & 1u;                                       // nonzero base + 63
    const uint64_t cur = c.sh < 0 ? lo : ((x >> 1) | (top << 63));
    const uint64_t prev = c.sh < 0 ? 0ull : (x & 1ull);
    const uint64_t hm = cur ^ ((cur << 1) | prev);
    return c.n >= 64 ? hm : (hm & ((1ull << c.n) - 1ull));
}

// Stream of a super-chunk of SC = 4 * LPN * K steps, read with 16-byte loads:
// vector k of lane j holds steps (k * LPN + j) * 4 .. + 3, so each lane
// group reads whole 16-byte pieces of its run (a full 128-byte line per
// index array when LPN = 8).  Device streams carry 4 entries of padding, so
// a vector that starts below the run end never reads past the allocation.
typedef int int4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef float float4a4 __attribute__((ext_vector_type(4), aligned(4)));

template <int K, int NPM>
struct SChunk {
    int4a4 idx[K][NPM];
    float4a4 v[K];
    uint32_t w0, w1, w2;
    int sh;
    int n;
};

template <int LPN, int SC, int K, int NPM>
__device__ __forceinline__ void load_schunk(const SegArgs &A, int j, int64_t base, int64_t re,
                                            SChunk<K, NPM> &c)
{
    const int64_t rem = re - base;
    c.n = rem < SC ? (int)rem : SC;
    const int64_t p1 = base - 1;
    const int64_t wi = p1 < 0 ? 0 : (p1 >> 5);
    c.sh = p1 < 0 ? -1 : (int)(p1 & 31);
    c.w0 = A.bf[wi];
    c.w1 = A.bf[wi + 1];
    c.w2 = A.bf[wi + 2];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int el = (k * LPN + j) * 4;
        const bool ev = el < c.n;
        const int64_t e = base + el;
#pragma unroll
        for (int qq = 0; qq < NPM; ++qq)
            c.idx[k][qq] = ev ? __builtin_nontemporal_load(reinterpret_cast<const int4a4 *>(A.pidx[qq] + e))
                              : int4a4{0, 0, 0, 0};
        c.v[k] = ev ? __builtin_nontemporal_load(reinterpret_cast<const float4a4 *>(A.vals + e))
                    : float4a4{0.f, 0.f, 0.f, 0.f};
    }
}

template <int K, int NPM>
__device__ __forceinline__ uint64_t schunk_heads(const SChunk<K, NPM> &c)
{
    const uint64_t lo = (uint64_t)c.w0 | ((uint64_t)c.w1 << 32);
    const int sh = c.sh < 0 ? 0 : c.sh;
    const uint64_t x = sh ? ((lo >> sh) | ((uint64_t)c.w2 << (64 - sh))) : lo;
    const uint64_t top = (c.w2 >> sh) & 1u;
    const uint64_t cur = c.sh < 0 ? lo : ((x >> 1) | (top << 63));
    const uint64_t prev = c.sh < 0 ? 0ull : (x & 1ull);
    const uint64_t hm = cur ^ ((cur << 1) | prev);
    return c.n >= 64 ? hm : (hm & ((1ull << c.n) - 1ull));
}

template <int LPN, int ST, int K, int NPM>
__device__ __forceinline__ int sc_idx(const SChunk<K, NPM> &c, int qq)
{
    return bcast_imm<LPN, (ST / 4) % LPN>(c.idx[ST / (4 * LPN)][qq][ST % 4]);
}

template <int LPN, int ST, int K, int NPM>
__device__ __forceinline__ float sc_val(const SChunk<K, NPM> &c)
{
    return bcast_imm_f<LPN, (ST / 4) % LPN>(c.v[ST / (4 * LPN)][ST % 4]);
}

template <typename FT, int VW>
__device__ __forceinline__ void select_raw(bool take_a, const Raw<FT, VW> &a, const Raw<FT, VW> &b,
                                           Raw<FT, VW> &out)
{
    out.v = take_a ? a.v : b.v;
}

// Waves per SIMD.  The gathers' latency is what the waves wait on, so the
// wave count is held up by launch bounds, with the gather batch (registers
// of rows in flight per lane) sized to fit: float32 SpMTTKRP runs 3 waves
// with a full batch (more rows in flight per wave than 4 waves with a half
// batch, once a batch's gathers issue back to back); the other float32
// forms run 4 waves (128 VGPRs; the fused residual spills a few registers
// there and is still faster) with a half batch, and so does bfloat16 in
// 4-column lane chunks (8-byte row pieces, so a quarter batch holds as many
// rows); bfloat16 in 8-column chunks runs 3 (133-168 VGPRs) with a half
// batch, except the fused residual form, which runs 4 with a quarter batch
// (it holds no repeated row; a few registers spill); the one-lane residual
// form is left unconstrained.
template <typename FT, int VW, int LPN, int NP, bool RESID, bool KRON>
struct TileShape {
    static constexpr bool F32PLAIN = sizeof(FT) == 4 && NP >= 1 && (!RESID || LPN > 1);
    // float32 SpMTTKRP (two or more product modes): 3 waves with a double batch
    static constexpr bool F32MULTI = F32PLAIN && !RESID && !KRON && NP >= 2;
    static constexpr bool B16HALF = sizeof(FT) == 2 && VW == 4 && NP >= 1 && !RESID && !KRON;
    static constexpr bool B16ONE = sizeof(FT) == 2 && NP == 1 && !RESID && !KRON;
    static constexpr bool B16RES = sizeof(FT) == 2 && RESID && NP >= 2;
    static constexpr int waves = F32MULTI ? 3 : (F32PLAIN || B16HALF || B16RES) ? 4 : B16ONE ? 3
                               : (((LPN > 1 || !RESID) && !(sizeof(FT) == 2 && NP == 1)) ? 3 : 1);
    // registers of raw rows per lane for one gather batch
    static constexpr int batch_regs = F32MULTI ? 64 : (B16HALF || B16RES) ? 16
                                    : (F32PLAIN || B16ONE || (sizeof(FT) == 2 && NP >= 2)) ? 32 : 64;
};

template <typename FT, int VW, int LPN, int NP, bool RESID, bool ROWMAP, bool KRON = false, int KB = 1>
__global__ __launch_bounds__(256, (TileShape<FT, VW, LPN, NP, RESID, KRON>::waves))
void seg_tile_kernel(SegArgs A)
{
    constexpr int Q = 64 / LPN;                       // lane groups per wave
    constexpr int NPM = NP > 0 ? NP : kMaxNP;         // product modes held per step
    constexpr int RAWREGS = (int)(sizeof(Raw<FT, VW>) / 4);
    // gathers in flight per lane: the batch that fits the wave count above
    constexpr int CH0 = NP > 0 ? pow2_floor(TileShape<FT, VW, LPN, NP, RESID, KRON>::batch_regs / (NPM * RAWREGS)) : 2;
    constexpr int CL = CH0 > LPN ? CH0 : LPN;         // steps per chunk (stream granule)
    constexpr int CH = CH0 < CL ? CH0 : CL;           // steps per gather batch
    constexpr int U = CL / LPN;                       // stream entries per lane per chunk
    // KRON with KB > 1: a lane owns KB blocks of VW columns, one per element of
    // a KB-wide piece of the second-to-last product mode's row
    static_assert(KB == 1 || (KRON && !RESID), "column blocks are for SpTTMc");
    constexpr int AW = VW * KB;                       // accumulated columns per lane
    constexpr int RT = LPN * AW;                      // columns of this rank tile

    __shared__ int s_f[4];
    // the four waves' boundary partials (a: rows 0-3, b: rows 4-7); the single
    // pass reuses the rows for its chain sums once they have been read
    __shared__ float s_ab[8][RT];
    float (*s_a)[RT] = s_ab;
    float (*s_b)[RT] = s_ab + 4;
    __shared__ double s_loss[4];
    __shared__ int s_hw[4];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int q = lane / LPN, j = lane % LPN;
    int64_t tile = blockIdx.x;
    int ry = (int)blockIdx.y;                         // rank tile
    if (A.sp_words) {
        // single pass: tiles in the order workgroups start (tickets), so every
        // tile this one may wait on is running or done
        __shared__ unsigned long long s_tk;
        if (threadIdx.x == 0) s_tk = atomicAdd(A.sp_ticket, 1ull) - A.sp_base;
        __syncthreads();
        if (s_tk >= (unsigned long long)A.ntiles * gridDim.y) {
            // ticket bookkeeping out of step with the launches: touch nothing
            if (threadIdx.x == 0)
                __hip_atomic_store(A.sp_err, (int)A.sp_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        tile = (int64_t)(s_tk / gridDim.y);
        ry = (int)(s_tk % gridDim.y);
    } else if (A.nblk > 1) {
        // XCD-aware order: every tile of block b runs on XCD b, whose L2 then
        // holds that block's rows of the split product mode
        const int x = (int)(blockIdx.x % kXcdBlocks);
        tile = A.blk_ts[x] + (int64_t)(blockIdx.x / kXcdBlocks);
        if (tile >= A.blk_ts[x + 1]) return;          // the whole workgroup leaves, before any barrier
    }
    const int T = A.tile_nnz;
    const int S = T / (4 * Q);                        // run length of one lane group
    const int64_t t0 = tile * (int64_t)T;
    const int64_t wstart = t0 + (int64_t)w * Q * S;
    const int64_t rs = wstart + (int64_t)q * S;
    const int64_t re = rs + S < A.nnz ? rs + S : A.nnz;
    const int np = NP > 0 ? NP : A.np;
    int col, colc;
    bool cval;
    if constexpr (KB == 1) {
        col = ry * RT + j * VW;
        cval = col < A.R;
        colc = cval ? col : 0;                        // lanes past R read column 0, never store
    } else {
        // lane gl: block gl % nb2 of the last mode, block (gl / nb2) % nb1 of
        // the one before, then the earlier modes' combined index
        const int gl = ry * LPN + j;
        const int nb2 = A.kr[np - 1] / VW, nb1 = A.kr[np - 2] / KB;
        cval = gl < A.R / AW;
        const int g2 = cval ? gl : 0;
        col = ((g2 / (nb2 * nb1)) * A.kr[np - 2] + ((g2 / nb2) % nb1) * KB) * A.kr[np - 1] + (g2 % nb2) * VW;
        colc = col;
    }
    const int R = A.R;
    // row bytes fit 32 bits (R <= 256), so a gather address is one 32 x 32 -> 64
    // multiply-add onto the factor's base
    const uint32_t R4 = (uint32_t)R * (uint32_t)sizeof(FT);
    // RESID: factor row of the index mode for an output row (blocks add block * rows)
    auto own_row = [&](int r) -> int64_t { return A.nblk > 1 ? (int64_t)(r % A.rows_own) : (int64_t)r; };
    const char *fb[NPM];
    uint32_t R4k[NPM];                                // KRON: row bytes of each product mode
    if constexpr (KRON) {
        // digits of this lane's first column, last product mode fastest (with
        // column blocks, the second-to-last digit starts this lane's KB-piece)
        int rem = colc;
#pragma unroll
        for (int qq = NPM - 1; qq >= 0; --qq) {
            if (qq < np) {
                const int d = rem % A.kr[qq];
                rem /= A.kr[qq];
                fb[qq] = reinterpret_cast<const char *>(A.fac[qq]) + (size_t)d * sizeof(FT);
                R4k[qq] = (uint32_t)A.kr[qq] * (uint32_t)sizeof(FT);
            } else {
                fb[qq] = nullptr;
                R4k[qq] = 0;
            }
        }
    } else {
#pragma unroll
        for (int qq = 0; qq < NPM; ++qq) {
            fb[qq] = reinterpret_cast<const char *>(A.fac[qq]) + (size_t)colc * sizeof(FT);
            R4k[qq] = R4;
        }
    }

    // store the lane's AW columns of one output (or carry) row
    const int kstride = KB > 1 ? A.kr[np - 1] : 0;   // column distance between a lane's blocks
    auto store_acc = [&](float *rowp, const float (&v)[AW]) {
        if constexpr (KB == 1 && !ROWMAP && !KRON) {
            store_row_stream<VW>(rowp + col, v);      // SpTTM: one row per fibre, never re-read
        } else if constexpr (KB == 1) {
            store_row<VW>(rowp + col, v);
        } else {
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                float tv[VW];
#pragma unroll
                for (int k = 0; k < VW; ++k) tv[k] = v[kb * VW + k];
                store_row<VW>(rowp + col + kb * kstride, tv);
            }
        }
    };

    // first chunk of the stream and the tile's segment ordinal: issued first
    // fast path: 16-byte stream vectors in super-chunks; generic path: chunks
    constexpr bool FAST = (NP > 0) && (VW > 1) && !KRON;
    constexpr int CLF = CH0;                                           // gather batch (register budget)
    constexpr int K = FAST ? ((CLF + 4 * LPN - 1) / (4 * LPN)) : 1;  // vectors per lane per array
    constexpr int SC = FAST ? 4 * LPN * K : CL;                        // steps per super-chunk
    static_assert(!FAST || (SC % CLF == 0 && SC <= 64), "super-chunk shape");
    // SpMTTKRP: consecutive nonzeros often share the first product-mode
    // index (its order within a segment is sorted); such rows are not re-read.
    // That saves cache requests at the price of a held row and a select per
    // step: it pays where one gather instruction covers 16 rows or more (4
    // lanes per row or fewer) or there are three product modes, but cost
    // float32 with two product modes at 8 or more lanes per row 4% on the
    // Zipf 20M tensor, and the fused residual form (which also holds the
    // segment's own row) 18% in bfloat16 on the 200M tensor, so those forms
    // re-read the row
    constexpr bool REUSE = FAST && ROWMAP && NP >= 2 && !RESID && !(sizeof(FT) == 4 && NP == 2 && LPN >= 8);
    Chunk<U, NPM> cur;
    SChunk<K, NPM> scur;
    if (rs < re) {
        if constexpr (FAST) load_schunk<LPN, SC, K, NPM>(A, j, rs, re, scur);
        else load_chunk<LPN, CL, U, NPM>(A, np, j, rs, re, cur);
    }
    const int ts0 = A.tile_seg0[tile];
    const int h0 = (int)head_at(A.bf, t0);

    // ---- 1. heads before each run.  Heads in [t0, wave start): counted by
    //         the whole wave; heads of the earlier runs of this wave: a scan
    //         across lane groups.  No barrier.
    int wc = 0;
    const int64_t wend = wstart < A.nnz ? wstart : A.nnz;   // no bits exist at or past Z
    for (int64_t p = t0 + 64 * (int64_t)lane; p < wend; p += 64 * 64) {
        const int n = (int)(wend - p < 64 ? wend - p : 64);
        wc += __popcll(head_window(A.bf, p, n));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wc += __shfl_xor(wc, o, 64);
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
    // heads strictly before the tile: ordinal of its first nonzero + 1, less
    // one if that nonzero is itself a head
    const int H_tile = ts0 + 1 - h0;
    const int H_wave = H_tile + wc;
    const int H_run = H_wave + inc - cnt;

    // ---- 2. walk the run, one chunk at a time: gather this chunk's rows,
    //         then put the next chunk's stream in flight, then reduce
    float acc[AW], pre[AW];
    zero(acc);
    zero(pre);
    int have = 0;
    int g = H_run - 1;                                // segment open before the run
    int currow = 0;                                   // ROWMAP: output row of segment g
    float own[VW];
    float lsum = 0.f;
    if constexpr (RESID) {
        zero(own);
        if (g >= 0 && rs < re) {
            currow = A.seg_row[g];
            load_row<FT, VW>(reinterpret_cast<const FT *>(A.own) + own_row(currow) * R + colc, own);
        }
    }

    // one step of the general path (a head may occur, the chunk may be short)
    auto on_head = [&](uint64_t hm, int st) {
        if ((hm >> st) & 1ull) {
            if (have && cval) {
                const int64_t row = ROWMAP ? (int64_t)currow : (int64_t)g;
                store_acc(A.out + row * R, acc);
            }
            if (!have) {
#pragma unroll
                for (int k = 0; k < AW; ++k) pre[k] = acc[k];
            }
            have = 1;
            zero(acc);
            ++g;
            if constexpr (ROWMAP) currow = A.seg_row[g];
            if constexpr (RESID)
                load_row<FT, VW>(reinterpret_cast<const FT *>(A.own) + own_row(currow) * R + colc, own);
        }
    };
    auto step = [&](const float (&h)[AW], float v, uint64_t hm, int st, int n) {
        on_head(hm, st);
        if (st < n) {
            if constexpr (RESID) {
                // lanes past R hold column 0 (clamped reads): kept out of the dot product
                float d = 0.f;
#pragma unroll
                for (int k = 0; k < VW; ++k) d += own[k] * h[k];
                d = group_sum<LPN>(cval ? d : 0.f);
                const float r = d - v;
                const float sc = r * A.inv_nnz;
#pragma unroll
                for (int k = 0; k < VW; ++k) acc[k] += sc * h[k];
                if (j == 0) lsum += r * r;
            } else {
#pragma unroll
                for (int k = 0; k < AW; ++k) acc[k] += v * h[k];
            }
        }
    };

    if constexpr (FAST) {
        int lastidx = -1;                              // REUSE: index of the row held in last0
        Raw<FT, VW> last0;
        set_one<FT, VW>(last0);
        for (int64_t base = rs; base < re; base += SC) {
            SChunk<K, NPM> snxt;
            const bool more = base + SC < re;
            const uint64_t hms = schunk_heads(scur);
            const int nsc = scur.n;
            static_for<SC / CLF>([&](auto cc) {
                constexpr int C0 = decltype(cc)::value * CLF;
                // gathers of this chunk, back to back (repeated first-mode rows skipped)
                Raw<FT, VW> rows[CLF][NPM];
                uint32_t dup = 0;
                static_for<CLF>([&](auto sc) {
                    constexpr int ST = decltype(sc)::value;
#pragma unroll
                    for (int qq = 0; qq < NPM; ++qq) {
                        const int idx = sc_idx<LPN, C0 + ST, K, NPM>(scur, qq);
                        const char *p = fb[qq] + (uint64_t)(uint32_t)idx * (uint64_t)R4;
                        if (REUSE && qq == 0) {
                            const bool d = idx == lastidx;
                            lastidx = idx;
                            dup |= (uint32_t)d << ST;
                            // a repeated row is taken from last0 when used, so the
                            // register is left as it is here
                            if (!d) load_raw<FT, VW>(reinterpret_cast<const FT *>(p), rows[ST][0]);
                        } else {
                            load_raw<FT, VW>(reinterpret_cast<const FT *>(p), rows[ST][qq]);
                        }
                    }
                });
                if constexpr (C0 == 0) {
                    if (more) load_schunk<LPN, SC, K, NPM>(A, j, base + SC, re, snxt);
                }
                if constexpr (REUSE) {
                    // hide from the optimiser that the repeat mask below is the
                    // branch condition above: otherwise it folds the choice
                    // between last0 and the new row into the branch's join, which
                    // then needs each conditional gather to land before the next
                    // one issues (a wait per step instead of one per batch)
                    __asm__ volatile("" : "+v"(dup));
                }
                float vv[CLF];
                static_for<CLF>([&](auto sc) {
                    constexpr int ST = decltype(sc)::value;
                    vv[ST] = sc_val<LPN, C0 + ST, K, NPM>(scur);
                });
                const uint64_t hm = (hms >> C0) & ((CLF >= 64) ? ~0ull : ((1ull << CLF) - 1ull));
                const int n = nsc - C0;
                const bool easy = !RESID && __ballot(hm != 0ull || n < CLF) == 0ull;
                auto hrow = [&](auto sc, float (&h)[VW]) {
                    constexpr int ST = decltype(sc)::value;
                    if constexpr (REUSE) {
                        Raw<FT, VW> r0;
                        select_raw<FT, VW>((dup >> ST) & 1u, last0, rows[ST][0], r0);
                        last0 = r0;
                        to_float<FT, VW>(r0, h);
                    } else {
                        to_float<FT, VW>(rows[ST][0], h);
                    }
#pragma unroll
                    for (int qq = 1; qq < NPM; ++qq) {
                        float x[VW];
                        to_float<FT, VW>(rows[ST][qq], x);
#pragma unroll
                        for (int k = 0; k < VW; ++k) h[k] *= x[k];
                    }
                };
                if (easy) {
                    static_for<CLF>([&](auto sc) {
                        constexpr int ST = decltype(sc)::value;
                        float h[VW];
                        hrow(sc, h);
#pragma unroll
                        for (int k = 0; k < VW; ++k) acc[k] += vv[ST] * h[k];
                    });
                } else if (NP == 1 && !RESID && __ballot(n < CLF) == 0ull) {
                    // every lane group holds the whole batch (only a run's end
                    // is short), so no step needs the bound check; kept to one
                    // product mode without the residual, where the copy of the
                    // loop body costs no spills
                    static_for<CLF>([&](auto sc) {
                        constexpr int ST = decltype(sc)::value;
                        float h[VW];
                        hrow(sc, h);
                        step(h, vv[ST], hm, ST, CLF);
                    });
                } else {
                    static_for<CLF>([&](auto sc) {
                        constexpr int ST = decltype(sc)::value;
                        float h[VW];
                        hrow(sc, h);
                        step(h, vv[ST], hm, ST, n);
                    });
                }
            });
            scur = snxt;
        }
    } else {
        for (int64_t base = rs; base < re; base += CL) {
            Chunk<U, NPM> nxt;
            const bool more = base + CL < re;
            // generic path: gathers in batches of CH steps, runtime mode count
            if (more) load_chunk<LPN, CL, U, NPM>(A, np, j, base + CL, re, nxt);
            const uint64_t hm = chunk_heads(cur);
            const int n = cur.n;
            static_for<CL / CH>([&](auto sbc) {
                constexpr int S0 = decltype(sbc)::value * CH;
                Raw<FT, VW> rows[CH][NPM];
                Raw<FT, 1> ks[CH][NPM];                 // KRON: one element of each non-last mode
                Raw<FT, KB> kp[CH];                     // KRON, KB > 1: KB elements of the second-to-last mode
                static_for<CH>([&](auto jjc) {
                    constexpr int ST = S0 + decltype(jjc)::value;
#pragma unroll
                    for (int qq = 0; qq < NPM; ++qq) {
                        const int idx = bcast_imm<LPN, ST % LPN>(cur.idx[ST / LPN][qq]);
                        const FT *p = reinterpret_cast<const FT *>(fb[qq] + (uint64_t)(uint32_t)idx * (uint64_t)R4k[qq]);
                        if constexpr (KRON && KB > 1) {
                            if (qq < np - 2) load_raw<FT, 1>(p, ks[ST - S0][qq]);
                            else if (qq == np - 2) load_raw<FT, KB>(p, kp[ST - S0]);
                            else if (qq == np - 1) load_raw<FT, VW>(p, rows[ST - S0][0]);
                        } else if constexpr (KRON) {
                            if (qq < np - 1) load_raw<FT, 1>(p, ks[ST - S0][qq]);
                            else if (qq == np - 1) load_raw<FT, VW>(p, rows[ST - S0][0]);
                        } else {
                            if (qq < np) load_raw<FT, VW>(p, rows[ST - S0][qq]);
                            else set_one<FT, VW>(rows[ST - S0][qq]);
                        }
                    }
                });
                static_for<CH>([&](auto jjc) {
                    constexpr int ST = S0 + decltype(jjc)::value;
                    const float v = bcast_imm_f<LPN, ST % LPN>(cur.v[ST / LPN]);
                    float h[AW];
                    if constexpr (KRON && KB > 1) {
                        (void)h;
                        float u2[VW], u1[KB];
                        to_float<FT, VW>(rows[ST - S0][0], u2);
                        to_float<FT, KB>(kp[ST - S0], u1);
                        float m = 1.f;
#pragma unroll
                        for (int qq = 0; qq < NPM - 2; ++qq) {
                            if (qq < np - 2) {
                                float x[1];
                                to_float<FT, 1>(ks[ST - S0][qq], x);
                                m *= x[0];
                            }
                        }
                        // column (kb, k) gains (v m u1[kb]) u2[k]: one multiply-add per column
                        on_head(hm, ST);
                        if (ST < n) {
                            const float vm = v * m;
#pragma unroll
                            for (int kb = 0; kb < KB; ++kb) {
                                const float c1 = vm * u1[kb];
#pragma unroll
                                for (int k = 0; k < VW; ++k) acc[kb * VW + k] += c1 * u2[k];
                            }
                        }
                        return;
                    } else {
                        to_float<FT, VW>(rows[ST - S0][0], h);
                    }
                    if constexpr (KRON) {
                        float m = 1.f;
#pragma unroll
                        for (int qq = 0; qq < NPM - 1; ++qq) {
                            if (qq < np - 1) {
                                float x[1];
                                to_float<FT, 1>(ks[ST - S0][qq], x);
                                m *= x[0];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < VW; ++k) h[k] *= m;
                    } else {
#pragma unroll
                        for (int qq = 1; qq < NPM; ++qq) {
                            float x[VW];
                            to_float<FT, VW>(rows[ST - S0][qq], x);
#pragma unroll
                            for (int k = 0; k < VW; ++k) h[k] *= x[k];
                        }
                    }
                    step(h, v, hm, ST, n);
                });
            });
            cur = nxt;
        }
    }

    // ---- 3. wave-level segmented scan of the runs' (f, a, b)
    const int fo = have;
    float ao[AW];
    int f = have;
    float a[AW], b[AW];
#pragma unroll
    for (int k = 0; k < AW; ++k) {
        ao[k] = have ? pre[k] : acc[k];
        a[k] = ao[k];
        b[k] = acc[k];
    }
    wave_segscan<LPN, AW>(f, a, b, q);
    {   // exclusive prefix of this group: the inclusive value of group q - 1
        const int fp = __shfl_up(f, LPN, 64);
        float bp[AW];
#pragma unroll
        for (int k = 0; k < AW; ++k) bp[k] = __shfl_up(b[k], LPN, 64);
        if (q >= 1 && fo && fp && cval) {
            float v[AW];
#pragma unroll
            for (int k = 0; k < AW; ++k) v[k] = bp[k] + ao[k];
            const int gc = H_run - 1;
            const int64_t row = ROWMAP ? (int64_t)A.seg_row[gc] : (int64_t)gc;
            store_acc(A.out + row * R, v);
        }
    }
    if (q == Q - 1) {
#pragma unroll
        for (int k = 0; k < AW; ++k) {
            s_a[w][j * AW + k] = a[k];
            s_b[w][j * AW + k] = b[k];
        }
        if (j == 0) s_f[w] = f;
    }
    if constexpr (RESID) {
        float l = lsum;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
        if (lane == 0) s_loss[w] = (double)l;
    }
    if (lane == 0) s_hw[w] = H_wave;
    __syncthreads();

    // ---- 4. tile level: a wave's first closing whose segment started in an
    //         earlier wave of the tile; then the tile's carries
    if (q == 0 && w >= 1 && s_f[w] && cval) {
        int fx = s_f[0];
        float bx[AW];
#pragma unroll
        for (int k = 0; k < AW; ++k) bx[k] = s_b[0][j * AW + k];
        for (int i = 1; i < w; ++i) {
#pragma unroll
            for (int k = 0; k < AW; ++k) bx[k] = s_f[i] ? s_b[i][j * AW + k] : bx[k] + s_a[i][j * AW + k];
            fx |= s_f[i];
        }
        if (fx) {
            float v[AW];
#pragma unroll
            for (int k = 0; k < AW; ++k) v[k] = bx[k] + s_a[w][j * AW + k];
            const int gc = s_hw[w] - 1;
            const int64_t row = ROWMAP ? (int64_t)A.seg_row[gc] : (int64_t)gc;
            store_acc(A.out + row * R, v);
        }
    }
    float at[AW], bt[AW];                             // the tile's carries (wave 0, group 0)
    if (w == 0 && q == 0 && cval) {
        int ft = s_f[0];
#pragma unroll
        for (int k = 0; k < AW; ++k) { at[k] = s_a[0][j * AW + k]; bt[k] = s_b[0][j * AW + k]; }
        for (int i = 1; i < 4; ++i) {
#pragma unroll
            for (int k = 0; k < AW; ++k) {
                const float ai = s_a[i][j * AW + k], bi = s_b[i][j * AW + k];
                const float na = ft ? at[k] : at[k] + ai;
                const float nb = s_f[i] ? bi : bt[k] + ai;
                at[k] = na;
                bt[k] = nb;
            }
            ft |= s_f[i];
        }
        if (A.sp_words) {
#pragma unroll
            for (int k = 0; k < AW; ++k) {
                const int c = col + (k / VW) * kstride + (k % VW);
                sp_put(A.sp_words + (tile * 2) * R + c, at[k], A.sp_epoch);
                sp_put(A.sp_words + (tile * 2 + 1) * R + c, bt[k], A.sp_epoch);
            }
        } else {
            store_acc(A.carry_a + tile * R, at);
            store_acc(A.carry_b + tile * R, bt);
        }
    }
    if (A.sp_words) {
        // chains this tile closes: the segment its first head closes (started
        // in tile sp_from[tile]), and at the last tile the segment open at the
        // end.  Up to 8 lane groups sum strided shares of the chain's middle
        // tiles for wave 0 group 0's columns, several words in flight each;
        // group 0 adds the shares in a fixed order to the chain start's closing
        // partial and the tile's own.
        constexpr int SPG = 4 * Q < 8 ? 4 * Q : 8;       // lane groups summing a chain
        constexpr int UW = AW >= 16 ? 1 : 16 / AW;       // tiles in flight per group
        const int G = w * Q + q;
        __syncthreads();                                  // s_ab has been read above
        auto chain = [&](int64_t from, bool tail) {
            float part[AW];
            zero(part);
            if (G < SPG && cval) {
                for (int64_t t0 = from + 1 + G; t0 < tile; t0 += (int64_t)UW * SPG) {
                    uint64_t wv[UW][AW];
#pragma unroll
                    for (int u = 0; u < UW; ++u) {
                        const int64_t tt = t0 + (int64_t)u * SPG;
#pragma unroll
                        for (int k = 0; k < AW; ++k) {
                            const int c = col + (k / VW) * kstride + (k % VW);
                            wv[u][k] = tt < tile ? __hip_atomic_load(A.sp_words + (tt * 2) * R + c, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT)
                                                 : ((uint64_t)A.sp_epoch << 32);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UW; ++u) {
                        const int64_t tt = t0 + (int64_t)u * SPG;
#pragma unroll
                        for (int k = 0; k < AW; ++k) {
                            float x = __uint_as_float((uint32_t)wv[u][k]);
                            if ((uint32_t)(wv[u][k] >> 32) != A.sp_epoch) {   // not published yet: wait
                                const int c = col + (k / VW) * kstride + (k % VW);
                                x = sp_get(A.sp_words + (tt * 2) * R + c, A.sp_epoch, A.sp_err);
                            }
                            part[k] += x;
                        }
                    }
                }
            }
            if (G < SPG) {
#pragma unroll
                for (int k = 0; k < AW; ++k) s_ab[G][j * AW + k] = part[k];
            }
            __syncthreads();
            if (G == 0 && cval) {
                float v[AW];
                if (tail && from == tile) {
                    // the last tile holds the last segment's head: its own closing partial
#pragma unroll
                    for (int k = 0; k < AW; ++k) v[k] = bt[k];
                } else {
#pragma unroll
                    for (int k = 0; k < AW; ++k) {
                        const int c = col + (k / VW) * kstride + (k % VW);
                        v[k] = sp_get(A.sp_words + (from * 2 + 1) * R + c, A.sp_epoch, A.sp_err);
                    }
                    for (int g2 = 0; g2 < SPG; ++g2) {
#pragma unroll
                        for (int k = 0; k < AW; ++k) v[k] += s_ab[g2][j * AW + k];
                    }
#pragma unroll
                    for (int k = 0; k < AW; ++k) v[k] += at[k];
                }
                const int gc = tail ? A.nseg - 1 : H_tile - 1;
                const int64_t row = ROWMAP ? (int64_t)A.seg_row[gc] : (int64_t)gc;
                store_acc(A.out + row * R, v);
            }
            __syncthreads();
        };
        const int64_t from1 = A.sp_from[tile];
        if (from1 >= 0) chain(from1, false);
        if (tile == A.ntiles - 1) chain(A.sp_tail_from, true);
    }
    if constexpr (RESID) {
        if (tid == 0 && ry == 0 && A.partial)
            A.partial[tile] = ((s_loss[0] + s_loss[1]) + s_loss[2]) + s_loss[3];
    }
}

}  // namespace dev
}  // namespace fcoo

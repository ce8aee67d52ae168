// Internal declarations shared by the host builder and the HIP launchers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fcoo.h"

namespace fcoo {

constexpr int kMaxOrder = 8;
constexpr int kMaxR = 256;
constexpr int kMaxKronWidth = 16384;   // SpTTMc output columns (prod of the product-mode ranks)
constexpr int kBlock = 256;        // threads per workgroup of the tile kernels (4 waves)
constexpr int kXcds = 8;           // XCDs of an MI355X: workgroup w runs on XCD w % 8

// error reporting (thread-local message, negative code returned)
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();

#define FCOO_HIP(call)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return ::fcoo::hip_fail(e_, #call); \
    } while (0)

// One (op, mode) F-COO build: host arrays (kept for export) and device copies.
struct Built {
    bool built = false;
    bool on_device = false;
    bool host_arrays = true;                  // false: built on the GPU, per-nonzero arrays on the device only
    int op = 0, mode = 0, threadlen = 0, tile_nnz = 0;
    int lane_cols = 0;                        // bfloat16 columns per lane chunk (4, 8; 0: default rule)
    int64_t nnz = 0, nseg = 0, npart = 0, ntiles = 0;
    std::vector<int> imodes, pmodes;

    // XCD blocks (SpMTTKRP): the nonzeros are split into nblk groups by ranges
    // of product mode bmode's index (blk_of), each group leading the sort key;
    // a segment is a (block, row) pair written to partial row block * I + row,
    // and block b's tiles [blk_ts[b], blk_ts[b+1]) run on XCD b
    int nblk = 1;
    int bmode = -1;
    int64_t rows = 0;                         // SpMTTKRP: dims[mode] (rows of the result)
    std::vector<int32_t> blk_of;              // dims[bmode]: block of each index
    std::vector<int64_t> blk_ts;              // nblk + 1 tile starts

    // F-COO arrays (Sec. IV-B) and per-segment / per-tile indexing
    std::vector<std::vector<int32_t>> pidx;   // |pmodes| x Z
    std::vector<float> val;                   // Z
    std::vector<uint8_t> bf;                  // ceil(Z/8)
    std::vector<uint32_t> sf;                 // ceil(P/32)
    std::vector<int32_t> seg;                 // MTTKRP: nseg rows; TTM: nseg x (N-1)
    std::vector<int32_t> tile_seg0;           // ntiles
    std::vector<int32_t> perm;                // Z: sorted position -> input position

    // carry fix-up list: (closing tile b, chain start tile a, output row) per entry
    std::vector<int32_t> fix;
    std::vector<int32_t> empty_rows;          // MTTKRP rows with no nonzero

    // device copies
    int32_t *d_pidx[kMaxOrder] = {};
    float *d_val = nullptr;
    uint32_t *d_bf = nullptr;                 // bit stream as uint32 words, +2 zero words
    uint32_t *d_sf = nullptr;                 // device builds only (where it is made), for export
    int32_t *d_seg_row = nullptr;             // MTTKRP only
    int32_t *d_tile_seg0 = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_fix = nullptr;
    int32_t *d_empty = nullptr;
    int64_t device_bytes = 0;

    // scratch owned by this build, grown on demand
    float *d_carry = nullptr;                 // 2 x ntiles x R floats
    int64_t carry_cap = 0;                    // floats
    float *d_gperm = nullptr;                 // Z floats (values in stored order)
    float *d_bpart = nullptr;                 // XCD blocks: nblk x I x width partial outputs
    int64_t bpart_cap = 0;                    // floats
    double *d_partial = nullptr;              // per-tile float64 partial sums
    int64_t partial_cap = 0;

    // single pass (fcoo_opts.single_pass): segments crossing tiles are finished
    // inside the tile kernel from published boundary partials, no fix-up pass
    bool sp = false;
    int32_t *d_sp_from = nullptr;             // ntiles: chain start tile of each tile's first head, or -1
    int sp_tail_from = -1;                    // chain start of the segment open at the end
    uint64_t *d_sp_words = nullptr;           // ntiles x 2 x R published partials
    int64_t sp_words_cap = 0;                 // words
    unsigned long long *d_sp_ticket = nullptr;   // ticket counter (never reset)
    int *d_sp_err = nullptr;                  // set by a wait that gave up
    unsigned long long sp_tickets = 0;        // tickets taken by earlier launches
    uint32_t sp_epoch = 0;                    // tag of the last launch

    int64_t nfix() const { return (int64_t)fix.size() / 3; }
    int64_t max_block_tiles() const;
    int64_t format_bytes() const;
    void free_device();
};

// Scratch for CP-ALS and small reductions, owned by the handle.
struct Workspace {
    float *M = nullptr;          int64_t M_cap = 0;      // floats
    double *dbl = nullptr;       int64_t dbl_cap = 0;    // doubles
    int *flags = nullptr;                               // device ints (pinv flags)
    double *host_pinned = nullptr;                      // fit readback
    void free_all();
};

}  // namespace fcoo

struct fcoo_tensor {
    int order = 0;
    int64_t dims[fcoo::kMaxOrder] = {};
    int64_t nnz = 0;
    std::vector<int32_t> idx[fcoo::kMaxOrder];
    std::vector<float> vals;
    double normX2 = 0.0;                         // sum of squared values (float64)
    fcoo::Built b[2][fcoo::kMaxOrder];

    // coordinate list on the device (model at the nonzeros), uploaded on first use
    int32_t *d_coo[fcoo::kMaxOrder] = {};
    float *d_coo_val = nullptr;
    bool coo_on_device = false;

    fcoo::Workspace ws;

    // optional events recorded around each tile kernel (caller-owned)
    hipEvent_t ev_before = nullptr, ev_after = nullptr;
    // CP-ALS: second stream for the R x R solve (default priority), created on first use
    hipStream_t aux = nullptr;
    hipEvent_t ev_dep = nullptr, ev_solved = nullptr;
};

namespace fcoo {

// helpers implemented in fcoo_host.cpp
int ensure_device_floats(float **p, int64_t *cap, int64_t need, hipStream_t s);
int ensure_device_doubles(double **p, int64_t *cap, int64_t need, hipStream_t s);
int upload_coo(fcoo_tensor *t, hipStream_t s);
int upload_i32(int32_t **dst, const std::vector<int32_t> &v, int64_t pad, hipStream_t s, int64_t *acct);
// carry fix-up chains and empty output rows from the per-tile head counts
// (heads_before[t] = heads before nonzero t * tile_nnz, t = 0 .. ntiles) and b.seg
void finish_tiles(const fcoo_tensor *t, Built &b, int mode, int op, const std::vector<int64_t> &heads_before);
// the F-COO build of one (op, mode) on the GPU (same arrays as the host build)
// Device primitives of the GPU build (fcoo_sort.hip).  sort_pairs_u64: stable
// radix sort of n (key, value) pairs by the key's bits below end_bit,
// ping-ponging between the two buffers; the result is in (k0, v0) if
// *passes is even, else in (k1, v1).  scan_i32: prefix sum of n int32 (out
// may not alias in).  `work` holds sort_work_ints(n) / scan_work_ints(n)
// int32 of device scratch.  Both enqueue on s and return an FCOO_* code.
int64_t sort_work_ints(int64_t n);
int64_t scan_work_ints(int64_t n);
int sort_pairs_u64(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int end_bit,
                   int32_t *work, hipStream_t s, int *passes);
int scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, int32_t *work, hipStream_t s);
int build_on_device(fcoo_tensor *t, Built &b, int mode, int op, int threadlen, int tile_nnz, int nblk,
                    int xmode, hipStream_t s);
// XCD blocks of a SpMTTKRP build (nblk 0 / 1: none), split by ranges of product
// mode xmode (-1: the product mode with the most rows); needs b.op, b.mode,
// b.pmodes, b.tile_nnz
int setup_blocks(const fcoo_tensor *t, Built &b, int nblk, int xmode);
// the single-pass chain table of a finished build (fix list -> per-tile chain starts) and its counters
int setup_single_pass(Built &b, hipStream_t s);
int check_factors(const fcoo_tensor *t, int skip_mode, const void *const *factors, int dtype, int R);
// the build of (op, mode), or NULL with *rc set (FCOO_EINVAL: null handle, mode
// or op out of range; FCOO_ENOTBUILT: no build, or none on the device if need_device)
Built *get_built(fcoo_tensor *t, int mode, int op, bool need_device, int *rc);

// launchers implemented in the .hip files (return FCOO_OK or an error code)
struct TileProblem {
    const Built *b;
    const void *fac[kMaxOrder];      // per product mode q: factor base pointer
    const float *vals;               // values in stored order (b->d_val or a permuted copy)
    int dtype;
    int R;
    float *out;                      // output rows, leading dimension R
    float *carry;                    // 2 x ntiles x R
    // fused MSE residual (resid_spmttkrp)
    const void *own = nullptr;       // factor of the index mode (dims[mode] x R)
    float inv_nnz = 0.f;
    double *partial = nullptr;       // per-tile partial losses (ntiles) or null
    hipEvent_t ev_before = nullptr;  // recorded around the tile kernel when set
    hipEvent_t ev_after = nullptr;
    float *bpart = nullptr;          // XCD blocks: nblk x rows x R partial output (segments land here)
    // SpTTMc: Kronecker rows; R is then the output width prod kr[q]
    bool kron = false;
    int kr[kMaxOrder] = {};          // per product mode q: columns of its factor
    // single pass (set by prep_single_pass; sp_words null: carries + fix-up)
    uint64_t *sp_words = nullptr;
    uint32_t sp_epoch = 0;
};
// single-pass words of a build for a launch of width R (no-op for other builds)
int prep_single_pass(Built *b, TileProblem &p, hipStream_t s);
int launch_segmented(const TileProblem &p, hipStream_t s, bool resid);
int launch_permute_values(const Built &b, const float *g, float *out, hipStream_t s);
int launch_reduce_partials(const double *partial, int64_t n, double scale, double *out, hipStream_t s);
int launch_model(const fcoo_tensor *t, const void *const *factors, int dtype, int R, float *xhat,
                 hipStream_t s);

}  // namespace fcoo

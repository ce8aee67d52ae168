/*
 * fcoo.h -- C ABI of the F-COO sparse tensor library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library implements the unified sparse tensor method of "A Unified
 * Optimization Approach for Sparse Tensor Operations on GPUs" (Liu, Wen,
 * Sarwate, Mehri Dehnavi): the flagged-coordinate (F-COO) storage format
 * (Sec. IV-B), and one-shot SpMTTKRP / SpTTM kernels that reduce with a
 * segmented scan instead of atomics (Sec. IV-C, IV-D), driving CP-ALS
 * (Algorithm 1).  It adds gradient-based sparse CP (model at the nonzeros,
 * residual SpMTTKRP) and a BF16 factor-storage form.
 *
 * Conventions for every entry point:
 *   - Modes are 0-based: the paper's "mode-1" is mode 0.
 *   - Dense matrices (factors, M, Y, U) are row-major with leading dimension
 *     R: element (i, r) is at offset i * R + r.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it and the call returns without waiting,
 *     except where stated (fcoo_build waits for its upload; fcoo_cp_als_iter
 *     waits for the 8-byte fit).
 *   - Return value: FCOO_OK (0) or a negative FCOO_E* code; the message of
 *     the last error on the calling thread is fcoo_last_error().  No call
 *     aborts or throws on bad input.
 *   - A handle is not re-entrant (it owns scratch buffers): use one handle
 *     per thread, or serialise calls on it.
 */
#ifndef FCOO_H
#define FCOO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FCOO_OK = 0,
    FCOO_EINVAL = -1,        /* null pointer, mode out of range, bad option value */
    FCOO_ENOMEM = -2,        /* host or device allocation failed */
    FCOO_EHIP = -3,          /* a HIP runtime call failed (message holds its text) */
    FCOO_ENOTBUILT = -4,     /* operation on an (op, mode) that fcoo_build has not built */
    FCOO_ERANGE = -5,        /* a coordinate is >= its dimension, or a size overflows */
    FCOO_EUNSUPPORTED = -6   /* order outside [2, 8], R outside [1, 256], unknown dtype */
};

/* Operation classes (Table I): decide which modes are index / product modes. */
enum fcoo_op {
    FCOO_OP_MTTKRP = 0,      /* index mode = {mode}, product modes = all others        */
    FCOO_OP_TTM = 1          /* index modes = all others, product mode = {mode}        */
};

/* Storage type of dense factor matrices read by the kernels. */
enum fcoo_dtype {
    FCOO_F32 = 0,            /* float32                                                */
    FCOO_BF16 = 1            /* bfloat16 (upper 16 bits of a float32); FP32 accumulate */
};

typedef struct fcoo_tensor fcoo_tensor;   /* opaque; owned by the library */

/* Build options.  A zero field selects the default. */
typedef struct {
    int threadlen;   /* nonzeros per partition: 8, 16, 32 or 64 (default 16).  One sf
                        bit per partition (Sec. IV-B, Table II). */
    int tile_nnz;    /* nonzeros per workgroup tile: a multiple of 256 and of
                        threadlen (default 4096). */
    int host_only;   /* 1: build the host arrays only (no device upload), e.g. to
                        fcoo_export them on a machine without a GPU. */
    int device;      /* 1: sort and encode on the GPU (same arrays, bit for bit);
                        needs the packed sort key within 64 bits, 0 < Z < 2^31,
                        and holds about 32 bytes per nonzero of scratch while it
                        runs.  The per-nonzero arrays then live on the device only
                        (fcoo_export copies them back).  Exclusive with host_only. */
    int xcd_blocks;  /* SpMTTKRP builds: 8 splits the nonzeros into 8 blocks of
                        about Z/8 nonzeros by ranges of the largest product
                        mode's index; block b leads the sort order, runs on
                        XCD b (whose L2 then holds that mode's rows of the
                        block), and writes partial rows summed at the end of
                        each call.  A segment is then a (block, row) pair and
                        fcoo_export's seg holds block * dims[mode] + row.
                        0 or 1: off (default). */
    int xcd_mode;    /* with xcd_blocks: 1 + the product mode whose index
                        ranges define the blocks (FCOO_EINVAL if it is not a
                        product mode of the build); 0: the product mode with
                        the most rows. */
    int lane_cols;   /* bfloat16 factors, SpMTTKRP / SpTTM: columns of a row
                        that one lane reads per gather, 4 (8-byte pieces; the
                        kernel then runs 4 waves per SIMD) or 8 (16-byte
                        pieces, 3 waves per SIMD; always so with R > 64 or R
                        not a multiple of 4, with the fused residual and with
                        SpTTMc).  0: 4 with exactly two product modes and R <=
                        64, else 8.  fcoo_autotune times both. */
    int single_pass; /* 1: finish the segments that cross tile boundaries inside
                        the tile kernel (the paper's adjacent synchronization,
                        Sec. IV-D): each tile publishes its two boundary
                        partials tagged with the launch, and the tile holding
                        a segment's closing head waits (bounded) for its
                        chain's partials and writes the row, so no fix-up pass
                        runs.  Workgroups take tiles in start order from a
                        ticket counter.  Plain layout only (FCOO_EINVAL with
                        xcd_blocks); fcoo_spmttkrp_noalloc keeps the fix-up
                        pass.  0: fix-up pass (default). */
} fcoo_opts;

/* Sizes of one built (op, mode). */
typedef struct {
    int64_t nnz;          /* Z */
    int64_t nseg;         /* segments: non-empty slices (MTTKRP) or fibres (TTM) */
    int64_t npart;        /* partitions P = ceil(Z / threadlen)                   */
    int64_t ntiles;       /* ceil(Z / tile_nnz)                                   */
    int64_t nfix;         /* segments finished by the carry fix-up pass           */
    int64_t nempty;       /* MTTKRP: output rows with no nonzero (written as 0)   */
    int64_t bytes_format; /* bytes of the F-COO arrays (pidx, val, bf, sf)        */
    int64_t bytes_device; /* all device bytes held for this (op, mode)            */
    int32_t threadlen;
    int32_t tile_nnz;
    int32_t order;
    int32_t on_device;    /* 1 if uploaded                                        */
    int32_t xcd_blocks;   /* 1, or the number of XCD blocks (SpMTTKRP)           */
    int32_t block_mode;   /* mode whose index ranges define the blocks, or -1    */
    int32_t lane_cols;    /* fcoo_opts.lane_cols of the build (0: default rule)  */
    int32_t single_pass;  /* 1 if built with fcoo_opts.single_pass              */
    int32_t sp_gave_up;   /* single pass: 1 if a wait for another tile's partial
                             gave up (its result is then wrong); fcoo_info
                             waits for the device to read it                    */
} fcoo_info_t;

/*
 * fcoo_create -- copy a COO tensor into a new handle.
 *   order   number of modes N, 2..8.
 *   dims    host, N dimension sizes, each in [1, 2^31 - 1].
 *   nnz     Z >= 0 (Z = 0 is valid: every result is zero).
 *   idx     host, N pointers to host int32 arrays of Z 0-based coordinates.
 *   vals    host, Z float32 values.  Repeated coordinates are kept as separate
 *           nonzeros and add (COO semantics).
 *   out     receives the handle; release it with fcoo_destroy.
 * Errors: FCOO_EINVAL (null), FCOO_EUNSUPPORTED (order), FCOO_ERANGE (a
 * coordinate outside [0, dims[m]) or a bad dimension), FCOO_ENOMEM.
 */
int fcoo_create(int order, const int64_t *dims, int64_t nnz, const int32_t *const *idx,
                const float *vals, fcoo_tensor **out);

/*
 * fcoo_build -- build the F-COO form of the tensor for (op, mode) on the
 * host and upload it once (Sec. IV-B; the paper prepares F-COO per mode on
 * the host and transfers it once, Sec. IV-D).
 *   The nonzeros are ordered by the index-mode tuple, then the product-mode
 *   tuple (stable; ties keep input order).  Stored per nonzero: the
 *   product-mode indices and the value.  bf: a parity bit per nonzero that
 *   starts at 1 and toggles at each new segment (slice for MTTKRP, fibre for
 *   TTM).  sf: one bit per partition of `threadlen` nonzeros, set iff a
 *   segment starts inside it.  Per segment: its output row (MTTKRP) or its
 *   fibre coordinates (TTM).  Per tile: the ordinal of the segment holding
 *   its first nonzero.
 *   opts may be NULL (defaults).  Rebuilding an (op, mode) replaces it.
 *   Waits for the upload to finish before returning.
 * Errors: FCOO_EINVAL, FCOO_ENOMEM, FCOO_EHIP.
 */
int fcoo_build(fcoo_tensor *t, int mode, int op, const fcoo_opts *opts, void *stream);

/* fcoo_info -- sizes of a built (op, mode).  Errors: FCOO_EINVAL, FCOO_ENOTBUILT. */
int fcoo_info(const fcoo_tensor *t, int mode, int op, fcoo_info_t *info);

/*
 * fcoo_export -- host copies of a built (op, mode)'s arrays (any pointer may
 * be NULL to skip it).  Sizes come from fcoo_info:
 *   pidx      |product modes| pointers to Z int32 each, in ascending mode order
 *   val       Z float32
 *   bf        ceil(Z / 8) bytes, bit s of the stream at byte s>>3, bit s&7
 *   sf        ceil(npart / 32) uint32 words, bit p at word p>>5, bit p&31
 *   seg       MTTKRP: nseg int32 output rows (strictly increasing);
 *             TTM: nseg x (N-1) int32 fibre coordinates, row-major, the
 *             index modes in ascending order (lexicographically increasing)
 *   tile_seg0 ntiles int32: ordinal of the segment holding nonzero t*tile_nnz
 *   perm      Z int32: input position of the nonzero stored at position s
 * Errors: FCOO_EINVAL, FCOO_ENOTBUILT.
 */
int fcoo_export(const fcoo_tensor *t, int mode, int op, int32_t *const *pidx, float *val,
                uint8_t *bf, uint32_t *sf, int32_t *seg, int32_t *tile_seg0, int32_t *perm);

/*
 * fcoo_autotune -- choose the layout of one (op, mode) by timing: each
 * candidate tile_nnz -- for op = MTTKRP each with xcd_blocks 0 and with
 * xcd_blocks 8 split by every product mode (xcd_mode), skipping blocked
 * layouts the build refuses -- is built (on the GPU when the sort key fits 64
 * bits, else on the host; the current threadlen is kept, default 16), and for
 * bfloat16 factors with R <= 64 a multiple of 4 both lane_cols 4 and 8 are
 * tried on it; each is run once to warm up, then `reps` times between two
 * HIP events on `stream`, and the fastest is left in place (the paper tunes
 * its launch shape per dataset, Sec. V, Table V).
 *   factors  as fcoo_spmttkrp (op = MTTKRP) or factors[mode] = U (op = TTM);
 *            device data of `dtype`, R columns.
 *   tiles    host array of `ncand` candidate tile sizes (each a multiple of
 *            256 and of threadlen), or NULL for {1024, 2048, 4096, 8192, 16384}.
 *   reps     timed repetitions per candidate (< 1: 3).
 *   best     host, out (may be NULL): the options of the kept build.
 *   best_ms  host, out (may be NULL): its mean time per operation (ms).
 * Allocates a temporary output (rows x R float32) and two events; waits on
 * `stream` after each candidate.  On error the (op, mode) may be left built
 * with any candidate or unbuilt.
 * Errors: as fcoo_build and fcoo_spmttkrp / fcoo_spttm.
 */
int fcoo_autotune(fcoo_tensor *t, int mode, int op, const void *const *factors, int dtype, int R,
                  const int *tiles, int ncand, int reps, fcoo_opts *best, float *best_ms, void *stream);

/*
 * fcoo_spmttkrp -- M = X_(mode) (Khatri-Rao product of the other factors),
 * computed over the nonzeros in one shot (Eq. 5 / Eq. 6):
 *   M[i, r] = sum over nonzeros e with i_mode(e) = i of
 *             val(e) * prod_{m != mode} A_m[i_m(e), r].
 *   factors  host array of N device pointers; factors[m] is dims[m] x R of
 *            `dtype`; factors[mode] is not read (may be NULL).
 *   M        device, dims[mode] x R float32, written fully (rows of empty
 *            slices are written as 0).  Must not alias a factor.
 * Requires fcoo_build(mode, FCOO_OP_MTTKRP).  Deterministic: repeated calls
 * give bitwise-identical results (no atomics).
 * Errors: FCOO_EINVAL, FCOO_ENOTBUILT, FCOO_EUNSUPPORTED, FCOO_EHIP, FCOO_ENOMEM.
 */
int fcoo_spmttkrp(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R,
                  float *M, void *stream);

/* Bytes of the fixed device scratch array behind fcoo_spmttkrp_noalloc. */
#define FCOO_NOALLOC_SCRATCH_BYTES (16ll << 20)

/*
 * fcoo_spmttkrp_noalloc -- fcoo_spmttkrp for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and result (bitwise equal
 * to fcoo_spmttkrp on the same build and inputs), but the call allocates
 * nothing: its scratch -- the tile carries, 2 x ntiles x R floats (rounded up
 * to 256 bytes), plus xcd_blocks x dims[mode] x R floats of partial rows for
 * an XCD-blocked build -- lives in one library-owned device array of
 * FCOO_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * (which looks its address up with the GPU current) until the process ends.
 * The caller still owns and passes factors and M.  Every scratch element the
 * call reads it first writes, so nothing needs clearing between calls.
 * All calls on one GPU share that array: calls that overlap on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the
 * caller.
 * Errors: as fcoo_spmttkrp; FCOO_ERANGE when the scratch needed exceeds
 * FCOO_NOALLOC_SCRATCH_BYTES (nothing is launched).
 */
int fcoo_spmttkrp_noalloc(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R,
                          float *M, void *stream);

/*
 * fcoo_spttm -- Y = X x_mode U (Eq. 3), semi-sparse result:
 *   Y[g, :] = sum over nonzeros e of fibre g of val(e) * U[i_mode(e), :]
 *   where fibre g is the g-th distinct tuple of the other modes' indices in
 *   lexicographic order (fcoo_export's `seg`).  Structurally present fibres
 *   are all listed, also when their sum cancels to zero.
 *   U   device, dims[mode] x R of `dtype`.
 *   Y   device, nseg x R float32, written fully.
 * Requires fcoo_build(mode, FCOO_OP_TTM).
 * Errors: as fcoo_spmttkrp.
 */
int fcoo_spttm(fcoo_tensor *t, int mode, const void *U, int dtype, int R, float *Y, void *stream);

/*
 * fcoo_spttmc -- tensor times a matrix chain on every mode but `mode` (Eq. 4,
 * Table I third row; the kernel of Tucker / HOOI), Y = Y_(mode):
 *   Y[i, c] = sum over nonzeros e with i_mode(e) = i of
 *             val(e) * U_{m1}[i_m1(e), p_1] * U_{m2}[i_m2(e), p_2] * ...
 *   where m1 < m2 < ... are the other modes and column c is the Kronecker
 *   (Eq. 1) position of (p_1, p_2, ...): the last mode's column runs fastest,
 *   c = (..(p_1 ranks[m2] + p_2) ranks[m3] + ..).
 *   factors  host array of N device pointers; factors[m] is dims[m] x
 *            ranks[m] of `dtype`; factors[mode] is not read (may be NULL).
 *   ranks    host array of N ints, each in [1, 256]; ranks[mode] is ignored;
 *            the width W = prod_{m != mode} ranks[m] must not exceed 16384.
 *   Y        device, dims[mode] x W float32, written fully (rows of empty
 *            slices are written as 0).
 * Uses the SpMTTKRP encoding of the mode (the index and product modes are the
 * same): requires fcoo_build(mode, FCOO_OP_MTTKRP).  Deterministic.
 * Errors: as fcoo_spmttkrp.
 */
int fcoo_spttmc(fcoo_tensor *t, int mode, const void *const *factors, int dtype, const int *ranks,
                float *Y, void *stream);

/*
 * fcoo_spmttkrp_values -- fcoo_spmttkrp with the tensor's values replaced
 * by `g` (device, Z float32 in the caller's input order of fcoo_create):
 *   M[i, r] = sum_{e : i_mode(e) = i} g[e] prod_{m != mode} A_m[i_m(e), r].
 * This is the adjoint of the CP model at the nonzeros (its gradient with
 * respect to A_mode when g = dL/dxhat).
 * Requires fcoo_build(mode, FCOO_OP_MTTKRP).  Errors: as fcoo_spmttkrp.
 */
int fcoo_spmttkrp_values(fcoo_tensor *t, int mode, const float *g, const void *const *factors,
                         int dtype, int R, float *M, void *stream);

/*
 * fcoo_model_at_nnz -- CP model at the nonzeros:
 *   xhat[e] = sum_r prod_m A_m[i_m(e), r], e in the caller's input order.
 *   xhat  device, Z float32.  The first call uploads the coordinate list.
 * Errors: FCOO_EINVAL, FCOO_EUNSUPPORTED, FCOO_EHIP, FCOO_ENOMEM.
 */
int fcoo_model_at_nnz(fcoo_tensor *t, const void *const *factors, int dtype, int R, float *xhat,
                      void *stream);

/*
 * fcoo_resid_spmttkrp -- fused gradient of the mean-squared error of the CP
 * model at the nonzeros, L = (1 / 2Z) sum_e (xhat_e - x_e)^2, for one mode:
 *   G[i, r] = (1/Z) sum_{e : i_mode(e) = i} (xhat_e - x_e) prod_{m != mode} A_m[i_m(e), r]
 *   recomputing xhat_e from the factor rows (nothing per nonzero is stored).
 *   G     device, dims[mode] x R float32, written fully.
 *   loss  device double* or NULL; if given, receives L (computed in the same
 *         pass, reduced deterministically).
 * Rank limit: one workgroup lane group holds a whole factor row (the residual
 * needs the full dot product), so R <= 64 for float32 factors, and for
 * bfloat16 R <= 128 when R is a multiple of 8, else R <= 64.  A larger R
 * returns FCOO_EUNSUPPORTED; fcoo_model_at_nnz followed by
 * fcoo_spmttkrp_values computes the same gradient at any R in [1, 256].
 * Requires fcoo_build(mode, FCOO_OP_MTTKRP).  Errors: as fcoo_spmttkrp.
 */
int fcoo_resid_spmttkrp(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R,
                        float *G, double *loss, void *stream);

/*
 * fcoo_cp_als_iter -- one sweep of CP-ALS (Algorithm 1, N modes, Gauss-Seidel):
 * for n = 0..N-1: M = SpMTTKRP_n; V = Hadamard product of the Grams G_m,
 * m != n (float64); A_n = M V^-1 (float64 inverse by elimination whose
 * pivots are those of the Cholesky factorisation; symmetric-eigen
 * pseudo-inverse when a pivot is <= 0 or below 1e-13 max diag V, R <= 64);
 * lambda = column 2-norms
 * of A_n; A_n columns divided by lambda (zero columns left zero); A_n stored
 * as `dtype` (round to nearest even); G_n = A_n^T A_n of the stored values.
 * Then fit = 1 - sqrt(max(0, |X|^2 + |Xhat|^2 - 2 <X, Xhat>)) / |X|.
 *   factors  host array of N device pointers, in/out, dims[m] x R of `dtype`.
 *   lambda   device, R float64 (out: the norms of the last mode).
 *   grams    device, N x R x R float64, in/out: G_m = A_m^T A_m.  Set
 *            `grams_valid` = 0 to have them computed from the factors first.
 *   fit      host double* (out); the call waits for it.
 *   used_pinv host int* or NULL (out): bit n set if mode n used the pseudo-inverse.
 * Requires fcoo_build(n, FCOO_OP_MTTKRP) for every mode n.  The R x R solve
 * of each mode runs on a second stream owned by the handle, beside that
 * mode's SpMTTKRP (it needs only the other modes' Grams); events order it
 * after the earlier work on `stream` and before the row solve, so for the
 * caller all the work is ordered on `stream`.
 * Errors: FCOO_EINVAL, FCOO_ENOTBUILT, FCOO_EUNSUPPORTED, FCOO_EHIP, FCOO_ENOMEM.
 */
int fcoo_cp_als_iter(fcoo_tensor *t, void *const *factors, int dtype, int R, double *lambda,
                     double *grams, int grams_valid, double *fit, int *used_pinv, void *stream);

/*
 * fcoo_gram -- G = A^T A (float64 R x R, device) of a dims[mode] x R factor
 * (device, `dtype`): matrix-core (MFMA) products per row block, float64 sum
 * across blocks.  Errors: FCOO_EINVAL, FCOO_EUNSUPPORTED, FCOO_EHIP, FCOO_ENOMEM.
 */
int fcoo_gram(fcoo_tensor *t, int mode, const void *A, int dtype, int R, double *G, void *stream);

/*
 * fcoo_device_copy -- copy `bytes` of device memory from src to dst with the
 * library's own plain copy kernel (16-byte streaming loads and stores): the device-copy
 * bandwidth the sparse kernels are measured against, and a kernel of known
 * traffic for calibrating hardware byte counters.  Not part of the method.
 *   src, dst  device, 16-byte aligned, not overlapping (caller-owned).
 *   bytes     a non-negative multiple of 16.
 * Errors: FCOO_EINVAL (null pointer, misalignment, size), FCOO_EHIP.
 */
int fcoo_device_copy(const void *src, void *dst, int64_t bytes, void *stream);

/*
 * fcoo_set_tile_events -- instrumentation for callers that time the tile
 * kernel alone.  While `before` and `after` (hipEvent_t values passed as
 * void*, created and owned by the caller) are non-NULL, every SpMTTKRP /
 * SpTTM / value-replaced / residual call on this handle records `before` on
 * its stream immediately before its tile kernel and `after` immediately
 * after it.  Passing NULL, NULL switches recording off.  Changes no result.
 * Errors: FCOO_EINVAL (null handle, or exactly one event NULL).
 */
int fcoo_set_tile_events(fcoo_tensor *t, void *before, void *after);

/* fcoo_destroy -- free the handle and every device buffer it owns (NULL is ignored). */
void fcoo_destroy(fcoo_tensor *t);

/* fcoo_last_error -- message of the calling thread's last failed call ("" if none). */
const char *fcoo_last_error(void);

/* fcoo_version -- ABI version (major * 100 + minor). */
int fcoo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FCOO_H */

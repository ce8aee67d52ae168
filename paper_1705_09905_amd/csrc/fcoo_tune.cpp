// Per-tensor tuning of one (operation, mode): the paper tunes its launch
// shape per dataset (Sec. V, Table V); here each candidate layout -- tile
// size; for SpMTTKRP plain or XCD blocks split by one of the product modes;
// for bfloat16 rows the lane chunk, which also sets the waves per SIMD -- is
// built, its operation is timed with HIP events on the caller's stream, and
// the fastest is kept.  Host code over the public entry points.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <vector>

#include "fcoo_internal.h"

using namespace fcoo;

namespace {

int run_op(fcoo_tensor *t, int mode, int op, const void *const *factors, int dtype, int R, float *out,
           void *stream)
{
    if (op == FCOO_OP_MTTKRP) return fcoo_spmttkrp(t, mode, factors, dtype, R, out, stream);
    return fcoo_spttm(t, mode, factors[mode], dtype, R, out, stream);
}

}  // namespace

extern "C" int fcoo_autotune(fcoo_tensor *t, int mode, int op, const void *const *factors, int dtype, int R,
                             const int *tiles, int ncand, int reps, fcoo_opts *best, float *best_ms,
                             void *stream)
{
    clear_error();
    if (!t || !factors) return fail(FCOO_EINVAL, "null argument");
    if (mode < 0 || mode >= t->order) return fail(FCOO_EINVAL, "mode %d out of range", mode);
    if (op != FCOO_OP_MTTKRP && op != FCOO_OP_TTM) return fail(FCOO_EINVAL, "unknown op %d", op);
    static const int kDefault[] = {1024, 2048, 4096, 8192, 16384};
    if (!tiles) {
        tiles = kDefault;
        ncand = (int)(sizeof(kDefault) / sizeof(kDefault[0]));
    }
    if (ncand < 1) return fail(FCOO_EINVAL, "no candidate tile sizes");
    if (reps < 1) reps = 3;
    hipStream_t s = (hipStream_t)stream;
    int threadlen = 16;
    fcoo_info_t inf{};
    if (fcoo_info(t, mode, op, &inf) == FCOO_OK) threadlen = inf.threadlen;

    // candidates: each tile size; for SpMTTKRP the plain layout and the XCD
    // blocks split by each product mode; for bfloat16 rows both lane chunks
    // (4 columns at 4 waves per SIMD, 8 columns at 3).  Builds run on the GPU
    // when the sort key allows it (same arrays).
    struct Cand { int tile, xcd, xmode; };
    std::vector<Cand> cands;
    for (int c = 0; c < ncand; ++c) {
        cands.push_back({tiles[c], 0, 0});
        if (op == FCOO_OP_MTTKRP && t->nnz > 0)
            for (int m = 0; m < t->order; ++m)
                if (m != mode) cands.push_back({tiles[c], kXcds, m + 1});
    }
    const int nprod = op == FCOO_OP_MTTKRP ? t->order - 1 : 1;
    std::vector<int> lanes = {0};
    if (dtype == FCOO_BF16 && R % 4 == 0 && R <= 64 && nprod <= 3) lanes = {4, 8};
    auto build = [&](const Cand &c) -> int {
        fcoo_opts o{threadlen, c.tile, 0, t->nnz > 0 ? 1 : 0, c.xcd, c.xmode, 0};
        int r = fcoo_build(t, mode, op, &o, stream);
        if (r == FCOO_EUNSUPPORTED && o.device) {   // sort key over 64 bits: host build
            o.device = 0;
            r = fcoo_build(t, mode, op, &o, stream);
        }
        return r;
    };
    int rc = build(cands[0]);
    if (rc) return rc;
    if ((rc = fcoo_info(t, mode, op, &inf))) return rc;
    const int64_t rows = op == FCOO_OP_MTTKRP ? t->dims[mode] : inf.nseg;
    float *out = nullptr;
    if (rows > 0 && hipMalloc((void **)&out, (size_t)rows * R * sizeof(float)) != hipSuccess)
        return fail(FCOO_ENOMEM, "autotune output (%lld x %d floats)", (long long)rows, R);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(out);
        return fail(FCOO_EHIP, "hipEventCreate");
    }
    float bms = FLT_MAX;
    size_t bi = 0, cur = 0;                          // best and currently built candidate
    int blane = 0;
    for (size_t c = 0; c < cands.size() && rc == FCOO_OK; ++c) {
        if (c > 0) {
            rc = build(cands[c]);
            cur = c;
            if (rc == FCOO_EUNSUPPORTED && cands[c].xcd) {   // e.g. 8 x rows past the int32 range
                rc = FCOO_OK;
                continue;
            }
            if (rc) break;
        }
        for (int lc : lanes) {
            t->b[op][mode].lane_cols = lc;           // a launch choice: no rebuild
            if ((rc = run_op(t, mode, op, factors, dtype, R, out, stream))) break;   // warm-up
            if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(FCOO_EHIP, "hipEventRecord"); break; }
            for (int r = 0; r < reps && rc == FCOO_OK; ++r) rc = run_op(t, mode, op, factors, dtype, R, out, stream);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(FCOO_EHIP, "timing");
                break;
            }
            ms /= (float)reps;
            if (ms < bms) {
                bms = ms;
                bi = c;
                blane = lc;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc) return rc;
    if (bi != cur && (rc = build(cands[bi]))) return rc;
    t->b[op][mode].lane_cols = blane;
    fcoo_opts o{threadlen, cands[bi].tile, 0, 0, cands[bi].xcd, cands[bi].xmode, blane};
    if (best) *best = o;
    if (best_ms) *best_ms = bms;
    return FCOO_OK;
}

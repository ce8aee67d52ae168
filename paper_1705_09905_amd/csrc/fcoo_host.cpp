// Host side of the F-COO library: the handle, the per-(op, mode) F-COO
// build (mode sort, bf / sf flags, per-segment and per-tile indexing, the
// carry fix-up list), the one-time upload, export, and argument checking of
// the C ABI.  F-COO itself is defined in Sec. IV-B; the build runs on the
// host once per mode and is uploaded once (Sec. IV-D, "complete tensor-based
// algorithms").
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>

#include "fcoo_internal.h"

namespace fcoo {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(FCOO_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(FCOO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// small parallel helpers (std::thread; the host build is a one-time cost)
// ---------------------------------------------------------------------------
static int host_threads()
{
    const char *e = getenv("FCOO_HOST_THREADS");
    int n = e ? atoi(e) : (int)std::thread::hardware_concurrency();
    if (n < 1) n = 1;
    if (n > 32) n = 32;
    return n;
}

template <class F>
static void parallel_chunks(int64_t n, int T, F fn)
{
    if (T <= 1 || n < 65536) {
        fn(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t)
        th.emplace_back([=]() { fn(t, n * t / T, n * (t + 1) / T); });
    for (auto &x : th) x.join();
}

// Stable LSD radix sort of (key, id) pairs, 11-bit digits, `bits` significant
// key bits.  Ties keep their incoming order.
static void radix_sort(std::vector<uint64_t> &k, std::vector<uint32_t> &v, int bits, int T)
{
    const int64_t n = (int64_t)k.size();
    if (n < 2 || bits <= 0) return;
    constexpr int DB = 11, NB = 1 << DB;
    std::vector<uint64_t> k2(n);
    std::vector<uint32_t> v2(n);
    if (n < 65536) T = 1;
    std::vector<int64_t> hist((size_t)T * NB);
    for (int shift = 0; shift < bits; shift += DB) {
        std::fill(hist.begin(), hist.end(), 0);
        parallel_chunks(n, T, [&](int t, int64_t b, int64_t e) {
            int64_t *h = hist.data() + (size_t)t * NB;
            for (int64_t i = b; i < e; ++i) h[(k[i] >> shift) & (NB - 1)]++;
        });
        bool trivial = false;
        for (int d = 0; d < NB && !trivial; ++d) {
            int64_t c = 0;
            for (int t = 0; t < T; ++t) c += hist[(size_t)t * NB + d];
            if (c == n) trivial = true;
            else if (c) break;
        }
        if (trivial) continue;
        int64_t run = 0;
        for (int d = 0; d < NB; ++d)
            for (int t = 0; t < T; ++t) {
                int64_t c = hist[(size_t)t * NB + d];
                hist[(size_t)t * NB + d] = run;
                run += c;
            }
        parallel_chunks(n, T, [&](int t, int64_t b, int64_t e) {
            int64_t *h = hist.data() + (size_t)t * NB;
            for (int64_t i = b; i < e; ++i) {
                int64_t p = h[(k[i] >> shift) & (NB - 1)]++;
                k2[p] = k[i];
                v2[p] = v[i];
            }
        });
        k.swap(k2);
        v.swap(v2);
    }
}

static int bit_width(int64_t d)  // bits to hold 0..d-1
{
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < d) ++b;
    return b;
}

int64_t Built::format_bytes() const
{
    return 4 * nnz * (int64_t)pmodes.size() + 4 * nnz + (nnz + 7) / 8 + 4 * ((npart + 31) / 32);
}

void Built::free_device()
{
    if (d_bpart) (void)hipFree(d_bpart);
    d_bpart = nullptr;
    bpart_cap = 0;
    for (auto &p : d_pidx) { if (p) (void)hipFree(p); p = nullptr; }
    void *ptrs[] = {d_val, d_bf, d_sf, d_seg_row, d_tile_seg0, d_perm, d_fix, d_empty, d_carry,
                    d_gperm, d_partial, d_sp_from, d_sp_words, d_sp_ticket, d_sp_err};
    for (void *p : ptrs) if (p) (void)hipFree(p);
    d_val = nullptr; d_bf = nullptr; d_sf = nullptr; d_seg_row = nullptr; d_tile_seg0 = nullptr;
    d_perm = nullptr; d_fix = nullptr; d_empty = nullptr; d_carry = nullptr; d_gperm = nullptr;
    d_partial = nullptr; d_sp_from = nullptr; d_sp_words = nullptr; d_sp_ticket = nullptr; d_sp_err = nullptr;
    carry_cap = 0; partial_cap = 0; device_bytes = 0; sp_words_cap = 0; sp_tickets = 0; sp_epoch = 0;
    on_device = false;
}

void Workspace::free_all()
{
    if (M) (void)hipFree(M);
    if (dbl) (void)hipFree(dbl);
    if (flags) (void)hipFree(flags);
    if (host_pinned) (void)hipHostFree(host_pinned);
    M = nullptr; dbl = nullptr; flags = nullptr; host_pinned = nullptr;
    M_cap = dbl_cap = 0;
}

// Grow a device scratch buffer.  The old buffer may still be read by work
// queued on `s`, so the stream is drained before it is released.
int ensure_device_floats(float **p, int64_t *cap, int64_t need, hipStream_t s)
{
    if (need <= *cap) return FCOO_OK;
    if (*p) {
        FCOO_HIP(hipStreamSynchronize(s));
        FCOO_HIP(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    FCOO_HIP(hipMalloc((void **)p, (size_t)need * sizeof(float)));
    *cap = need;
    return FCOO_OK;
}

int ensure_device_doubles(double **p, int64_t *cap, int64_t need, hipStream_t s)
{
    if (need <= *cap) return FCOO_OK;
    if (*p) {
        FCOO_HIP(hipStreamSynchronize(s));
        FCOO_HIP(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    FCOO_HIP(hipMalloc((void **)p, (size_t)need * sizeof(double)));
    *cap = need;
    return FCOO_OK;
}

template <class T>
static int upload(T **dst, const T *src, int64_t n, int64_t pad_elems, hipStream_t s, int64_t *acct)
{
    const size_t bytes = (size_t)(n + pad_elems) * sizeof(T);
    FCOO_HIP(hipMalloc((void **)dst, bytes ? bytes : sizeof(T)));
    if (pad_elems) FCOO_HIP(hipMemsetAsync(*dst, 0, bytes, s));
    if (n) FCOO_HIP(hipMemcpyAsync(*dst, src, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
    *acct += (int64_t)bytes;
    return FCOO_OK;
}

int upload_i32(int32_t **dst, const std::vector<int32_t> &v, int64_t pad, hipStream_t s, int64_t *acct)
{
    return upload(dst, v.data(), (int64_t)v.size(), pad, s, acct);
}

int upload_coo(fcoo_tensor *t, hipStream_t s)
{
    if (t->coo_on_device) return FCOO_OK;
    int64_t acct = 0;
    for (int m = 0; m < t->order; ++m) {
        int rc = upload(&t->d_coo[m], t->idx[m].data(), t->nnz, 0, s, &acct);
        if (rc) return rc;
    }
    int rc = upload(&t->d_coo_val, t->vals.data(), t->nnz, 0, s, &acct);
    if (rc) return rc;
    FCOO_HIP(hipStreamSynchronize(s));
    t->coo_on_device = true;
    return FCOO_OK;
}

int check_factors(const fcoo_tensor *t, int skip_mode, const void *const *factors, int dtype, int R)
{
    if (!factors) return fail(FCOO_EINVAL, "factors is NULL");
    if (dtype != FCOO_F32 && dtype != FCOO_BF16) return fail(FCOO_EUNSUPPORTED, "unknown dtype %d", dtype);
    if (R < 1 || R > kMaxR) return fail(FCOO_EUNSUPPORTED, "R = %d outside [1, %d]", R, kMaxR);
    for (int m = 0; m < t->order; ++m)
        if (m != skip_mode && !factors[m]) return fail(FCOO_EINVAL, "factors[%d] is NULL", m);
    return FCOO_OK;
}

// XCD blocks: the product mode with the most rows is split into nblk index
// ranges holding about Z / nblk nonzeros each; block b's nonzeros lead the
// sort order as a group, and its tiles are those that start inside it.
int setup_blocks(const fcoo_tensor *t, Built &b, int nblk, int xmode)
{
    b.nblk = 1;
    b.bmode = -1;
    b.blk_of.clear();
    b.blk_ts.clear();
    b.rows = b.op == FCOO_OP_MTTKRP ? t->dims[b.mode] : 0;
    if (nblk <= 1) return FCOO_OK;
    if (nblk != kXcds) return fail(FCOO_EINVAL, "xcd_blocks must be 0, 1 or %d (got %d)", kXcds, nblk);
    if (b.op != FCOO_OP_MTTKRP) return fail(FCOO_EINVAL, "xcd_blocks applies to SpMTTKRP builds");
    if ((int64_t)nblk * t->dims[b.mode] > (int64_t)0x7fffffff)
        return fail(FCOO_EUNSUPPORTED, "xcd_blocks: %d x dims[mode] exceeds the int32 row range", nblk);
    int bm = -1;
    if (xmode >= 0) {
        for (int m : b.pmodes) if (m == xmode) bm = m;
        if (bm < 0) return fail(FCOO_EINVAL, "xcd_mode: mode %d is not a product mode of this build", xmode);
    } else {
        bm = b.pmodes[0];
        for (int m : b.pmodes) if (t->dims[m] > t->dims[bm]) bm = m;
    }
    const int64_t D = t->dims[bm], Z = t->nnz;
    std::vector<int64_t> cnt(D, 0);
    for (int64_t e = 0; e < Z; ++e) cnt[t->idx[bm][e]]++;
    b.blk_of.resize(D);
    std::vector<int64_t> zs(nblk + 1, 0);
    int64_t before = 0;
    for (int64_t i = 0; i < D; ++i) {
        int blk = Z > 0 ? (int)((before * nblk) / Z) : 0;
        if (blk >= nblk) blk = nblk - 1;
        b.blk_of[i] = blk;
        zs[blk + 1] += cnt[i];
        before += cnt[i];
    }
    for (int k = 0; k < nblk; ++k) zs[k + 1] += zs[k];
    const int64_t T = b.tile_nnz, ntiles = (Z + T - 1) / T;
    b.blk_ts.assign(nblk + 1, 0);
    for (int k = 1; k < nblk; ++k) {
        int64_t ts = zs[k] / T;
        if (ts > ntiles) ts = ntiles;
        b.blk_ts[k] = ts < b.blk_ts[k - 1] ? b.blk_ts[k - 1] : ts;
    }
    b.blk_ts[nblk] = ntiles;
    b.nblk = nblk;
    b.bmode = bm;
    return FCOO_OK;
}

int setup_single_pass(Built &b, hipStream_t s)
{
    if (b.nblk > 1) return fail(FCOO_EINVAL, "single_pass needs the plain layout (no xcd_blocks)");
    if (b.ntiles > (int64_t)0x7fffffff) return fail(FCOO_EUNSUPPORTED, "single_pass: too many tiles");
    std::vector<int32_t> from(b.ntiles + 1, -1);
    b.sp_tail_from = -1;
    for (int64_t e = 0; e < b.nfix(); ++e) {
        const int32_t tb = b.fix[3 * e], ta = b.fix[3 * e + 1];
        if (tb < b.ntiles) from[tb] = ta;
        else b.sp_tail_from = ta;
    }
    int64_t acct = 0;
    int rc = upload_i32(&b.d_sp_from, from, 0, s, &acct);
    if (rc) return rc;
    FCOO_HIP(hipMalloc((void **)&b.d_sp_ticket, sizeof(unsigned long long)));
    FCOO_HIP(hipMalloc((void **)&b.d_sp_err, sizeof(int)));
    FCOO_HIP(hipMemsetAsync(b.d_sp_ticket, 0, sizeof(unsigned long long), s));
    FCOO_HIP(hipMemsetAsync(b.d_sp_err, 0, sizeof(int), s));
    FCOO_HIP(hipStreamSynchronize(s));
    b.device_bytes += acct + (int64_t)sizeof(unsigned long long) + (int64_t)sizeof(int);
    b.sp_tickets = 0;
    b.sp_epoch = 0;
    b.sp = true;
    return FCOO_OK;
}

int prep_single_pass(Built *b, TileProblem &p, hipStream_t s)
{
    if (!b->sp || b->nnz == 0) return FCOO_OK;
    const int64_t need = 2 * b->ntiles * (int64_t)p.R;
    if (need > b->sp_words_cap) {
        // fresh words hold tag 0, which no launch uses
        if (b->d_sp_words) {
            FCOO_HIP(hipStreamSynchronize(s));
            FCOO_HIP(hipFree(b->d_sp_words));
            b->d_sp_words = nullptr;
            b->sp_words_cap = 0;
        }
        FCOO_HIP(hipMalloc((void **)&b->d_sp_words, (size_t)need * sizeof(uint64_t)));
        FCOO_HIP(hipMemsetAsync(b->d_sp_words, 0, (size_t)need * sizeof(uint64_t), s));
        b->sp_words_cap = need;
    }
    if (++b->sp_epoch == 0) b->sp_epoch = 1;
    p.sp_words = b->d_sp_words;
    p.sp_epoch = b->sp_epoch;
    return FCOO_OK;
}

int64_t Built::max_block_tiles() const
{
    int64_t m = 0;
    for (int k = 0; k < nblk; ++k) m = blk_ts[k + 1] - blk_ts[k] > m ? blk_ts[k + 1] - blk_ts[k] : m;
    return m;
}

// ---------------------------------------------------------------------------
// the F-COO build for one (op, mode)
// ---------------------------------------------------------------------------
static int build_host(fcoo_tensor *t, Built &b, int mode, int op, int threadlen, int tile_nnz, int nblk,
                      int xmode)
{
    const int N = t->order;
    const int64_t Z = t->nnz;
    const int T = host_threads();
    b = Built();
    b.op = op; b.mode = mode; b.threadlen = threadlen; b.tile_nnz = tile_nnz; b.nnz = Z;
    for (int m = 0; m < N; ++m) {
        if (m == mode) continue;
        if (op == FCOO_OP_MTTKRP) b.pmodes.push_back(m); else b.imodes.push_back(m);
    }
    if (op == FCOO_OP_MTTKRP) b.imodes.insert(b.imodes.begin(), mode); else b.pmodes.push_back(mode);
    int rc0 = setup_blocks(t, b, nblk, xmode);
    if (rc0) return rc0;
    const bool blocked = b.nblk > 1;
    const int bbits = blocked ? bit_width(b.nblk) : 0;

    // 1. stable lexicographic order of (block, index-mode tuple, product-mode tuple)
    std::vector<int> order_modes(b.imodes);
    order_modes.insert(order_modes.end(), b.pmodes.begin(), b.pmodes.end());
    int total_bits = bbits, pbits = 0;
    for (int m : b.imodes) total_bits += bit_width(t->dims[m]);
    for (int m : b.pmodes) { int w = bit_width(t->dims[m]); total_bits += w; pbits += w; }
    std::vector<uint32_t> perm(Z);
    std::vector<uint64_t> key;
    const bool packed = total_bits <= 64;
    if (packed) {
        key.resize(Z);
        parallel_chunks(Z, T, [&](int, int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e) {
                uint64_t k = blocked ? (uint64_t)b.blk_of[t->idx[b.bmode][e]] : 0;
                for (int m : order_modes) k = (bit_width(t->dims[m]) ? (k << bit_width(t->dims[m])) : k) | (uint64_t)t->idx[m][e];
                key[e] = k;
                perm[e] = (uint32_t)e;
            }
        });
        radix_sort(key, perm, total_bits, T);
    } else {
        for (int64_t e = 0; e < Z; ++e) perm[e] = (uint32_t)e;
        std::stable_sort(perm.begin(), perm.end(), [&](uint32_t x, uint32_t y) {
            if (blocked) {
                const int bx = b.blk_of[t->idx[b.bmode][x]], by = b.blk_of[t->idx[b.bmode][y]];
                if (bx != by) return bx < by;
            }
            for (int m : order_modes) {
                int32_t a = t->idx[m][x], c = t->idx[m][y];
                if (a != c) return a < c;
            }
            return false;
        });
    }

    // 2. per-nonzero arrays in sorted order, and segment heads
    b.perm.resize(Z);
    b.val.resize(Z);
    b.pidx.assign(b.pmodes.size(), std::vector<int32_t>(Z));
    std::vector<uint8_t> head(Z);
    parallel_chunks(Z, T, [&](int, int64_t lo, int64_t hi) {
        for (int64_t s = lo; s < hi; ++s) {
            const uint32_t e = perm[s];
            b.perm[s] = (int32_t)e;
            b.val[s] = t->vals[e];
            for (size_t q = 0; q < b.pmodes.size(); ++q) b.pidx[q][s] = t->idx[b.pmodes[q]][e];
            bool h = (s == 0);
            if (!h) {
                if (packed) {
                    h = pbits < 64 && (key[s] >> pbits) != (key[s - 1] >> pbits);
                } else {
                    if (blocked) h = b.blk_of[t->idx[b.bmode][e]] != b.blk_of[t->idx[b.bmode][perm[s - 1]]];
                    for (int m : b.imodes)
                        if (!h && t->idx[m][e] != t->idx[m][perm[s - 1]]) { h = true; break; }
                }
            }
            head[s] = h;
        }
    });
    key.clear(); key.shrink_to_fit();

    // 3. bf (parity toggled at each head, starting at 1), sf, segments, tiles
    const int64_t P = (Z + threadlen - 1) / threadlen;
    const int64_t ntiles = (Z + tile_nnz - 1) / tile_nnz;
    b.npart = P; b.ntiles = ntiles;
    b.bf.assign((Z + 7) / 8, 0);
    b.sf.assign((P + 31) / 32, 0);
    b.tile_seg0.resize(ntiles);
    std::vector<int64_t> seg_start;  // position of each head
    std::vector<int64_t> heads_before_tile(ntiles + 1, 0);
    std::vector<uint8_t> tile_has_head(ntiles, 0);
    int64_t cnt = 0;
    for (int64_t s = 0; s < Z; ++s) {
        if (s % tile_nnz == 0) heads_before_tile[s / tile_nnz] = cnt;
        if (head[s]) {
            ++cnt;
            seg_start.push_back(s);
            b.sf[(s / threadlen) >> 5] |= 1u << ((s / threadlen) & 31);
            tile_has_head[s / tile_nnz] = 1;
        }
        if (cnt & 1) b.bf[s >> 3] |= (uint8_t)(1u << (s & 7));
        if (s % tile_nnz == 0) b.tile_seg0[s / tile_nnz] = (int32_t)(cnt - 1);
    }
    heads_before_tile[ntiles] = cnt;
    b.nseg = cnt;
    const int nim = (int)b.imodes.size();
    b.seg.resize((size_t)cnt * nim);
    for (int64_t g = 0; g < cnt; ++g) {
        const uint32_t e = perm[seg_start[g]];
        for (int q = 0; q < nim; ++q) b.seg[(size_t)g * nim + q] = t->idx[b.imodes[q]][e];
        if (blocked) b.seg[g] += b.blk_of[t->idx[b.bmode][e]] * (int32_t)t->dims[mode];
    }

    // 4. carry fix-up list: a segment that is still open at the end of a tile
    //    is finished by the first head of a later tile (or by the end of the
    //    tensor).  Entry (b, a, row): tiles a+1 .. b-1 hold no head, tile a
    //    holds the segment's start.  The segment closed at tile b's first
    //    head is the last one that starts before tile b.
    auto out_row = [&](int64_t g) -> int32_t {
        return op == FCOO_OP_MTTKRP ? b.seg[(size_t)g] : (int32_t)g;
    };
    int64_t last = -1;
    for (int64_t tb = 0; tb < ntiles; ++tb) {
        if (!tile_has_head[tb]) continue;
        if (tb >= 1) {
            const int64_t g = heads_before_tile[tb] - 1;
            b.fix.push_back((int32_t)tb);
            b.fix.push_back((int32_t)last);
            b.fix.push_back(out_row(g));
        }
        last = tb;
    }
    if (Z > 0) {
        b.fix.push_back((int32_t)ntiles);
        b.fix.push_back((int32_t)last);
        b.fix.push_back(out_row(cnt - 1));
    }

    // 5. output rows of MTTKRP that no nonzero touches (with XCD blocks: rows
    //    of the nblk x dims[mode] partial output)
    if (op == FCOO_OP_MTTKRP) {
        const int64_t rows = (int64_t)b.nblk * t->dims[mode];
        std::vector<uint8_t> present(rows, 0);
        for (int64_t g = 0; g < cnt; ++g) present[b.seg[g]] = 1;
        for (int64_t i = 0; i < rows; ++i)
            if (!present[i]) b.empty_rows.push_back((int32_t)i);
    }
    b.built = true;
    return FCOO_OK;
}

void finish_tiles(const fcoo_tensor *t, Built &b, int mode, int op, const std::vector<int64_t> &hb)
{
    const int64_t ntiles = b.ntiles, cnt = b.nseg;
    auto out_row = [&](int64_t g) -> int32_t {
        return op == FCOO_OP_MTTKRP ? b.seg[(size_t)g] : (int32_t)g;
    };
    b.fix.clear();
    int64_t last = -1;
    for (int64_t tb = 0; tb < ntiles; ++tb) {
        if (hb[tb + 1] == hb[tb]) continue;          // no head in tile tb
        if (tb >= 1) {
            b.fix.push_back((int32_t)tb);
            b.fix.push_back((int32_t)last);
            b.fix.push_back(out_row(hb[tb] - 1));
        }
        last = tb;
    }
    if (b.nnz > 0) {
        b.fix.push_back((int32_t)ntiles);
        b.fix.push_back((int32_t)last);
        b.fix.push_back(out_row(cnt - 1));
    }
    b.empty_rows.clear();
    if (op == FCOO_OP_MTTKRP) {
        const int64_t rows = (int64_t)b.nblk * t->dims[mode];
        std::vector<uint8_t> present(rows, 0);
        for (int64_t g = 0; g < cnt; ++g) present[b.seg[g]] = 1;
        for (int64_t i = 0; i < rows; ++i)
            if (!present[i]) b.empty_rows.push_back((int32_t)i);
    }
}

static int build_device(Built &b, hipStream_t s)
{
    int64_t acct = 0;
    int rc;
    for (size_t q = 0; q < b.pidx.size(); ++q)
        if ((rc = upload(&b.d_pidx[q], b.pidx[q].data(), b.nnz, 4, s, &acct))) return rc;
    // 4 entries of zero padding: 16-byte stream vectors never read past the allocation
    if ((rc = upload(&b.d_val, b.val.data(), b.nnz, 4, s, &acct))) return rc;
    {   // bit stream as uint32 words plus two zero words (64-bit windows never read past it)
        const int64_t words = (b.nnz + 31) / 32;
        std::vector<uint32_t> w(words, 0);
        if (!b.bf.empty()) memcpy(w.data(), b.bf.data(), b.bf.size());
        if ((rc = upload(&b.d_bf, w.data(), words, 2, s, &acct))) return rc;
        FCOO_HIP(hipStreamSynchronize(s));
    }
    // sf stays on the host (exported with the format): the kernels count the
    // segment heads before each run from bf popcounts, so no device work reads it
    if (b.op == FCOO_OP_MTTKRP)
        if ((rc = upload(&b.d_seg_row, b.seg.data(), b.nseg, 1, s, &acct))) return rc;
    if ((rc = upload(&b.d_tile_seg0, b.tile_seg0.data(), b.ntiles, 1, s, &acct))) return rc;
    if ((rc = upload(&b.d_perm, b.perm.data(), b.nnz, 0, s, &acct))) return rc;
    if ((rc = upload(&b.d_fix, b.fix.data(), (int64_t)b.fix.size(), 3, s, &acct))) return rc;
    if ((rc = upload(&b.d_empty, b.empty_rows.data(), (int64_t)b.empty_rows.size(), 1, s, &acct)))
        return rc;
    FCOO_HIP(hipStreamSynchronize(s));
    b.device_bytes = acct;
    b.on_device = true;
    return FCOO_OK;
}

// The build of (op, mode), or NULL with *rc set: FCOO_EINVAL for a null
// handle, a mode outside [0, order) or an unknown op; FCOO_ENOTBUILT when
// that (op, mode) has no build (on the device, if need_device).
Built *get_built(fcoo_tensor *t, int mode, int op, bool need_device, int *rc)
{
    if (!t) { *rc = fail(FCOO_EINVAL, "null handle"); return nullptr; }
    if (mode < 0 || mode >= t->order) { *rc = fail(FCOO_EINVAL, "mode %d out of range", mode); return nullptr; }
    if (op != FCOO_OP_MTTKRP && op != FCOO_OP_TTM) { *rc = fail(FCOO_EINVAL, "unknown op %d", op); return nullptr; }
    Built &b = t->b[op][mode];
    if (!b.built || (need_device && !b.on_device)) {
        *rc = fail(FCOO_ENOTBUILT, "(op %d, mode %d) is not built%s", op, mode,
                   b.built ? " on the device" : "");
        return nullptr;
    }
    *rc = FCOO_OK;
    return &b;
}

}  // namespace fcoo

using namespace fcoo;

extern "C" {

int fcoo_version(void) { return 101; }

const char *fcoo_last_error(void) { return fcoo::g_err.c_str(); }

int fcoo_create(int order, const int64_t *dims, int64_t nnz, const int32_t *const *idx,
                const float *vals, fcoo_tensor **out)
{
    clear_error();
    if (!out) return fail(FCOO_EINVAL, "out is NULL");
    *out = nullptr;
    if (order < 2 || order > kMaxOrder) return fail(FCOO_EUNSUPPORTED, "order %d outside [2, 8]", order);
    if (!dims) return fail(FCOO_EINVAL, "dims is NULL");
    if (nnz < 0) return fail(FCOO_EINVAL, "nnz < 0");
    if (nnz > 0 && (!idx || !vals)) return fail(FCOO_EINVAL, "idx or vals is NULL");
    if (nnz > (int64_t)INT32_MAX) return fail(FCOO_ERANGE, "nnz %lld exceeds 2^31 - 1", (long long)nnz);
    for (int m = 0; m < order; ++m) {
        if (dims[m] < 1 || dims[m] > (int64_t)INT32_MAX)
            return fail(FCOO_ERANGE, "dims[%d] = %lld outside [1, 2^31 - 1]", m, (long long)dims[m]);
        if (nnz > 0 && !idx[m]) return fail(FCOO_EINVAL, "idx[%d] is NULL", m);
    }
    fcoo_tensor *t = new (std::nothrow) fcoo_tensor();
    if (!t) return fail(FCOO_ENOMEM, "handle");
    try {
        t->order = order;
        t->nnz = nnz;
        for (int m = 0; m < order; ++m) {
            t->dims[m] = dims[m];
            t->idx[m].assign(idx ? idx[m] : nullptr, idx ? idx[m] + nnz : nullptr);
        }
        t->vals.assign(vals, vals + nnz);
    } catch (const std::bad_alloc &) {
        delete t;
        return fail(FCOO_ENOMEM, "copying %lld nonzeros", (long long)nnz);
    }
    for (int m = 0; m < order; ++m) {
        const int32_t *c = t->idx[m].data();
        const int64_t d = dims[m];
        for (int64_t e = 0; e < nnz; ++e)
            if (c[e] < 0 || (int64_t)c[e] >= d) {
                int rc = fail(FCOO_ERANGE, "idx[%d][%lld] = %d outside [0, %lld)", m, (long long)e,
                              c[e], (long long)d);
                delete t;
                return rc;
            }
    }
    double s = 0.0;
    for (int64_t e = 0; e < nnz; ++e) s += (double)t->vals[e] * (double)t->vals[e];
    t->normX2 = s;
    *out = t;
    return FCOO_OK;
}

int fcoo_build(fcoo_tensor *t, int mode, int op, const fcoo_opts *opts, void *stream)
{
    clear_error();
    if (!t) return fail(FCOO_EINVAL, "null handle");
    if (mode < 0 || mode >= t->order) return fail(FCOO_EINVAL, "mode %d out of range", mode);
    if (op != FCOO_OP_MTTKRP && op != FCOO_OP_TTM) return fail(FCOO_EINVAL, "unknown op %d", op);
    int threadlen = opts && opts->threadlen ? opts->threadlen : 16;
    int tile_nnz = opts && opts->tile_nnz ? opts->tile_nnz : 4096;
    const bool host_only = opts && opts->host_only;
    const bool on_gpu = opts && opts->device;
    const int nblk = opts ? opts->xcd_blocks : 0;
    const int xmode = opts ? opts->xcd_mode - 1 : -1;
    const int lane_cols = opts ? opts->lane_cols : 0;
    const bool single_pass = opts && opts->single_pass;
    if (host_only && on_gpu) return fail(FCOO_EINVAL, "host_only and device are exclusive");
    if (lane_cols != 0 && lane_cols != 4 && lane_cols != 8)
        return fail(FCOO_EINVAL, "lane_cols %d not in {0, 4, 8}", lane_cols);
    if (threadlen != 8 && threadlen != 16 && threadlen != 32 && threadlen != 64)
        return fail(FCOO_EINVAL, "threadlen %d not in {8, 16, 32, 64}", threadlen);
    if (tile_nnz <= 0 || tile_nnz % 256 || tile_nnz % threadlen || tile_nnz > (1 << 20))
        return fail(FCOO_EINVAL, "tile_nnz %d must be a positive multiple of 256 and threadlen, <= 2^20",
                    tile_nnz);
    Built &b = t->b[op][mode];
    b.free_device();
    int rc;
    if (on_gpu) {
        try {
            rc = build_on_device(t, b, mode, op, threadlen, tile_nnz, nblk, xmode, (hipStream_t)stream);
        } catch (const std::bad_alloc &) {
            rc = fail(FCOO_ENOMEM, "device build (host side)");
        }
        if (!rc && single_pass) rc = setup_single_pass(b, (hipStream_t)stream);
        if (rc) {
            b.free_device();
            b = Built();
        }
        b.lane_cols = lane_cols;
        return rc;
    }
    try {
        rc = build_host(t, b, mode, op, threadlen, tile_nnz, nblk, xmode);
    } catch (const std::bad_alloc &) {
        b = Built();
        return fail(FCOO_ENOMEM, "host build");
    }
    if (rc) return rc;
    b.lane_cols = lane_cols;
    if (host_only) return FCOO_OK;
    rc = build_device(b, (hipStream_t)stream);
    if (!rc && single_pass) rc = setup_single_pass(b, (hipStream_t)stream);
    if (rc) { b.free_device(); return rc; }
    return FCOO_OK;
}

int fcoo_info(const fcoo_tensor *t, int mode, int op, fcoo_info_t *info)
{
    clear_error();
    if (!info) return fail(FCOO_EINVAL, "info is NULL");
    int rc;
    const Built *b = get_built(const_cast<fcoo_tensor *>(t), mode, op, false, &rc);
    if (!b) return rc;
    info->nnz = b->nnz;
    info->nseg = b->nseg;
    info->npart = b->npart;
    info->ntiles = b->ntiles;
    info->nfix = b->nfix();
    info->nempty = (int64_t)b->empty_rows.size();
    info->bytes_format = b->format_bytes();
    info->bytes_device = b->device_bytes;
    info->threadlen = b->threadlen;
    info->tile_nnz = b->tile_nnz;
    info->order = t->order;
    info->on_device = b->on_device ? 1 : 0;
    info->xcd_blocks = b->nblk;
    info->block_mode = b->bmode;
    info->lane_cols = b->lane_cols;
    info->single_pass = b->sp ? 1 : 0;
    info->sp_gave_up = 0;
    if (b->sp && b->d_sp_err) {
        // reads the flag a bounded wait of the single-pass kernel sets (synchronous)
        int e = 0;
        FCOO_HIP(hipMemcpy(&e, b->d_sp_err, sizeof(int), hipMemcpyDeviceToHost));
        info->sp_gave_up = e != 0;
    }
    return FCOO_OK;
}

int fcoo_export(const fcoo_tensor *t, int mode, int op, int32_t *const *pidx, float *val,
                uint8_t *bf, uint32_t *sf, int32_t *seg, int32_t *tile_seg0, int32_t *perm)
{
    clear_error();
    int rc;
    const Built *b = get_built(const_cast<fcoo_tensor *>(t), mode, op, false, &rc);
    if (!b) return rc;
    if (!b->host_arrays) {
        // built on the GPU: the per-nonzero arrays live on the device only
        const int64_t Z = b->nnz;
        if (pidx)
            for (size_t q = 0; q < b->pmodes.size(); ++q)
                if (pidx[q]) FCOO_HIP(hipMemcpy(pidx[q], b->d_pidx[q], (size_t)Z * 4, hipMemcpyDeviceToHost));
        if (val) FCOO_HIP(hipMemcpy(val, b->d_val, (size_t)Z * 4, hipMemcpyDeviceToHost));
        if (bf) FCOO_HIP(hipMemcpy(bf, b->d_bf, (size_t)(Z + 7) / 8, hipMemcpyDeviceToHost));
        if (sf) FCOO_HIP(hipMemcpy(sf, b->d_sf, (size_t)((b->npart + 31) / 32) * 4, hipMemcpyDeviceToHost));
        if (perm) FCOO_HIP(hipMemcpy(perm, b->d_perm, (size_t)Z * 4, hipMemcpyDeviceToHost));
        if (seg) memcpy(seg, b->seg.data(), b->seg.size() * 4);
        if (tile_seg0) memcpy(tile_seg0, b->tile_seg0.data(), b->tile_seg0.size() * 4);
        return FCOO_OK;
    }
    if (pidx)
        for (size_t q = 0; q < b->pidx.size(); ++q)
            if (pidx[q]) memcpy(pidx[q], b->pidx[q].data(), b->pidx[q].size() * 4);
    if (val) memcpy(val, b->val.data(), b->val.size() * 4);
    if (bf) memcpy(bf, b->bf.data(), b->bf.size());
    if (sf) memcpy(sf, b->sf.data(), b->sf.size() * 4);
    if (seg) memcpy(seg, b->seg.data(), b->seg.size() * 4);
    if (tile_seg0) memcpy(tile_seg0, b->tile_seg0.data(), b->tile_seg0.size() * 4);
    if (perm) memcpy(perm, b->perm.data(), b->perm.size() * 4);
    return FCOO_OK;
}

void fcoo_destroy(fcoo_tensor *t)
{
    if (!t) return;
    for (auto &row : t->b)
        for (auto &b : row) b.free_device();
    for (auto &p : t->d_coo) if (p) (void)hipFree(p);
    if (t->d_coo_val) (void)hipFree(t->d_coo_val);
    t->ws.free_all();
    if (t->ev_dep) (void)hipEventDestroy(t->ev_dep);
    if (t->ev_solved) (void)hipEventDestroy(t->ev_solved);
    if (t->aux) (void)hipStreamDestroy(t->aux);
    delete t;
}

// ---------------------------------------------------------------------------
// sparse operations: argument checks, then the HIP launchers
// ---------------------------------------------------------------------------

// XCD blocks: the partial output (nblk x rows x width floats) of this build
static int prep_blocks(Built *b, TileProblem &p, hipStream_t s)
{
    if (b->nblk <= 1) return FCOO_OK;
    int rc = ensure_device_floats(&b->d_bpart, &b->bpart_cap, (int64_t)b->nblk * b->rows * p.R, s);
    if (rc) return rc;
    p.bpart = b->d_bpart;
    return FCOO_OK;
}
int fcoo_spmttkrp(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R, float *M,
                  void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_MTTKRP, true, &rc);
    if (!b) return rc;
    rc = check_factors(t, mode, factors, dtype, R);
    if (rc) return rc;
    if (!M) return fail(FCOO_EINVAL, "M is NULL");
    hipStream_t s = (hipStream_t)stream;
    TileProblem p{};
    p.b = b;
    for (size_t q = 0; q < b->pmodes.size(); ++q) p.fac[q] = factors[b->pmodes[q]];
    p.vals = b->d_val;
    p.dtype = dtype;
    p.R = R;
    p.out = M;
    if ((rc = ensure_device_floats(&b->d_carry, &b->carry_cap, 2 * b->ntiles * (int64_t)R, s))) return rc;
    p.carry = b->d_carry;
    if ((rc = prep_blocks(b, p, s))) return rc;
    if ((rc = prep_single_pass(b, p, s))) return rc;
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    return launch_segmented(p, s, false);
}

int fcoo_spttmc(fcoo_tensor *t, int mode, const void *const *factors, int dtype, const int *ranks,
                float *Y, void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_MTTKRP, true, &rc);
    if (!b) return rc;
    if (!ranks) return fail(FCOO_EINVAL, "ranks is NULL");
    int64_t W = 1;
    for (int m = 0; m < t->order; ++m) {
        if (m == mode) continue;
        if (ranks[m] < 1 || ranks[m] > kMaxR)
            return fail(FCOO_EUNSUPPORTED, "ranks[%d] = %d outside [1, %d]", m, ranks[m], kMaxR);
        W *= ranks[m];
        if (W > kMaxKronWidth)
            return fail(FCOO_EUNSUPPORTED, "SpTTMc width (product of the ranks) above %d", kMaxKronWidth);
    }
    rc = check_factors(t, mode, factors, dtype, 1);
    if (rc) return rc;
    if (!Y) return fail(FCOO_EINVAL, "Y is NULL");
    hipStream_t s = (hipStream_t)stream;
    TileProblem p{};
    p.b = b;
    p.kron = true;
    for (size_t q = 0; q < b->pmodes.size(); ++q) {
        p.fac[q] = factors[b->pmodes[q]];
        p.kr[q] = ranks[b->pmodes[q]];
    }
    p.vals = b->d_val;
    p.dtype = dtype;
    p.R = (int)W;
    p.out = Y;
    if ((rc = ensure_device_floats(&b->d_carry, &b->carry_cap, 2 * b->ntiles * W, s))) return rc;
    p.carry = b->d_carry;
    if ((rc = prep_blocks(b, p, s))) return rc;
    if ((rc = prep_single_pass(b, p, s))) return rc;
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    return launch_segmented(p, s, false);
}

int fcoo_spttm(fcoo_tensor *t, int mode, const void *U, int dtype, int R, float *Y, void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_TTM, true, &rc);
    if (!b) return rc;
    if ((!U && b->nnz) || (!Y && b->nseg)) return fail(FCOO_EINVAL, "U or Y is NULL");
    if (dtype != FCOO_F32 && dtype != FCOO_BF16) return fail(FCOO_EUNSUPPORTED, "unknown dtype %d", dtype);
    if (R < 1 || R > kMaxR) return fail(FCOO_EUNSUPPORTED, "R = %d outside [1, %d]", R, kMaxR);
    hipStream_t s = (hipStream_t)stream;
    TileProblem p{};
    p.b = b;
    p.fac[0] = U;
    p.vals = b->d_val;
    p.dtype = dtype;
    p.R = R;
    p.out = Y;
    if ((rc = ensure_device_floats(&b->d_carry, &b->carry_cap, 2 * b->ntiles * (int64_t)R, s))) return rc;
    p.carry = b->d_carry;
    if ((rc = prep_blocks(b, p, s))) return rc;
    if ((rc = prep_single_pass(b, p, s))) return rc;
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    return launch_segmented(p, s, false);
}

int fcoo_spmttkrp_values(fcoo_tensor *t, int mode, const float *g, const void *const *factors,
                         int dtype, int R, float *M, void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_MTTKRP, true, &rc);
    if (!b) return rc;
    rc = check_factors(t, mode, factors, dtype, R);
    if (rc) return rc;
    if (!M || (!g && b->nnz)) return fail(FCOO_EINVAL, "M or g is NULL");
    hipStream_t s = (hipStream_t)stream;
    int64_t cap = b->d_gperm ? b->nnz : 0;
    if (!b->d_gperm && b->nnz) {
        if ((rc = ensure_device_floats(&b->d_gperm, &cap, b->nnz, s))) return rc;
    }
    if (b->nnz && (rc = launch_permute_values(*b, g, b->d_gperm, s))) return rc;
    TileProblem p{};
    p.b = b;
    for (size_t q = 0; q < b->pmodes.size(); ++q) p.fac[q] = factors[b->pmodes[q]];
    p.vals = b->d_gperm;
    p.dtype = dtype;
    p.R = R;
    p.out = M;
    if ((rc = ensure_device_floats(&b->d_carry, &b->carry_cap, 2 * b->ntiles * (int64_t)R, s))) return rc;
    p.carry = b->d_carry;
    if ((rc = prep_blocks(b, p, s))) return rc;
    if ((rc = prep_single_pass(b, p, s))) return rc;
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    return launch_segmented(p, s, false);
}

int fcoo_resid_spmttkrp(fcoo_tensor *t, int mode, const void *const *factors, int dtype, int R,
                        float *G, double *loss, void *stream)
{
    clear_error();
    int rc;
    Built *b = get_built(t, mode, FCOO_OP_MTTKRP, true, &rc);
    if (!b) return rc;
    rc = check_factors(t, -1, factors, dtype, R);
    if (rc) return rc;
    if (!G) return fail(FCOO_EINVAL, "G is NULL");
    hipStream_t s = (hipStream_t)stream;
    TileProblem p{};
    p.b = b;
    for (size_t q = 0; q < b->pmodes.size(); ++q) p.fac[q] = factors[b->pmodes[q]];
    p.vals = b->d_val;
    p.dtype = dtype;
    p.R = R;
    p.out = G;
    p.own = factors[mode];
    p.inv_nnz = b->nnz ? (float)(1.0 / (double)b->nnz) : 0.f;
    if ((rc = ensure_device_floats(&b->d_carry, &b->carry_cap, 2 * b->ntiles * (int64_t)R, s))) return rc;
    p.carry = b->d_carry;
    if ((rc = prep_blocks(b, p, s))) return rc;
    if ((rc = prep_single_pass(b, p, s))) return rc;
    if (loss) {
        if ((rc = ensure_device_doubles(&b->d_partial, &b->partial_cap, b->ntiles + 1, s))) return rc;
        p.partial = b->d_partial;
    }
    p.ev_before = t->ev_before;
    p.ev_after = t->ev_after;
    if ((rc = launch_segmented(p, s, true))) return rc;
    if (loss) return launch_reduce_partials(b->d_partial, b->ntiles,
                                            b->nnz ? 0.5 / (double)b->nnz : 0.0, loss, s);
    return FCOO_OK;
}

int fcoo_set_tile_events(fcoo_tensor *t, void *before, void *after)
{
    clear_error();
    if (!t) return fail(FCOO_EINVAL, "null handle");
    if ((before == nullptr) != (after == nullptr)) return fail(FCOO_EINVAL, "give both events or neither");
    t->ev_before = (hipEvent_t)before;
    t->ev_after = (hipEvent_t)after;
    return FCOO_OK;
}

int fcoo_model_at_nnz(fcoo_tensor *t, const void *const *factors, int dtype, int R, float *xhat,
                      void *stream)
{
    clear_error();
    if (!t) return fail(FCOO_EINVAL, "null handle");
    int rc = check_factors(t, -1, factors, dtype, R);
    if (rc) return rc;
    if (!xhat && t->nnz) return fail(FCOO_EINVAL, "xhat is NULL");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = upload_coo(t, s))) return rc;
    return launch_model(t, factors, dtype, R, xhat, s);
}

}  // extern "C"

// F-COO build on the GPU (Sec. IV-B; the paper preprocesses on the host).
// Same arrays as the host builder, bit for bit:
//   1. packed 64-bit key per nonzero (index modes, then product modes, each
//      in ascending mode order, lower modes in the higher bits) and a stable
//      radix sort of (key, input position) (fcoo_sort.hip);
//   2. product-mode indices decoded from the sorted keys (their low bits),
//      values gathered through the sorted positions, and the segment heads
//      (index-mode part of the key changes);
//   3. inclusive scan of the heads: segment ordinal of every nonzero;
//   4. bf words (parity of the running head count, so the bit starts at 1
//      and toggles at every head), sf words (any head in a partition), both
//      by wave ballots; output row / fibre coordinates of every segment;
//      per-tile head counts and first-segment ordinals.
// The host then derives the carry fix-up chains from the per-tile counts and
// the rows no segment covers (O(tiles + rows) work), as the host builder does.
#include <hip/hip_runtime.h>

#include <cstring>

#include <vector>

#include "fcoo_internal.h"

namespace fcoo {
namespace dev {

struct KeyArgs {
    const int32_t *idx[kMaxOrder];   // coordinate arrays in key order (index modes, then product modes)
    int width[kMaxOrder];            // bits of each
    int nmodes;
    int64_t nnz;
    const int32_t *blk_of;           // XCD blocks: block of each index of bidx (else null)
    const int32_t *bidx;             // coordinates of the block mode
};

__global__ __launch_bounds__(256) void key_kernel(KeyArgs a, uint64_t *__restrict__ key,
                                                  uint32_t *__restrict__ pos)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.nnz; e += (int64_t)gridDim.x * 256) {
        uint64_t k = a.blk_of ? (uint64_t)a.blk_of[a.bidx[e]] : 0;
        for (int i = 0; i < a.nmodes; ++i) {
            const int w = a.width[i];
            k = (w ? (k << w) : k) | (uint64_t)(uint32_t)a.idx[i][e];
        }
        key[e] = k;
        pos[e] = (uint32_t)e;
    }
}

struct GatherArgs {
    const float *vals;
    const uint64_t *key;             // sorted keys
    const uint32_t *pos;             // input position of each sorted nonzero
    int32_t *pidx[kMaxOrder];        // per product mode q
    int pshift[kMaxOrder];           // bit offset of product mode q in the key
    int pwidth[kMaxOrder];           // its bits (0 for a mode of extent 1)
    int np;
    int pbits;                       // bits of the product-mode part of the key
    float *val;
    int32_t *perm;
    int32_t *head;
    int64_t nnz;
};

__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a)
{
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < a.nnz; s += (int64_t)gridDim.x * 256) {
        const uint32_t e = a.pos[s];
        const uint64_t k = a.key[s];
        for (int q = 0; q < a.np; ++q) {
            const int w = a.pwidth[q];
            a.pidx[q][s] = w ? (int32_t)((k >> a.pshift[q]) & ((1ull << w) - 1)) : 0;
        }
        a.val[s] = a.vals[e];
        a.perm[s] = (int32_t)e;
        int h = s == 0;
        if (!h && a.pbits < 64) h = (k >> a.pbits) != (a.key[s - 1] >> a.pbits);
        a.head[s] = h;
    }
}

// bf word w: bit i = parity of the heads up to nonzero 32 w + i (0 past Z).
// One lane per nonzero; a wave's ballot is two words.
__global__ __launch_bounds__(256) void bf_kernel(const int32_t *__restrict__ cum, int64_t nnz, int64_t nwords,
                                                 uint32_t *__restrict__ bf)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool bit = s < nnz && (cum[s] & 1);
    const uint64_t m = __ballot(bit);
    const int lane = threadIdx.x & 63;
    const int64_t w = (s - lane) >> 5;                     // first word of this wave
    if (lane == 0 && w < nwords) bf[w] = (uint32_t)m;
    if (lane == 32 && w + 1 < nwords) bf[w + 1] = (uint32_t)(m >> 32);
}

// sf word w: bit i = some head in partition 32 w + i (partitions of L nonzeros).
__global__ __launch_bounds__(256) void sf_kernel(const int32_t *__restrict__ head, int64_t nnz, int L,
                                                 int64_t npart, int64_t nwords, uint32_t *__restrict__ sf)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool any = false;
    if (p < npart) {
        const int64_t s0 = p * L;
        const int64_t s1 = s0 + L < nnz ? s0 + L : nnz;
        for (int64_t s = s0; s < s1 && !any; ++s) any = head[s] != 0;
    }
    const uint64_t m = __ballot(any);
    const int lane = threadIdx.x & 63;
    const int64_t w = (p - lane) >> 5;
    if (lane == 0 && w < nwords) sf[w] = (uint32_t)m;
    if (lane == 32 && w + 1 < nwords) sf[w + 1] = (uint32_t)(m >> 32);
}

struct SegArgsB {
    const uint64_t *key;             // sorted keys
    const int32_t *head;
    const int32_t *cum;
    int ishift[kMaxOrder];           // bit offset of index mode q in the key
    int iwidth[kMaxOrder];           // its bits (0 for a mode of extent 1)
    int nim;
    int32_t *seg;                    // nseg x nim
    int64_t nnz;
    int bshift;                      // XCD blocks (SpMTTKRP): block number = key >> bshift,
    int32_t rows;                    // row = block * rows + index (rows = 0: no blocks)
};

// Coordinates of every segment, decoded from the key of its head nonzero.
__global__ __launch_bounds__(256) void seg_kernel(SegArgsB a)
{
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < a.nnz; s += (int64_t)gridDim.x * 256) {
        if (!a.head[s]) continue;
        const int64_t g = a.cum[s] - 1;
        const uint64_t k = a.key[s];
        for (int q = 0; q < a.nim; ++q) {
            const int w = a.iwidth[q];
            a.seg[g * a.nim + q] = w ? (int32_t)((k >> a.ishift[q]) & ((1ull << w) - 1)) : 0;
        }
        if (a.rows) a.seg[g] += (int32_t)(a.bshift < 64 ? k >> a.bshift : 0) * a.rows;
    }
}

// hb[t] = heads before nonzero t T (t = 0 .. ntiles; hb[ntiles] = all heads),
// ts0[t] = ordinal of the segment holding nonzero t T.
__global__ __launch_bounds__(256) void tiles_kernel(const int32_t *__restrict__ cum, int64_t nnz, int T,
                                                    int64_t ntiles, int32_t *__restrict__ hb,
                                                    int32_t *__restrict__ ts0)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t > ntiles) return;
    const int64_t s = t * T;
    hb[t] = s == 0 ? 0 : cum[(s < nnz ? s : nnz) - 1];
    if (t < ntiles) ts0[t] = cum[s] - 1;
}

}  // namespace dev

namespace {

int bits_of(int64_t d)  // bits to hold 0 .. d-1
{
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < d) ++b;
    return b;
}

int grid_of(int64_t n, int cap = 65535 * 16)
{
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

// device temporaries of one build, freed on every exit path
struct Scratch {
    std::vector<void *> p;
    ~Scratch() { for (void *x : p) (void)hipFree(x); }
    template <typename T>
    int get(T **out, int64_t n)
    {
        void *x = nullptr;
        if (hipMalloc(&x, (size_t)(n > 0 ? n : 1) * sizeof(T)) != hipSuccess)
            return fail(FCOO_ENOMEM, "device build scratch (%lld elements)", (long long)n);
        p.push_back(x);
        *out = (T *)x;
        return FCOO_OK;
    }
};

template <typename T>
int alloc_dev(T **dst, int64_t n, int64_t pad, hipStream_t s, int64_t *acct)
{
    const size_t bytes = (size_t)(n + pad > 0 ? n + pad : 1) * sizeof(T);
    FCOO_HIP(hipMalloc((void **)dst, bytes));
    if (pad) FCOO_HIP(hipMemsetAsync(*dst, 0, bytes, s));
    *acct += (int64_t)bytes;
    return FCOO_OK;
}

}  // namespace

int build_on_device(fcoo_tensor *t, Built &b, int mode, int op, int L, int T, int nblk, int xmode, hipStream_t s)
{
    const int N = t->order;
    const int64_t Z = t->nnz;
    b = Built();
    b.op = op; b.mode = mode; b.threadlen = L; b.tile_nnz = T; b.nnz = Z;
    b.host_arrays = false;
    for (int m = 0; m < N; ++m) {
        if (m == mode) continue;
        if (op == FCOO_OP_MTTKRP) b.pmodes.push_back(m); else b.imodes.push_back(m);
    }
    if (op == FCOO_OP_MTTKRP) b.imodes.insert(b.imodes.begin(), mode); else b.pmodes.push_back(mode);
    int rc = setup_blocks(t, b, nblk, xmode);
    if (rc) return rc;
    const bool blocked = b.nblk > 1;
    int total = blocked ? bits_of(b.nblk) : 0, pbits = 0;
    dev::KeyArgs ka{};
    ka.nnz = Z;
    for (int m : b.imodes) { ka.idx[ka.nmodes] = nullptr; ka.width[ka.nmodes++] = bits_of(t->dims[m]); }
    for (int m : b.pmodes) { const int w = bits_of(t->dims[m]); ka.width[ka.nmodes++] = w; pbits += w; }
    for (int i = 0; i < ka.nmodes; ++i) total += ka.width[i];
    if (total > 64)
        return fail(FCOO_EUNSUPPORTED, "device build needs the sort key within 64 bits (%d bits)", total);
    if (Z == 0) return fail(FCOO_EUNSUPPORTED, "device build of an empty tensor (build it on the host)");
    if (Z > (int64_t)0x7fffffff) return fail(FCOO_EUNSUPPORTED, "device build supports Z < 2^31");
    rc = upload_coo(t, s);
    if (rc) return rc;
    {
        int i = 0;
        for (int m : b.imodes) ka.idx[i++] = t->d_coo[m];
        for (int m : b.pmodes) ka.idx[i++] = t->d_coo[m];
    }
    const int64_t P = (Z + L - 1) / L;
    const int64_t ntiles = (Z + T - 1) / T;
    b.npart = P;
    b.ntiles = ntiles;

    Scratch tmp;
    uint64_t *k0, *k1;
    uint32_t *p0, *p1;
    int32_t *head, *cum, *hb;
    if ((rc = tmp.get(&k0, Z)) || (rc = tmp.get(&k1, Z)) || (rc = tmp.get(&p0, Z)) || (rc = tmp.get(&p1, Z)) ||
        (rc = tmp.get(&head, Z)) || (rc = tmp.get(&cum, Z)) || (rc = tmp.get(&hb, ntiles + 1)))
        return rc;

    int32_t *blk_d = nullptr;
    if (blocked) {
        if ((rc = tmp.get(&blk_d, (int64_t)b.blk_of.size()))) return rc;
        FCOO_HIP(hipMemcpyAsync(blk_d, b.blk_of.data(), b.blk_of.size() * 4, hipMemcpyHostToDevice, s));
        ka.blk_of = blk_d;
        ka.bidx = t->d_coo[b.bmode];
    }

    // 1. keys and the stable radix sort
    hipLaunchKernelGGL(dev::key_kernel, dim3(grid_of(Z)), dim3(256), 0, s, ka, k0, p0);
    FCOO_HIP(hipGetLastError());
    const int end_bit = total > 0 ? total : 1;
    const int64_t wsort = sort_work_ints(Z), wscan = scan_work_ints(Z);
    int32_t *work;
    if ((rc = tmp.get(&work, wsort > wscan ? wsort : wscan))) return rc;
    int passes = 0;
    if ((rc = sort_pairs_u64(k0, k1, p0, p1, Z, end_bit, work, s, &passes))) return rc;
    uint64_t *ks = (passes & 1) ? k1 : k0;            // the sorted pairs
    uint32_t *ps = (passes & 1) ? p1 : p0;

    // 2. sorted per-nonzero arrays (4 zero entries of padding, as uploaded by the host builder)
    int64_t acct = 0;
    dev::GatherArgs ga{};
    ga.vals = t->d_coo_val;
    ga.key = ks;
    ga.pos = ps;
    ga.np = (int)b.pmodes.size();
    for (int q = ga.np - 1, sh = 0; q >= 0; --q) {   // last product mode in the lowest bits
        if ((rc = alloc_dev(&b.d_pidx[q], Z, 4, s, &acct))) return rc;
        ga.pidx[q] = b.d_pidx[q];
        ga.pwidth[q] = bits_of(t->dims[b.pmodes[q]]);
        ga.pshift[q] = sh;
        sh += ga.pwidth[q];
    }
    ga.pbits = pbits;
    if ((rc = alloc_dev(&b.d_val, Z, 4, s, &acct))) return rc;
    if ((rc = alloc_dev(&b.d_perm, Z, 0, s, &acct))) return rc;
    ga.val = b.d_val;
    ga.perm = b.d_perm;
    ga.head = head;
    ga.nnz = Z;
    hipLaunchKernelGGL(dev::gather_kernel, dim3(grid_of(Z)), dim3(256), 0, s, ga);
    FCOO_HIP(hipGetLastError());

    // 3. segment ordinals
    if ((rc = scan_i32(head, cum, Z, true, work, s))) return rc;

    // 4. flags, tiles, segments
    const int64_t bfw = (Z + 31) / 32, sfw = (P + 31) / 32;
    if ((rc = alloc_dev(&b.d_bf, bfw, 2, s, &acct))) return rc;
    if ((rc = alloc_dev(&b.d_sf, sfw, 1, s, &acct))) return rc;
    if ((rc = alloc_dev(&b.d_tile_seg0, ntiles, 1, s, &acct))) return rc;
    hipLaunchKernelGGL(dev::bf_kernel, dim3((unsigned)((bfw * 32 + 255) / 256)), dim3(256), 0, s, cum, Z, bfw,
                       b.d_bf);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::sf_kernel, dim3((unsigned)((sfw * 32 + 255) / 256)), dim3(256), 0, s, head, Z, L, P,
                       sfw, b.d_sf);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::tiles_kernel, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0, s, cum, Z, T,
                       ntiles, hb, b.d_tile_seg0);
    FCOO_HIP(hipGetLastError());
    std::vector<int32_t> hbh(ntiles + 1);
    FCOO_HIP(hipMemcpyAsync(hbh.data(), hb, (size_t)(ntiles + 1) * 4, hipMemcpyDeviceToHost, s));
    FCOO_HIP(hipStreamSynchronize(s));
    const int64_t nseg = hbh[ntiles];
    b.nseg = nseg;
    const int nim = (int)b.imodes.size();
    int32_t *segd;
    if (op == FCOO_OP_MTTKRP) {
        if ((rc = alloc_dev(&b.d_seg_row, nseg, 1, s, &acct))) return rc;
        segd = b.d_seg_row;
    } else if ((rc = tmp.get(&segd, nseg * nim))) {
        return rc;
    }
    dev::SegArgsB sa{};
    sa.key = ks;
    sa.head = head;
    sa.cum = cum;
    int sh = pbits;
    for (int q = nim - 1; q >= 0; --q) {   // index modes above the product modes, last one lowest
        sa.iwidth[q] = bits_of(t->dims[b.imodes[q]]);
        sa.ishift[q] = sh;
        sh += sa.iwidth[q];
    }
    sa.nim = nim;
    sa.seg = segd;
    sa.nnz = Z;
    if (blocked) {
        sa.bshift = sh;
        sa.rows = (int32_t)t->dims[mode];
    }
    hipLaunchKernelGGL(dev::seg_kernel, dim3(grid_of(Z)), dim3(256), 0, s, sa);
    FCOO_HIP(hipGetLastError());
    b.seg.resize((size_t)nseg * nim);
    b.tile_seg0.resize(ntiles);
    FCOO_HIP(hipMemcpyAsync(b.seg.data(), segd, (size_t)nseg * nim * 4, hipMemcpyDeviceToHost, s));
    FCOO_HIP(hipMemcpyAsync(b.tile_seg0.data(), b.d_tile_seg0, (size_t)ntiles * 4, hipMemcpyDeviceToHost, s));
    FCOO_HIP(hipStreamSynchronize(s));

    // 5. carry chains and empty rows on the host (per tile / per row)
    std::vector<int64_t> hb64(hbh.begin(), hbh.end());
    finish_tiles(t, b, mode, op, hb64);
    if ((rc = upload_i32(&b.d_fix, b.fix, 3, s, &acct))) return rc;
    if ((rc = upload_i32(&b.d_empty, b.empty_rows, 1, s, &acct))) return rc;
    FCOO_HIP(hipStreamSynchronize(s));
    b.device_bytes = acct;
    b.built = true;
    b.on_device = true;
    return FCOO_OK;
}

}  // namespace fcoo

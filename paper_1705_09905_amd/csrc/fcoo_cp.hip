// CP-ALS dense steps (Algorithm 1): Gram products on the matrix cores, the
// R x R float64 solve, the row solve with column normalisation, the fit, and
// the sweep driver fcoo_cp_als_iter.
//
// Per mode n of a sweep: M = SpMTTKRP_n (segmented-scan kernels);
// V = Hadamard product of the Grams G_m, m != n (float64);
// W = V^-1 by Gauss-Jordan elimination (its pivots are the squared pivots of
// the Cholesky factorisation V = L L^T), or the pseudo-inverse from a
// symmetric eigendecomposition (cyclic Jacobi) when V is not numerically
// positive definite; A_n = M W with column 2-norms lambda,
// A_n / lambda stored as float32 or bfloat16 (round to nearest even);
// G_n = A_n^T A_n from the stored values.  After the last mode:
// fit = 1 - sqrt(max(0, |X|^2 + |Xhat|^2 - 2 <X, Xhat>)) / |X|, with
// |Xhat|^2 = lambda^T (Hadamard of all Grams) lambda and
// <X, Xhat> = sum_r lambda_r sum_i M_{N-1}(i, r) A_{N-1}(i, r).
// Every reduction runs in a fixed order: results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include "fcoo_device.h"
#include "fcoo_internal.h"

namespace fcoo {
namespace dev {

constexpr int kGramRows = 1024;        // rows of A per Gram workgroup (256 per wave)
constexpr int kMaxCpR = 64;            // R bound of the in-LDS solve

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// Partial Gram of rows [blk * kGramRows, ...) for the 32 x 32 tile pair
// (tr, tc): each wave accumulates its quarter of the rows on the matrix
// cores (float32 inputs: 32x32x2; bfloat16: 32x32x8), the four waves are
// summed in float64 and written to partial[blk][R x R].  The operands of the
// next GU matrix steps are loaded while the current ones run.
template <typename FT>
__global__ __launch_bounds__(256) void gram_partial_kernel(const FT *__restrict__ A, int64_t I, int R,
                                                           double *__restrict__ partial)
{
    __shared__ float red[4][32][33];
    const int ntile = (R + 31) / 32;
    const int tr = blockIdx.y / ntile, tc = blockIdx.y % ntile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * kGramRows;
    const int64_t r0 = b0 + (int64_t)w * (kGramRows / 4);
    int64_t r1 = r0 + kGramRows / 4;
    if (r1 > I) r1 = I;
    const int ca = tr * 32 + (lane & 31), cb = tc * 32 + (lane & 31);
    const bool va = ca < R, vb = cb < R;
    const int kk = lane >> 5;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    constexpr int GU = 8;                                    // matrix steps per operand batch
    if constexpr (sizeof(FT) == 4) {
        const float *Af = reinterpret_cast<const float *>(A);
        constexpr int STEP = 2 * GU;                         // rows per batch
        auto ld = [&](int64_t i, float (&a)[GU], float (&b)[GU]) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int64_t row = i + 2 * u + kk;
                a[u] = (row < r1 && va) ? Af[row * R + ca] : 0.f;
                b[u] = (row < r1 && vb) ? Af[row * R + cb] : 0.f;
            }
        };
        float a0[GU], b0v[GU];
        ld(r0, a0, b0v);
        for (int64_t i = r0; i < r1; i += STEP) {
            float a1[GU], b1[GU];
            ld(i + STEP, a1, b1);
#pragma unroll
            for (int u = 0; u < GU; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[u], b0v[u], acc, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < GU; ++u) { a0[u] = a1[u]; b0v[u] = b1[u]; }
        }
    } else {
        const uint16_t *Ab = reinterpret_cast<const uint16_t *>(A);
        constexpr int GB = GU / 2;
        constexpr int STEP = 8 * GB;
        auto ld = [&](int64_t i, shortx4 (&a)[GB], shortx4 (&b)[GB]) {
#pragma unroll
            for (int u = 0; u < GB; ++u) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t row = i + 8 * u + 4 * kk + t;
                    a[u][t] = (short)((row < r1 && va) ? Ab[row * R + ca] : 0);
                    b[u][t] = (short)((row < r1 && vb) ? Ab[row * R + cb] : 0);
                }
            }
        };
        shortx4 a0[GB], b0v[GB];
        ld(r0, a0, b0v);
        for (int64_t i = r0; i < r1; i += STEP) {
            shortx4 a1[GB], b1[GB];
            ld(i + STEP, a1, b1);
#pragma unroll
            for (int u = 0; u < GB; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0[u], b0v[u], acc, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < GB; ++u) { a0[u] = a1[u]; b0v[u] = b1[u]; }
        }
    }
    // accumulator v of lane l holds tile element (8 (v/4) + 4 (l/32) + v%4, l%32)
#pragma unroll
    for (int v = 0; v < 16; ++v) red[w][8 * (v >> 2) + 4 * kk + (v & 3)][lane & 31] = acc[v];
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const int i = e >> 5, jj = e & 31;
        const int gi = tr * 32 + i, gj = tc * 32 + jj;
        if (gi < R && gj < R) {
            const double s = ((double)red[0][i][jj] + (double)red[1][i][jj]) + ((double)red[2][i][jj] + (double)red[3][i][jj]);
            partial[(int64_t)blockIdx.x * R * R + (int64_t)gi * R + gj] = s;
        }
    }
}

// out[e] = sum_b partial[b][e] (b < nblk): one wave per element, lane t sums
// b = t, t + 64, ..., then a butterfly; fixed order, so repeatable.
__global__ __launch_bounds__(64) void sum_blocks_kernel(const double *__restrict__ partial, int64_t nblk,
                                                        int64_t n_per, double *__restrict__ out)
{
    const int64_t e = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 64) s += partial[b * n_per + e];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) out[e] = s;
}

// One workgroup: V = Hadamard of the Grams but mode n; W = V^-1 by
// Gauss-Jordan elimination without row exchanges (lane k of each wave owns
// column k, the four waves share its rows; the pivots are the
// Schur-complement diagonal, i.e. the squared Cholesky pivots of V = L L^T), or V^+ from a cyclic Jacobi eigendecomposition when
// a pivot is <= 0 or below 1e-13 * max(diag V).  flags[n] = 1 when the
// pseudo-inverse was used.  R <= kMaxCpR.  V is inverted in place in LDS;
// the Jacobi fallback keeps its eigenvectors in tmp (global, R x R).
__device__ void form_hadamard(const double *__restrict__ grams, int N, int n, int R,
                              double (*V)[kMaxCpR + 1])
{
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        double h = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != n) h *= grams[(int64_t)m * R * R + e];
        V[e / R][e % R] = h;
    }
}

__global__ __launch_bounds__(256) void als_solve_kernel(const double *__restrict__ grams, int N, int n,
                                                        int R, double *__restrict__ W,
                                                        double *__restrict__ tmp, int *__restrict__ flags)
{
    __shared__ double V[kMaxCpR][kMaxCpR + 1];
    __shared__ double rj[kMaxCpR], cj[kMaxCpR];
    __shared__ double cs_s[2];
    const int tid = threadIdx.x;
    const int k = tid & 63;                         // column of this lane
    const int q = tid >> 6;                         // rows q, q + 4, q + 8, ... of that column
    form_hadamard(grams, N, n, R, V);
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < R; ++i) dmax = V[i][i] > dmax ? V[i][i] : dmax;
    bool fail = false;
    constexpr int RPL = kMaxCpR / 4;                // rows per lane at most
    for (int j = 0; j < R; ++j) {
        const double p = V[j][j];                   // Schur-complement pivot (same on every lane)
        if (!(p > 0.0) || p <= 1e-13 * dmax) { fail = true; break; }
        if (tid < R) {
            rj[tid] = V[j][tid];
            cj[tid] = V[tid][j];
        }
        __syncthreads();
        const double ip = 1.0 / p;
        if (k < R) {
            const double rjk = rj[k] * ip;
            // rows i != j: a - c_i rjk (column j: -c_i / p); row j is set below
            double a[RPL], c[RPL];
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int i = q + 4 * u;
                const int ic = i < R ? i : 0;
                a[u] = V[ic][k];
                c[u] = cj[ic];
            }
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int i = q + 4 * u;
                const double t = a[u] - c[u] * rjk;
                const double tc = -c[u] * ip;
                if (i < R) V[i][k] = k == j ? tc : t;
            }
        }
        __syncthreads();
        if (tid < R) V[j][tid] = tid == j ? ip : rj[tid] * ip;
        __syncthreads();
    }
    if (!fail) {
        for (int e = tid; e < R * R; e += 256) W[e] = V[e / R][e % R];
        if (tid == 0) flags[n] = 0;
        return;
    }
    // ---- pseudo-inverse: cyclic Jacobi on V (symmetric), eigenvectors in tmp
    __syncthreads();
    form_hadamard(grams, N, n, R, V);
    for (int e = tid; e < R * R; e += 256) tmp[e] = (e / R == e % R) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int p = 0; p < R - 1; ++p) {
            for (int q = p + 1; q < R; ++q) {
                if (tid == 0) {
                    const double apq = V[p][q];
                    double c = 1.0, sn = 0.0;
                    if (fabs(apq) > 1e-300) {
                        const double theta = (V[q][q] - V[p][p]) / (2.0 * apq);
                        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                    cs_s[0] = c;
                    cs_s[1] = sn;
                }
                __syncthreads();
                const double c = cs_s[0], sn = cs_s[1];
                if (sn != 0.0) {
                    // V <- J^T V J, J the rotation in the (p, q) plane; eigenvectors <- Q J
                    for (int k = tid; k < R; k += 256) {
                        const double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - sn * vkq;
                        V[k][q] = sn * vkp + c * vkq;
                    }
                    __syncthreads();
                    for (int k = tid; k < R; k += 256) {
                        const double vpk = V[p][k], vqk = V[q][k];
                        V[p][k] = c * vpk - sn * vqk;
                        V[q][k] = sn * vpk + c * vqk;
                        const double qkp = tmp[k * R + p], qkq = tmp[k * R + q];
                        tmp[k * R + p] = c * qkp - sn * qkq;
                        tmp[k * R + q] = sn * qkp + c * qkq;
                    }
                }
                __syncthreads();
            }
        }
        // stop once the off-diagonal mass is negligible
        if (tid == 0) {
            double off = 0.0, dia = 0.0;
            for (int i = 0; i < R; ++i)
                for (int j = 0; j < R; ++j) {
                    if (i == j) dia += V[i][j] * V[i][j];
                    else off += V[i][j] * V[i][j];
                }
            cs_s[0] = (off <= 1e-30 * (dia > 0 ? dia : 1.0)) ? 1.0 : 0.0;
        }
        __syncthreads();
        const bool done = cs_s[0] != 0.0;
        __syncthreads();
        if (done) break;
    }
    double dm = 0.0;
    for (int i = 0; i < R; ++i) dm = V[i][i] > dm ? V[i][i] : dm;
    const double cut = (double)R * 2.220446049250313e-16 * dm;
    __syncthreads();
    for (int e = tid; e < R * R; e += 256) {
        const int i = e / R, j = e % R;
        double se = 0.0;
        for (int k = 0; k < R; ++k) {
            const double d = V[k][k];
            if (d > cut) se += tmp[i * R + k] * tmp[j * R + k] / d;
        }
        W[e] = se;
    }
    if (tid == 0) flags[n] = 1;
}


// Row solve, Y = M W (I x R, float64 accumulation), in row tiles staged in
// LDS with W.  Lane layout: 256 / RC row slots x RC columns (RC = R rounded
// up to a power of two, R <= kMaxCpR); a tile has RPT rows per slot.
//   STORE = false: per block, the column sums of Y^2 -> partial[blk][R];
//   STORE = true:  A(i, c) = Y(i, c) / lambda_c (0 when lambda_c = 0), stored
//                  as FT (bfloat16: round to nearest even).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int RC> struct RowTile {
    static constexpr int SLOTS = 256 / RC;
    static constexpr int RPT = RC >= 4 ? RC / 4 : 1;          // rows per slot per tile
    static constexpr int ROWS = SLOTS * RPT;                  // rows per tile (64 .. 256)
};

template <typename FT, int RC, bool STORE>
__global__ __launch_bounds__(256) void rowsolve_kernel(const float *__restrict__ M, const double *__restrict__ W,
                                                       const double *__restrict__ lambda, int64_t I, int R,
                                                       int tiles_per_block, double *__restrict__ partial,
                                                       FT *__restrict__ A)
{
    using RT = RowTile<RC>;
    __shared__ double sW[RC * RC];
    __shared__ float sM[RT::ROWS * (RC + 1)];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int slot = tid / RC, c = tid % RC;
    for (int e = tid; e < RC * RC; e += 256) {
        const int k = e / RC, cc = e % RC;
        sW[e] = (k < R && cc < R) ? W[k * R + cc] : 0.0;
    }
    const double lam = (STORE && c < R) ? lambda[c] : 0.0;
    double ss = 0.0;
    const int64_t first = (int64_t)blockIdx.x * tiles_per_block * RT::ROWS;
    for (int tt = 0; tt < tiles_per_block; ++tt) {
        const int64_t i0 = first + (int64_t)tt * RT::ROWS;
        if (i0 >= I) break;
        const int nrow = I - i0 < RT::ROWS ? (int)(I - i0) : RT::ROWS;
        __syncthreads();                                   // sW written / previous tile consumed
        for (int e = tid; e < nrow * R; e += 256) sM[(e / R) * (RC + 1) + e % R] = M[i0 * R + e];
        __syncthreads();
        double y[RT::RPT];
#pragma unroll
        for (int u = 0; u < RT::RPT; ++u) y[u] = 0.0;
        for (int k = 0; k < R; ++k) {
            const double wk = sW[k * RC + c];
#pragma unroll
            for (int u = 0; u < RT::RPT; ++u) y[u] += (double)sM[(u * RT::SLOTS + slot) * (RC + 1) + k] * wk;
        }
#pragma unroll
        for (int u = 0; u < RT::RPT; ++u) {
            const int r = u * RT::SLOTS + slot;
            if (r < nrow && c < R) {
                if constexpr (STORE) {
                    const double a = lam > 0.0 ? y[u] / lam : 0.0;
                    const int64_t o = (i0 + r) * R + c;
                    if constexpr (sizeof(FT) == 4) reinterpret_cast<float *>(A)[o] = (float)a;
                    else reinterpret_cast<uint16_t *>(A)[o] = f32_to_bf16_rne((float)a);
                } else {
                    ss += y[u] * y[u];
                }
            }
        }
    }
    if constexpr (!STORE) {
        red[tid] = ss;
        __syncthreads();
        if (tid < R) {
            double s = 0.0;
            for (int k = 0; k < RT::SLOTS; ++k) s += red[k * RC + tid];
            partial[(int64_t)blockIdx.x * R + tid] = s;
        }
    }
}

// lambda_c = sqrt(sum_b partial[b][c]): one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void lambda_kernel(const double *__restrict__ partial, int64_t nblk, int R,
                                                     double *__restrict__ lambda)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) s += partial[b * R + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lambda[c] = sqrt(red[0]);
}


// Fit, pass 1: per block, sum_i sum_r lambda_r M(i, r) A(i, r) in float64.
template <typename FT>
__global__ __launch_bounds__(256) void inner_kernel(const float *__restrict__ M, const FT *__restrict__ A,
                                                    const double *__restrict__ lambda, int64_t I, int R,
                                                    int rows_per_block, double *__restrict__ partial)
{
    __shared__ double red[256];
    const int64_t b0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t b1 = b0 + rows_per_block;
    if (b1 > I) b1 = I;
    double s = 0.0;
    for (int64_t e = b0 * R + threadIdx.x; e < b1 * R; e += 256) {
        const int r = (int)(e % R);
        float a;
        if constexpr (sizeof(FT) == 4) a = reinterpret_cast<const float *>(A)[e];
        else a = bf16_to_f32(reinterpret_cast<const uint16_t *>(A)[e]);
        s += lambda[r] * (double)M[e] * (double)a;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Fit, pass 2 (one workgroup).
__global__ __launch_bounds__(256) void fit_kernel(const double *__restrict__ partial, int64_t nblk,
                                                  const double *__restrict__ grams, int N, int R,
                                                  const double *__restrict__ lambda, double normX2,
                                                  double *__restrict__ fit)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) s += partial[b];
    double x2 = 0.0;
    for (int e = threadIdx.x; e < R * R; e += 256) {
        double h = 1.0;
        for (int m = 0; m < N; ++m) h *= grams[(int64_t)m * R * R + e];
        x2 += lambda[e / R] * h * lambda[e % R];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double inner = red[0];
    __syncthreads();
    red[threadIdx.x] = x2;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double xhat2 = red[0];
        double res2 = normX2 + xhat2 - 2.0 * inner;
        if (res2 < 0.0) res2 = 0.0;
        fit[0] = normX2 > 0.0 ? 1.0 - sqrt(res2) / sqrt(normX2) : 0.0;
    }
}

}  // namespace dev

static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

static int pow2_ceil(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Rows per row-solve tile for RC = R rounded up to a power of two.
static int rowsolve_rows(int RC)
{
    switch (RC) {
        case 1: return dev::RowTile<1>::ROWS;
        case 2: return dev::RowTile<2>::ROWS;
        case 4: return dev::RowTile<4>::ROWS;
        case 8: return dev::RowTile<8>::ROWS;
        case 16: return dev::RowTile<16>::ROWS;
        case 32: return dev::RowTile<32>::ROWS;
        default: return dev::RowTile<64>::ROWS;
    }
}

template <typename FT, bool STORE>
static hipError_t rowsolve_launch(int RC, int nblk, hipStream_t s, const float *M, const double *W,
                                  const double *lambda, int64_t I, int R, double *partial, FT *A)
{
    const dim3 g((unsigned)nblk), b(256);
    switch (RC) {
        case 1: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 1, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        case 2: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 2, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        case 4: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 4, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        case 8: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 8, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        case 16: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 16, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        case 32: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 32, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
        default: hipLaunchKernelGGL((dev::rowsolve_kernel<FT, 64, STORE>), g, b, 0, s, M, W, lambda, I, R, 1, partial, A); break;
    }
    return hipGetLastError();
}

// G = A^T A (float64) of an I x R factor; partials in ws->dbl.
static int gram_launch(fcoo_tensor *t, const void *A, int dtype, int64_t I, int R, double *G, hipStream_t s)
{
    const int nblk = ceil_div(I, dev::kGramRows);
    const int ntile = (R + 31) / 32;
    int rc = ensure_device_doubles(&t->ws.dbl, &t->ws.dbl_cap, (int64_t)nblk * R * R + 16, s);
    if (rc) return rc;
    if (dtype == FCOO_F32)
        hipLaunchKernelGGL(dev::gram_partial_kernel<float>, dim3(nblk, ntile * ntile), dim3(256), 0, s,
                           (const float *)A, I, R, t->ws.dbl);
    else
        hipLaunchKernelGGL(dev::gram_partial_kernel<dev::bf16raw>, dim3(nblk, ntile * ntile), dim3(256), 0, s,
                           (const dev::bf16raw *)A, I, R, t->ws.dbl);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::sum_blocks_kernel, dim3((unsigned)((int64_t)R * R)), dim3(64), 0, s,
                       t->ws.dbl, (int64_t)nblk, (int64_t)R * R, G);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}

}  // namespace fcoo

using namespace fcoo;

extern "C" {

int fcoo_gram(fcoo_tensor *t, int mode, const void *A, int dtype, int R, double *G, void *stream)
{
    clear_error();
    if (!t || !A || !G) return fail(FCOO_EINVAL, "null argument");
    if (mode < 0 || mode >= t->order) return fail(FCOO_EINVAL, "mode %d out of range", mode);
    if (dtype != FCOO_F32 && dtype != FCOO_BF16) return fail(FCOO_EUNSUPPORTED, "unknown dtype %d", dtype);
    if (R < 1 || R > kMaxR) return fail(FCOO_EUNSUPPORTED, "R = %d outside [1, %d]", R, kMaxR);
    return gram_launch(t, A, dtype, t->dims[mode], R, G, (hipStream_t)stream);
}

int fcoo_cp_als_iter(fcoo_tensor *t, void *const *factors, int dtype, int R, double *lambda,
                     double *grams, int grams_valid, double *fit, int *used_pinv, void *stream)
{
    clear_error();
    if (!t) return fail(FCOO_EINVAL, "null handle");
    int rc = check_factors(t, -1, (const void *const *)factors, dtype, R);
    if (rc) return rc;
    if (!lambda || !grams || !fit) return fail(FCOO_EINVAL, "lambda, grams or fit is NULL");
    if (R > dev::kMaxCpR) return fail(FCOO_EUNSUPPORTED, "cp_als_iter supports R <= %d (R = %d)", dev::kMaxCpR, R);
    const int N = t->order;
    for (int n = 0; n < N; ++n)
        if (!t->b[FCOO_OP_MTTKRP][n].built || !t->b[FCOO_OP_MTTKRP][n].on_device)
            return fail(FCOO_ENOTBUILT, "cp_als_iter needs the MTTKRP build of every mode (mode %d missing)", n);
    hipStream_t s = (hipStream_t)stream;
    int64_t maxI = 0;
    for (int n = 0; n < N; ++n) maxI = t->dims[n] > maxI ? t->dims[n] : maxI;
    if ((rc = ensure_device_floats(&t->ws.M, &t->ws.M_cap, maxI * R, s))) return rc;
    // scratch doubles: gram partials | W | tmp | block partials | fit
    const int RC = pow2_ceil(R);
    const int rows_tile = rowsolve_rows(RC);
    const int inner_rows = R < 8192 ? 8192 / R : 1;              // rows per fit-partial block
    const int64_t nblk_max = ceil_div(maxI, rows_tile < inner_rows ? rows_tile : inner_rows) + 1;
    const int64_t gram_need = (int64_t)ceil_div(maxI, dev::kGramRows) * R * R + 16;
    const int64_t need = 2 * (int64_t)R * R + nblk_max * R + 64 + gram_need;
    if ((rc = ensure_device_doubles(&t->ws.dbl, &t->ws.dbl_cap, need, s))) return rc;
    if (!t->ws.flags) FCOO_HIP(hipMalloc((void **)&t->ws.flags, 16 * sizeof(int)));
    if (!t->ws.host_pinned) FCOO_HIP(hipHostMalloc((void **)&t->ws.host_pinned, 64, hipHostMallocDefault));
    double *Wd = t->ws.dbl + gram_need;
    double *tmpd = Wd + (int64_t)R * R;
    double *part = tmpd + (int64_t)R * R;
    double *fitd = part + nblk_max * R;

    if (!grams_valid)
        for (int m = 0; m < N; ++m)
            if ((rc = gram_launch(t, factors[m], dtype, t->dims[m], R, grams + (int64_t)m * R * R, s))) return rc;

    // V_n needs only the Grams of the other modes, which are final before
    // SpMTTKRP_n starts: the solve runs on a second stream beside it
    if (!t->aux) {
        FCOO_HIP(hipStreamCreateWithFlags(&t->aux, hipStreamNonBlocking));
        FCOO_HIP(hipEventCreateWithFlags(&t->ev_dep, hipEventDisableTiming));
        FCOO_HIP(hipEventCreateWithFlags(&t->ev_solved, hipEventDisableTiming));
    }
    for (int n = 0; n < N; ++n) {
        const int64_t I = t->dims[n];
        FCOO_HIP(hipEventRecord(t->ev_dep, s));
        FCOO_HIP(hipStreamWaitEvent(t->aux, t->ev_dep, 0));
        hipLaunchKernelGGL(dev::als_solve_kernel, dim3(1), dim3(256), 0, t->aux, grams, N, n, R, Wd, tmpd,
                           t->ws.flags);
        FCOO_HIP(hipGetLastError());
        FCOO_HIP(hipEventRecord(t->ev_solved, t->aux));
        if ((rc = fcoo_spmttkrp(t, n, (const void *const *)factors, dtype, R, t->ws.M, stream))) return rc;
        FCOO_HIP(hipStreamWaitEvent(s, t->ev_solved, 0));
        const int nblk = ceil_div(I, rows_tile);
        hipError_t e = rowsolve_launch<float, false>(RC, nblk, s, t->ws.M, Wd, nullptr, I, R, part, nullptr);
        if (e != hipSuccess) return hip_fail(e, "row solve (norms)");
        hipLaunchKernelGGL(dev::lambda_kernel, dim3(R), dim3(256), 0, s, part, (int64_t)nblk, R, lambda);
        FCOO_HIP(hipGetLastError());
        if (dtype == FCOO_F32)
            e = rowsolve_launch<float, true>(RC, nblk, s, t->ws.M, Wd, lambda, I, R, nullptr, (float *)factors[n]);
        else
            e = rowsolve_launch<dev::bf16raw, true>(RC, nblk, s, t->ws.M, Wd, lambda, I, R, nullptr,
                                                    (dev::bf16raw *)factors[n]);
        if (e != hipSuccess) return hip_fail(e, "row solve (store)");
        if ((rc = gram_launch(t, factors[n], dtype, I, R, grams + (int64_t)n * R * R, s))) return rc;
    }
    const int64_t IN = t->dims[N - 1];
    const int nblk = ceil_div(IN, inner_rows);
    if (dtype == FCOO_F32)
        hipLaunchKernelGGL(dev::inner_kernel<float>, dim3(nblk), dim3(256), 0, s, t->ws.M,
                           (const float *)factors[N - 1], lambda, IN, R, inner_rows, part);
    else
        hipLaunchKernelGGL(dev::inner_kernel<dev::bf16raw>, dim3(nblk), dim3(256), 0, s, t->ws.M,
                           (const dev::bf16raw *)factors[N - 1], lambda, IN, R, inner_rows, part);
    FCOO_HIP(hipGetLastError());
    hipLaunchKernelGGL(dev::fit_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)nblk, grams, N, R, lambda,
                       t->normX2, fitd);
    FCOO_HIP(hipGetLastError());
    FCOO_HIP(hipMemcpyAsync(t->ws.host_pinned, fitd, sizeof(double), hipMemcpyDeviceToHost, s));
    int *hflags = reinterpret_cast<int *>(t->ws.host_pinned + 1);
    FCOO_HIP(hipMemcpyAsync(hflags, t->ws.flags, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, s));
    FCOO_HIP(hipStreamSynchronize(s));
    *fit = t->ws.host_pinned[0];
    if (used_pinv) {
        int bits = 0;
        for (int n = 0; n < N; ++n) bits |= (hflags[n] ? 1 : 0) << n;
        *used_pinv = bits;
    }
    return FCOO_OK;
}

}  // extern "C"

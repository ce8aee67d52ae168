// CP-ALS dense steps (Algorithm 1): Gram products on the matrix cores, the
// R x R float64 solve, the row solve with column normalisation, the fit, and
// the sweep driver fcoo_cp_als_iter.
//
// Per mode n of a sweep: M = SpMTTKRP_n (segmented-scan kernels);
// V = Hadamard product of the Grams G_m, m != n (float64);
// W = V^-1 by Cholesky (V = L L^T, W = L^-T L^-1), or the pseudo-inverse
// from a symmetric eigendecomposition (cyclic Jacobi) when V is not
// numerically positive definite; A_n = M W with column 2-norms lambda,
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
// summed in float64 and written to partial[blk][R x R].
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
    const int kk = lane >> 5;
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    if constexpr (sizeof(FT) == 4) {
        for (int64_t i = r0; i < r1; i += 2) {
            const int64_t row = i + kk;
            const float a = (row < r1 && ca < R) ? reinterpret_cast<const float *>(A)[row * R + ca] : 0.f;
            const float b = (row < r1 && cb < R) ? reinterpret_cast<const float *>(A)[row * R + cb] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    } else {
        const uint16_t *Ab = reinterpret_cast<const uint16_t *>(A);
        for (int64_t i = r0; i < r1; i += 8) {
            shortx4 a, b;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t row = i + 4 * kk + t;
                a[t] = (short)((row < r1 && ca < R) ? Ab[row * R + ca] : 0);
                b[t] = (short)((row < r1 && cb < R) ? Ab[row * R + cb] : 0);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
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

// out[e] = scale * sum_b partial[b][e], e < n_per, b in order.
__global__ __launch_bounds__(256) void sum_blocks_kernel(const double *__restrict__ partial, int64_t nblk,
                                                         int64_t n_per, double *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_per; e += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int64_t b = 0; b < nblk; ++b) s += partial[b * n_per + e];
        out[e] = s;
    }
}

// One workgroup: V = Hadamard of the Grams but mode n; W = V^-1 (Cholesky)
// or V^+ (cyclic Jacobi eigendecomposition) when a Cholesky pivot is <= 0
// or below 1e-13 * max(diag V).  flags[n] = 1 when the pseudo-inverse was
// used.  R <= kMaxCpR.  V lives in LDS (the Cholesky factor overwrites its
// lower triangle); tmp (R x R, global) holds L^-1 or the eigenvectors.
__device__ void form_hadamard(const double *__restrict__ grams, int N, int n, int R,
                              double (*V)[kMaxCpR + 1])
{
    for (int e = threadIdx.x; e < R * R; e += 256) {
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
    __shared__ double dmax_s, cs_s[2];
    __shared__ int fail_s;
    const int tid = threadIdx.x;
    form_hadamard(grams, N, n, R, V);
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        for (int i = 0; i < R; ++i) d = V[i][i] > d ? V[i][i] : d;
        dmax_s = d;
        fail_s = 0;
    }
    __syncthreads();
    // Cholesky in place (lower triangle), column by column
    for (int j = 0; j < R; ++j) {
        if (tid == 0) {
            double sj = V[j][j];
            for (int k = 0; k < j; ++k) sj -= V[j][k] * V[j][k];
            if (!(sj > 0.0) || sj <= 1e-13 * dmax_s) fail_s = 1;
            else V[j][j] = sqrt(sj);
        }
        __syncthreads();
        if (fail_s) break;
        for (int i = j + 1 + tid; i < R; i += 256) {
            double si = V[i][j];
            for (int k = 0; k < j; ++k) si -= V[i][k] * V[j][k];
            V[i][j] = si / V[j][j];
        }
        __syncthreads();
    }
    if (!fail_s) {
        // tmp = L^-1 (lower triangular): column c solves L x = e_c
        for (int c = tid; c < R; c += 256) {
            for (int i = 0; i < R; ++i) {
                if (i < c) { tmp[i * R + c] = 0.0; continue; }
                double si = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) si -= V[i][k] * tmp[k * R + c];
                tmp[i * R + c] = si / V[i][i];
            }
        }
        __syncthreads();
        // W = L^-T L^-1
        for (int e = tid; e < R * R; e += 256) {
            const int i = e / R, j = e % R;
            const int k0 = i > j ? i : j;
            double se = 0.0;
            for (int k = k0; k < R; ++k) se += tmp[k * R + i] * tmp[k * R + j];
            W[e] = se;
        }
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
    if (tid == 0) {
        double d = 0.0;
        for (int i = 0; i < R; ++i) d = V[i][i] > d ? V[i][i] : d;
        dmax_s = d;
    }
    __syncthreads();
    const double cut = (double)R * 2.220446049250313e-16 * dmax_s;
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

// Pass 1 of the row solve: per block of rows, sum_i (M W)(i, c)^2 in float64.
// Thread layout: 256 / RC row slots x RC columns (RC = R rounded up to a
// power of two, R <= kMaxCpR).
__global__ __launch_bounds__(256) void rowsolve_norm_kernel(const float *__restrict__ M,
                                                            const double *__restrict__ W, int64_t I,
                                                            int R, int RC, int rows_per_block,
                                                            double *__restrict__ partial)
{
    __shared__ double red[256];
    const int slots = 256 / RC;
    const int slot = threadIdx.x / RC, c = threadIdx.x % RC;
    const int64_t b0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t b1 = b0 + rows_per_block;
    if (b1 > I) b1 = I;
    double ss = 0.0;
    if (c < R) {
        for (int64_t i = b0 + slot; i < b1; i += slots) {
            const float *m = M + i * R;
            double y = 0.0;
            for (int k = 0; k < R; ++k) y += (double)m[k] * W[k * R + c];
            ss += y * y;
        }
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int k = 0; k < slots; ++k) s += red[k * RC + threadIdx.x];
        partial[(int64_t)blockIdx.x * R + threadIdx.x] = s;
    }
}

__global__ void lambda_kernel(const double *__restrict__ partial, int64_t nblk, int R,
                              double *__restrict__ lambda)
{
    const int c = threadIdx.x;
    if (c >= R) return;
    double s = 0.0;
    for (int64_t b = 0; b < nblk; ++b) s += partial[b * R + c];
    lambda[c] = sqrt(s);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Pass 2: A(i, c) = (M W)(i, c) / lambda_c (0 when lambda_c = 0), stored as FT.
template <typename FT>
__global__ __launch_bounds__(256) void rowsolve_store_kernel(const float *__restrict__ M,
                                                             const double *__restrict__ W,
                                                             const double *__restrict__ lambda, int64_t I,
                                                             int R, int RC, FT *__restrict__ A)
{
    const int slots = 256 / RC;
    const int slot = threadIdx.x / RC, c = threadIdx.x % RC;
    if (c >= R) return;
    const double lam = lambda[c];
    for (int64_t i = (int64_t)blockIdx.x * slots + slot; i < I; i += (int64_t)gridDim.x * slots) {
        const float *m = M + i * R;
        double y = 0.0;
        for (int k = 0; k < R; ++k) y += (double)m[k] * W[k * R + c];
        const double a = lam > 0.0 ? y / lam : 0.0;
        if constexpr (sizeof(FT) == 4) reinterpret_cast<float *>(A)[i * R + c] = (float)a;
        else reinterpret_cast<uint16_t *>(A)[i * R + c] = f32_to_bf16_rne((float)a);
    }
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
    hipLaunchKernelGGL(dev::sum_blocks_kernel, dim3(ceil_div((int64_t)R * R, 256)), dim3(256), 0, s,
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
    // scratch doubles: W (R*R) + lambda partials / inner partials + gram partials
    const int rows_pb = 4096;
    const int64_t nblk_max = ceil_div(maxI, rows_pb) + 1;
    const int64_t gram_need = (int64_t)ceil_div(maxI, dev::kGramRows) * R * R + 16;
    const int64_t need = 2 * (int64_t)R * R + nblk_max * R + 64 + gram_need;
    if ((rc = ensure_device_doubles(&t->ws.dbl, &t->ws.dbl_cap, need, s))) return rc;
    if (!t->ws.flags) FCOO_HIP(hipMalloc((void **)&t->ws.flags, 16 * sizeof(int)));
    if (!t->ws.host_pinned) FCOO_HIP(hipHostMalloc((void **)&t->ws.host_pinned, 64, hipHostMallocDefault));
    // layout of ws.dbl: [gram partials | W | block partials | fit]
    double *Wd = t->ws.dbl + gram_need;
    double *tmpd = Wd + (int64_t)R * R;
    double *part = tmpd + (int64_t)R * R;
    double *fitd = part + nblk_max * R;

    if (!grams_valid)
        for (int m = 0; m < N; ++m)
            if ((rc = gram_launch(t, factors[m], dtype, t->dims[m], R, grams + (int64_t)m * R * R, s))) return rc;

    const int RC = pow2_ceil(R);
    for (int n = 0; n < N; ++n) {
        const int64_t I = t->dims[n];
        if ((rc = fcoo_spmttkrp(t, n, (const void *const *)factors, dtype, R, t->ws.M, stream))) return rc;
        hipLaunchKernelGGL(dev::als_solve_kernel, dim3(1), dim3(256), 0, s, grams, N, n, R, Wd, tmpd,
                           t->ws.flags);
        FCOO_HIP(hipGetLastError());
        const int nblk = ceil_div(I, rows_pb);
        hipLaunchKernelGGL(dev::rowsolve_norm_kernel, dim3(nblk), dim3(256), 0, s, t->ws.M, Wd, I, R, RC,
                           rows_pb, part);
        FCOO_HIP(hipGetLastError());
        hipLaunchKernelGGL(dev::lambda_kernel, dim3(1), dim3(kMaxR), 0, s, part, (int64_t)nblk, R, lambda);
        FCOO_HIP(hipGetLastError());
        const int sgrid = ceil_div(I, 256 / RC) < 65535 * 4 ? ceil_div(I, 256 / RC) : 65535 * 4;
        if (dtype == FCOO_F32)
            hipLaunchKernelGGL(dev::rowsolve_store_kernel<float>, dim3(sgrid), dim3(256), 0, s, t->ws.M, Wd,
                               lambda, I, R, RC, (float *)factors[n]);
        else
            hipLaunchKernelGGL(dev::rowsolve_store_kernel<dev::bf16raw>, dim3(sgrid), dim3(256), 0, s, t->ws.M,
                               Wd, lambda, I, R, RC, (dev::bf16raw *)factors[n]);
        FCOO_HIP(hipGetLastError());
        if ((rc = gram_launch(t, factors[n], dtype, I, R, grams + (int64_t)n * R * R, s))) return rc;
    }
    const int64_t IN = t->dims[N - 1];
    const int nblk = ceil_div(IN, rows_pb);
    if (dtype == FCOO_F32)
        hipLaunchKernelGGL(dev::inner_kernel<float>, dim3(nblk), dim3(256), 0, s, t->ws.M,
                           (const float *)factors[N - 1], lambda, IN, R, rows_pb, part);
    else
        hipLaunchKernelGGL(dev::inner_kernel<dev::bf16raw>, dim3(nblk), dim3(256), 0, s, t->ws.M,
                           (const dev::bf16raw *)factors[N - 1], lambda, IN, R, rows_pb, part);
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

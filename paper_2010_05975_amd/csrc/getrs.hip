// Solve A X = B from the factors A = P L U (the problem statement of Sec. 2.2
// applied to a right-hand side; LAPACK getrs conventions).
//
// 1. perm: the ipiv interchanges composed into one gather (one workgroup,
//    the index array in LDS).
// 2. X = B[perm] (gather into a temporary, then back).
// 3. Forward substitution with unit L and back substitution with U, blocked
//    by 256 rows: a one-workgroup kernel solves the diagonal triangle, and the
//    FP64 MFMA update kernel applies the off-diagonal block to the remaining
//    rows (C -= L_block * X_block).
#include "cfx_internal.h"

namespace cfx {
namespace {

constexpr int kPermLds = 36864;   // n up to this uses the LDS permutation (144 KiB)
constexpr int TRB = 256;          // triangle block

__global__ __launch_bounds__(256) void perm_lds_kernel(const int32_t *ipiv, int n, int32_t *perm)
{
    __shared__ int32_t p[kPermLds];
    for (int i = threadIdx.x; i < n; i += 256) p[i] = i;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < n; ++i) {
            const int r = ipiv[i];
            if (r != i) { const int t = p[i]; p[i] = p[r]; p[r] = t; }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) perm[i] = p[i];
}

__global__ void perm_global_kernel(const int32_t *ipiv, int64_t n, int32_t *perm)
{
    if (threadIdx.x != 0) return;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = ipiv[i];
        if (r != i) { const int32_t t = perm[i]; perm[i] = perm[r]; perm[r] = t; }
    }
}

__global__ void gather_rows_kernel(const double *B, int64_t ldb, const int32_t *perm, int64_t n,
                                   int64_t nrhs, double *T)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e / nrhs, c = e - i * nrhs;
    T[e] = B[(int64_t)perm[i] * ldb + c];
}

__global__ void copy_back_kernel(const double *T, int64_t n, int64_t nrhs, double *B, int64_t ldb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e / nrhs, c = e - i * nrhs;
    B[i * ldb + c] = T[e];
}

// Triangle solve of the block rows r0 .. r0+bs of X (n x nrhs, stride ldx)
// in place.  lower != 0: unit lower L; else upper U (non-unit).
__global__ __launch_bounds__(256) void trsv_block_kernel(const double *LU, int64_t lda, double *X,
                                                         int64_t ldx, int64_t r0, int bs, int nrhs,
                                                         int lower)
{
    const int tid = threadIdx.x;
    if (lower) {
        for (int j = 0; j < bs; ++j) {
            // rows below j inside the block get x_i -= L_ij x_j
            for (int e = tid; e < (bs - j - 1) * nrhs; e += 256) {
                const int i = j + 1 + e / nrhs, c = e % nrhs;
                X[(r0 + i) * ldx + c] -= LU[(r0 + i) * lda + r0 + j] * X[(r0 + j) * ldx + c];
            }
            __syncthreads();
        }
    } else {
        for (int j = bs - 1; j >= 0; --j) {
            const double d = LU[(r0 + j) * lda + r0 + j];
            for (int c = tid; c < nrhs; c += 256) X[(r0 + j) * ldx + c] /= d;
            __syncthreads();
            for (int e = tid; e < j * nrhs; e += 256) {
                const int i = e / nrhs, c = e % nrhs;
                X[(r0 + i) * ldx + c] -= LU[(r0 + i) * lda + r0 + j] * X[(r0 + j) * ldx + c];
            }
            __syncthreads();
        }
    }
}

}  // namespace

int launch_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda, const int32_t *ipiv,
                 double *B, int64_t ldb, int32_t *perm, double *tmp, hipStream_t st)
{
    if (n == 0 || nrhs == 0) return CFX_OK;
    if (n <= kPermLds)
        hipLaunchKernelGGL(perm_lds_kernel, dim3(1), dim3(256), 0, st, ipiv, (int)n, perm);
    else
        hipLaunchKernelGGL(perm_global_kernel, dim3(1), dim3(64), 0, st, ipiv, n, perm);
    CFX_HIP(hipGetLastError());
    const int64_t tot = n * nrhs;
    const unsigned g = (unsigned)((tot + 255) / 256);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(g), dim3(256), 0, st, B, ldb, perm, n, nrhs, tmp);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(copy_back_kernel, dim3(g), dim3(256), 0, st, tmp, n, nrhs, B, ldb);
    CFX_HIP(hipGetLastError());

    // forward: L y = P b
    for (int64_t r0 = 0; r0 < n; r0 += TRB) {
        const int bs = (int)((n - r0) < TRB ? (n - r0) : TRB);
        hipLaunchKernelGGL(trsv_block_kernel, dim3(1), dim3(256), 0, st, LU, lda, B, ldb, r0, bs,
                           (int)nrhs, 1);
        CFX_HIP(hipGetLastError());
        const int64_t below = n - r0 - bs;
        if (below > 0) {
            int rc = launch_schur_f64(LU + (r0 + bs) * lda + r0, lda, B + r0 * ldb, ldb,
                                      B + (r0 + bs) * ldb, ldb, below, nrhs, bs, st);
            if (rc) return rc;
        }
    }
    // backward: U x = y
    int64_t nb = (n + TRB - 1) / TRB;
    for (int64_t b = nb - 1; b >= 0; --b) {
        const int64_t r0 = b * TRB;
        const int bs = (int)((n - r0) < TRB ? (n - r0) : TRB);
        hipLaunchKernelGGL(trsv_block_kernel, dim3(1), dim3(256), 0, st, LU, lda, B, ldb, r0, bs,
                           (int)nrhs, 0);
        CFX_HIP(hipGetLastError());
        if (r0 > 0) {
            int rc = launch_schur_f64(LU + r0, lda, B + r0 * ldb, ldb, B, ldb, r0, nrhs, bs, st);
            if (rc) return rc;
        }
    }
    return CFX_OK;
}

}  // namespace cfx

// Row interchanges of a panel and the two triangular solves (FactorizeA10,
// FactorizeA01 of Alg. 1; Sec. 7.2) on gfx950.
//
// The interchanges are the root's plan: at most 2*vb (destination, source)
// row pairs, applied to all n columns at once (the net effect of the vb
// sequential LAPACK-style interchanges).  Each workgroup owns a stripe of 16
// columns, reads every source value of its stripe into registers, then
// writes every destination, so no stripe depends on another.  The diagonal
// block of the panel is written from the root's factored block (L00\U00).
//
// L21 = A21 U00^{-1}: a workgroup owns 32 rows and the whole panel width,
// sweeps 32-column blocks left to right (update by the finished blocks, then
// substitution against the diagonal 32 x 32 triangle).  U12 = L00^{-1} A12:
// a workgroup owns 32 columns and sweeps 32-row blocks top to bottom.  Both
// work in LDS and write their strip back in place.
#include "cfx_internal.h"

namespace cfx {
namespace {

// ---------------------------------------------------------------------------
// laswp
// ---------------------------------------------------------------------------
constexpr int SW_COLS = 16;
constexpr int SW_SLOTS = 2 * kMaxV / (256 / SW_COLS);   // 32 pairs per thread

__global__ __launch_bounds__(256) void laswp_kernel(double *A, int64_t lda, int64_t n, int64_t k,
                                                    int vb, const int32_t *plan, const double *lu00)
{
    const int np = plan[0];
    const int32_t *dst = plan + 1;
    const int32_t *src = plan + 1 + 2 * kMaxV;
    const int64_t c = (int64_t)blockIdx.x * SW_COLS + (threadIdx.x & (SW_COLS - 1));
    const int q0 = threadIdx.x / SW_COLS;
    const bool in_panel = c >= k && c < k + vb;
    double vals[SW_SLOTS];
#pragma unroll
    for (int s = 0; s < SW_SLOTS; ++s) {
        const int q = q0 + s * (256 / SW_COLS);
        if (q < np && c < n) vals[s] = A[(int64_t)src[q] * lda + c];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SW_SLOTS; ++s) {
        const int q = q0 + s * (256 / SW_COLS);
        if (q < np && c < n) {
            const int64_t d = dst[q];
            if (!(in_panel && d < k + vb)) A[d * lda + c] = vals[s];
        }
    }
    if (in_panel)
        for (int j = q0; j < vb; j += 256 / SW_COLS)
            A[(k + j) * lda + c] = lu00[(int64_t)j * vb + (c - k)];
}

// ---------------------------------------------------------------------------
// triangular solves
// ---------------------------------------------------------------------------
constexpr int TB = 32;          // strip size and inner block
constexpr int XLD = kMaxV + 1;  // padded strip row (L21 kernel)

// L21 strip: rows i0 .. i0+rows of A21 (m x vb), U00 upper (non-unit).
__device__ void trsm_l21_strip(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t i0,
                               double *smem)
{
    const int tid = threadIdx.x;
    double *Xs = smem;                    // TB x XLD
    double *Ub = smem + TB * XLD;         // (vb) x (TB+1): U[0:jb+TB, jb:jb+TB]
    const double *U = A + k * lda + k;
    double *X = A + (k + vb) * lda + k;
    const int rows = (int)((m - i0) < TB ? (m - i0) : TB);

    for (int e = tid; e < rows * vb; e += 256) {
        const int i = e / vb, c = e - i * vb;
        Xs[i * XLD + c] = X[(i0 + i) * lda + c];
    }
    for (int jb = 0; jb < vb; jb += TB) {
        const int bc = (vb - jb) < TB ? (vb - jb) : TB;
        for (int e = tid; e < (jb + bc) * bc; e += 256) {
            const int l = e / bc, c = e - l * bc;
            Ub[l * (TB + 1) + c] = U[l * lda + jb + c];
        }
        __syncthreads();
        // update by finished blocks: T = X[:, jb:jb+bc] - X[:, 0:jb] U[0:jb, jb:jb+bc]
        {
            const int i = tid >> 3, c4 = (tid & 7) * 4;
            if (i < rows && jb > 0) {
                double acc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = (c4 + q < bc) ? Xs[i * XLD + jb + c4 + q] : 0.0;
                for (int l = 0; l < jb; ++l) {
                    const double x = Xs[i * XLD + l];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] -= x * Ub[l * (TB + 1) + c4 + q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (c4 + q < bc) Xs[i * XLD + jb + c4 + q] = acc[q];
            }
        }
        __syncthreads();
        // substitution against the diagonal triangle
        if (tid < rows) {
            double *xi = Xs + tid * XLD + jb;
            for (int j = 0; j < bc; ++j) {
                double s = xi[j];
                for (int l = 0; l < j; ++l) s -= xi[l] * Ub[(jb + l) * (TB + 1) + j];
                const double d = Ub[(jb + j) * (TB + 1) + j];
                xi[j] = d != 0.0 ? s / d : s;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < rows * vb; e += 256) {
        const int i = e / vb, c = e - i * vb;
        X[(i0 + i) * lda + c] = Xs[i * XLD + c];
    }
}

// U12 strip: columns j0 .. j0+cols of A12 (vb x m), L00 unit lower.
__device__ void trsm_u12_strip(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t j0,
                               double *smem)
{
    const int tid = threadIdx.x;
    double *Xs = smem;                       // vb x (TB+1)
    double *Lb = smem + kMaxV * (TB + 1);    // TB x XLD: L[jb:jb+TB, 0:jb+TB]
    const double *L = A + k * lda + k;
    double *X = A + k * lda + (k + vb);
    const int cols = (int)((m - j0) < TB ? (m - j0) : TB);

    for (int e = tid; e < vb * TB; e += 256) {
        const int l = e / TB, c = e - l * TB;
        if (c < cols) Xs[l * (TB + 1) + c] = X[l * lda + j0 + c];
    }
    for (int jb = 0; jb < vb; jb += TB) {
        const int bc = (vb - jb) < TB ? (vb - jb) : TB;
        for (int e = tid; e < bc * (jb + bc); e += 256) {
            const int j = e / (jb + bc), l = e - j * (jb + bc);
            Lb[j * XLD + l] = L[(jb + j) * lda + l];
        }
        __syncthreads();
        {
            const int c = tid & 31, j4 = (tid >> 5) * 4;
            if (c < cols && jb > 0) {
                double acc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = (j4 + q < bc) ? Xs[(jb + j4 + q) * (TB + 1) + c] : 0.0;
                for (int l = 0; l < jb; ++l) {
                    const double x = Xs[l * (TB + 1) + c];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] -= Lb[(j4 + q) * XLD + l] * x;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j4 + q < bc) Xs[(jb + j4 + q) * (TB + 1) + c] = acc[q];
            }
        }
        __syncthreads();
        if (tid < cols) {
            for (int j = 1; j < bc; ++j) {
                double s = Xs[(jb + j) * (TB + 1) + tid];
                for (int l = 0; l < j; ++l) s -= Lb[j * XLD + jb + l] * Xs[(jb + l) * (TB + 1) + tid];
                Xs[(jb + j) * (TB + 1) + tid] = s;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < vb * TB; e += 256) {
        const int l = e / TB, c = e - l * TB;
        if (c < cols) X[l * lda + j0 + c] = Xs[l * (TB + 1) + c];
    }
}

constexpr size_t kTrsmLds = (size_t)(TB * XLD + kMaxV * (TB + 1)) * sizeof(double);

__global__ __launch_bounds__(256) void trsm_kernel(double *A, int64_t lda, int64_t k, int vb, int64_t m,
                                                   int nstrips)
{
    extern __shared__ double smem[];
    if ((int)blockIdx.x < nstrips)
        trsm_l21_strip(A, lda, k, vb, m, (int64_t)blockIdx.x * TB, smem);
    else
        trsm_u12_strip(A, lda, k, vb, m, (int64_t)(blockIdx.x - nstrips) * TB, smem);
}

__global__ void set_int_kernel(int32_t *p, int32_t v) { *p = v; }

}  // namespace

int launch_laswp(double *A, int64_t lda, int64_t n, int64_t k, int vb, const Workspace &ws,
                 hipStream_t st)
{
    const int64_t grid = (n + SW_COLS - 1) / SW_COLS;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)grid), dim3(256), 0, st, A, lda, n, k, vb,
                       (const int32_t *)ws.plan, (const double *)ws.lu00);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_trsm(double *A, int64_t lda, int64_t k, int vb, int64_t m, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        CFX_HIP(hipFuncSetAttribute((const void *)trsm_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrsmLds));
        attr_set = true;
    }
    if (m <= 0) return CFX_OK;
    const int nstrips = (int)((m + TB - 1) / TB);
    hipLaunchKernelGGL(trsm_kernel, dim3(2 * nstrips), dim3(256), kTrsmLds, st, A, lda, k, vb, m, nstrips);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_set_int(int32_t *p, int32_t value, hipStream_t st)
{
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, value);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

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
// L21 = A21 U00^{-1} and U12 = L00^{-1} A12 are one solve shape: X U = B
// with U upper triangular, for X = L21 (U = U00) and for X = U12^T
// (U = L00^T, unit diagonal).  One wavefront owns a strip of 16 rows of X
// (16 rows of L21, or 16 columns of U12 read transposed) in LDS and sweeps
// 32-column blocks left to right: the finished blocks are applied on the
// FP64 matrix cores (X_b -= X_{<b} U_{<b,b}), then each lane solves one row
// against the 32 x 32 diagonal triangle by substitution with true division
// (a zero diagonal leaves that column unscaled).
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
constexpr int TSB = 32;               // diagonal block of the solve
constexpr int TSR = 16;               // rows of X per wavefront
constexpr int XLD = kMaxV + 4;        // padded LDS row of the strip

typedef double d4t __attribute__((ext_vector_type(4)));

// U(r, c) of the solve: U00 for L21 (mode 0), L00^T for U12 (mode 1).
template <int MODE>
__device__ __forceinline__ double uval(const double *P, int64_t lda, int r, int c)
{
    if constexpr (MODE == 0) return P[(int64_t)r * lda + c];
    else return r == c ? 1.0 : P[(int64_t)c * lda + r];
}

template <int MODE>
__global__ __launch_bounds__(64) void trsm_kernel(double *A, int64_t lda, int64_t k, int vb, int64_t m)
{
    __shared__ double X[TSR][XLD];
    __shared__ double Ub[TSB][TSB + 1];
    const int lane = threadIdx.x;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * TSR;
    const int rows = (m - r0) < TSR ? (int)(m - r0) : TSR;
    const double *P = A + k * lda + k;     // the panel's diagonal block
    // X[i][c]: L21 row r0+i (mode 0) or U12 column r0+i (mode 1)
    auto xaddr = [&](int i, int c) -> double * {
        if constexpr (MODE == 0) return A + (k + vb + r0 + i) * lda + k + c;
        else return A + (k + c) * lda + k + vb + r0 + i;
    };
    for (int e = lane; e < TSR * vb; e += 64) {
        int i, c;
        if constexpr (MODE == 0) { i = e / vb; c = e - i * vb; }
        else { c = e / TSR; i = e - c * TSR; }      // 16 consecutive columns of A12 per row
        X[i][c] = i < rows ? *xaddr(i, c) : 0.0;
    }
    __syncthreads();
    for (int b0 = 0; b0 < vb; b0 += TSB) {
        const int bc = (vb - b0) < TSB ? (vb - b0) : TSB;
        // X_b -= X[:, 0:b0] U[0:b0, b0:b0+bc] (two 16 x 16 tiles)
        if (b0 > 0) {
            d4t acc[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[t][q] = X[lk + 4 * q][b0 + 16 * t + lr];
            // b0 is a multiple of 32: chunks of 8 k-steps, all operand loads
            // of a chunk issued before its matrix-core operations
            const bool c0ok = b0 + lr < vb, c1ok = b0 + 16 + lr < vb;
            for (int kc = 0; kc < b0; kc += 32) {
                double av[8], bv[8][2];
#pragma unroll
                for (int s8 = 0; s8 < 8; ++s8) {
                    const int kr = kc + 4 * s8 + lk;
                    av[s8] = -X[lr][kr];
                    bv[s8][0] = c0ok ? uval<MODE>(P, lda, kr, b0 + lr) : 0.0;
                    bv[s8][1] = c1ok ? uval<MODE>(P, lda, kr, b0 + 16 + lr) : 0.0;
                }
#pragma unroll
                for (int s8 = 0; s8 < 8; ++s8)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s8], bv[s8][t], acc[t], 0, 0, 0);
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = b0 + 16 * t + lr;
                    if (c < vb) X[lk + 4 * q][c] = acc[t][q];
                }
        }
        // the diagonal block of U
        for (int e = lane; e < bc * bc; e += 64) {
            const int r = e / bc, c = e - r * bc;
            Ub[r][c] = uval<MODE>(P, lda, b0 + r, b0 + c);
        }
        __syncthreads();
        if (lane < TSR) {
            double x[TSB];
#pragma unroll
            for (int j = 0; j < TSB; ++j) x[j] = j < bc ? X[lane][b0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < TSB; ++j) {
                if (j < bc) {
                    double sj = x[j];
#pragma unroll
                    for (int l = 0; l < j; ++l) sj -= x[l] * Ub[l][j];
                    if constexpr (MODE == 0) {
                        const double d = Ub[j][j];
                        x[j] = d != 0.0 ? sj / d : sj;
                    } else {
                        x[j] = sj;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < TSB; ++j)
                if (j < bc) X[lane][b0 + j] = x[j];
        }
        __syncthreads();
    }
    for (int e = lane; e < TSR * vb; e += 64) {
        int i, c;
        if constexpr (MODE == 0) { i = e / vb; c = e - i * vb; }
        else { c = e / TSR; i = e - c * TSR; }
        if (i < rows) *xaddr(i, c) = X[i][c];
    }
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
    if (m <= 0) return CFX_OK;
    const unsigned g = (unsigned)((m + TSR - 1) / TSR);
    hipLaunchKernelGGL(trsm_kernel<0>, dim3(g), dim3(64), 0, st, A, lda, k, vb, m);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(trsm_kernel<1>, dim3(g), dim3(64), 0, st, A, lda, k, vb, m);
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

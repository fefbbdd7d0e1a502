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
// With row masking (Sec. 7.3, "Row Swapping vs. Row Masking") rows are not
// moved: a row map rm (logical row -> physical row) takes the place of the
// interchanges (rowmap_apply_kernel applies the plan to it, lu00_scatter
// writes the root's L00\U00 into the pivot rows where they are), and every
// kernel reaches logical row i at physical row rm[i].
//
// L21 = A21 U00^{-1} and U12 = L00^{-1} A12 are one solve shape: X U = B
// with U upper triangular, for X = L21 (U = U00) and for X = U12^T
// (U = L00^T, unit diagonal).  A workgroup of 4 wavefronts owns 64 rows of
// X (rows of L21, or columns of U12 read transposed), 16 per wavefront,
// kept in registers in the matrix cores' operand layout, and sweeps
// 32-column blocks left to right.  Per block the workgroup stages the U
// columns of the block once in LDS; each wavefront applies its finished
// blocks on the FP64 matrix cores (X_b -= X_{<b} U_{<b,b}), then solves its
// 16 rows against the 32 x 32 diagonal triangle by substitution, four lanes
// per row, with true division (a zero diagonal leaves that column
// unscaled).
#include <utility>

#include "cfx_internal.h"

namespace cfx {
namespace {

// ---------------------------------------------------------------------------
// laswp
// ---------------------------------------------------------------------------
constexpr int SW_COLS = 16;
constexpr int SW_SLOTS = 2 * kMaxV / (256 / SW_COLS);   // 32 pairs per thread

// Columns c0 + s for stripe positions s < split, c0 + skip + s after them,
// below n: the interchanges of one column range, or of all columns outside a
// window.
__global__ __launch_bounds__(256) void laswp_kernel(double *A, int64_t lda, int64_t n, int64_t k,
                                                    int vb, const int32_t *plan, const double *lu00,
                                                    int64_t c0, int64_t split, int64_t skip)
{
    // the plan's row indices are staged in LDS first, so that the row loads
    // below are all in flight together instead of each waiting for its index
    __shared__ int32_t s_src[2 * kMaxV], s_dst[2 * kMaxV];
    const int np = plan[0];
    for (int q = threadIdx.x; q < np; q += 256) {
        s_dst[q] = plan[1 + q];
        s_src[q] = plan[1 + 2 * kMaxV + q];
    }
    __syncthreads();
    const int64_t sp = (int64_t)blockIdx.x * SW_COLS + (threadIdx.x & (SW_COLS - 1));
    const int64_t c = c0 + sp + (sp >= split ? skip : 0);
    const int q0 = threadIdx.x / SW_COLS;
    const bool in_panel = c >= k && c < k + vb;
    double vals[SW_SLOTS];
#pragma unroll
    for (int s = 0; s < SW_SLOTS; ++s) {
        const int q = q0 + s * (256 / SW_COLS);
        if (q < np && c < n) vals[s] = A[(int64_t)s_src[q] * lda + c];
    }
    // one wait for every row load, on every path: the stores below then
    // need no wait of their own (a store's wait would also wait for the
    // stores before it)
    __builtin_amdgcn_s_waitcnt(0x0F70);           // vmcnt(0)
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SW_SLOTS; ++s) {
        const int q = q0 + s * (256 / SW_COLS);
        if (q < np && c < n) {
            const int64_t d = s_dst[q];
            if (!(in_panel && d < k + vb)) A[d * lda + c] = vals[s];
        }
    }
    if (in_panel)
        for (int j = q0; j < vb; j += 256 / SW_COLS)
            A[(k + j) * lda + c] = lu00[(int64_t)j * vb + (c - k)];
}

// Row masking: the plan's moves applied to the row map instead of the rows
// (all sources read before any destination is written; one workgroup).
__global__ __launch_bounds__(256) void rowmap_apply_kernel(int32_t *rm, const int32_t *plan)
{
    const int np = plan[0];
    const int32_t *dst = plan + 1;
    const int32_t *src = plan + 1 + 2 * kMaxV;
    int v[2 * kMaxV / 256];
#pragma unroll
    for (int s = 0; s < 2 * kMaxV / 256; ++s) {
        const int q = threadIdx.x + 256 * s;
        if (q < np) v[s] = rm[src[q]];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2 * kMaxV / 256; ++s) {
        const int q = threadIdx.x + 256 * s;
        if (q < np) rm[dst[q]] = v[s];
    }
}

// Row masking: the root's factored block L00\U00 into the panel columns of
// the pivot rows, where they are (one workgroup per pivot row).
__global__ __launch_bounds__(256) void lu00_scatter_kernel(double *A, int64_t lda, const int32_t *rm, int64_t k,
                                                           int vb, const double *lu00)
{
    const int j = blockIdx.x;
    double *row = A + (int64_t)rm[k + j] * lda + k;
    for (int c = threadIdx.x; c < vb; c += 256) row[c] = lu00[(int64_t)j * vb + c];
}

// Physical row of logical row i (identity without a row map).
__device__ __forceinline__ int64_t phys(const int32_t *rm, int64_t i) { return rm ? (int64_t)rm[i] : i; }

// ---------------------------------------------------------------------------
// triangular solves
// ---------------------------------------------------------------------------
constexpr int TSB = 32;               // diagonal block of the solve
constexpr int TSW = 16;               // rows of X per wavefront
constexpr int TSR = 4 * TSW;          // rows of X per workgroup
constexpr int ULD = TSB + 1;          // padded LDS row of the staged U block
constexpr int NCH = kMaxV / 4;        // 4-column chunks of a row of X

typedef double d4t __attribute__((ext_vector_type(4)));

template <typename F, int... J>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Lane q of every group of four lanes (DPP quad permutation), 64 bits.
template <int Q>
__device__ __forceinline__ double quad_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, Q * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Q * 0x55, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// U(r, c) of the solve: U00 for L21 (mode 0), L00^T for U12 (mode 1), from
// the panel's diagonal block (rows k.. through the row map, columns k..).
// Only r <= c is ever read.
// rmk: the panel rows' physical rows (rm[k + i], staged in LDS), or null.
__device__ __forceinline__ int64_t pk(const int32_t *rmk, int64_t k, int i) { return rmk ? (int64_t)rmk[i] : k + i; }
template <int MODE>
__device__ __forceinline__ double uval(const double *A, int64_t lda, const int32_t *rmk, int64_t k, int r, int c)
{
    if constexpr (MODE == 0) return A[pk(rmk, k, r) * lda + k + c];
    else return r == c ? 1.0 : A[pk(rmk, k, c) * lda + k + r];
}

// One workgroup: rows rbase .. rbase+64 (below rend) of X.  LDS:
//   Us  U[0 : c0+32, c0 : c0+32] of the current block (kMaxV x ULD)
//   Sb  per wavefront: the block's rows (inputs, then the solution)
//   Sg  per wavefront: X_{<b} U_{<b,b} of the block
template <int MODE>
__device__ __forceinline__ void trsm_body(double *A, int64_t lda, const int32_t *rm, const int32_t *rmk, int64_t k,
                                          int vb, int64_t rbase, int64_t rend, double *Us,
                                          double (*Sb)[TSW][ULD], double (*Sg)[TSW][ULD])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row = rbase + wave * TSW + lr;   // this lane's row of X
    const bool rok = row < rend;
    // L21: this lane's row of A21 (one physical row); U12^T: the panel
    // rows, column k + vb + row
    const int64_t xrow = MODE == 0 ? phys(rm, k + vb + (rok ? row : 0)) : 0;
    auto xaddr = [&](int c) -> double * {
        if constexpr (MODE == 0) return A + xrow * lda + k + c;
        else return A + pk(rmk, k, c) * lda + k + vb + row;
    };
    // xa[s] = X[row][4s + lk]: the A operand layout of v_mfma_f64_16x16x4f64
    // (lane l holds row l%16, column l/16 of each 16 x 4 slice)
    double xa[NCH];
    sfor<NCH>([&](auto SC) {
        constexpr int sc = decltype(SC)::value;
        const int c = 4 * sc + lk;
        xa[sc] = (rok && c < vb) ? *xaddr(c) : 0.0;
    });

    // U[0 : c0+32, c0 : c0+32] of block b, this thread's share in registers;
    // the next block's share is fetched while the current block computes
    // element i of this thread: (r, c) = (e / 32, e % 32) with e = tid + 256 i
    // for U00 (rows of 32 consecutive doubles), (tid, i) for L00^T (columns
    // of L00 read down, consecutive threads on consecutive addresses)
    constexpr int NPRE = kMaxV * TSB / 256;
    auto elem = [&](int i, int &r, int &c) {
        if constexpr (MODE == 0) { r = (tid + 256 * i) >> 5; c = tid & 31; }
        else { r = tid; c = i; }
    };
    double pre[NPRE];
    auto fetch_u = [&](int c0f) {
        const int bcf = (vb - c0f) < TSB ? (vb - c0f) : TSB;
        const int krf = c0f + bcf;
#pragma unroll
        for (int i = 0; i < NPRE; ++i) {
            int r, c;
            elem(i, r, c);
            pre[i] = (r < krf && c < bcf && r <= c0f + c) ? uval<MODE>(A, lda, rmk, k, r, c0f + c) : 0.0;
        }
    };
    fetch_u(0);

    sfor<kMaxV / TSB>([&](auto BC) {
        constexpr int b = decltype(BC)::value;
        constexpr int c0 = TSB * b;
        if (c0 < vb) {
            const int bc = (vb - c0) < TSB ? (vb - c0) : TSB;
            const int kr = c0 + bc;
            __syncthreads();                    // the previous block's readers are done
#pragma unroll
            for (int i = 0; i < NPRE; ++i) {
                int r, c;
                elem(i, r, c);
                if (r < kr) Us[r * ULD + c] = pre[i];
            }
            if (c0 + TSB < vb) fetch_u(c0 + TSB);
            // the block's current values, operand layout -> rows
            sfor<TSB / 4>([&](auto SC) {
                constexpr int sc = decltype(SC)::value;
                Sb[wave][lr][4 * sc + lk] = xa[TSB / 4 * b + sc];
            });
            __syncthreads();
            // X_{<b} U_{<b,b} on the matrix cores (two 16 x 16 tiles)
            d4t g0 = {0.0, 0.0, 0.0, 0.0}, g1 = {0.0, 0.0, 0.0, 0.0};
            sfor<TSB / 4 * b>([&](auto SC) {
                constexpr int sc = decltype(SC)::value;
                const double u0 = Us[(4 * sc + lk) * ULD + lr];
                const double u1 = Us[(4 * sc + lk) * ULD + 16 + lr];
                g0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[sc], u0, g0, 0, 0, 0);
                g1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[sc], u1, g1, 0, 0, 0);
            });
            // result layout: lane l holds rows l/16 + 4q of column l%16
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Sg[wave][lk + 4 * q][lr] = g0[q];
                Sg[wave][lk + 4 * q][16 + lr] = g1[q];
            }
            __syncthreads();
            {
                // substitution against the diagonal triangle by all 64 lanes:
                // lanes 4r .. 4r+3 hold row r of the wave's 16, eight columns
                // each (lane group sg: columns 8 sg .. 8 sg + 7).  Step j: the
                // lane holding column j finishes x_j (mode 0: divides it by
                // U[j][j]), a quad broadcast hands x_j to the row's other
                // lanes, and each lane applies x_c -= x_j U[j][c] to its
                // columns c > j; row j + 1 of the triangle is requested from
                // LDS meanwhile.  Per element: the same operations in the
                // same order (increasing j) as a row-by-row substitution.
                const int sr = lane >> 2, sg = lane & 3;
                double x[8], u[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    x[c] = Sb[wave][sr][8 * sg + c] - Sg[wave][sr][8 * sg + c];
                    u[c] = Us[c0 * ULD + 8 * sg + c];
                }
                sfor<TSB>([&](auto JC) {
                    constexpr int j = decltype(JC)::value;
                    constexpr int gj = j / 8, cj = j % 8;
                    if (j < bc) {
                        double un[8];
                        if (j + 1 < bc) {
#pragma unroll
                            for (int c = 0; c < 8; ++c) un[c] = Us[(c0 + j + 1) * ULD + 8 * sg + c];
                        }
                        if constexpr (MODE == 0) {
                            if (sg == gj) {
                                const double d = u[cj];
                                x[cj] = d != 0.0 ? x[cj] / d : x[cj];
                            }
                        }
                        const double xj = quad_bcast<gj>(x[cj]);
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            if (8 * sg + c > j) x[c] -= xj * u[c];
#pragma unroll
                        for (int c = 0; c < 8; ++c) u[c] = un[c];
                    }
                });
#pragma unroll
                for (int c = 0; c < 8; ++c) Sb[wave][sr][8 * sg + c] = x[c];
            }
            __syncthreads();
            sfor<TSB / 4>([&](auto SC) {
                constexpr int sc = decltype(SC)::value;
                xa[TSB / 4 * b + sc] = Sb[wave][lr][4 * sc + lk];
            });
        }
    });
    sfor<NCH>([&](auto SC) {
        constexpr int sc = decltype(SC)::value;
        const int c = 4 * sc + lk;
        if (rok && c < vb) *xaddr(c) = xa[sc];
    });
}

// With a row map, the panel rows' physical rows (rm[k .. k + vb)) are read
// once into LDS, so that the solve's loads of the panel rows do not each
// wait for a row-map lookup.
__device__ __forceinline__ void stage_panel_rows(const int32_t *rm, int64_t k, int vb, int32_t *rmk)
{
    if (!rm) return;
    for (int i = threadIdx.x; i < vb; i += blockDim.x) rmk[i] = rm[k + i];
    __syncthreads();
}

// Rows i0 .. i1 of one solve.
template <int MODE>
__global__ __launch_bounds__(256) void trsm_kernel(double *A, int64_t lda, const int32_t *rm, int64_t k, int vb,
                                                   int64_t i0, int64_t i1)
{
    __shared__ double Us[kMaxV * ULD];
    __shared__ double Sb[4][TSW][ULD];
    __shared__ double Sg[4][TSW][ULD];
    __shared__ int32_t rmk[kMaxV];
    stage_panel_rows(rm, k, vb, rmk);
    trsm_body<MODE>(A, lda, rm, rm ? rmk : nullptr, k, vb, i0 + (int64_t)blockIdx.x * TSR, i1, Us, Sb, Sg);
}

// Both solves in one launch: workgroups 0 .. g0 take the m rows of L21,
// the others the first n1 columns of U12.
__global__ __launch_bounds__(256) void trsm_pair_kernel(double *A, int64_t lda, const int32_t *rm, int64_t k,
                                                        int vb, int64_t m, int g0, int64_t n1)
{
    __shared__ double Us[kMaxV * ULD];
    __shared__ double Sb[4][TSW][ULD];
    __shared__ double Sg[4][TSW][ULD];
    __shared__ int32_t rmk[kMaxV];
    stage_panel_rows(rm, k, vb, rmk);
    const int32_t *rk = rm ? rmk : nullptr;
    if ((int)blockIdx.x < g0)
        trsm_body<0>(A, lda, rm, rk, k, vb, (int64_t)blockIdx.x * TSR, m, Us, Sb, Sg);
    else
        trsm_body<1>(A, lda, rm, rk, k, vb, (int64_t)(blockIdx.x - g0) * TSR, n1, Us, Sb, Sg);
}

__global__ void set_int_kernel(int32_t *p, int32_t v) { *p = v; }

}  // namespace

int launch_laswp(double *A, int64_t lda, int64_t n, int64_t k, int vb, const Workspace &ws,
                 hipStream_t st, int64_t w0, int64_t w1, bool window)
{
    // all n columns (w1 <= w0); the columns [w0, w1) (window); or all
    // columns but those
    int64_t c0 = 0, cols = n, split = n, skip = 0, end = n;
    if (w1 > w0) {
        if (window) {
            c0 = w0;
            cols = w1 - w0;
            split = cols;
            end = w1;
        } else {
            cols = n - (w1 - w0);
            split = w0;
            skip = w1 - w0;
        }
    }
    if (cols <= 0) return CFX_OK;
    const int64_t grid = (cols + SW_COLS - 1) / SW_COLS;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)grid), dim3(256), 0, st, A, lda, end, k, vb,
                       (const int32_t *)ws.plan, (const double *)ws.lu00, c0, split, skip);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_rowmap_apply(double *A, int64_t lda, int32_t *rm, int64_t k, int vb, const Workspace &ws,
                        hipStream_t st)
{
    hipLaunchKernelGGL(rowmap_apply_kernel, dim3(1), dim3(256), 0, st, rm, (const int32_t *)ws.plan);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(lu00_scatter_kernel, dim3((unsigned)vb), dim3(256), 0, st, A, lda, (const int32_t *)rm, k,
                       vb, (const double *)ws.lu00);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

__global__ void rowmap_init_kernel(int32_t *rm, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rm[i] = (int32_t)i;
}

int launch_rowmap_init(int32_t *rm, int64_t n, hipStream_t st)
{
    if (n <= 0) return CFX_OK;
    hipLaunchKernelGGL(rowmap_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rm, n);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_trsm_first(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t n1, hipStream_t st,
                      const int32_t *rm)
{
    if (m <= 0) return CFX_OK;
    n1 = n1 < m ? n1 : m;
    const int64_t g0 = (m + TSR - 1) / TSR, g1 = (n1 + TSR - 1) / TSR;
    if (g0 + g1 > INT32_MAX) return CFX_ENOTSUP;
    hipLaunchKernelGGL(trsm_pair_kernel, dim3((unsigned)(g0 + g1)), dim3(256), 0, st, A, lda, rm, k, vb, m,
                       (int)g0, n1);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_trsm_rest(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t n1, hipStream_t st,
                     const int32_t *rm)
{
    if (n1 >= m) return CFX_OK;
    const unsigned g = (unsigned)((m - n1 + TSR - 1) / TSR);
    hipLaunchKernelGGL(trsm_kernel<1>, dim3(g), dim3(256), 0, st, A, lda, rm, k, vb, n1, m);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_trsm(double *A, int64_t lda, int64_t k, int vb, int64_t m, hipStream_t st, const int32_t *rm)
{
    return launch_trsm_first(A, lda, k, vb, m, m, st, rm);
}

int launch_set_int(int32_t *p, int32_t value, hipStream_t st)
{
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, value);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

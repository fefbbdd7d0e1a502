// FP64 GMRES-based iterative refinement around a (possibly mixed-precision)
// tournament-pivoted LU: the factorisation of Alg. 1 with its Schur updates
// in BF16/FP16 serves as the preconditioner M = U^{-1} L^{-1} P of GMRES on
// M A d = M r, and the solution is refined in FP64 until the normwise
// backward error eta = |b - A x|_inf / (|A|_inf |x|_inf + |b|_inf) reaches
// the target.  This is GMRES-IR in the form of Carson and Higham (SIAM J.
// Sci. Comput. 2018); the paper itself does not treat refinement.
//
// Device kernels here: the residual r = b - A x with compensated (Dot2,
// Ogita-Rump-Oishi) row sums, so that eta is not limited by the rounding
// of the residual itself; plain FP64 A v; deterministic block dot products
// and vector combinations for classical Gram-Schmidt with one
// re-orthogonalisation.  The small Hessenberg least-squares problem is
// solved on the host with Givens rotations.
#include <cmath>
#include <new>
#include <vector>

#include "cfx_internal.h"

// The compensated sums below rely on each product and sum being rounded
// separately: no contraction into fused multiply-adds in this file.
#pragma clang fp contract(off)

namespace cfx {
namespace {

constexpr int kDotBlocks = 256;

// max that propagates NaN (fmax would drop it and hide a failed solve)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// One wavefront per row.  RES: out_i = b_i - A_i x with a compensated dot
// product, and rowabs_i = sum_j |A_ij| when rowabs is not null.  Otherwise
// out_i = A_i x in plain FP64.
template <bool RES>
__global__ __launch_bounds__(256) void gemv_kernel(const double *__restrict__ A, int64_t lda, int64_t n,
                                                   const double *__restrict__ x, const double *__restrict__ b,
                                                   double *__restrict__ out, double *__restrict__ rowabs)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double *row = A + i * lda;
    if constexpr (RES) {
        double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0, ab = 0.0;
        int64_t j = lane;
        if (((((uintptr_t)row) | (uintptr_t)x) & 15) == 0) {
            // 16-byte loads: the two elements of a pair go to the two sums
            const double2 *row2 = reinterpret_cast<const double2 *>(row);
            const double2 *x2 = reinterpret_cast<const double2 *>(x);
            int64_t j2 = lane;
#pragma unroll 4
            for (; j2 < n / 2; j2 += 64) {
                const double2 a = row2[j2], xv = x2[j2];
                const double p0 = a.x * xv.x, p1 = a.y * xv.y;
                const double e0 = fma(a.x, xv.x, -p0), e1 = fma(a.y, xv.y, -p1);
                double t0, t1;
                two_sum(s0, p0, s0, t0);
                two_sum(s1, p1, s1, t1);
                c0 += t0 + e0;
                c1 += t1 + e1;
                ab += fabs(a.x) + fabs(a.y);
            }
            j = (n & 1) && lane == 0 ? n - 1 : n;   // the odd last element
        }
        for (; j + 64 < n; j += 128) {
            const double a0 = row[j], a1 = row[j + 64];
            const double p0 = a0 * x[j], p1 = a1 * x[j + 64];
            const double e0 = fma(a0, x[j], -p0), e1 = fma(a1, x[j + 64], -p1);
            double t0, t1;
            two_sum(s0, p0, s0, t0);
            two_sum(s1, p1, s1, t1);
            c0 += t0 + e0;
            c1 += t1 + e1;
            ab += fabs(a0) + fabs(a1);
        }
        if (j < n) {
            const double a0 = row[j];
            const double p0 = a0 * x[j];
            const double e0 = fma(a0, x[j], -p0);
            double t0;
            two_sum(s0, p0, s0, t0);
            c0 += t0 + e0;
            ab += fabs(a0);
        }
        double s, t;
        two_sum(s0, s1, s, t);
        double c = c0 + c1 + t;
        for (int off = 32; off >= 1; off >>= 1) {
            const double so = __shfl_xor(s, off), co = __shfl_xor(c, off);
            two_sum(s, so, s, t);
            c += co + t;
            ab += __shfl_xor(ab, off);
        }
        if (lane == 0) {
            double u, e;
            two_sum(b[i], -s, u, e);
            out[i] = u + (e - c);
            if (rowabs) rowabs[i] = ab;
        }
    } else {
        double s0 = 0.0, s1 = 0.0;
        int64_t j = lane;
        for (; j + 64 < n; j += 128) {
            s0 += row[j] * x[j];
            s1 += row[j + 64] * x[j + 64];
        }
        if (j < n) s0 += row[j] * x[j];
        double s = s0 + s1;
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) out[i] = s;
    }
}

// out_i = A_i x in plain FP64, one wavefront per row, for rows and x
// aligned to 16 bytes: each lane loads two consecutive elements at a time
// and keeps four loads of the row in flight (four partial sums), so that
// more of the row is requested at once than with one 8-byte load per lane.
__global__ __launch_bounds__(256) void gemv_plain_kernel(const double *__restrict__ A, int64_t lda, int64_t n,
                                                         const double *__restrict__ x, double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double2 *row = reinterpret_cast<const double2 *>(A + i * lda);
    const double2 *x2 = reinterpret_cast<const double2 *>(x);
    const int64_t n2 = n / 2;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t j = lane;
    for (; j + 192 < n2; j += 256) {
        double2 a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = row[j + 64 * q];
            b[q] = x2[j + 64 * q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += a[q].x * b[q].x + a[q].y * b[q].y;
    }
    for (; j < n2; j += 64) {
        const double2 a = row[j], b = x2[j];
        s[0] += a.x * b.x + a.y * b.y;
    }
    if ((n & 1) && lane == 0) s[1] += A[i * lda + n - 1] * x[n - 1];
    double t = (s[0] + s[1]) + (s[2] + s[3]);
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) out[i] = t;
}

// partial[k * nblk + blk] = sum over this block's slice of V_k . w
// (V_k = V + k * ldv), k < nv; fixed reduction order.
__global__ __launch_bounds__(256) void dots_kernel(const double *__restrict__ V, int64_t ldv, int nv,
                                                   const double *__restrict__ w, int64_t n, int64_t chunk,
                                                   double *__restrict__ partial)
{
    __shared__ double red[256];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int k = 0; k < nv; ++k) {
        const double *vk = V + (int64_t)k * ldv;
        double s = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += vk[i] * w[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[k] = sum_b partial[k * nblk + b] (MAX: max instead of sum).
template <bool MAX>
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial, int nblk, int nv,
                                                     double *__restrict__ out)
{
    __shared__ double red[256];
    for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) {
            const double p = partial[(int64_t)k * nblk + b];
            s = MAX ? nanmax(s, p) : s + p;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o)
                red[threadIdx.x] = MAX ? nanmax(red[threadIdx.x], red[threadIdx.x + o])
                                       : red[threadIdx.x] + red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

// partial[v * nblk + blk] = max |vec_v| over this block's slice, for the
// nv vectors vec_v = X + v * ldv.
__global__ __launch_bounds__(256) void amax_kernel(const double *__restrict__ X, int64_t ldv, int nv, int64_t n,
                                                   int64_t chunk, double *__restrict__ partial)
{
    __shared__ double red[256];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int k = 0; k < nv; ++k) {
        const double *vk = X + (int64_t)k * ldv;
        double s = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s = nanmax(s, fabs(vk[i]));
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// w_i += sign * sum_{k < nv} coef[k] V_k[i]   (k in order)
__global__ void vcomb_kernel(double *__restrict__ w, const double *__restrict__ V, int64_t ldv, int nv,
                             const double *__restrict__ coef, double sign, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < nv; ++k) s += coef[k] * V[(int64_t)k * ldv + i];
    w[i] += sign * s;
}

__global__ void scale_kernel(double *__restrict__ dst, const double *__restrict__ src, double alpha, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = alpha * src[i];
}

unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int launch_gemv(const double *A, int64_t lda, int64_t n, const double *x, double *y, hipStream_t st)
{
    if (n <= 0) return CFX_OK;
    if ((((uintptr_t)A | (uintptr_t)x) & 15) == 0 && lda % 2 == 0)
        hipLaunchKernelGGL(gemv_plain_kernel, dim3(blocks_of(n, 4)), dim3(256), 0, st, A, lda, n, x, y);
    else
        hipLaunchKernelGGL(gemv_kernel<false>, dim3(blocks_of(n, 4)), dim3(256), 0, st, A, lda, n, x,
                           (const double *)nullptr, y, (double *)nullptr);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_residual(const double *A, int64_t lda, int64_t n, const double *x, const double *b, double *r,
                    double *rowabs, hipStream_t st)
{
    if (n <= 0) return CFX_OK;
    hipLaunchKernelGGL(gemv_kernel<true>, dim3(blocks_of(n, 4)), dim3(256), 0, st, A, lda, n, x, b, r, rowabs);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

// ---------------------------------------------------------------------------
// Device vectors of one refinement (all n doubles unless stated).
// ---------------------------------------------------------------------------
size_t ir_vec_bytes(int64_t n, int restart)
{
    const size_t vec = ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
    const size_t small = (((size_t)kDotBlocks * (restart + 3) + 8 * (restart + 3)) * sizeof(double) + 255) &
                         ~(size_t)255;
    return vec * (8 + (size_t)restart + 1) + small + kTrsvSyncBytes;
}

IrVectors carve_ir(void *base, int64_t n, int restart)
{
    const size_t vec = ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
    char *p = static_cast<char *>(base);
    IrVectors v;
    v.n = n;
    v.restart = restart;
    v.x = reinterpret_cast<double *>(p); p += vec;
    v.r = reinterpret_cast<double *>(p); p += vec;
    v.b = reinterpret_cast<double *>(p); p += vec;
    v.w = reinterpret_cast<double *>(p); p += vec;
    v.z = reinterpret_cast<double *>(p); p += vec;
    v.rowabs = reinterpret_cast<double *>(p); p += vec;
    v.tmp = reinterpret_cast<double *>(p); p += vec;
    v.ys = reinterpret_cast<double *>(p); p += vec;
    v.V = reinterpret_cast<double *>(p); p += vec * ((size_t)restart + 1);
    v.ldv = (int64_t)(vec / sizeof(double));
    v.partial = reinterpret_cast<double *>(p);
    v.out = v.partial + (size_t)kDotBlocks * (restart + 3);
    const size_t small = (((size_t)kDotBlocks * (restart + 3) + 8 * (restart + 3)) * sizeof(double) + 255) &
                         ~(size_t)255;
    v.sync = reinterpret_cast<int32_t *>(p + small);
    return v;
}

namespace {

struct Ctx {
    const double *A;
    int64_t lda;
    const double *F;   // factors
    int64_t ldf;
    const int32_t *perm;
    IrVectors v;
    hipStream_t st;
    int spin_limit;
};

// dst = M src = U^{-1} L^{-1} P src
int apply_m(const Ctx &c, const double *src, double *dst)
{
    int rc = launch_gather_rows(c.v.n, 1, src, 1, c.perm, dst, 1, c.st);
    if (rc) return rc;
    return launch_trsv(c.v.n, 1, c.F, c.ldf, dst, 1, c.v.sync, c.v.ys, c.st, c.spin_limit);
}

// out[0..nv) = V_k . w, k < nv (device result at `out`)
int dots(const Ctx &c, const double *V, int64_t ldv, int nv, const double *w, double *out)
{
    const int64_t n = c.v.n;
    int nblk = (int)((n + 255) / 256);
    if (nblk > kDotBlocks) nblk = kDotBlocks;
    const int64_t chunk = (n + nblk - 1) / nblk;
    hipLaunchKernelGGL(dots_kernel, dim3(nblk), dim3(256), 0, c.st, V, ldv, nv, w, n, chunk, c.v.partial);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(reduce_kernel<false>, dim3(1), dim3(256), 0, c.st, c.v.partial, nblk, nv, out);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

// out[0..nv) = max |X_k|
int amax(const Ctx &c, const double *X, int64_t ldv, int nv, double *out)
{
    const int64_t n = c.v.n;
    int nblk = (int)((n + 255) / 256);
    if (nblk > kDotBlocks) nblk = kDotBlocks;
    const int64_t chunk = (n + nblk - 1) / nblk;
    hipLaunchKernelGGL(amax_kernel, dim3(nblk), dim3(256), 0, c.st, X, ldv, nv, n, chunk, c.v.partial);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(reduce_kernel<true>, dim3(1), dim3(256), 0, c.st, c.v.partial, nblk, nv, out);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int vcomb(const Ctx &c, double *w, const double *V, int64_t ldv, int nv, const double *coef, double sign)
{
    hipLaunchKernelGGL(vcomb_kernel, dim3(blocks_of(c.v.n, 256)), dim3(256), 0, c.st, w, V, ldv, nv, coef, sign,
                       c.v.n);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int scale(const Ctx &c, double *dst, const double *src, double alpha)
{
    hipLaunchKernelGGL(scale_kernel, dim3(blocks_of(c.v.n, 256)), dim3(256), 0, c.st, dst, src, alpha, c.v.n);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int to_host(const Ctx &c, double *h, const double *d, size_t count)
{
    CFX_HIP(hipMemcpyAsync(h, d, count * sizeof(double), hipMemcpyDeviceToHost, c.st));
    CFX_HIP(hipStreamSynchronize(c.st));
    return CFX_OK;
}

// eta of the current x (residual r = b - A x left in v.r).  anorm < 0 on
// entry: compute |A|_inf as well.
int backward_error(const Ctx &c, double &anorm, double &eta)
{
    const IrVectors &v = c.v;
    int rc = launch_residual(c.A, c.lda, v.n, v.x, v.b, v.r, anorm < 0 ? v.rowabs : nullptr, c.st);
    if (rc) return rc;
    // r, x, b, rowabs are consecutive vectors at stride ldv: r = x + ldv,
    // b = x + 2 ldv; rowabs = x + 5 ldv.
    if ((rc = amax(c, v.x, v.ldv, 3, v.out))) return rc;
    if (anorm < 0 && (rc = amax(c, v.rowabs, v.ldv, 1, v.out + 3))) return rc;
    double hm[4];
    if ((rc = to_host(c, hm, v.out, anorm < 0 ? 4 : 3))) return rc;
    if (anorm < 0) anorm = hm[3];
    const double xn = hm[0], rn = hm[1], bn = hm[2];
    const double den = anorm * xn + bn;
    if (!std::isfinite(xn) || !std::isfinite(rn) || !std::isfinite(den))
        eta = NAN;   // a non-finite solution never counts as converged
    else
        eta = den > 0 ? rn / den : (rn > 0 ? INFINITY : 0.0);
    return CFX_OK;
}

}  // namespace

// Refine x (in v.x, initial guess already there) for right-hand side v.b.
int ir_refine(const double *A, int64_t lda, const double *F, int64_t ldf, const int32_t *perm,
              const IrVectors &v, const IrParams &p, IrResult *res, hipStream_t st)
{
    Ctx c{A, lda, F, ldf, perm, v, st, p.spin_limit};
    const int m = v.restart;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hh(2 * (m + 1) + 1);
    double anorm = -1.0, eta = 0.0;
    double eta_hist[2] = {0.0, 0.0};   // eta one and two steps back
    int rc;
    res->outer = 0;
    res->inner = 0;
    res->converged = 0;
    for (int outer = 0;; ++outer) {
        if ((rc = backward_error(c, anorm, eta))) return rc;
        if (outer == 0) res->eta_first = eta;
        res->eta = eta;
        res->outer = outer;
        if (!(eta > p.tol)) {
            res->converged = std::isfinite(eta) ? 1 : 0;
            break;
        }
        if (outer >= p.max_outer || !std::isfinite(eta)) break;
        // stagnation: eta did not halve over the last two steps
        if (outer >= 2 && eta > 0.5 * eta_hist[1]) break;
        eta_hist[1] = eta_hist[0];
        eta_hist[0] = eta;

        // GMRES on M A d = M r from d = 0
        if ((rc = apply_m(c, v.r, v.z))) return rc;
        if ((rc = dots(c, v.z, 0, 1, v.z, v.out))) return rc;
        double beta2;
        if ((rc = to_host(c, &beta2, v.out, 1))) return rc;
        const double beta = std::sqrt(beta2);
        if (!(beta > 0) || !std::isfinite(beta)) break;
        if ((rc = scale(c, v.V, v.z, 1.0 / beta))) return rc;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < m; ++j) {
            double *Vj = v.V + (int64_t)j * v.ldv;
            if ((rc = launch_gemv(A, lda, v.n, Vj, v.tmp, st))) return rc;
            if ((rc = apply_m(c, v.tmp, v.w))) return rc;
            // classical Gram-Schmidt, twice
            double *h1 = v.out, *h2 = v.out + (m + 1), *nw = v.out + 2 * (m + 1);
            if ((rc = dots(c, v.V, v.ldv, j + 1, v.w, h1))) return rc;
            if ((rc = vcomb(c, v.w, v.V, v.ldv, j + 1, h1, -1.0))) return rc;
            if ((rc = dots(c, v.V, v.ldv, j + 1, v.w, h2))) return rc;
            if ((rc = vcomb(c, v.w, v.V, v.ldv, j + 1, h2, -1.0))) return rc;
            if ((rc = dots(c, v.w, 0, 1, v.w, nw))) return rc;
            if ((rc = to_host(c, hh.data(), v.out, 2 * (m + 1) + 1))) return rc;
            const double hn = std::sqrt(hh[2 * (m + 1)]);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[(m + 1) + i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double rr = std::hypot(a, b);
            cs[j] = rr > 0 ? a / rr : 1.0;
            sn[j] = rr > 0 ? b / rr : 0.0;
            H[(size_t)j * m + j] = rr;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++res->inner;
            jend = j + 1;
            if (std::fabs(g[j + 1]) <= p.gmres_tol * beta || !(hn > 0)) break;
            if (j + 1 < m && (rc = scale(c, v.V + (int64_t)(j + 1) * v.ldv, v.w, 1.0 / hn))) return rc;
        }
        // y = H^{-1} g (upper triangular jend x jend), then x += V y
        for (int i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jend; ++k) s -= H[(size_t)i * m + k] * y[k];
            const double d = H[(size_t)i * m + i];
            y[i] = d != 0 ? s / d : 0.0;
        }
        CFX_HIP(hipMemcpyAsync(v.out, y.data(), (size_t)jend * sizeof(double), hipMemcpyHostToDevice, st));
        if ((rc = vcomb(c, v.x, v.V, v.ldv, jend, v.out, 1.0))) return rc;
    }
    // a triangular solve of this refinement (or of the initial solve, whose
    // flag is sticky too) that gave up waiting leaves NaN behind: an error
    bool gave_up = false;
    if ((rc = read_solve_flag(v.sync, st, &gave_up))) return rc;
    return gave_up ? CFX_ESOLVE : CFX_OK;
}

}  // namespace cfx

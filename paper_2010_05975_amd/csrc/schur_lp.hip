// Low-precision Schur-complement update for the mixed-precision
// factorisation: A22 -= L21 U12 with L21 and U12 rounded to BF16 or FP16,
// products accumulated in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_{bf16,f16}) and subtracted from the FP64 trailing
// matrix.  The pivot search, interchanges and triangular solves stay FP64;
// the accuracy lost here is recovered by FP64 iterative refinement.
//
// The operands are packed once per panel into the workspace: L21 row-major
// (m x Kp, k contiguous) and U12 transposed (m x Kp, k contiguous), Kp = vb
// rounded up to 32 and zero-padded, so every lane fetches its 8-element
// k-run with one 16-byte load.  The kernel is bound by the FP64 read and
// write of A22 (16 bytes per element per panel); the operand tiles come
// from L2.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "cfx_internal.h"

namespace cfx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, KB = 32;
constexpr int GROUP_M = 8;
constexpr int NXCD = 8;

template <typename T> struct Lp;
template <> struct Lp<__bf16> {
    typedef bf8 v8;
    static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Lp<_Float16> {
    typedef h8 v8;
    static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Position `pos` of the regrouped order -> tile (ti, tj): grouped row-major,
// GROUP_M tile rows at a time.
__device__ __forceinline__ void tile_at(int pos, int tm, int tn, int &ti, int &tj)
{
    const int group = pos / (GROUP_M * tn);
    const int first = group * GROUP_M;
    const int gsz = (tm - first) < GROUP_M ? (tm - first) : GROUP_M;
    const int r = pos - group * GROUP_M * tn;
    ti = first + r % gsz;
    tj = r / gsz;
}

// FP64 -> T rounded once, to nearest with ties to even (no intermediate
// FP32 rounding).  BF16: round to FP32 by truncation toward zero with the
// sticky "odd" bit (round-to-odd keeps the information a second rounding
// needs), then to BF16 by round-to-nearest-even on the bits; FP16: the
// direct conversion.
template <typename T> __device__ __forceinline__ T to_lowp(double x);
template <> __device__ __forceinline__ __bf16 to_lowp<__bf16>(double x)
{
    if (x != x) return __builtin_bit_cast(__bf16, (unsigned short)0x7FC0);
    float f = (float)x;                               // nearest
    unsigned b = __float_as_uint(f);
    const double back = (double)f;
    if (back != x && !__builtin_isinf(f)) {
        // step to the neighbour on x's side if f is even: the odd one of
        // the two FP32 values around x
        if ((b & 1u) == 0u) b = (fabs(x) > fabs(back)) ? b + 1u : b - 1u;
    }
    const unsigned r = (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
    return __builtin_bit_cast(__bf16, (unsigned short)r);
}
template <> __device__ __forceinline__ _Float16 to_lowp<_Float16>(double x) { return (_Float16)x; }

// Round an FP64 panel to T: Lp[i][k] = T(L[i][k]) for i < m, k < K, zero for
// K <= k < Kp.
template <typename T>
__global__ void pack_rows_kernel(const double *__restrict__ L, int64_t ldl, int64_t m, int K, int Kp,
                                 T *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * Kp) return;
    const int64_t i = e / Kp;
    const int k = (int)(e - i * Kp);
    out[e] = to_lowp<T>(k < K ? L[i * ldl + k] : 0.0);
}

// Ut[j][k] = T(U[k][j]) for j < n, k < K (transposed through LDS in FP64),
// zero for K <= k < Kp.
template <typename T>
__global__ __launch_bounds__(256) void pack_cols_kernel(const double *__restrict__ U, int64_t ldu, int64_t n,
                                                        int K, int Kp, T *__restrict__ out)
{
    __shared__ double tile[32][33];
    const int64_t j0 = (int64_t)blockIdx.x * 32;
    const int k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int k = k0 + r;
        const int64_t j = j0 + tx;
        tile[r][tx] = (k < K && j < n) ? U[(int64_t)k * ldu + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + r;
        const int k = k0 + tx;
        if (j < n && k < Kp) out[j * Kp + k] = to_lowp<T>(tile[tx][r]);
    }
}

template <typename T, bool EDGE>
__global__ __launch_bounds__(256, 2) void schur_lp_kernel(const T *__restrict__ Lp_, const T *__restrict__ Ut_,
                                                          int Kp, double *__restrict__ C, int64_t ldc,
                                                          int64_t mr, int64_t nc, int tm, int tn)
{
    typedef typename Lp<T>::v8 v8;
    // XCD-aware persistent schedule (as the FP64 update): workgroup b runs
    // on XCD b % 8, which owns a contiguous range of tile positions; with
    // one workgroup per tile each takes exactly one position
    const int nb = tm * tn;
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
    const int nsl = ((int)gridDim.x - xcd + NXCD - 1) / NXCD;
    const int per = nb / NXCD;
    const int cnt = per + (xcd < nb - per * NXCD ? 1 : 0);
#pragma unroll 1
    for (int it = slot; it < cnt; it += nsl) {
    int ti, tj;
    tile_at(it < per ? xcd * per + it : NXCD * per + xcd, tm, tn, ti, tj);
    const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;

    const v8 *ap[4], *bp[4];
    bool aok[4], bok[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t gi = i0 + wm + a * 16 + lr;
        aok[a] = !EDGE || gi < mr;
        ap[a] = reinterpret_cast<const v8 *>(Lp_ + (aok[a] ? gi : 0) * Kp + 8 * lk);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t gj = j0 + wn + b * 16 + lr;
        bok[b] = !EDGE || gj < nc;
        bp[b] = reinterpret_cast<const v8 *>(Ut_ + (bok[b] ? gj : 0) * Kp + 8 * lk);
    }
    // the C tile is read first: the kernel is bound by these reads and
    // writes, and their latency then overlaps the operand loads and the
    // matrix-core work (f32 16x16 accumulator layout: lane l holds rows
    // 4*(l/16) + q of column l%16)
    // (whole tiles only; an edge tile reads C at the end, which keeps its
    // guarded addressing within the register budget).  Whole tiles move C
    // non-temporally, so that it does not evict the operands from L2.
    double cv[4][4][4];
    if constexpr (!EDGE) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    cv[a][b][q] = __builtin_nontemporal_load(&C[(i0 + wm + a * 16 + 4 * lk + q) * ldc + j0 + wn + b * 16 + lr]);
    }
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int k0 = 0; k0 < Kp; k0 += KB) {
        v8 af[4], bf[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = ap[a][k0 / 8];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = bp[b][k0 / 8];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = Lp<T>::mfma(af[a], bf[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = j0 + wn + b * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = i0 + wm + a * 16 + 4 * lk + q;
                if constexpr (!EDGE) {
                    __builtin_nontemporal_store(cv[a][b][q] - (double)acc[a][b][q], &C[gi * ldc + gj]);
                } else if (gi < mr && gj < nc) {
                    double *c = C + gi * ldc + gj;
                    *c = *c - (double)acc[a][b][q];
                }
            }
        }
    }   // tiles of this workgroup
}

template <typename T>
int pack_impl(const double *L21, const double *U12, int64_t lda, int64_t m, int K, void *buf,
              hipStream_t st)
{
    const int Kp = (K + KB - 1) / KB * KB;
    T *Lp_ = static_cast<T *>(buf);
    T *Ut_ = Lp_ + (size_t)m * Kp;
    const int64_t tot = m * Kp;
    hipLaunchKernelGGL(pack_rows_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L21, lda,
                       m, K, Kp, Lp_);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(pack_cols_kernel<T>, dim3((unsigned)((m + 31) / 32), (unsigned)(Kp / 32)), dim3(256), 0,
                       st, U12, lda, m, K, Kp, Ut_);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

template <typename T>
int schur_impl(const void *buf, int64_t m, int K, int64_t col0, int64_t ncols, double *C, int64_t ldc,
               int max_wgs, hipStream_t st)
{
    const int Kp = (K + KB - 1) / KB * KB;
    const T *Lp_ = static_cast<const T *>(buf);
    const T *Ut_ = Lp_ + (size_t)m * Kp + (size_t)col0 * Kp;
    if (m <= 0 || ncols <= 0) return CFX_OK;
    const int tm = (int)((m + BM - 1) / BM), tn = (int)((ncols + BN - 1) / BN);
    if ((int64_t)tm * tn > INT32_MAX) return CFX_ENOTSUP;
    int64_t nb = (int64_t)tm * tn;
    if (max_wgs > 0 && max_wgs < nb) nb = max_wgs < NXCD ? NXCD : max_wgs;
    const bool full = (m % BM == 0) && (ncols % BN == 0);
    if (full)
        hipLaunchKernelGGL((schur_lp_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, st, Lp_, Ut_, Kp,
                           C + col0, ldc, m, ncols, tm, tn);
    else
        hipLaunchKernelGGL((schur_lp_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, st, Lp_, Ut_, Kp,
                           C + col0, ldc, m, ncols, tm, tn);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace

size_t lp_pack_bytes(int64_t m, int K)
{
    const int Kp = (K + KB - 1) / KB * KB;
    return 2 * (size_t)m * Kp * 2;
}

int launch_pack_lp(int precision, const double *L21, const double *U12, int64_t lda, int64_t m, int K,
                   void *buf, hipStream_t st)
{
    if (m <= 0) return CFX_OK;
    if (precision == CFX_PREC_BF16) return pack_impl<__bf16>(L21, U12, lda, m, K, buf, st);
    return pack_impl<_Float16>(L21, U12, lda, m, K, buf, st);
}

int launch_schur_lp(int precision, const void *buf, int64_t m, int K, int64_t col0, int64_t ncols, double *C,
                    int64_t ldc, int max_wgs, hipStream_t st)
{
    if (precision == CFX_PREC_BF16) return schur_impl<__bf16>(buf, m, K, col0, ncols, C, ldc, max_wgs, st);
    return schur_impl<_Float16>(buf, m, K, col0, ncols, C, ldc, max_wgs, st);
}

}  // namespace cfx

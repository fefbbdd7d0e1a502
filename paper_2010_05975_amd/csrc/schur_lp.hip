// Low-precision Schur-complement update for the mixed-precision
// factorisation: A22 -= L21 U12 with L21 and U12 rounded to BF16 or FP16,
// products accumulated in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_{bf16,f16}) and subtracted from the FP64 trailing
// matrix.  The pivot search, interchanges and triangular solves stay FP64;
// the accuracy lost here is recovered by FP64 iterative refinement.
//
// The operands are packed once per panel into the workspace: L21 row-major
// (m x Kp, k contiguous) and U12 transposed (n x Kp, k contiguous), Kp = vb
// rounded up to 32 and zero-padded, so every lane fetches its 8-element
// k-run with one 16-byte (8-byte for FP8) load.  The kernel is bound by the
// FP64 read and write of A22 (16 bytes per element per panel); the operand
// tiles come from L2.
//
// FP8 (OCP E4M3: 4 exponent bits, bias 7, 3 fraction bits, largest finite
// 448, no infinities) has too little range for unscaled operands, so each
// row i of L21 and each column j of U12 is first scaled by a power of two,
// 2^sL_i and 2^sU_j, that brings its largest magnitude into [128, 256); the
// scaled values are rounded to E4M3 (to nearest, ties to even; the scaled
// range never overflows) and stored as bytes.  In registers each E4M3 byte
// is widened exactly to FP16 (every E4M3 value, times 2^-8, is an FP16
// value: the byte's exponent and fraction fields land in the FP16 fields
// unchanged), multiplied on the FP16 matrix cores with FP32 accumulation,
// and every sum is scaled back by 2^(16 - sL_i - sU_j), exactly, before it
// is subtracted.  (The FP8 matrix-core instruction was measured to
// accumulate less accurately than FP32 rounding allows, by up to 4x the
// bound K 2^-23 sum|l||u|; the exact widening keeps the FP32 bound.)  A row
// of L21 or column of U12 holding a non-finite value makes its row or
// column of the update NaN.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "cfx_internal.h"

namespace cfx {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// One E4M3 value as a byte (the storage type of the FP8 operands).
struct e4m3 {
    unsigned char bits;
};

constexpr int BM = 128, BN = 128, KB = 32;
constexpr int GROUP_M = 8;
constexpr int NXCD = 8;

// Scale exponent of a row / column holding a non-finite value.
constexpr int kNonFinite = 1 << 20;

// Bytes 0 and 1 of w (E4M3) -> two FP16 values, each 2^-8 times the E4M3
// value: sign to bit 15, exponent and fraction fields shifted left by 7
// (E4M3 exponent e with bias 7 becomes FP16 exponent e with bias 15, a
// factor 2^-8; E4M3 subnormals M 2^-9 become FP16 subnormals M 2^-17).
__device__ __forceinline__ unsigned e4m3x2_to_f16x2(unsigned w)
{
    return ((w & 0x7Fu) << 7) | ((w & 0x80u) << 8) | ((w & 0x7F00u) << 15) | ((w & 0x8000u) << 16);
}

template <typename T> struct Lp;
template <> struct Lp<e4m3> {
    typedef long v8;        // 8 E4M3 values
    static __device__ __forceinline__ f4 mfma(v8 a, v8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(widen(a), widen(b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ h8 widen(v8 v)
    {
        const unsigned long long u = (unsigned long long)v;
        const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const u4 r = {e4m3x2_to_f16x2(lo), e4m3x2_to_f16x2(lo >> 16), e4m3x2_to_f16x2(hi),
                      e4m3x2_to_f16x2(hi >> 16)};
        return __builtin_bit_cast(h8, r);
    }
};
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

// FP64 -> E4M3 (bias 7), to nearest with ties to even (the scaled operands
// stay below 256): the quantum of x's binade (clamped at the subnormal
// binade 2^-6) is a power of two, so x / q is exact and rint rounds it to
// nearest even; the rounded value is then encoded field by field.  |x| up
// to 464 rounds to 448 (the tie goes to the even 448); beyond it, and for
// NaN or infinite inputs, the result is the E4M3 NaN (0x7F / 0xFF).
template <> __device__ __forceinline__ e4m3 to_lowp<e4m3>(double x)
{
    if (!(fabs(x) <= 464.0)) return e4m3{(unsigned char)((x != x || x > 0) ? 0x7F : 0xFF)};
    const unsigned sign = __builtin_signbit(x) ? 0x80u : 0u;
    const double a = fabs(x);
    if (a == 0.0) return e4m3{(unsigned char)sign};
    int e2;
    (void)frexp(a, &e2);                       // a = f 2^e2, f in [0.5, 1)
    const int e = e2 - 1 < -6 ? -6 : e2 - 1;   // binade exponent (subnormals: -6)
    const double r = rint(ldexp(a, 3 - e));    // quantum 2^(e-3): r in [0, 16]
    unsigned bits;
    if (e == -6 && r < 8.0) {
        bits = (unsigned)r;                    // subnormal: r * 2^-9
    } else if (r >= 16.0) {
        bits = (unsigned)(e + 1 + 7) << 3;     // rounded up to the next binade
    } else {
        bits = ((unsigned)(e + 7) << 3) | ((unsigned)r - 8u);
    }
    return e4m3{(unsigned char)(sign | bits)};
}

// Power-of-two scale exponent of a row or column: 8 - E for a largest
// magnitude M = f 2^E (f in [0.5, 1)), so that M 2^s lies in [128, 256);
// 0 for an all-zero vector, kNonFinite when M is not finite.
__device__ __forceinline__ int scale_exp(double M)
{
    if (!(M < INFINITY)) return kNonFinite;     // also NaN
    if (!(M > 0.0)) return 0;
    int e2;
    (void)frexp(M, &e2);
    return 8 - e2;
}

// max(m, |a|) that keeps a NaN once it has met one
__device__ __forceinline__ double absmax_nan(double m, double a)
{
    a = fabs(a);
    return (a > m || a != a) ? a : m;
}

// Physical row of logical row i (identity without a row map).
__device__ __forceinline__ int64_t phys(const int32_t *rm, int64_t i) { return rm ? (int64_t)rm[i] : i; }

// sL[i] for the rows of L (m x K, stride ldl): one wavefront per row.
__global__ __launch_bounds__(256) void row_scale_kernel(const double *__restrict__ L, int64_t ldl, int64_t m,
                                                        int K, const int32_t *__restrict__ rmap,
                                                        int32_t *__restrict__ sL)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    const double *row = L + phys(rmap, i) * ldl;
    double mx = 0.0;
    for (int k = lane; k < K; k += 64) mx = absmax_nan(mx, row[k]);
    for (int off = 32; off >= 1; off >>= 1) mx = absmax_nan(mx, __shfl_xor(mx, off));
    if (lane == 0) sL[i] = scale_exp(mx);
}

// sU[j] for the columns of U (K x n, stride ldu): one thread per column.
__global__ __launch_bounds__(256) void col_scale_kernel(const double *__restrict__ U, int64_t ldu, int64_t n,
                                                        int K, const int32_t *__restrict__ umap,
                                                        int32_t *__restrict__ sU)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double mx = 0.0;
    for (int k = 0; k < K; ++k) mx = absmax_nan(mx, U[phys(umap, k) * ldu + j]);
    sU[j] = scale_exp(mx);
}

// Round an FP64 panel to T: Lp[i][k] = T(L[i][k] 2^sL[i]) for i < m, k < K
// (sL null: no scaling), zero for K <= k < Kp.
template <typename T>
__global__ void pack_rows_kernel(const double *__restrict__ L, int64_t ldl, int64_t m, int K, int Kp,
                                 const int32_t *__restrict__ rmap, const int32_t *__restrict__ sL,
                                 T *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * Kp) return;
    const int64_t i = e / Kp;
    const int k = (int)(e - i * Kp);
    double x = k < K ? L[phys(rmap, i) * ldl + k] : 0.0;
    if (sL) x = sL[i] == kNonFinite ? 0.0 : ldexp(x, sL[i]);
    out[e] = to_lowp<T>(x);
}

// Ut[j][k] = T(U[k][j] 2^sU[j]) for j < n, k < K (transposed through LDS in
// FP64; sU null: no scaling), zero for K <= k < Kp.
template <typename T>
__global__ __launch_bounds__(256) void pack_cols_kernel(const double *__restrict__ U, int64_t ldu, int64_t n,
                                                        int K, int Kp, const int32_t *__restrict__ umap,
                                                        const int32_t *__restrict__ sU, T *__restrict__ out)
{
    __shared__ double tile[32][33];
    const int64_t j0 = (int64_t)blockIdx.x * 32;
    const int k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int k = k0 + r;
        const int64_t j = j0 + tx;
        tile[r][tx] = (k < K && j < n) ? U[phys(umap, k) * ldu + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + r;
        const int k = k0 + tx;
        if (j < n && k < Kp) {
            double x = tile[tx][r];
            if (sU) x = sU[j] == kNonFinite ? 0.0 : ldexp(x, sU[j]);
            out[j * Kp + k] = to_lowp<T>(x);
        }
    }
}

template <typename T, bool EDGE>
__global__ __launch_bounds__(256, 2) void schur_lp_kernel(const T *__restrict__ Lp_, const T *__restrict__ Ut_,
                                                          int Kp, const int32_t *__restrict__ sL,
                                                          const int32_t *__restrict__ sU,
                                                          double *__restrict__ C, int64_t ldc,
                                                          int64_t mr, int64_t nc, int tm, int tn,
                                                          const int32_t *__restrict__ rmap)
{
    // FP8: every FP32 sum is scaled back by 2^-(sL_i + sU_j)
    constexpr bool SCALED = sizeof(T) == 1;
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
                    cv[a][b][q] = __builtin_nontemporal_load(
                        &C[phys(rmap, i0 + wm + a * 16 + 4 * lk + q) * ldc + j0 + wn + b * 16 + lr]);
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
    int se[4][4], sj[4];
    if constexpr (SCALED) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = j0 + wn + b * 16 + lr;
            sj[b] = (!EDGE || gj < nc) ? sU[gj] : 0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = i0 + wm + a * 16 + 4 * lk + q;
                se[a][q] = (!EDGE || gi < mr) ? sL[gi] : 0;
            }
    }
    auto sum_at = [&](int a, int b, int q) -> double {
        const double v = (double)acc[a][b][q];
        if constexpr (SCALED) {
            // products of the widened operands carry 2^-16
            if (se[a][q] == kNonFinite || sj[b] == kNonFinite) return __builtin_nan("");
            return ldexp(v, 16 - se[a][q] - sj[b]);
        }
        return v;
    };
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = j0 + wn + b * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = i0 + wm + a * 16 + 4 * lk + q;
                if constexpr (!EDGE) {
                    __builtin_nontemporal_store(cv[a][b][q] - sum_at(a, b, q), &C[phys(rmap, gi) * ldc + gj]);
                } else if (gi < mr && gj < nc) {
                    double *c = C + phys(rmap, gi) * ldc + gj;
                    *c = *c - sum_at(a, b, q);
                }
            }
        }
    }   // tiles of this workgroup
}

// Layout of the packed operands in `buf`: Lp (m x Kp), Ut (n x Kp), then
// for FP8 the scale exponents sL (m) and sU (n).
struct PackLayout {
    int Kp;
    size_t esz, off_ut, off_sl, off_su, total;
};

PackLayout pack_layout(int precision, int64_t m, int64_t n, int K)
{
    PackLayout p{};
    p.Kp = (K + KB - 1) / KB * KB;
    p.esz = precision == CFX_PREC_FP8 ? 1 : 2;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    p.off_ut = al((size_t)m * p.Kp * p.esz);
    p.off_sl = p.off_ut + al((size_t)n * p.Kp * p.esz);
    p.off_su = p.off_sl + (precision == CFX_PREC_FP8 ? al((size_t)m * 4) : 0);
    p.total = p.off_su + (precision == CFX_PREC_FP8 ? al((size_t)n * 4) : 0);
    return p;
}

template <typename T>
int pack_impl(const PackLayout &pl, const double *L21, int64_t ldl, int64_t m, const double *U12, int64_t ldu,
              int64_t n, int K, char *buf, hipStream_t st, const int32_t *rmap, const int32_t *umap)
{
    const int Kp = pl.Kp;
    T *Lp_ = reinterpret_cast<T *>(buf);
    T *Ut_ = reinterpret_cast<T *>(buf + pl.off_ut);
    int32_t *sL = nullptr, *sU = nullptr;
    if (sizeof(T) == 1) {
        sL = reinterpret_cast<int32_t *>(buf + pl.off_sl);
        sU = reinterpret_cast<int32_t *>(buf + pl.off_su);
        if (m > 0) {
            hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, L21, ldl, m, K,
                               rmap, sL);
            CFX_HIP(hipGetLastError());
        }
        if (n > 0) {
            hipLaunchKernelGGL(col_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U12, ldu, n,
                               K, umap, sU);
            CFX_HIP(hipGetLastError());
        }
    }
    const int64_t tot = m * Kp;
    if (tot > 0) {
        hipLaunchKernelGGL(pack_rows_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L21, ldl,
                           m, K, Kp, rmap, sL, Lp_);
        CFX_HIP(hipGetLastError());
    }
    if (n > 0) {
        hipLaunchKernelGGL(pack_cols_kernel<T>, dim3((unsigned)((n + 31) / 32), (unsigned)(Kp / 32)), dim3(256), 0,
                           st, U12, ldu, n, K, Kp, umap, sU, Ut_);
        CFX_HIP(hipGetLastError());
    }
    return CFX_OK;
}

template <typename T>
int schur_impl(const PackLayout &pl, const char *buf, int64_t m, int64_t col0, int64_t ncols, double *C,
               int64_t ldc, int max_wgs, hipStream_t st, const int32_t *rmap)
{
    const int Kp = pl.Kp;
    const T *Lp_ = reinterpret_cast<const T *>(buf);
    const T *Ut_ = reinterpret_cast<const T *>(buf + pl.off_ut) + (size_t)col0 * Kp;
    const int32_t *sL = nullptr, *sU = nullptr;
    if (sizeof(T) == 1) {
        sL = reinterpret_cast<const int32_t *>(buf + pl.off_sl);
        sU = reinterpret_cast<const int32_t *>(buf + pl.off_su) + col0;
    }
    if (m <= 0 || ncols <= 0) return CFX_OK;
    const int tm = (int)((m + BM - 1) / BM), tn = (int)((ncols + BN - 1) / BN);
    if ((int64_t)tm * tn > INT32_MAX) return CFX_ENOTSUP;
    int64_t nb = (int64_t)tm * tn;
    if (max_wgs > 0 && max_wgs < nb) nb = max_wgs < NXCD ? NXCD : max_wgs;
    const bool full = (m % BM == 0) && (ncols % BN == 0);
    if (full)
        hipLaunchKernelGGL((schur_lp_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, st, Lp_, Ut_, Kp, sL, sU,
                           C + col0, ldc, m, ncols, tm, tn, rmap);
    else
        hipLaunchKernelGGL((schur_lp_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, st, Lp_, Ut_, Kp, sL, sU,
                           C + col0, ldc, m, ncols, tm, tn, rmap);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace

size_t lp_pack_bytes(int precision, int64_t m, int64_t n, int K)
{
    return pack_layout(precision, m, n, K).total;
}

int launch_pack_lp(int precision, const double *L21, int64_t ldl, int64_t m, const double *U12, int64_t ldu,
                   int64_t n, int K, void *buf, hipStream_t st, const int32_t *rmap, const int32_t *umap)
{
    const PackLayout pl = pack_layout(precision, m, n, K);
    char *b = static_cast<char *>(buf);
    if (precision == CFX_PREC_BF16) return pack_impl<__bf16>(pl, L21, ldl, m, U12, ldu, n, K, b, st, rmap, umap);
    if (precision == CFX_PREC_FP16) return pack_impl<_Float16>(pl, L21, ldl, m, U12, ldu, n, K, b, st, rmap, umap);
    if (precision == CFX_PREC_FP8) return pack_impl<e4m3>(pl, L21, ldl, m, U12, ldu, n, K, b, st, rmap, umap);
    return CFX_ENOTSUP;
}

int launch_schur_lp(int precision, const void *buf, int64_t m, int64_t n, int K, int64_t col0, int64_t ncols,
                    double *C, int64_t ldc, int max_wgs, hipStream_t st, const int32_t *rmap)
{
    const PackLayout pl = pack_layout(precision, m, n, K);
    const char *b = static_cast<const char *>(buf);
    if (precision == CFX_PREC_BF16) return schur_impl<__bf16>(pl, b, m, col0, ncols, C, ldc, max_wgs, st, rmap);
    if (precision == CFX_PREC_FP16) return schur_impl<_Float16>(pl, b, m, col0, ncols, C, ldc, max_wgs, st, rmap);
    if (precision == CFX_PREC_FP8) return schur_impl<e4m3>(pl, b, m, col0, ncols, C, ldc, max_wgs, st, rmap);
    return CFX_ENOTSUP;
}

}  // namespace cfx

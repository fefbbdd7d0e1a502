// Solve A X = B from the factors A = P L U (the problem statement of Sec. 2.2
// applied to right-hand sides; LAPACK getrs conventions).
//
// 1. perm: the ipiv interchanges composed into one gather (one wavefront,
//    the index array in LDS; runs of interchanges on disjoint rows are
//    applied together).
// 2. X = B[perm] into a contiguous temporary.
// 3. Forward substitution with unit L, then back substitution with U,
//    blocked by SB = 128 rows.  One launch per block: every workgroup
//    subtracts the just-solved block's contribution from its rows
//    (x_i -= LU[i, blk] x_blk, an HBM-bound sweep over the factor), and
//    workgroup 0, whose rows are the next diagonal block, then solves that
//    block in registers.  No workgroup ever waits on another; the stream
//    order between launches carries the dependency.  Each factor element
//    is read once per triangular solve (8 n^2 bytes per getrs).
// 4. B = X.
#include <utility>

#include "cfx_internal.h"

namespace cfx {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kPermLds = 36864;   // n up to this uses the LDS permutation (144 KiB)
static_assert(kPermLds <= 0x10000, "row indices and the tags of perm_lds_kernel share a 32-bit entry");

// Physical row of factor row i: rm[i] for factors stored with row masking
// (rows never interchanged), else i.
__device__ __forceinline__ int64_t fr(const int32_t *rm, int64_t i) { return rm ? (int64_t)rm[i] : i; }
constexpr int SB = 128;           // block of the substitution
constexpr int HB = 64;            // half block solved by one wavefront's lanes
constexpr int RPW = 256;          // rows per updating workgroup (64: 34.6 ms, 256: 29.8 ms for 64 RHS at N = 32768)

template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F &&f)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

__device__ __forceinline__ double bcast(double x, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One wavefront; lane l holds interchange i0 + l of the current window of
// 64.  A run of consecutive interchanges is tried at once: each of its
// lanes tags the two rows of its interchange (an LDS add of 1 << 16; the
// entries themselves are < 2^16).  No row tagged twice means that the run
// touches disjoint rows, so its interchanges commute and every lane applies
// its own; the next run is then twice as long.  Otherwise the tags are
// removed and the run is halved; a run of at most 2 is applied in order by
// lane 0.  An entry outside [i, n) is no interchange.
__global__ __launch_bounds__(64) void perm_lds_kernel(const int32_t *ipiv, int n, int32_t *perm)
{
    __shared__ int32_t p[kPermLds];
    const int lane = threadIdx.x;
    for (int i = lane; i < n; i += 64) p[i] = i;
    __syncthreads();
    int nxt = lane < n ? ipiv[lane] : 0;
    int run = 64;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int cnt = n - i0 < 64 ? n - i0 : 64;
        const int i = i0 + lane;
        const int r = nxt;
        if (i0 + 64 + lane < n) nxt = ipiv[i0 + 64 + lane];    // the next window, ahead of its use
        const bool valid = lane < cnt && r > i && r < n;
        int b = 0;      // interchanges [i0, i0 + b) are applied (uniform)
        while (b < cnt) {
            const int e = b + run < cnt ? b + run : cnt;
            const bool act = valid && lane >= b && lane < e;
            int oi = 0, orr = 0;
            if (act) {
                oi = atomicAdd(&p[i], 0x10000);
                orr = atomicAdd(&p[r], 0x10000);
            }
            const bool clash = act && (((oi | orr) >> 16) != 0);
            if (__ballot(clash) == 0) {
                if (act) {      // untagged old entries: the swap, tags dropped
                    p[i] = orr;
                    p[r] = oi;
                }
                b = e;
                run = run < 32 ? 2 * run : 64;
            } else {
                if (act) {
                    atomicSub(&p[i], 0x10000);
                    atomicSub(&p[r], 0x10000);
                }
                if (e - b <= 2) {
                    for (int j = b; j < e; ++j) {
                        const int rj = __builtin_amdgcn_readlane(r, j);
                        const int ij = i0 + j;
                        if (lane == 0 && rj > ij && rj < n) {
                            const int t = p[ij];
                            p[ij] = p[rj];
                            p[rj] = t;
                        }
                    }
                    b = e;
                } else {
                    run = (e - b) / 2;
                }
            }
        }
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) perm[i] = p[i];
}

__global__ void perm_global_kernel(const int32_t *ipiv, int64_t n, int32_t *perm)
{
    if (threadIdx.x != 0) return;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = ipiv[i];
        if (r > i && r < n) { const int32_t t = perm[i]; perm[i] = perm[r]; perm[r] = t; }
    }
}

__global__ void gather_rows_kernel(const double *B, int64_t ldb, const int32_t *perm, int64_t n,
                                   int64_t nrhs, double *T, int64_t ldt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e / nrhs, c = e - i * nrhs;
    T[i * ldt + c] = B[(int64_t)perm[i] * ldb + c];
}

__global__ void copy_rows_kernel(const double *T, int64_t ldt, int64_t n, int64_t nrhs, double *B,
                                 int64_t ldb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e / nrhs, c = e - i * nrhs;
    B[i * ldb + c] = T[i * ldt + c];
}

// x_i[c] -= sum_{k < bs} LU[i][c0 + k] * ys[k][c] for rows rbeg <= i < rend
// and the nc right-hand sides cc .. cc+nc of this chunk.  One right-hand
// side: a wavefront takes 4 rows at a time, 16 lanes per row; 16 right-hand
// sides: 16 rows at a time on the FP64 matrix cores.
template <int NRC>
__device__ __forceinline__ void update_rows(const double *__restrict__ LU, int64_t lda, const int32_t *rm,
                                            double *X, int64_t ldx, int cc, int nc, int64_t rbeg, int64_t rend,
                                            int64_t c0, int bs, const double *ys)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane >> 4, q = lane & 15;
    constexpr int RW = NRC == 1 ? 4 : 16;       // rows per wavefront pass
    for (int64_t i0 = rbeg + wave * RW; i0 < rend; i0 += 4 * RW) {
        if constexpr (NRC == 1) {
            const int64_t i = i0 + sub;
            const bool ok = i < rend;
            const double *row = LU + fr(rm, ok ? i : rbeg) * lda + c0;
            // lane q owns the 8 consecutive columns 8q .. 8q+7
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * q + e;
                if (k < bs) s += row[k] * ys[k];
            }
            s += __shfl_xor(s, 8, 16);
            s += __shfl_xor(s, 4, 16);
            s += __shfl_xor(s, 2, 16);
            s += __shfl_xor(s, 1, 16);
            if (ok && q == 0) X[i * ldx + cc] -= s;
        } else {
            static_assert(NRC == 16, "the matrix-core update takes 16 right-hand sides");
            // 16 rows x 16 right-hand sides per wavefront on the FP64 matrix
            // cores, K = bs: A lane l = (row l%16, k l/16), B lane l =
            // (k l/16, right-hand side l%16) from the staged block, D lane l
            // element q = (row l/16 + 4q, right-hand side l%16).  Every factor
            // value of the 16 rows is requested before the first product.
            const int lr = lane & 15, lk = lane >> 4;
            const int64_t ia = i0 + lr;
            const double *arow = LU + fr(rm, ia < rend ? ia : rbeg) * lda + c0;
            double av[SB / 4];
#pragma unroll
            for (int t = 0; t < SB / 4; ++t) {
                const int k = 4 * t + lk;
                av[t] = (ia < rend && k < bs) ? arow[k] : 0.0;
            }
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < SB / 4; ++t)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], ys[(4 * t + lk) * NRC + lr], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t ir = i0 + lk + 4 * e;
                if (ir < rend && lr < nc) X[ir * ldx + cc + lr] -= acc[e];
            }
        }
    }
}

// Unit lower triangular solve of the diagonal block rows r0 .. r0+bs
// (bs <= SB) in place in X, as two halves of HB rows.  Lane t of a
// wavefront owns row t of the half and keeps that row of L in registers;
// column j is eliminated by broadcasting lane j's finished value.
template <int NRC>
__device__ void diag_lower(const double *__restrict__ LU, int64_t lda, const int32_t *rm, double *X, int64_t ldx,
                           int cc, int nc, int64_t r0, int bs, double *yh)
{
    constexpr int CPW = NRC == 1 ? 1 : NRC / 4;   // right-hand sides per wavefront
    const int t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool active = wave * CPW < NRC;
    for (int h = 0; h < 2; ++h) {
        const int hb = bs - HB * h < HB ? bs - HB * h : HB;
        if (hb <= 0) break;
        const int64_t rb = r0 + HB * h;
        const bool okr = t < hb;
        if (active) {
            const double *row = LU + fr(rm, rb + (okr ? t : 0)) * lda;
            double Lr[HB];
            static_for<HB>([&](auto J) {
                constexpr int j = decltype(J)::value;
                Lr[j] = (okr && j < t) ? row[rb + j] : 0.0;
            });
            double xv[CPW];
#pragma unroll
            for (int e = 0; e < CPW; ++e) {
                const int c = wave * CPW + e;
                xv[e] = (okr && c < nc) ? X[(rb + t) * ldx + cc + c] : 0.0;
            }
            if (h == 1) {
                // contribution of the solved first half (rows r0 .. r0+HB)
                for (int k = 0; k < HB; ++k) {
                    const double l = okr ? row[r0 + k] : 0.0;
#pragma unroll
                    for (int e = 0; e < CPW; ++e) xv[e] -= l * yh[k * NRC + wave * CPW + e];
                }
            }
            static_for<HB>([&](auto J) {
                constexpr int j = decltype(J)::value;
#pragma unroll
                for (int e = 0; e < CPW; ++e) xv[e] -= Lr[j] * bcast(xv[e], j);
            });
#pragma unroll
            for (int e = 0; e < CPW; ++e) {
                const int c = wave * CPW + e;
                if (okr && c < nc) X[(rb + t) * ldx + cc + c] = xv[e];
                if (h == 0) yh[t * NRC + c] = xv[e];
            }
        }
        __syncthreads();
    }
}

// Upper (non-unit) triangular solve of the diagonal block rows r0 .. r0+bs
// in place in X: the second half first, then the first.
template <int NRC>
__device__ void diag_upper(const double *__restrict__ LU, int64_t lda, const int32_t *rm, double *X, int64_t ldx,
                           int cc, int nc, int64_t r0, int bs, double *yh)
{
    constexpr int CPW = NRC == 1 ? 1 : NRC / 4;
    const int t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool active = wave * CPW < NRC;
    for (int h = 1; h >= 0; --h) {
        const int hb = bs - HB * h < HB ? bs - HB * h : HB;
        if (hb <= 0) continue;
        const int64_t rb = r0 + HB * h;
        const bool okr = t < hb;
        if (active) {
            const double *row = LU + fr(rm, rb + (okr ? t : 0)) * lda;
            double Ur[HB];
            static_for<HB>([&](auto J) {
                constexpr int j = decltype(J)::value;
                Ur[j] = (okr && j > t && j < hb) ? row[rb + j] : 0.0;
            });
            const double d = okr ? row[rb + t] : 1.0;
            double xv[CPW];
#pragma unroll
            for (int e = 0; e < CPW; ++e) {
                const int c = wave * CPW + e;
                xv[e] = (okr && c < nc) ? X[(rb + t) * ldx + cc + c] : 0.0;
            }
            if (h == 0 && bs > HB) {
                // contribution of the solved second half (rows r0+HB .. r0+bs)
                for (int k = 0; k < bs - HB; ++k) {
                    const double u = okr ? row[r0 + HB + k] : 0.0;
#pragma unroll
                    for (int e = 0; e < CPW; ++e) xv[e] -= u * yh[k * NRC + wave * CPW + e];
                }
            }
            static_for<HB>([&](auto J) {
                constexpr int j = HB - 1 - decltype(J)::value;
                if (j < hb) {
#pragma unroll
                    for (int e = 0; e < CPW; ++e) {
                        if (t == j) xv[e] = xv[e] / d;
                        xv[e] -= Ur[j] * bcast(xv[e], j);
                    }
                }
            });
#pragma unroll
            for (int e = 0; e < CPW; ++e) {
                const int c = wave * CPW + e;
                if (okr && c < nc) X[(rb + t) * ldx + cc + c] = xv[e];
                if (h == 1) yh[t * NRC + c] = xv[e];
            }
        }
        __syncthreads();
    }
}

template <int NRC>
__device__ __forceinline__ void stage_block(const double *X, int64_t ldx, int cc, int nc, int64_t c0, int bs,
                                            double *ys)
{
    for (int e = threadIdx.x; e < SB * NRC; e += 256) {
        const int k = e / NRC, c = e - k * NRC;
        ys[e] = (k < bs && c < nc) ? X[(c0 + k) * ldx + cc + c] : 0.0;
    }
    __syncthreads();
}

// Forward step: when c0 >= 0 the block rows c0 .. c0+bs are solved and
// every row below is updated with them; workgroup 0 owns the next block
// rows r0 .. r0+bsn (r0 = c0 + bs) and then solves it.  Workgroup g >= 1
// owns rows r0 + bsn + (g-1) RPW .. + RPW.
template <int NRC>
__global__ __launch_bounds__(256) void fwd_step_kernel(const double *__restrict__ LU, int64_t lda,
                                                       const int32_t *rm, double *X, int64_t ldx, int64_t n,
                                                       int nrhs, int64_t c0, int bs, int64_t r0, int bsn)
{
    __shared__ double ys[SB * NRC];
    __shared__ double yh[HB * NRC];
    const int cc = blockIdx.y * NRC;
    const int nc = nrhs - cc < NRC ? nrhs - cc : NRC;
    if (c0 >= 0) {
        stage_block<NRC>(X, ldx, cc, nc, c0, bs, ys);
        int64_t rbeg, rend;
        if (blockIdx.x == 0) {
            rbeg = r0;
            rend = r0 + bsn;
        } else {
            rbeg = r0 + bsn + (int64_t)(blockIdx.x - 1) * RPW;
            rend = rbeg + RPW < n ? rbeg + RPW : n;
        }
        update_rows<NRC>(LU, lda, rm, X, ldx, cc, nc, rbeg, rend, c0, bs, ys);
    }
    if (blockIdx.x != 0 || bsn <= 0) return;
    __syncthreads();
    diag_lower<NRC>(LU, lda, rm, X, ldx, cc, nc, r0, bsn, yh);
}

// Backward step: when c0 >= 0 the block rows c0 .. c0+bs are solved and
// every row above is updated with them; workgroup 0 owns the block rows
// r0 .. r0+bsn just above (r0 + bsn = c0) and then solves it.  Workgroup
// g >= 1 owns rows (g-1) RPW .. + RPW below r0.
template <int NRC>
__global__ __launch_bounds__(256) void bwd_step_kernel(const double *__restrict__ LU, int64_t lda,
                                                       const int32_t *rm, double *X, int64_t ldx, int nrhs,
                                                       int64_t c0, int bs, int64_t r0, int bsn)
{
    __shared__ double ys[SB * NRC];
    __shared__ double yh[HB * NRC];
    const int cc = blockIdx.y * NRC;
    const int nc = nrhs - cc < NRC ? nrhs - cc : NRC;
    if (c0 >= 0) {
        stage_block<NRC>(X, ldx, cc, nc, c0, bs, ys);
        int64_t rbeg, rend;
        if (blockIdx.x == 0) {
            rbeg = r0;
            rend = r0 + bsn;
        } else {
            rbeg = (int64_t)(blockIdx.x - 1) * RPW;
            rend = rbeg + RPW < r0 ? rbeg + RPW : r0;
        }
        update_rows<NRC>(LU, lda, rm, X, ldx, cc, nc, rbeg, rend, c0, bs, ys);
    }
    if (blockIdx.x != 0 || bsn <= 0) return;
    __syncthreads();
    diag_upper<NRC>(LU, lda, rm, X, ldx, cc, nc, r0, bsn, yh);
}

// ---------------------------------------------------------------------------
// One right-hand side: one launch per triangle.  Blocks of TB rows take
// tickets in solve order (top down for L, bottom up for U).  Each triangle
// reads its right-hand side from one vector and writes its solution to the
// other, whose entries hold a mark (a signalling-NaN bit pattern that no
// arithmetic result carries) until they are solved: a block applies the
// solved blocks as their values appear, each wavefront polling the values
// themselves (one relaxed device-scope load per lane; a value is final once
// it is not the mark), so no counter and no fence lies between a block's
// result and the blocks that use it.  Then the block solves its diagonal
// block in one wavefront and stores its values.  A block only waits for
// blocks with smaller tickets, which were taken by running workgroups, so
// every wait ends; each factor element is still read once.  Per row the sum
// runs over the blocks in solve order, 16 columns per lane, then a fixed
// quad reduction: the result does not depend on timing.
// ---------------------------------------------------------------------------
constexpr int TB = 64;
constexpr unsigned long long kUnsolved = 0xFFF05EB71E5E17A1ull;   // exponent all ones, quiet bit clear
constexpr unsigned long long kQuietNaN = 0x7FF8000000000000ull;

// Clears the tickets and marks every entry of `out` unsolved; sync[4] (a
// wait gave up) is sticky until the host reads and clears it.
__global__ void trsv_reset_kernel(int32_t *sync, double *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4) sync[i] = 0;
    if (i < n) out[i] = __longlong_as_double((long long)kUnsolved);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double a)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(a), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(a), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double poll_value(const double *p)
{
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ bool is_unsolved(double v)
{
    return (unsigned long long)__double_as_longlong(v) == kUnsolved;
}

// LOWER: L y = x with unit L (forward, in = x, out = y); else U x = y
// (backward, in = y, out = x).  `out` holds the mark in every entry on
// entry.  The forward solve also marks `in` once its block has read its
// right-hand side, so `in` is ready to be the backward solve's `out`.
// sync[0] / sync[2] are the forward / backward tickets, sync[4] is set when
// a wait gave up after spin_limit polls (never, when the tickets order the
// blocks and the device runs every resident workgroup; the bound only
// guarantees that every workgroup exits).  A block that gave up writes NaN
// for its rows, so an invalid solution is never mistaken for a result, and
// waits no more.
template <bool LOWER>
__global__ __launch_bounds__(256) void trsv_sf_kernel(const double *__restrict__ LU, int64_t lda,
                                                      const int32_t *rm, double *in, double *out, int64_t n,
                                                      int nb, int32_t *sync, int spin_limit)
{
    __shared__ double part[TB];
    __shared__ double Ts[TB][TB + 1];   // the diagonal block (padded rows), zero on and off its triangle
    __shared__ double Dg[TB];           // U: its diagonal
    __shared__ int sh_t, sh_gaveup;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t *ticket = sync + (LOWER ? 0 : 2);
    if (tid == 0) {
        sh_t = atomicAdd(ticket, 1);
        sh_gaveup = 0;
    }
    __syncthreads();
    const int t = sh_t;
    const int J = LOWER ? t : nb - 1 - t;
    const int64_t r0 = (int64_t)J * TB;
    const int rows = (n - r0) < TB ? (int)(n - r0) : TB;
    const int rr = 16 * wave + (lane >> 2);     // this lane's row of the block
    const int cq = (lane & 3) * 16;              // its 16 columns of a block
    const bool rok = rr < rows;
    const double *lrow = LU + fr(rm, r0 + (rok ? rr : 0)) * lda;
    const int nk = t;                            // blocks to apply, in solve order
    auto kcol = [&](int i) -> int64_t { return (int64_t)(LOWER ? i : nb - 1 - i) * TB + cq; };
    // Every load is issued, its address clamped into the matrix (a row past
    // the block's rows reads the block's first row, whose sums are never
    // used), and what lies past column n is replaced by zero only where the
    // values are used: no branch around a load, and no wait until the use.
    auto load_l = [&](int i, double *lv) {
        const int64_t c0 = kcol(i);
#pragma unroll
        for (int e = 0; e < 16; ++e) lv[e] = lrow[c0 + e < n ? c0 + e : n - 1];
    };
    // one value of block i of the solution per lane (lane l: column l)
    auto xcol = [&](int i) -> int64_t { return (int64_t)(LOWER ? i : nb - 1 - i) * TB + lane; };
    auto load_x = [&](int i) -> double {
        const int64_t c = xcol(i);
        return poll_value(out + (c < n ? c : n - 1));
    };
    // the diagonal block (L: strictly lower; U: strictly upper, its
    // diagonal apart) is staged in LDS before any wait (every load in
    // bounds, so they are all in flight at once); wave 0 takes it into
    // registers only for the solve.  For U the coefficients above the
    // diagonal are divided by the diagonal element of their column (the
    // unit triangle U D^-1), so that no division waits on the previous row
    // in the substitution.
    double tv[TB * TB / 256];
#pragma unroll
    for (int rep = 0; rep < TB * TB / 256; ++rep) {
        const int e = tid + 256 * rep;
        const int i = e / TB, j = e - i * TB;
        const int ic = i < rows ? i : rows - 1, jc = j < rows ? j : rows - 1;
        tv[rep] = LU[fr(rm, r0 + ic) * lda + r0 + jc];
    }
#pragma unroll
    for (int rep = 0; rep < TB * TB / 256; ++rep) {
        const int e = tid + 256 * rep;
        const int i = e / TB, j = e - i * TB;
        const bool in_tri = i < rows && j < rows && (LOWER ? j < i : j > i);
        Ts[i][j] = in_tri ? tv[rep] : 0.0;
        if (!LOWER && i == j) Dg[i] = i < rows ? tv[rep] : 1.0;
    }
    if constexpr (!LOWER) {
        __syncthreads();
#pragma unroll
        for (int rep = 0; rep < TB * TB / 256; ++rep) {
            const int e = tid + 256 * rep;
            const int i = e / TB, j = e - i * TB;
            if (j > i && j < rows) Ts[i][j] = Ts[i][j] / Dg[j];
        }
    }
    __syncthreads();                              // the staged block is visible to wave 0
    const bool ok = wave == 0 && lane < rows;
    const int64_t gi = r0 + (ok ? lane : 0);
    const double rhs = ok ? in[gi] : 0.0;

    // per row: block sums (16 products each, one lane) accumulated over the
    // blocks with Neumaier's compensation.  The factor tile and the
    // solution values of block i + D are requested when block i has been
    // applied (a ring of D slots, unrolled by D so that every slot keeps its
    // registers and the wait before a slot's use covers only that slot's
    // loads); a value still marked is loaded again when its block is
    // reached, until it is not.  D = 1 measured fastest (deeper rings, 2, 3
    // and 4 slots: 5.0, 5.4 and 5.6 ms against 4.9 ms for the solve at
    // N = 32768; they keep more streaming loads in flight beside the polls
    // and stores of the chain), and a row behind the head still catches up
    // faster than the chain moves.
    constexpr int D = 1;
    double acc = 0.0, cmp = 0.0;
    double lq[D][16];
    double xq[D];
    bool gave = false;
    auto refill = [&](int q, int i) {
        load_l(i, lq[q]);
        xq[q] = load_x(i);
    };
    auto apply = [&](int q, int i) {
        double xi = xq[q];
        if (!gave && __ballot(is_unsolved(xi))) {
            int spins = 0;
            do {
                if (spins++ >= spin_limit) {
                    gave = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                xi = load_x(i);
            } while (__ballot(is_unsolved(xi)));
        }
        if (xcol(i) >= n) xi = 0.0;
        if (kcol(i) - cq + TB > n) {              // the block reaches past column n
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (kcol(i) + e >= n) lq[q][e] = 0.0;
        }
        double bsum = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) bsum += lq[q][e] * __shfl(xi, cq + e);
        const double tsum = acc + bsum;
        cmp += fabs(acc) >= fabs(bsum) ? (acc - tsum) + bsum : (bsum - tsum) + acc;
        acc = tsum;
    };
    if (nk > 0) {
        static_for<D>([&](auto S) {
            if (decltype(S)::value < nk) refill(decltype(S)::value, decltype(S)::value);
        });
        for (int i = 0; i < nk; i += D) {
            static_for<D>([&](auto S) {
                constexpr int q = decltype(S)::value;
                if (i + q < nk) {
                    apply(q, i + q);
                    if (i + q + D < nk) refill(q, i + q + D);
                }
            });
        }
    }
    // wave 0 requests its rows of the diagonal block now, so that the reads
    // are in flight during the reduction and the barrier
    double Tr[TB];
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < TB; ++j) Tr[j] = Ts[lane][j];
    }
    acc += cmp;
    acc += dpp_d<0xB1>(acc);                      // quad_perm [1,0,3,2]
    acc += dpp_d<0x4E>(acc);                      // quad_perm [2,3,0,1]
    if ((lane & 3) == 0) part[rr] = acc;
    if (gave && lane == 0) {
        sh_gaveup = 1;
        atomicOr(sync + 4, 1);
    }
    __syncthreads();
    if (wave != 0) return;
    // Lane l holds row l; at step j (solve order) the value of row j is
    // final, is broadcast, and every lane subtracts its coefficient of
    // column j times it.  The coefficients of a lane's own and later columns
    // are zero, so the step is one broadcast and one fused multiply-add over
    // the whole wavefront: a row already final takes v - 0 * x_j, which is v
    // unless x_j is not finite or v is a zero of the other sign than the
    // product.  The wavefront is issue-bound here, so this form (no per-step
    // selection of the final values) is the fast one; when any result is
    // zero or not finite, the block is solved again keeping each row's value
    // at its own step, which is exact in every case.  U is solved as U D^-1
    // (unit diagonal) for D x; x follows by one division per row.
    const double dg = LOWER ? 1.0 : Dg[lane];
    const double v0 = ok ? rhs - part[lane] : 0.0;
    double v = v0;
#pragma unroll
    for (int s = 0; s < TB; ++s) {
        const int j = LOWER ? s : TB - 1 - s;
        if (j < rows) v = v - Tr[j] * bcast(v, j);
    }
    double fin = v;
    if (__ballot(ok && (v == 0.0 || !__builtin_isfinite(v)))) {
        v = v0;
#pragma unroll 1
        for (int s = 0; s < rows; ++s) {
            const int j = LOWER ? s : rows - 1 - s;
            const double xj = bcast(v, j);
            fin = lane == j ? v : fin;
            v = v - Ts[lane][j] * xj;
        }
    }
    if constexpr (!LOWER) fin = fin / dg;
    v = fin;
    if (ok) {
        unsigned long long u = sh_gaveup ? kQuietNaN : (unsigned long long)__double_as_longlong(v);
        if (u == kUnsolved) u = kQuietNaN;
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(out + gi), u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (LOWER) in[gi] = __longlong_as_double((long long)kUnsolved);
    }
}

// x (n doubles, contiguous) holds P b on entry and the solution on return;
// y (n doubles) is the intermediate vector.
int trsv_one(int64_t n, const double *LU, int64_t lda, const int32_t *rm, double *x, double *y, int32_t *sync,
             int spin_limit, hipStream_t st)
{
    const int64_t nb = (n + TB - 1) / TB;
    if (nb > INT32_MAX) return CFX_ENOTSUP;
    hipLaunchKernelGGL(trsv_reset_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sync, y, n);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(trsv_sf_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, LU, lda, rm, x, y, n, (int)nb,
                       sync, spin_limit);
    CFX_HIP(hipGetLastError());
    hipLaunchKernelGGL(trsv_sf_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, LU, lda, rm, y, x, n, (int)nb,
                       sync, spin_limit);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

template <int NRC>
int trsv_impl(int64_t n, int nrhs, const double *LU, int64_t lda, const int32_t *rm, double *X, int64_t ldx,
              hipStream_t st)
{
    const int64_t nb = (n + SB - 1) / SB;
    const unsigned gy = (unsigned)((nrhs + NRC - 1) / NRC);
    auto bsz = [&](int64_t J) { return (int)((n - J * SB) < SB ? (n - J * SB) : SB); };
    auto cdiv = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    // forward: L y = x
    hipLaunchKernelGGL(fwd_step_kernel<NRC>, dim3(1, gy), dim3(256), 0, st, LU, lda, rm, X, ldx, n, nrhs,
                       (int64_t)-1, 0, (int64_t)0, bsz(0));
    CFX_HIP(hipGetLastError());
    for (int64_t J = 0; J + 1 < nb; ++J) {
        const int64_t c0 = J * SB, r0 = c0 + SB;
        const int bsn = bsz(J + 1);
        const int64_t below = n - r0 - bsn;
        const unsigned gx = (unsigned)(1 + cdiv(below, RPW));
        hipLaunchKernelGGL(fwd_step_kernel<NRC>, dim3(gx, gy), dim3(256), 0, st, LU, lda, rm, X, ldx, n, nrhs,
                           c0, SB, r0, bsn);
        CFX_HIP(hipGetLastError());
    }
    // backward: U x = y
    hipLaunchKernelGGL(bwd_step_kernel<NRC>, dim3(1, gy), dim3(256), 0, st, LU, lda, rm, X, ldx, nrhs,
                       (int64_t)-1, 0, (nb - 1) * SB, bsz(nb - 1));
    CFX_HIP(hipGetLastError());
    for (int64_t J = nb - 1; J >= 1; --J) {
        const int64_t c0 = J * SB, r0 = c0 - SB;
        const unsigned gx = (unsigned)(1 + cdiv(r0, RPW));
        hipLaunchKernelGGL(bwd_step_kernel<NRC>, dim3(gx, gy), dim3(256), 0, st, LU, lda, rm, X, ldx, nrhs, c0,
                           bsz(J), r0, SB);
        CFX_HIP(hipGetLastError());
    }
    return CFX_OK;
}

}  // namespace

int read_solve_flag(int32_t *sync, hipStream_t st, bool *gave_up)
{
    int32_t f = 0;
    CFX_HIP(hipMemcpyAsync(&f, sync + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CFX_HIP(hipStreamSynchronize(st));
    *gave_up = f != 0;
    if (f) {
        int rc = launch_set_int(sync + 4, 0, st);
        if (rc) return rc;
    }
    return CFX_OK;
}

int launch_perm(int64_t n, const int32_t *ipiv, int32_t *perm, hipStream_t st)
{
    if (n <= 0) return CFX_OK;
    if (n <= kPermLds)
        hipLaunchKernelGGL(perm_lds_kernel, dim3(1), dim3(64), 0, st, ipiv, (int)n, perm);
    else
        hipLaunchKernelGGL(perm_global_kernel, dim3(1), dim3(64), 0, st, ipiv, n, perm);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_gather_rows(int64_t n, int64_t nrhs, const double *B, int64_t ldb, const int32_t *perm, double *T,
                       int64_t ldt, hipStream_t st)
{
    const int64_t tot = n * nrhs;
    if (tot <= 0) return CFX_OK;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, B, ldb, perm,
                       n, nrhs, T, ldt);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_copy_rows(int64_t n, int64_t nrhs, const double *T, int64_t ldt, double *B, int64_t ldb,
                     hipStream_t st)
{
    const int64_t tot = n * nrhs;
    if (tot <= 0) return CFX_OK;
    hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, T, ldt, n, nrhs,
                       B, ldb);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_trsv(int64_t n, int64_t nrhs, const double *LU, int64_t lda, double *X, int64_t ldx, int32_t *sync,
                double *Y, hipStream_t st, int spin_limit, const int32_t *rm)
{
    if (n <= 0 || nrhs <= 0) return CFX_OK;
    if (nrhs == 1 && sync && Y && (ldx == 1 || n == 1)) return trsv_one(n, LU, lda, rm, X, Y, sync, spin_limit, st);
    if (nrhs == 1) return trsv_impl<1>(n, 1, LU, lda, rm, X, ldx, st);
    return trsv_impl<16>(n, (int)nrhs, LU, lda, rm, X, ldx, st);
}

int launch_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda, const int32_t *ipiv, double *B,
                 int64_t ldb, int32_t *perm, double *tmp, int32_t *sync, hipStream_t st, int spin_limit,
                 const int32_t *rm)
{
    if (n == 0 || nrhs == 0) return CFX_OK;
    int rc;
    // row masking: the row map is the permutation of P B itself
    const int32_t *pb = rm;
    if (!rm) {
        if ((rc = launch_perm(n, ipiv, perm, st))) return rc;
        pb = perm;
    }
    if ((rc = launch_gather_rows(n, nrhs, B, ldb, pb, tmp, nrhs, st))) return rc;
    // one right-hand side: the second n doubles of tmp are the solve's
    // intermediate vector
    if ((rc = launch_trsv(n, nrhs, LU, lda, tmp, nrhs, sync, nrhs == 1 ? tmp + n : nullptr, st, spin_limit, rm)))
        return rc;
    return launch_copy_rows(n, nrhs, tmp, nrhs, B, ldb, st);
}

}  // namespace cfx

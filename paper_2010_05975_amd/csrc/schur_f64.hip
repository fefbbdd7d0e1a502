// Schur-complement update A22 -= L21 U12 (FactorizeA11 of Alg. 1, the
// statement S2 of Sec. 6 that carries the leading 2N^3/3 flops) on the FP64
// matrix cores of gfx950.
//
// A workgroup of 4 wavefronts owns a 128 x 128 tile of C; each wavefront a
// 64 x 64 sub-tile held as 4 x 4 accumulators of v_mfma_f64_16x16x4f64.
// The K = vb reduction is staged through LDS in chunks of 16, double
// buffered: the next chunk is fetched into registers while the current one
// feeds the matrix cores.  Both operand tiles are stored k-major in LDS so
// that the 16 lanes of an MFMA operand row read 16 consecutive doubles.
// C is read once into the accumulators before the reduction (the L tile is
// staged negated, so the matrix cores accumulate C - L U) and written once,
// both non-temporal: C streams through without evicting the operand strips
// from L2, nor the data of the tournament kernels that run beside the
// update.
//
// With row masking (rows never interchanged) the rows of L21 and C, and of
// U12, are reached through row maps (logical row -> physical row): the
// MAPPED variants look up each tile row's physical row once per use.
//
// Tiles are mapped XCD-aware: consecutive workgroup ids land on different
// XCDs (each with its own L2), so ids are regrouped to give each XCD a
// contiguous, row-grouped range of tiles that share L21 and U12 strips.
#include "cfx_internal.h"

namespace cfx {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDA_S = BM + 16;   // padded k-major rows of the L tile
constexpr int LDB_S = BN + 16;
constexpr int GROUP_M = 8;
constexpr int NXCD = 8;

// Position `pos` of the regrouped order -> tile (ti, tj): grouped row-major,
// GROUP_M tile rows at a time, so that consecutive positions share L21 and
// U12 strips.
__device__ __forceinline__ void tile_at(int pos, int tm, int tn, int &ti, int &tj)
{
    const int group = pos / (GROUP_M * tn);
    const int first = group * GROUP_M;
    const int gsz = (tm - first) < GROUP_M ? (tm - first) : GROUP_M;
    const int r = pos - group * GROUP_M * tn;
    ti = first + r % gsz;
    tj = r / gsz;
}

// One 128 x 128 tile (ti, tj) of C -= L U.
// EDGE: the tile may cross the matrix edge or K is not a multiple of BK
// (every access is guarded).  VEC: operands are 16-byte aligned with even
// strides, so a thread fetches its 8 contiguous doubles as 4 x 16 bytes.
// The arithmetic is the same in every variant (the guards only substitute
// zeros and skip stores), so a tile's values do not depend on the variant.
template <bool EDGE, bool VEC, bool MAPPED>
__device__ __forceinline__ void schur_tile(const double *__restrict__ L, int64_t ldl, const double *__restrict__ U,
                                           int64_t ldu, double *__restrict__ C, int64_t ldc, int64_t mr, int64_t nc,
                                           int K, int ti, int tj, const int32_t *__restrict__ rmap,
                                           const int32_t *__restrict__ umap, double (*As)[BK * LDA_S],
                                           double (*Bs)[BK * LDB_S])
{
    // physical row of tile row i of L / C, and of row l of U
    auto crow = [&](int64_t i) -> int64_t {
        if constexpr (MAPPED) return (int64_t)rmap[(!EDGE || i < mr) ? i : 0];
        return i;
    };
    auto urow = [&](int64_t l) -> int64_t {
        if constexpr (MAPPED) return (int64_t)umap[(!EDGE || l < K) ? l : 0];
        return l;
    };
    const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;

    // global -> register staging assignment
    const int a_row = tid >> 1, a_col = (tid & 1) * 8;     // L tile: 128 rows x 16
    const int b_row = tid >> 4, b_col = (tid & 15) * 8;    // U tile: 16 rows x 128
    const int64_t lrow = crow(i0 + a_row);
    const double *Lp = L + lrow * ldl + a_col;
    const double *Up = U + (int64_t)b_row * ldu + j0 + b_col;
    double ra[8], rb[8];

    auto fetch = [&](int kc) {
        const int k0 = kc * BK;
        if constexpr (!EDGE && VEC) {
            const d2 *la = reinterpret_cast<const d2 *>(Lp + k0);
            const d2 *ub = reinterpret_cast<const d2 *>(
                MAPPED ? U + urow(k0 + b_row) * ldu + j0 + b_col : Up + (int64_t)k0 * ldu);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const d2 x = la[q], y = ub[q];
                ra[2 * q] = x[0]; ra[2 * q + 1] = x[1];
                rb[2 * q] = y[0]; rb[2 * q + 1] = y[1];
            }
        } else if constexpr (!EDGE) {
            const double *ub = MAPPED ? U + urow(k0 + b_row) * ldu + j0 + b_col : Up + (int64_t)k0 * ldu;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                ra[q] = Lp[k0 + q];
                rb[q] = ub[q];
            }
        } else {
            const int64_t gi = i0 + a_row;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = k0 + a_col + q;
                ra[q] = (gi < mr && kk < K) ? L[lrow * ldl + kk] : 0.0;
            }
            const int kb = k0 + b_row;
            const int64_t ur = urow(kb);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t gj = j0 + b_col + q;
                rb[q] = (kb < K && gj < nc) ? U[ur * ldu + gj] : 0.0;
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[buf][(a_col + q) * LDA_S + a_row] = -ra[q];
#pragma unroll
        for (int q = 0; q < 8; q += 2)
            *reinterpret_cast<d2 *>(&Bs[buf][b_row * LDB_S + b_col + q]) = d2{rb[q], rb[q + 1]};
    };

    // The accumulators start from C and the L tile is staged negated, so the
    // matrix cores produce C - L U directly and the epilogue only stores.
    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = j0 + wn + b * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = i0 + wm + a * 16 + lk + 4 * q;
                acc[a][b][q] = (!EDGE || (gi < mr && gj < nc)) ? __builtin_nontemporal_load(&C[crow(gi) * ldc + gj])
                                                                : 0.0;
            }
        }

    const int nk = (K + BK - 1) / BK;
    fetch(0);
    stash(0);
    __syncthreads();
    // every load of the prologue (C into the accumulators included) lands
    // here: otherwise the compiler may let some accumulator loads reach
    // into the loop, and the waits it then places inside the loop body
    // would also hold back every later chunk's prefetch
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) fetch(kc + 1);
        const double *as = As[buf];
        const double *bs = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[4], bf[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = as[(kk + lk) * LDA_S + wm + a * 16 + lr];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = bs[(kk + lk) * LDB_S + wn + b * 16 + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        if (kc + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }

    // epilogue: for v_mfma_f64_16x16x4f64 lane l holds rows l/16 + 4q
    // (q = 0..3) of column l%16 of each 16 x 16 block
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t gj = j0 + wn + b * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = i0 + wm + a * 16 + lk + 4 * q;
                if (!EDGE || (gi < mr && gj < nc)) __builtin_nontemporal_store(acc[a][b][q], &C[crow(gi) * ldc + gj]);
            }
        }
}

// Tiles are walked XCD-aware (below).  A ragged launch (EDGE) runs its
// interior tiles, which lie wholly inside the matrix, through the unguarded
// body and only the tiles on the edge through the guarded one.
template <bool EDGE, bool VEC, bool MAPPED>
__global__ __launch_bounds__(256, 2) void schur_f64_kernel(const double *__restrict__ L, int64_t ldl,
                                                           const double *__restrict__ U, int64_t ldu,
                                                           double *__restrict__ C, int64_t ldc,
                                                           int64_t mr, int64_t nc, int K, int tm, int tn,
                                                           const int32_t *__restrict__ rmap,
                                                           const int32_t *__restrict__ umap)
{
    __shared__ double As[2][BK * LDA_S];
    __shared__ double Bs[2][BK * LDB_S];

    // XCD-aware persistent schedule: the hardware sends workgroup b to XCD
    // b % 8.  XCD x owns the contiguous positions [x*per, (x+1)*per) (plus
    // position 8*per + x of the ragged end), and its workgroups walk them
    // with a stride of their count, so the tiles that share operand strips
    // stay in one L2.  With one workgroup per tile every workgroup takes
    // exactly one position.  Each tile ends with a barrier after its last K
    // chunk, so the next tile may refill the LDS buffers.
    const int nb = tm * tn;
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
    const int nsl = ((int)gridDim.x - xcd + NXCD - 1) / NXCD;   // workgroups on this XCD
    const int per = nb / NXCD;
    const int cnt = per + (xcd < nb - per * NXCD ? 1 : 0);
    const bool kfull = K % BK == 0;
#pragma unroll 1
    for (int it = slot; it < cnt; it += nsl) {
        int ti, tj;
        tile_at(it < per ? xcd * per + it : NXCD * per + xcd, tm, tn, ti, tj);
        if constexpr (EDGE) {
            if (kfull && (int64_t)(ti + 1) * BM <= mr && (int64_t)(tj + 1) * BN <= nc)
                schur_tile<false, VEC, MAPPED>(L, ldl, U, ldu, C, ldc, mr, nc, K, ti, tj, rmap, umap, As, Bs);
            else
                schur_tile<true, VEC, MAPPED>(L, ldl, U, ldu, C, ldc, mr, nc, K, ti, tj, rmap, umap, As, Bs);
        } else {
            schur_tile<false, VEC, MAPPED>(L, ldl, U, ldu, C, ldc, mr, nc, K, ti, tj, rmap, umap, As, Bs);
        }
    }
}

}  // namespace

int launch_schur_f64(const double *L, int64_t ldl, const double *U, int64_t ldu, double *C,
                     int64_t ldc, int64_t mr, int64_t nc, int K, int max_wgs, hipStream_t st,
                     const int32_t *rmap, const int32_t *umap)
{
    if (mr <= 0 || nc <= 0 || K <= 0) return CFX_OK;
    const int tm = (int)((mr + BM - 1) / BM), tn = (int)((nc + BN - 1) / BN);
    if ((int64_t)tm * tn > INT32_MAX) return CFX_ENOTSUP;
    int64_t nb = (int64_t)tm * tn;
    // a bounded grid (at least one workgroup per XCD) walks the tiles
    // persistently and leaves the rest of the device to concurrent work
    if (max_wgs > 0 && max_wgs < nb) nb = max_wgs < NXCD ? NXCD : max_wgs;
    const bool full = (mr % BM == 0) && (nc % BN == 0) && (K % BK == 0);
    const bool vec = ((reinterpret_cast<uintptr_t>(L) | reinterpret_cast<uintptr_t>(U)) & 15) == 0 &&
                     (ldl % 2 == 0) && (ldu % 2 == 0);
    if ((rmap == nullptr) != (umap == nullptr)) return CFX_ENOTSUP;   // both maps or none
    const dim3 grid((unsigned)nb), block(256);
#define CFX_SCHUR_LAUNCH(E, V, M)                                                                          \
    hipLaunchKernelGGL((schur_f64_kernel<E, V, M>), grid, block, 0, st, L, ldl, U, ldu, C, ldc, mr, nc, K, tm, tn, \
                       rmap, umap)
    if (rmap) {
        if (full) {
            if (vec) CFX_SCHUR_LAUNCH(false, true, true);
            else CFX_SCHUR_LAUNCH(false, false, true);
        } else {
            if (vec) CFX_SCHUR_LAUNCH(true, true, true);
            else CFX_SCHUR_LAUNCH(true, false, true);
        }
    } else if (full) {
        if (vec) CFX_SCHUR_LAUNCH(false, true, false);
        else CFX_SCHUR_LAUNCH(false, false, false);
    } else {
        if (vec) CFX_SCHUR_LAUNCH(true, true, false);
        else CFX_SCHUR_LAUNCH(true, false, false);
    }
#undef CFX_SCHUR_LAUNCH
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

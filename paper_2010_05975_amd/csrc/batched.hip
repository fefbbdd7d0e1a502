// Batched LU + solve of many independent small systems in one persistent
// launch.  Each system is the factorisation of Alg. 1 with one tournament
// leaf per panel (TP(v, 1): the leaf's GEPP is the panel's pivot search,
// Sec. 7.3), followed by the solve with its right-hand sides.
//
// Scheduling: a one-workgroup prologue sorts the systems by order n,
// largest first (counting sort), and clears the queue counter; the
// persistent kernel's workgroups then take systems from the sorted queue
// with an atomic ticket until it is empty (longest-processing-time-first
// keeps the tail short).  Every workgroup exits once the queue is drained.
//
// One system on one workgroup of 256 threads (n <= 512); the kernel needs
// about 460 registers per lane, so one workgroup is resident per compute
// unit and the persistent grid is one workgroup per compute unit.
//   panel    thread t owns rows t and t + 256; the panel's vb columns of
//            those rows live in registers (a window rotating by one column
//            per step).  Each pivot step is a wavefront argmax on integer
//            keys (DPP; ties to the smaller row) combined across the 4
//            wavefronts in LDS; rows move between owners through LDS.
//   swaps    the panel's interchanges, composed into (destination, source)
//            pairs, applied to the columns outside the panel (8 loads in
//            flight per thread before the values are staged in LDS).
//   U12      L11^{-1} A12, one column per thread, L11 in LDS.
//   Schur    A22 -= L21 U12 on the FP64 matrix cores (16x16x4 blocks,
//            32x32 per wavefront per pass): U12 staged once in LDS, each
//            wavefront walks tile rows with the row's L21 block in
//            registers and the next C block requested ahead.
//   solve    B gathered by the row permutation into LDS, forward and back
//            substitution in 32-row blocks (off-diagonal parts as dot
//            products with 16 factor values requested at once, diagonal
//            blocks by lane broadcast), written back.
// The panel width v per size class comes from the handle's tuning table.
#include <climits>
#include <utility>

#include "cfx_internal.h"

namespace cfx {
namespace {

constexpr int NT = 256;
constexpr int kMaxN = 512;
constexpr int kMaxRhs = 16;
constexpr int kMaxVB = 32;
constexpr int SBK = 32;   // substitution block

typedef double d4 __attribute__((ext_vector_type(4)));

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

struct Smem {
    // solve: permuted right-hand sides (stride kMaxRhs); factorisation:
    // staging of the interchanged rows, then of the panel's U12 rows
    double X[kMaxN * kMaxVB];
    double L11[kMaxVB * (kMaxVB + 1)];
    double rowP[kMaxVB], rowC[kMaxVB];
    unsigned long long redk[4];
    int redr[4];
    int perm[kMaxN];                  // position -> original row
    int iperm[kMaxN];                 // original row -> position before the panel
    int pivs[kMaxVB];
    int tdst[2 * kMaxVB], tsrc[2 * kMaxVB];
    int ntouch;
    int info;
    int ticket;
};

// The pivot order as an unsigned key: |a|'s bits + 1 (non-negative
// doubles order as their bit patterns), 0 for NaN and for rows that are not
// candidates, so a NaN never wins.
__device__ __forceinline__ unsigned long long piv_key(double a)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(a) & 0x7FFFFFFFFFFFFFFFull;
    return b > 0x7FF0000000000000ull ? 0ull : b + 1ull;
}

// Largest / smallest 32-bit value over the wavefront, uniform across lanes:
// a DPP butterfly inside each row of 16 lanes (xor 1, xor 2, half-mirror,
// mirror), then row broadcasts (lane 15 into rows 1 and 3, lane 31 into
// rows 2 and 3) leave the result in lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned a)
{
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0xB1, 0xF, 0xF, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x4E, 0xF, 0xF, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x141, 0xF, 0xF, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x140, 0xF, 0xF, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x142, 0xA, 0xF, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x143, 0xC, 0xF, false));
    return (unsigned)__builtin_amdgcn_readlane((int)a, 63);
}
__device__ __forceinline__ int wave_min_i32(int a)
{
    const int big = INT_MAX;
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0xB1, 0xF, 0xF, false));
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0x4E, 0xF, 0xF, false));
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0x141, 0xF, 0xF, false));
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0x140, 0xF, 0xF, false));
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0x142, 0xA, 0xF, false));
    a = min(a, __builtin_amdgcn_update_dpp(big, a, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(a, 63);
}

// The workgroup-wide pivot of column j of the panel: the largest key (the
// largest |value|), ties to the smaller row; INT_MAX when no row is a
// candidate or every candidate is NaN.  The wave's largest key (high
// words first, the low words only among lanes holding the largest high
// word), the lane holding it found by a ballot (a minimum over rows only
// when several lanes tie), then the 4 wavefronts' winners through LDS.
__device__ __forceinline__ int wg_argmax(unsigned long long key, int row, Smem &s)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(hi);
    const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
    const unsigned long long km = ((unsigned long long)mh << 32) | ml;
    const int cand = (key == km && km != 0ull) ? row : INT_MAX;
    const unsigned long long hits = __ballot(cand != INT_MAX);
    const int wr = hits == 0ull ? INT_MAX
                   : __popcll(hits) == 1 ? __builtin_amdgcn_readlane(cand, __ffsll((long long)hits) - 1)
                                         : wave_min_i32(cand);
    if (lane == 0) {
        s.redk[wave] = km;
        s.redr[wave] = wr;
    }
    __syncthreads();
    unsigned long long bk = s.redk[0];
    int br = s.redr[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        const unsigned long long ok = s.redk[w];
        const int orow = s.redr[w];
        if (ok > bk || (ok == bk && orow < br)) {
            bk = ok;
            br = orow;
        }
    }
    return bk == 0ull ? INT_MAX : br;
}

// One 32x32 block of A22 -= L21 U12 per wavefront pass, K = vb (zero
// padded to a multiple of 4).  f64 16x16x4 MFMA: A lane l = (row l%16,
// k l/16), B lane l = (k l/16, col l%16), D lane l element q = (row
// l/16 + 4q, col l%16).
template <int VB>
__device__ __forceinline__ void schur_tiles(double *A, int64_t lda, int n, int k, Smem &s)
{
    constexpr int KS = (VB + 3) / 4;     // k steps of 4
    const int m = n - k - VB;
    if (m <= 0) return;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int tiles = (m + 31) / 32;
    const int r0 = k + VB;
    // the panel's U12 rows (VB x m) staged once in LDS, zero beyond m and
    // VB; every tile then reads its U operand from there
    const int ldu = tiles * 32 + 4;
    double *Us = s.X;
    for (int e = t; e < 4 * KS * ldu; e += NT) {
        const int kk = e / ldu, j = e - kk * ldu;
        Us[e] = (kk < VB && j < m) ? A[(int64_t)(k + kk) * lda + r0 + j] : 0.0;
    }
    __syncthreads();
    // each wavefront walks whole tile rows: the tile row's L21 block is
    // loaded once into registers; the next tile's C block is requested
    // while the current one is on the matrix cores
    auto load_c = [&](int i0, int j0, d4 (&acc)[2][2]) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int gi = i0 + a * 16 + lk + 4 * q, gj = j0 + b * 16 + lr;
                    acc[a][b][q] = (gi < n && gj < n) ? A[(int64_t)gi * lda + gj] : 0.0;
                }
    };
    for (int ti = wave; ti < tiles; ti += 4) {
        const int i0 = r0 + ti * 32;
        double af[KS][2];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int kc = 4 * ks + lk;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int gi = i0 + a * 16 + lr;
                af[ks][a] = (gi < n && kc < VB) ? -A[(int64_t)gi * lda + k + kc] : 0.0;
            }
        }
        d4 acc[2][2];
        load_c(i0, r0, acc);
        for (int tj = 0; tj < tiles; ++tj) {
            const int j0 = r0 + tj * 32;
            d4 nxt[2][2];
            const bool more = tj + 1 < tiles;
            if (more) load_c(i0, j0 + 32, nxt);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                double bf[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) bf[b] = Us[(4 * ks + lk) * ldu + tj * 32 + b * 16 + lr];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks][a], bf[b], acc[a][b], 0, 0, 0);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int gi = i0 + a * 16 + lk + 4 * q, gj = j0 + b * 16 + lr;
                        if (gi < n && gj < n) A[(int64_t)gi * lda + gj] = acc[a][b][q];
                    }
            if (!more) break;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = nxt[a][b];
        }
    }
}

// One full-width panel of W columns at column k (k + W <= n): GEPP on rows
// k..n in registers, interchanges on the other columns, U12, Schur update.
// No loop unrolled over a compile-time range tests a run-time bound here
// (such masks are loop invariant and would be hoisted out of the
// persistent loop, all live at once).
template <int W>
__device__ __forceinline__ void panel(double *A, int64_t lda, int n, int k, int32_t *ipiv, Smem &s)
{
    const int t = threadIdx.x;
    double P[2][W];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = t + NT * q;
        const bool ok = r >= k && r < n;
        const double *row = A + (int64_t)(ok ? r : k) * lda + k;
        static_for<W>([&](auto C) {
            constexpr int c = decltype(C)::value;
            P[q][c] = row[c];
        });
    }
    // The pivot steps run as a loop (one copy of its body: the kernel's code
    // must stay small enough for the instruction cache), on a register
    // window that rotates left by one column per step: at step j, P[q][0]
    // holds column j, P[q][c] column j + c for c < W - j, and the finished
    // columns sit at the end; after W steps the window is back in order.
#pragma unroll 1
    for (int j = 0; j < W; ++j) {
        const int col = k + j;
        unsigned long long bk = 0ull;
        int br = INT_MAX;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = t + NT * q;
            const unsigned long long kq = (r >= col && r < n) ? piv_key(P[q][0]) : 0ull;
            if (kq > bk) {          // rows in increasing order: a tie keeps the smaller row
                bk = kq;
                br = r;
            }
        }
        int p = wg_argmax(bk, br, s);
        if (p == INT_MAX) p = col;
        // exchange rows col and p between their owners (whole rows, in the
        // window's order, which every thread shares)
        if (t == (p & (NT - 1))) {
            const int q = p >> 8;
            static_for<W>([&](auto C) {
                constexpr int c = decltype(C)::value;
                s.rowP[c] = q ? P[1][c] : P[0][c];
            });
        }
        if (t == (col & (NT - 1))) {
            const int q = col >> 8;
            static_for<W>([&](auto C) {
                constexpr int c = decltype(C)::value;
                s.rowC[c] = q ? P[1][c] : P[0][c];
            });
        }
        __syncthreads();
        if (p != col) {
            // value selects only (a store through a selected element address
            // would keep P out of registers)
            const bool own_c = t == (col & (NT - 1)), own_p = t == (p & (NT - 1));
            const int qc = col >> 8, qp = p >> 8;
            static_for<W>([&](auto C) {
                constexpr int c = decltype(C)::value;
                const double vp = s.rowP[c], vc = s.rowC[c];
                P[0][c] = (own_c && qc == 0) ? vp : (own_p && qp == 0) ? vc : P[0][c];
                P[1][c] = (own_c && qc == 1) ? vp : (own_p && qp == 1) ? vc : P[1][c];
            });
        }
        if (t == 0) {
            s.pivs[j] = p;
            ipiv[col] = p;
            const int a = s.perm[col];
            s.perm[col] = s.perm[p];
            s.perm[p] = a;
        }
        const double piv = s.rowP[0];
        if (piv != 0.0) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int r = t + NT * q;
                if (r > col && r < n) {
                    const double l = P[q][0] / piv;
                    P[q][0] = l;
                    static_for<W>([&](auto C) {
                        constexpr int c = decltype(C)::value;
                        if constexpr (c > 0)
                            if (c < W - j) P[q][c] -= l * s.rowP[c];
                    });
                }
            }
        } else if (t == 0 && s.info == 0) {
            s.info = col + 1;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double f = P[q][0];
            static_for<W - 1>([&](auto C) {
                constexpr int c = decltype(C)::value;
                P[q][c] = P[q][c + 1];
            });
            P[q][W - 1] = f;
        }
        __syncthreads();
    }
    // ---- write the panel back
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = t + NT * q;
        if (r >= k && r < n) {
            double *row = A + (int64_t)r * lda + k;
            static_for<W>([&](auto C) {
                constexpr int c = decltype(C)::value;
                row[c] = P[q][c];
            });
        }
    }
    // ---- the panel's interchanges on the other columns: destinations
    // k..k+W and every pivot row beyond; source = old position of the row
    // that now sits at the destination.
    if (t == 0) {
        int nt = 0;
        for (int j = 0; j < W; ++j) {
            s.tdst[nt] = k + j;
            s.tsrc[nt] = s.iperm[s.perm[k + j]];
            ++nt;
        }
        for (int j = 0; j < W; ++j) {
            const int p = s.pivs[j];
            if (p >= k + W) {
                bool seen = false;
                for (int e = W; e < nt; ++e) seen |= s.tdst[e] == p;
                if (!seen) {
                    s.tdst[nt] = p;
                    s.tsrc[nt] = s.iperm[s.perm[p]];
                    ++nt;
                }
            }
        }
        s.ntouch = nt;
    }
    __syncthreads();
    {
        // all sources of a column are read (staged in LDS) before any
        // destination is written; columns in chunks that fit the stage
        const int nt = s.ntouch;
        const int cw = (kMaxN * kMaxVB) / nt;
        for (int c0 = 0; c0 < n; c0 += cw) {
            const int cn = n - c0 < cw ? n - c0 : cw;
            const int tot = nt * cn;
            // 8 loads in flight per thread before their values are staged
            for (int e0 = t; e0 < tot; e0 += 8 * NT) {
                double val[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT;
                    if (e < tot) {
                        const int i = e / cn, cc = e - i * cn;
                        val[u] = A[(int64_t)s.tsrc[i] * lda + c0 + cc];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT;
                    if (e < tot) s.X[e] = val[u];
                }
            }
            __syncthreads();
            for (int e = t; e < nt * cn; e += NT) {
                const int i = e / cn, cc = e - i * cn, c = c0 + cc;
                if (c < k || c >= k + W) A[(int64_t)s.tdst[i] * lda + c] = s.X[e];
            }
            __syncthreads();
        }
    }
    // positions of the moved rows, for the next panel
    for (int e = t; e < s.ntouch; e += NT) {
        const int d = s.tdst[e];
        s.iperm[s.perm[d]] = d;
    }
    // L11 (unit lower) into LDS
    for (int e = t; e < W * W; e += NT) {
        const int i = e / W, j = e - i * W;
        s.L11[i * (kMaxVB + 1) + j] = A[(int64_t)(k + i) * lda + k + j];
    }
    __syncthreads();
    // ---- U12 = L11^{-1} A12, one column per thread
    for (int c = k + W + t; c < n; c += NT) {
        double x[W];
        static_for<W>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            x[q] = A[(int64_t)(k + q) * lda + c];
        });
        static_for<W>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            static_for<q>([&](auto R) {
                constexpr int r = decltype(R)::value;
                x[q] -= s.L11[q * (kMaxVB + 1) + r] * x[r];
            });
        });
        static_for<W>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            A[(int64_t)(k + q) * lda + c] = x[q];
        });
    }
    __syncthreads();
    schur_tiles<W>(A, lda, n, k, s);
    __syncthreads();
}

// Panels of width VB while they fit, then of 8, then single columns (every
// panel full width).
template <int VB>
__device__ __forceinline__ void factor(double *A, int64_t lda, int n, int32_t *ipiv, Smem &s)
{
    int k = 0;
    for (; k + VB <= n; k += VB) panel<VB>(A, lda, n, k, ipiv, s);
    if constexpr (VB > 8)
        for (; k + 8 <= n; k += 8) panel<8>(A, lda, n, k, ipiv, s);
    for (; k < n; ++k) panel<1>(A, lda, n, k, ipiv, s);
}

// sum_{j0 <= j < j1} row[j] X[j][c]: 16 factor values requested at once
// (each round one memory latency instead of one per element), four
// partial sums.
__device__ __forceinline__ double dot_rows(const double *row, int j0, int j1, const double *X, int c)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = j0;
    for (; j + 16 <= j1; j += 16) {
        double r[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) r[u] = row[j + u];
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
            s0 += r[u] * X[(j + u) * kMaxRhs + c];
            s1 += r[u + 1] * X[(j + u + 1) * kMaxRhs + c];
            s2 += r[u + 2] * X[(j + u + 2) * kMaxRhs + c];
            s3 += r[u + 3] * X[(j + u + 3) * kMaxRhs + c];
        }
    }
    for (; j < j1; ++j) s0 += row[j] * X[j * kMaxRhs + c];
    return (s0 + s1) + (s2 + s3);
}

// X (LDS, stride kMaxRhs) <- U^{-1} L^{-1} X with the factors in A.  The
// diagonal blocks are staged zero-padded in LDS (s.L11), so the unrolled
// elimination has no run-time tests.
__device__ __forceinline__ void solve(const double *A, int64_t lda, int n, int nrhs, Smem &s)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int LD = kMaxVB + 1;
    static_assert(SBK <= kMaxVB, "diagonal block must fit the L11 stage");
    // forward, unit L
    for (int I0 = 0; I0 < n; I0 += SBK) {
        const int bs = n - I0 < SBK ? n - I0 : SBK;
        for (int e = t; e < bs * nrhs; e += NT) {
            const int i = I0 + e / nrhs, c = e % nrhs;
            const double *row = A + (int64_t)i * lda;
            s.X[i * kMaxRhs + c] -= dot_rows(row, 0, I0, s.X, c);
        }
        // strictly lower part of the diagonal block, zero elsewhere
        for (int e = t; e < SBK * SBK; e += NT) {
            const int i = e / SBK, j = e - i * SBK;
            s.L11[i * LD + j] = (i < bs && j < i) ? A[(int64_t)(I0 + i) * lda + I0 + j] : 0.0;
        }
        __syncthreads();
        if (lane < SBK) {
            const bool okr = lane < bs;
            for (int c = wave; c < nrhs; c += 4) {
                double x = okr ? s.X[(I0 + lane) * kMaxRhs + c] : 0.0;
                static_for<SBK>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    x -= s.L11[lane * LD + j] * bcast(x, j);
                });
                if (okr) s.X[(I0 + lane) * kMaxRhs + c] = x;
            }
        }
        __syncthreads();
    }
    // backward, U: lane j's value is final (undivided) at step j; every
    // other lane uses x_j / u_jj, and each lane divides its own at the end
    for (int I0 = ((n - 1) / SBK) * SBK; I0 >= 0; I0 -= SBK) {
        const int bs = n - I0 < SBK ? n - I0 : SBK;
        const int j1 = I0 + bs;
        for (int e = t; e < bs * nrhs; e += NT) {
            const int i = I0 + e / nrhs, c = e % nrhs;
            const double *row = A + (int64_t)i * lda;
            s.X[i * kMaxRhs + c] -= dot_rows(row, j1, n, s.X, c);
        }
        // strictly upper part (zero elsewhere) and the diagonal (1 outside)
        for (int e = t; e < SBK * SBK; e += NT) {
            const int i = e / SBK, j = e - i * SBK;
            double v = 0.0;
            if (i < bs && j < bs && j >= i) v = A[(int64_t)(I0 + i) * lda + I0 + j];
            if (j == i && i >= bs) v = 1.0;
            s.L11[i * LD + j] = v;
        }
        __syncthreads();
        if (lane < SBK) {
            const bool okr = lane < bs;
            const double d = s.L11[lane * LD + lane];
            for (int c = wave; c < nrhs; c += 4) {
                double x = okr ? s.X[(I0 + lane) * kMaxRhs + c] : 0.0;
                static_for<SBK>([&](auto J) {
                    constexpr int j = SBK - 1 - decltype(J)::value;
                    const double xj = bcast(x, j) / s.L11[j * LD + j];
                    // lanes above j subtract u_ij x_j; lane j and below see
                    // a zero (u_jj is excluded: the diagonal is applied below)
                    const double u = j > lane ? s.L11[lane * LD + j] : 0.0;
                    x -= u * xj;
                });
                x = x / d;
                if (okr) s.X[(I0 + lane) * kMaxRhs + c] = x;
            }
        }
        __syncthreads();
    }
}

struct BatchArgs {
    int count;
    const int32_t *n, *nrhs;
    double *const *A;
    const int64_t *lda;
    double *const *B;
    const int64_t *ldb;
    int32_t *const *ipiv;
    int32_t *info;
    int32_t *order;
    int32_t *counter;
    int32_t vb_class[kBatchClasses];
};

__device__ __forceinline__ int size_class(int n)
{
    return n <= 32 ? 0 : n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 3 : 4;
}

// Counting sort of the systems by n, descending (invalid sizes last), and
// the queue counter reset.  One workgroup.
__global__ __launch_bounds__(1024) void batched_prep_kernel(BatchArgs a)
{
    __shared__ int hist[kMaxN + 2];
    __shared__ int base[kMaxN + 2];
    for (int b = threadIdx.x; b < kMaxN + 2; b += 1024) hist[b] = 0;
    if (threadIdx.x == 0) a.counter[0] = 0;
    __syncthreads();
    // bucket 0 holds n = kMaxN, ..., bucket kMaxN holds n = 0, kMaxN + 1 invalid
    for (int i = threadIdx.x; i < a.count; i += 1024) {
        const int nn = a.n[i];
        const int b = (nn < 0 || nn > kMaxN) ? kMaxN + 1 : kMaxN - nn;
        atomicAdd(&hist[b], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int b = 0; b < kMaxN + 2; ++b) {
            base[b] = run;
            run += hist[b];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.count; i += 1024) {
        const int nn = a.n[i];
        const int b = (nn < 0 || nn > kMaxN) ? kMaxN + 1 : kMaxN - nn;
        const int pos = atomicAdd(&base[b], 1);
        a.order[pos] = i;
    }
}

__global__ __launch_bounds__(NT) void batched_gesv_kernel(BatchArgs a)
{
    __shared__ Smem s;
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) s.ticket = atomicAdd(a.counter, 1);
        __syncthreads();
        const int idx = s.ticket;
        __syncthreads();
        if (idx >= a.count) break;
        const int sys = a.order[idx];
        const int n = a.n[sys], nrhs = a.nrhs[sys];
        const int64_t lda = a.lda[sys], ldb = a.ldb[sys];
        double *A = a.A[sys];
        double *B = a.B[sys];
        int32_t *ipiv = a.ipiv[sys];
        int bad = 0;
        if (n < 0 || n > kMaxN) bad = 1;
        else if (n > 0 && (A == nullptr || ipiv == nullptr)) bad = 2;
        else if (lda < (n > 1 ? n : 1)) bad = 3;
        else if (nrhs < 0 || nrhs > kMaxRhs) bad = 4;
        else if (n > 0 && nrhs > 0 && B == nullptr) bad = 5;
        else if (ldb < (nrhs > 1 ? nrhs : 1)) bad = 6;
        if (bad) {
            if (t == 0) a.info[sys] = -bad;
            continue;
        }
        if (n == 0) {
            if (t == 0) a.info[sys] = 0;
            continue;
        }
        for (int i = t; i < n; i += NT) {
            s.perm[i] = i;
            s.iperm[i] = i;
        }
        if (t == 0) s.info = 0;
        __syncthreads();
        const int vb = a.vb_class[size_class(n)];
        if (vb <= 8) factor<8>(A, lda, n, ipiv, s);
        else if (vb <= 16) factor<16>(A, lda, n, ipiv, s);
        else factor<32>(A, lda, n, ipiv, s);
        if (nrhs > 0) {
            for (int e = t; e < n * nrhs; e += NT) {
                const int i = e / nrhs, c = e % nrhs;
                s.X[i * kMaxRhs + c] = B[(int64_t)s.perm[i] * ldb + c];
            }
            __syncthreads();
            solve(A, lda, n, nrhs, s);
            for (int e = t; e < n * nrhs; e += NT) {
                const int i = e / nrhs, c = e % nrhs;
                B[(int64_t)i * ldb + c] = s.X[i * kMaxRhs + c];
            }
        }
        if (t == 0) a.info[sys] = s.info;
        __syncthreads();
    }
}

}  // namespace

size_t batched_work_bytes(int32_t count)
{
    return 256 + (((size_t)(count > 0 ? count : 0) * sizeof(int32_t) + 255) & ~(size_t)255);
}

int launch_gesv_batched(int32_t count, const int32_t *n, const int32_t *nrhs, double *const *A,
                        const int64_t *lda, double *const *B, const int64_t *ldb, int32_t *const *ipiv,
                        int32_t *info, void *work, const int32_t *vb_class, int grid, hipStream_t st)
{
    if (count <= 0) return CFX_OK;
    BatchArgs a;
    a.count = count;
    a.n = n;
    a.nrhs = nrhs;
    a.A = A;
    a.lda = lda;
    a.B = B;
    a.ldb = ldb;
    a.ipiv = ipiv;
    a.info = info;
    a.counter = static_cast<int32_t *>(work);
    a.order = reinterpret_cast<int32_t *>(static_cast<char *>(work) + 256);
    for (int c = 0; c < kBatchClasses; ++c) a.vb_class[c] = vb_class[c];
    hipLaunchKernelGGL(batched_prep_kernel, dim3(1), dim3(1024), 0, st, a);
    CFX_HIP(hipGetLastError());
    const int g = grid < count ? grid : count;
    hipLaunchKernelGGL(batched_gesv_kernel, dim3(g), dim3(NT), 0, st, a);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

namespace cfx {
namespace {

// Tuner input: entries in [-1, 1) from a counter hash (splitmix64 of the
// element index and seed) plus 2 sqrt(n) on the diagonal.
__global__ void synth_kernel(double *A, int n, int64_t total, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    uint64_t z = (uint64_t)e + seed * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    double v = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const int64_t local = e % ((int64_t)n * n);
    if (local / n == local % n) v += 2.0 * sqrt((double)n);
    A[e] = v;
}

}  // namespace

int launch_batched_synth(double *A, int n, int64_t count, uint64_t seed, hipStream_t st)
{
    const int64_t total = count * n * n;
    if (total <= 0) return CFX_OK;
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, A, n, total, seed);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

namespace cfx {
namespace {

__device__ __forceinline__ void two_sum_b(double a, double b, double &s, double &e)
{
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// eta_i = max over the right-hand sides c of system i of
// |b - A x|_inf / (|A|_inf |x|_inf + |b|_inf), residual rows summed with
// compensated (Dot2) sums.  One workgroup per system, one wavefront per
// row at a time.
__global__ __launch_bounds__(256) void batched_eta_kernel(int count, const int32_t *nv, const int32_t *rv,
                                                          double *const *Av, const int64_t *ldav,
                                                          double *const *Bv, const int64_t *ldbv,
                                                          double *const *Xv, const int64_t *ldxv, double *eta)
{
#pragma clang fp contract(off)
    __shared__ double red[4][4];
    const int sys = blockIdx.x;
    if (sys >= count) return;
    const int n = nv[sys], nrhs = rv[sys];
    const double *A = Av[sys];
    const double *B = Bv[sys];
    const double *X = Xv[sys];
    const int64_t lda = ldav[sys], ldb = ldbv[sys], ldx = ldxv[sys];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        double rmax = 0.0, xmax = 0.0, bmax = 0.0, amax = 0.0;
        for (int i = wave; i < n; i += 4) {
            const double *row = A + (int64_t)i * lda;
            double s = 0.0, cc = 0.0, ab = 0.0;
            for (int j = lane; j < n; j += 64) {
                const double a = row[j], x = X[(int64_t)j * ldx + c];
                const double p = a * x;
                const double e = fma(a, x, -p);
                double t;
                two_sum_b(s, p, s, t);
                cc += t + e;
                ab += fabs(a);
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const double so = __shfl_xor(s, off), co = __shfl_xor(cc, off);
                double t;
                two_sum_b(s, so, s, t);
                cc += co + t;
                ab += __shfl_xor(ab, off);
            }
            double u, e;
            const double bi = B[(int64_t)i * ldb + c];
            two_sum_b(bi, -s, u, e);
            const double r = fabs(u + (e - cc));
            const double xi = fabs(X[(int64_t)i * ldx + c]);
            rmax = (r > rmax || r != r) ? r : rmax;
            xmax = (xi > xmax || xi != xi) ? xi : xmax;
            bmax = fabs(bi) > bmax ? fabs(bi) : bmax;
            amax = ab > amax ? ab : amax;
        }
        if (lane == 0) {
            red[wave][0] = rmax;
            red[wave][1] = xmax;
            red[wave][2] = bmax;
            red[wave][3] = amax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m[4] = {0, 0, 0, 0};
            for (int w = 0; w < 4; ++w)
                for (int q = 0; q < 4; ++q) {
                    const double v = red[w][q];
                    m[q] = (v > m[q] || v != v) ? v : m[q];
                }
            const double den = m[3] * m[1] + m[2];
            double e;
            if (m[0] != m[0] || m[1] != m[1] || !(m[1] < INFINITY)) e = NAN;
            else e = den > 0 ? m[0] / den : (m[0] > 0 ? INFINITY : 0.0);
            worst = (e > worst || e != e) ? e : worst;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) eta[sys] = worst;
}

}  // namespace

int launch_batched_eta(int count, const int32_t *n, const int32_t *nrhs, double *const *A, const int64_t *lda,
                       double *const *B, const int64_t *ldb, double *const *X, const int64_t *ldx, double *eta,
                       hipStream_t st)
{
    if (count <= 0) return CFX_OK;
    hipLaunchKernelGGL(batched_eta_kernel, dim3(count), dim3(256), 0, st, count, n, nrhs, A, lda, B, ldb, X, ldx,
                       eta);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

}  // namespace cfx

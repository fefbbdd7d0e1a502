// Tournament pivoting (TournPivot of Alg. 1; Sec. 7.3 "Pivoting in COnfLUX";
// Sec. 7.4, Step 1) on gfx950.
//
// Each node of the tournament is a leaf (h consecutive rows of the panel)
// or a merge of two children's candidate rows, stacked left child first and
// taken with their current-step panel values.  A node selects min(vb, rows)
// rows by Gaussian elimination with partial pivoting, ties to the smallest
// global row.  The elimination of a node is blocked by BW = 32 columns; each
// block of one tree level is two launches:
//
//  P (one workgroup of 256 threads per node): thread t owns physical rows
//    t, t+NT, ... and keeps their block columns in registers.  Pivot steps:
//    each thread scores its unselected rows; two branch-free DPP/readlane
//    reductions give the wave's best score and the smallest global row
//    holding it; that row publishes the rest of its sub-panel into a
//    double-buffered LDS slot; one barrier; every thread picks the overall
//    winner from the slots and eliminates its rows against it.  Selected
//    rows are frozen, so their owners publish them whole once per
//    sub-panel, for the U rows of the rest of the block.  The node's state
//    (selection, row mask, negated U rows) is kept in the workspace between
//    launches.
//  E (many workgroups, all nodes of the level): the rank-BW update of the
//    trailing columns on the FP64 matrix cores, C^T -= U^T L^T, in 64 x 64
//    tiles; a node's update is spread over the whole GPU instead of being
//    bound by one compute unit's memory bandwidth.
//
// The node's panel block lives in a column-major scratch block (element
// (c, p) at c*rc + p): a wavefront touching one column of 64 consecutive
// rows makes one coalesced access, and the matrix-core tiles read and write
// 128-byte row runs.  Rows are never moved: selected rows are marked, and the
// selection order is kept.  In exact arithmetic this is the unblocked
// elimination, so the selection is the same.
//
// The root also turns its selection into LAPACK-style interchanges (ipiv)
// and a row-move plan for the swap kernel, and copies its factored top
// vb x vb block (L00 and U00 of the panel) out.
#include <climits>
#include <utility>

#include "cfx_internal.h"

namespace cfx {
namespace {


typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

struct NodeArgs {
    const double *W;        // panel origin: global row row0, first panel column
    int64_t ldw;
    int64_t row0;           // global index of panel row 0
    int64_t rows;           // panel rows
    int vb;                 // panel width (<= kMaxV)
    int leaf;               // 1: leaf level, 0: merge level
    int64_t h;              // leaf height
    const int32_t *cand_in; // merge level: children's candidates
    const int32_t *ccnt_in;
    int nn_in;              // merge level: number of child nodes
    int32_t *cand_out;
    int32_t *ccnt_out;
    double *S;              // node scratch (column-major per node)
    int64_t s_node;
    int rc;                 // scratch column stride = max rows of a node
    int root;               // this launch is the root
    int32_t *piv_out;       // root: selected global rows (may be null)
    double *lu00;           // root: factored top block
    int32_t *ipiv;          // root: interchanges, global indexing (may be null)
    int32_t *plan;          // root: row-move plan (may be null)
    int32_t *info;          // root: first zero pivot (may be null)
    const int32_t *rm;      // row masking: global row g is physical row rm[g] of W (else g - row0)
    int32_t *selg;          // per node: selected global rows [kMaxV], physical rows [kMaxV]
    unsigned char *rsel;    // per node: row already selected [rs_node]
    int rs_node;
    double *utg;            // per node: U rows of the previous block [32 x kMaxV]
    double *rtg;            // per node: the block's unit-lower triangle [32 x 40]
    int jb;                 // first column of the current block
};

// Compile-time loop: f(std::integral_constant<int, 0>) ... f(<N-1>), so that
// register arrays are only ever indexed by constants.
template <typename F, int... J>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ double max2(double a, double b) { return b > a ? b : a; }

// Smallest integer over the wavefront, uniform across lanes (same pattern).
__device__ __forceinline__ int wave_min(int g)
{
    g = min(g, __builtin_amdgcn_update_dpp(0, g, 0xB1, 0xF, 0xF, false));
    g = min(g, __builtin_amdgcn_update_dpp(0, g, 0x4E, 0xF, 0xF, false));
    g = min(g, __builtin_amdgcn_update_dpp(0, g, 0x141, 0xF, 0xF, false));
    g = min(g, __builtin_amdgcn_update_dpp(0, g, 0x140, 0xF, 0xF, false));
    return min(min(__builtin_amdgcn_readlane(g, 0), __builtin_amdgcn_readlane(g, 16)),
               min(__builtin_amdgcn_readlane(g, 32), __builtin_amdgcn_readlane(g, 48)));
}

// Score of a candidate value: |a|; NaN ranks below every number but above
// "not a candidate" (-1), so a block of NaNs still yields a pivot.
__device__ __forceinline__ double score(double a)
{
    const double s = fabs(a);
    return s == s ? s : -0.5;
}

// The same order as an unsigned integer key (the bit patterns of
// non-negative doubles order as the values do): 0 = not a candidate,
// 1 = NaN, |a| -> its bits + 2.  Integer reductions keep the argmax off the
// FP64 pipeline.
__device__ __forceinline__ unsigned long long score_key(double a)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(a) & 0x7FFFFFFFFFFFFFFFull;
    return b > 0x7FF0000000000000ull ? 1ull : b + 2ull;
}

// Largest unsigned value over the wavefront, uniform across lanes: a DPP
// butterfly inside each row of 16 lanes (xor 1, xor 2, half-mirror,
// mirror leave the row's maximum in every lane of the row), then row
// broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3) leave
// the wave's maximum in lane 63.
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

// Largest 64-bit key over the wavefront: the high words first; the low
// words only among the lanes holding the largest high word (one lane in
// the usual case, read directly).
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long k)
{
    const unsigned hi = (unsigned)(k >> 32), lo = (unsigned)k;
    const unsigned mh = wave_max_u32(hi);
    const unsigned long long at = __ballot(hi == mh);
    const unsigned ml = __popcll(at) == 1 ? (unsigned)__builtin_amdgcn_readlane((int)lo, __ffsll((long long)at) - 1)
                                          : wave_max_u32(hi == mh ? lo : 0u);
    return ((unsigned long long)mh << 32) | ml;
}

constexpr int UTLD = kMaxV;                 // row stride of the saved U rows

template <int RPT>
struct BlockW {
    static constexpr int value = (64 / RPT) < 32 ? (64 / RPT) : 32;
};

struct __attribute__((aligned(16))) Slot {
    double v;   // the wave's best row's value in the pivot column
    int g;      // smallest global row with the best score
    int p;      // its physical row in the node (-1: no candidate in the wave)
};

template <int BW, int NWV>
struct Lds {
    double cand[2][NWV][8];     // each wave's best row: its current sub-panel values
    Slot slot[2][NWV];          // each wave's best score, row and physical row
    double RT[BW][BW + 8];      // RT[l][i] = multiplier of block pivot i on pivot l
    double PR[8][BW + 2];       // the current sub-panel's pivot rows
    union {
        double tile[64 * 65];   // gather: transpose staging
        int plan_tmp[2 * kMaxV];
    };
    int sel[kMaxV];             // selected global rows, in order
    int selp[kMaxV];            // physical scratch row of each selected row
    unsigned char rowsel[kMaxLeafRows];   // physical row already selected
};

// Rows of node `node` at this level; 0 for a promoted (unpaired) node.
struct NodeRows {
    int r = 0;
    int cl = 0;
    int64_t leaf_first = 0;
    const int32_t *cl_list = nullptr, *cr_list = nullptr;
    bool promoted = false;
};

__device__ __forceinline__ NodeRows node_rows(const NodeArgs &p, int node)
{
    NodeRows n;
    if (p.leaf) {
        n.leaf_first = (int64_t)node * p.h;
        const int64_t last = n.leaf_first + p.h < p.rows ? n.leaf_first + p.h : p.rows;
        n.r = (int)(last - n.leaf_first);
    } else {
        const int a = 2 * node;
        if (a + 1 >= p.nn_in) {
            n.promoted = true;
            return n;
        }
        n.cl = p.ccnt_in[a];
        n.r = n.cl + p.ccnt_in[a + 1];
        n.cl_list = p.cand_in + (size_t)a * p.vb;
        n.cr_list = p.cand_in + (size_t)(a + 1) * p.vb;
    }
    return n;
}

__device__ __forceinline__ int node_gid(const NodeArgs &p, const NodeRows &n, int pr)
{
    if (p.leaf) return (int)(p.row0 + n.leaf_first + pr);
    return pr < n.cl ? n.cl_list[pr] : n.cr_list[pr - n.cl];
}

// ---------------------------------------------------------------------------
// P: pivot steps and U rows of one block, one workgroup per node.
// ---------------------------------------------------------------------------
template <int RPT, int NT>
__device__ __forceinline__ void panel_block(const NodeArgs &p, const int node, const int jb,
                                            Lds<BlockW<RPT>::value, NT / 64> &s)
{
    constexpr int BW = BlockW<RPT>::value;
    constexpr int NW = NT / 64;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int vb = p.vb;
    const int rc = p.rc;

    const NodeRows nr = node_rows(p, node);
    if (nr.promoted) {                        // unpaired: promoted unchanged
        if (jb == 0) {
            const int a = 2 * node;
            const int c = p.ccnt_in[a];
            for (int i = tid; i < c; i += NT) p.cand_out[(size_t)node * vb + i] = p.cand_in[(size_t)a * vb + i];
            if (tid == 0) p.ccnt_out[node] = c;
        }
        return;
    }
    const int r = nr.r;
    const int nsel = r < vb ? r : vb;
    if (jb >= nsel) return;
    const int bwc = (nsel - jb) < BW ? (nsel - jb) : BW;
    const int tc0 = jb + bwc;            // first trailing column
    const int ncol = nsel - tc0;         // trailing columns that matter

    double *Sn = p.S + (size_t)node * p.s_node;
    int32_t *selg = p.selg + (size_t)node * 2 * kMaxV;
    unsigned char *rselg = p.rsel + (size_t)node * p.rs_node;
    double *utg = p.utg + (size_t)node * 32 * UTLD;
    double *rtg = p.rtg + (size_t)node * 32 * 40;

    // this thread's rows and their block columns are requested first: they
    // do not depend on the node state below, so the loads overlap (rows
    // selected in earlier blocks are loaded too but never used; the root's
    // U-row copy below only writes such rows)
    int gid[RPT];
    static_for<RPT>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        const int pr = tid + q * NT;
        gid[q] = pr < r ? node_gid(p, nr, pr) : INT_MAX;
    });
    // x: the block columns of this thread's rows.  The block is eliminated
    // in sub-panels of SP columns: x[q][0..SP) always holds the current
    // sub-panel (the register window shifts left by SP after each one), so
    // only SP pivot steps are unrolled.
    constexpr int SP = BW < 8 ? BW : 8;
    double x[RPT][BW];
    static_for<RPT>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        const int pr = tid + q * NT;
#pragma unroll
        for (int c = 0; c < BW; ++c)
            x[q][c] = (pr < r && c < bwc) ? Sn[(size_t)(jb + c) * rc + pr] : 0.0;
    });
    if (jb > 0) {
        for (int i = tid; i < jb; i += NT) {
            s.sel[i] = selg[i];
            s.selp[i] = selg[kMaxV + i];
        }
    }
    for (int i = tid; i < r; i += NT) s.rowsel[i] = rselg[i];
    __syncthreads();
    if (jb > 0 && p.root) {
        // the previous block's U rows (computed by the update launch) go
        // into their pivot rows of the scratch block; only the root's
        // factored block is an output (other nodes hand on their selection
        // alone, and a selected row is never read again by its node)
        // One column per thread, all its loads issued before its stores (the
        // two arrays could alias, so a load-store loop would run one global
        // round trip per element).
        const int pj0 = jb - BW, ncp = nsel - jb;
        for (int c = tid; c < ncp; c += NT) {
            double u[BW];
#pragma unroll
            for (int i = 0; i < BW; ++i) u[i] = utg[(size_t)i * UTLD + c];
#pragma unroll
            for (int i = 0; i < BW; ++i) Sn[(size_t)(jb + c) * rc + s.selp[pj0 + i]] = u[i];
        }
        __syncthreads();    // the copies above land before the block's outputs
    }

    bool live[RPT];     // a real row that is not selected yet
    static_for<RPT>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        const int pr = tid + q * NT;
        live[q] = pr < r && !s.rowsel[pr];
    });

    {
        for (int sp0 = 0; sp0 < bwc; sp0 += SP) {
            const int spc = (bwc - sp0) < SP ? (bwc - sp0) : SP;   // steps in this sub-panel
            const int rem = bwc - sp0 - SP;                        // block columns right of it
            bool open[RPT];     // live when the sub-panel starts: writes its columns back
            int selstep[RPT];   // step of this sub-panel that selected the row, or -1
            static_for<RPT>([&](auto QC) {
                constexpr int q = decltype(QC)::value;
                open[q] = live[q];
                selstep[q] = -1;
            });
            static_for<SP>([&](auto JC) {
                constexpr int j = decltype(JC)::value;
                if (j < spc) {
                    const int par = j & 1;
                    // this thread's scores and the wave's best score (exact,
                    // as integer keys of the same order)
                    unsigned long long kq[RPT];
                    unsigned long long km = 0;
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        kq[q] = live[q] ? score_key(x[q][j]) : 0ull;
                        km = kq[q] > km ? kq[q] : km;
                    });
                    km = wave_max_key(km);
                    // the smallest global row of this lane scoring km; one
                    // lane holding it (the usual case) needs no reduction
                    int lg = INT_MAX;
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        lg = kq[q] == km ? min(lg, gid[q]) : lg;
                    });
                    const unsigned long long hits = __ballot(lg != INT_MAX);
                    const int wg = __popcll(hits) == 1 ? __builtin_amdgcn_readlane(lg, __ffsll((long long)hits) - 1)
                                                       : wave_min(lg);
                    // the row (unique: global rows are distinct) publishes its
                    // sub-panel values from column j on; a wave without
                    // candidates publishes an empty slot
                    if (wg != INT_MAX) {
                        static_for<RPT>([&](auto QC) {
                            constexpr int q = decltype(QC)::value;
                            if (gid[q] == wg) {
                                // km == 0: no candidate in this wave
                                s.slot[par][wave] = Slot{x[q][j], wg, km ? tid + q * NT : -1};
#pragma unroll
                                for (int cc = j; cc < SP; ++cc) s.cand[par][wave][cc] = x[q][cc];
                            }
                        });
                    } else if (lane == 0) {
                        s.slot[par][wave] = Slot{0.0, INT_MAX, -1};
                    }
                    __syncthreads();
                    // the node's winner: best score, ties to the smallest
                    // global row (some row is live at every step, so the
                    // best score is at least -0.5)
                    Slot sl[NW];
                    double sw[NW];      // the waves' best scores (-1: none)
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        sl[w] = s.slot[par][w];
                        sw[w] = sl[w].p < 0 ? -1.0 : score(sl[w].v);
                    }
                    double M = sw[0];
#pragma unroll
                    for (int w = 1; w < NW; ++w) M = max2(M, sw[w]);
                    int Gw = INT_MAX;
#pragma unroll
                    for (int w = 0; w < NW; ++w) Gw = sw[w] == M ? min(Gw, sl[w].g) : Gw;
                    int mw = 0, pw = sl[0].p;
                    double piv = sl[0].v;
#pragma unroll
                    for (int w = 1; w < NW; ++w) {
                        mw = sl[w].g == Gw ? w : mw;
                        pw = sl[w].g == Gw ? sl[w].p : pw;
                        piv = sl[w].g == Gw ? sl[w].v : piv;
                    }
                    // the rest of the pivot row is requested now; the pivot
                    // itself came with the slot
                    const double *prow = &s.cand[par][mw][0];
                    double pv[SP];
#pragma unroll
                    for (int cc = j + 1; cc < SP; ++cc) pv[cc] = prow[cc];
                    if (tid == 0) {
                        s.sel[jb + sp0 + j] = Gw;
                        s.selp[jb + sp0 + j] = pw;
                        s.rowsel[pw] = 1;
                    }
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        if (tid + q * NT == pw) {
                            live[q] = false;
                            selstep[q] = j;
                        }
                    });
                    if (piv != 0.0) {
                        static_for<RPT>([&](auto QC) {
                            constexpr int q = decltype(QC)::value;
                            if (live[q]) {
                                const double l = x[q][j] / piv;
                                x[q][j] = l;
#pragma unroll
                                for (int cc = j + 1; cc < SP; ++cc) x[q][cc] -= l * pv[cc];
                            }
                        });
                    }
                }
            });

            // the sub-panel's columns are final for this block
            static_for<RPT>([&](auto QC) {
                constexpr int q = decltype(QC)::value;
                const int pr = tid + q * NT;
                if (open[q]) {
#pragma unroll
                    for (int c = 0; c < SP; ++c)
                        if (c < spc) Sn[(size_t)(jb + sp0 + c) * rc + pr] = x[q][c];
                }
            });
            if (rem > 0) {
                // the sub-panel's pivot rows as they were when selected
                // (frozen since), from the threads that hold them
                static_for<RPT>([&](auto QC) {
                    constexpr int q = decltype(QC)::value;
                    if (selstep[q] >= 0) {
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc) s.PR[selstep[q]][cc] = x[q][cc];
                    }
                });
                __syncthreads();
                // U rows of the sub-panel's pivots at the rest of the block:
                // PR[i][SP + c] -= sum_{l<i} PR[i][l] * U[l][SP + c]
                if (tid < rem) {
                    // one column per thread, kept in registers (the same
                    // operations in the same order as updating PR in place)
                    const int c = SP + tid;
                    double uc[SP];
#pragma unroll
                    for (int i = 0; i < SP; ++i) uc[i] = s.PR[i][c];
#pragma unroll
                    for (int i = 1; i < SP; ++i) {
#pragma unroll
                        for (int l = 0; l < SP; ++l)
                            if (l < i) uc[i] -= s.PR[i][l] * uc[l];
                    }
                    // the sub-panel's pivot rows hold U rows in the rest of the block
#pragma unroll
                    for (int i = 0; i < SP; ++i) {
                        s.PR[i][c] = uc[i];
                        Sn[(size_t)(jb + sp0 + c) * rc + s.selp[jb + sp0 + i]] = uc[i];
                    }
                }
                __syncthreads();
                // rank-SP update of the rest of the block: pivot by pivot,
                // the pivot's U row (up to BW - SP values) requested from
                // LDS at once, then every remaining column of this thread's
                // live rows (per element the same subtractions in the same
                // order as a column-by-column loop)
                constexpr int RW = BW - SP;
#pragma unroll
                for (int l = 0; l < SP; ++l) {
                    double ur[RW > 0 ? RW : 1];
#pragma unroll
                    for (int c = 0; c < RW; c += 2) {
                        const d2 t = *reinterpret_cast<const d2 *>(&s.PR[l][SP + c]);
                        ur[c] = t[0];
                        if (c + 1 < RW) ur[c + 1] = t[1];
                    }
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        if (live[q]) {
#pragma unroll
                            for (int c = 0; c < RW; ++c) x[q][SP + c] -= x[q][l] * ur[c];
                        }
                    });
                }
                // shift the window
                static_for<RPT>([&](auto QC) {
                    constexpr int q = decltype(QC)::value;
#pragma unroll
                    for (int c = 0; c + SP < BW; ++c) x[q][c] = x[q][c + SP];
                });
            }
        }
    }
    __syncthreads();
    // the block's unit-lower triangle for the update launch:
    // RT[l][i] = multiplier of pivot i on pivot l (l < i)
    for (int e = tid; e < bwc * bwc; e += NT) {
        const int i = e / bwc, l = e - i * bwc;
        if (l < i) s.RT[l][i] = Sn[(size_t)(jb + l) * rc + s.selp[jb + i]];
    }
    __syncthreads();

    // save the node state for the next launches
    for (int i = tid; i < r; i += NT) rselg[i] = s.rowsel[i];
    for (int i = tid; i < bwc; i += NT) {
        selg[jb + i] = s.sel[jb + i];
        selg[kMaxV + jb + i] = s.selp[jb + i];
    }

    for (int e = tid; e < BW * (BW + 8); e += NT) rtg[e] = (&s.RT[0][0])[e];

    if (jb + bwc < nsel) return;

    // ---- last block: outputs --------------------------------------------
    __syncthreads();
    for (int j = tid; j < nsel; j += NT) p.cand_out[(size_t)node * vb + j] = s.sel[j];
    if (tid == 0) p.ccnt_out[node] = nsel;
    if (!p.root) return;

    const int64_t k = p.row0;   // the panel's diagonal row
    if (p.piv_out)
        for (int j = tid; j < vb; j += NT) p.piv_out[j] = s.sel[j];
    // the factored top block: one column per thread, loads in batches of
    // 32 ahead of their stores (see the U-row copy)
    for (int c = tid; c < vb; c += NT) {
        const size_t col = (size_t)c * rc;
        for (int j0 = 0; j0 < vb; j0 += 32) {
            double t[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) t[q] = j0 + q < vb ? Sn[col + s.selp[j0 + q]] : 0.0;
#pragma unroll
            for (int q = 0; q < 32; ++q)
                if (j0 + q < vb) p.lu00[(size_t)(j0 + q) * vb + c] = t[q];
        }
    }
    // first exactly zero pivot of the panel, all diagonal entries at once
    if (p.info) {
        int *zfirst = s.plan_tmp + 2 * kMaxV - 1;
        if (tid == 0) *zfirst = INT_MAX;
        __syncthreads();
        for (int j = tid; j < vb; j += NT)
            if (Sn[(size_t)j * rc + s.selp[j]] == 0.0) atomicMin(zfirst, j);
        __syncthreads();
        if (tid == 0 && *zfirst != INT_MAX && *p.info == 0) *p.info = (int32_t)(k + *zfirst + 1);
        __syncthreads();    // zfirst is plan scratch below
    }
    if (p.ipiv && p.plan) {
        int *loc = s.plan_tmp;
        int *at = loc + vb;
        if (tid == 0) {
            // Sequential interchanges k+j <-> (current position of pivot j).
            // loc[t]: current position of the row that started at k+t;
            // at[q]:  which starting top row sits at top position k+q.
            for (int t = 0; t < vb; ++t) { loc[t] = (int)(k + t); at[t] = t; }
            for (int j = 0; j < vb; ++j) {
                const int pj = s.sel[j];
                const bool top = pj < k + vb;
                const int pos = top ? loc[pj - k] : pj;
                p.ipiv[k + j] = pos;
                const int tcur = at[j];
                if (pos != k + j) {
                    loc[tcur] = pos;
                    if (pos < k + vb) at[pos - k] = tcur;
                }
                if (top) loc[pj - k] = (int)(k + j);
            }
        }
        __syncthreads();
        // the row-move plan: selected rows into the top positions (in pivot
        // order), then the displaced top rows (in starting order); one
        // wavefront compacts each list with ballots
        if (tid < 64) {
            int *dst = p.plan + 1, *src = p.plan + 1 + 2 * kMaxV;
            const unsigned long long below = (1ull << lane) - 1;
            int np = 0;
            for (int j0 = 0; j0 < vb; j0 += 64) {
                const int j = j0 + lane;
                const bool mv = j < vb && s.sel[j] != k + j;
                const unsigned long long bal = __ballot(mv);
                const int at_ = np + __popcll(bal & below);
                if (mv) { dst[at_] = (int)(k + j); src[at_] = s.sel[j]; }
                np += __popcll(bal);
            }
            for (int t0 = 0; t0 < vb; t0 += 64) {
                const int t = t0 + lane;
                const bool mv = t < vb && loc[t] >= k + vb;
                const unsigned long long bal = __ballot(mv);
                const int at_ = np + __popcll(bal & below);
                if (mv) { dst[at_] = loc[t]; src[at_] = (int)(k + t); }
                np += __popcll(bal);
            }
            if (lane == 0) p.plan[0] = np;
        }
    }
}

template <int RPT, int NT>
__global__ __launch_bounds__(NT) void tslu_panel_kernel(NodeArgs p)
{
    // The tournament is the critical path and runs beside the Schur update:
    // its (latency-bound) waves go first when they share a SIMD with the
    // update's matrix-core waves.
    __builtin_amdgcn_s_setprio(3);
    extern __shared__ double smem_raw[];
    auto &s = *reinterpret_cast<Lds<BlockW<RPT>::value, NT / 64> *>(smem_raw);
    panel_block<RPT, NT>(p, blockIdx.x, p.jb, s);
}

// ---------------------------------------------------------------------------
// E: rank-BW update of the trailing columns of every node of the level.
// Workgroup = one 64-row x 64-column tile of one node; wave w owns rows
// 16w .. 16w+15 of the tile.  A = -U^T (16 columns x 4 pivots), B = L^T
// (4 pivots x 16 rows, zero for selected rows), D = C^T (16 x 16).
// ---------------------------------------------------------------------------
template <int BW>
struct UpdLds {
    double Ut[BW][64 + 1];   // -U rows of the block at the tile's columns
    double Rt[BW][BW + 8];
    int sp[BW];
};

// One 64 x 64 tile (trow, tcol) of node `node`'s rank-BW update; 256
// threads (4 wavefronts), which all take the same early returns.
template <int BW>
__device__ __forceinline__ void update_tile(const NodeArgs &p, const int node, const int jb, const int trow,
                                            const int tcol, UpdLds<BW> &u)
{
    auto &Ut = u.Ut;
    auto &Rt = u.Rt;
    auto &sp = u.sp;
    const NodeRows nr = node_rows(p, node);
    if (nr.promoted) return;
    const int r = nr.r;
    const int nsel = r < p.vb ? r : p.vb;
    if (jb >= nsel) return;
    const int bwc = (nsel - jb) < BW ? (nsel - jb) : BW;
    const int tc0 = jb + bwc, ncol = nsel - tc0;
    const int c00 = tcol * 64, r00 = trow * 64;
    if (c00 >= ncol || r00 >= r) return;

    const int rc = p.rc;
    const int tid = threadIdx.x;
    double *Sn = p.S + (size_t)node * p.s_node;
    const unsigned char *rselg = p.rsel + (size_t)node * p.rs_node;
    const int32_t *selg = p.selg + (size_t)node * 2 * kMaxV;
    double *utg = p.utg + (size_t)node * 32 * UTLD;
    const double *rtg = p.rtg + (size_t)node * 32 * 40;

    for (int e = tid; e < BW * (BW + 8); e += 256) (&Rt[0][0])[e] = rtg[e];
    if (tid < BW) sp[tid] = selg[kMaxV + jb + tid];
    __syncthreads();

    // U rows of the block's pivots at this tile's columns: unit-lower
    // substitution, one column per thread
    if (tid < 64) {
        const int cc = c00 + tid;
        if (cc < ncol) {
            const size_t col = (size_t)(tc0 + cc) * rc;
            for (int h = 0; h < BW; h += 8) {
                double u[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) u[i] = (h + i < bwc) ? Sn[col + sp[h + i]] : 0.0;
                for (int l = 0; l < h; ++l) {
                    const double ul = -Ut[l][tid];
#pragma unroll
                    for (int i = 0; i < 8; ++i) u[i] -= Rt[l][h + i] * ul;
                }
#pragma unroll
                for (int l = 0; l < 8; ++l)
#pragma unroll
                    for (int i = l + 1; i < 8; ++i) u[i] -= Rt[h + l][h + i] * u[l];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    Ut[h + i][tid] = (h + i < bwc) ? -u[i] : 0.0;
                    if (p.root && trow == 0 && h + i < bwc) utg[(size_t)(h + i) * UTLD + cc] = u[i];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < BW; ++i) Ut[i][tid] = 0.0;
        }
    }
    __syncthreads();

    // rank-BW update: A = -U^T (16 columns x 4 pivots), B = L^T (4 pivots x
    // 16 rows, zero for selected rows), D = C^T (16 x 16)
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int pr = r00 + wave * 16 + lr;
    const bool rowin = pr < r;
    const bool rowok = rowin && !rselg[pr];
    constexpr int KS = (BW + 3) / 4;
    double bop[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int l = 4 * ks + lk;
        bop[ks] = (rowok && l < bwc) ? Sn[(size_t)(jb + l) * rc + pr] : 0.0;
    }
    d4 acc[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cc = c00 + 16 * tt + lk + 4 * q;
            acc[tt][q] = (cc < ncol && rowin) ? Sn[(size_t)(tc0 + cc) * rc + pr] : 0.0;
        }
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int l = 4 * ks + lk;
            const double aop = (l < bwc) ? Ut[l][16 * tt + lr] : 0.0;
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[ks], acc[tt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cc = c00 + 16 * tt + lk + 4 * q;
            if (cc < ncol && rowin) Sn[(size_t)(tc0 + cc) * rc + pr] = acc[tt][q];
        }
}

template <int BW>
__global__ __launch_bounds__(256) void tslu_update_kernel(NodeArgs p, int tiles_r, int tiles_c)
{
    __builtin_amdgcn_s_setprio(3);      // critical path (see tslu_panel_kernel)
    __shared__ UpdLds<BW> u;
    const int tile = blockIdx.x;
    const int per_node = tiles_r * tiles_c;
    const int node = tile / per_node;
    const int t = tile - node * per_node;
    const int trow = t / tiles_c, tcol = t - trow * tiles_c;
    update_tile<BW>(p, node, p.jb, trow, tcol, u);
}

// The rank-BW update of one node's remaining columns after block jb, by
// the node's own workgroup (256 threads): the block triangle and pivot
// positions are staged once; the U rows of the block are computed for up to
// UPC columns at a time (one column per thread, the same substitution as
// update_tile) into Ut (BW x (UPC + 2) doubles), and every 64 x 64 tile of
// those columns is updated on the matrix cores as in update_tile (the
// block's L rows of a 64-row strip are loaded once per strip).  Same
// operations per element as update_tile, so the same values.
template <int BW>
struct UpdStage {
    double Rt[BW][BW + 8];
    int sp[BW];
};
constexpr int UPC = 128;

template <int BW>
__device__ __forceinline__ void update_node(const NodeArgs &p, const int node, const int jb, const int tiles_r,
                                            double (*Ut)[UPC + 2], UpdStage<BW> &u)
{
    auto &Rt = u.Rt;
    auto &sp = u.sp;
    const NodeRows nr = node_rows(p, node);
    const int r = nr.r;
    const int nsel = r < p.vb ? r : p.vb;
    const int bwc = (nsel - jb) < BW ? (nsel - jb) : BW;
    const int tc0 = jb + bwc, ncol = nsel - tc0;
    const int rc = p.rc;
    const int tid = threadIdx.x;
    double *Sn = p.S + (size_t)node * p.s_node;
    const unsigned char *rselg = p.rsel + (size_t)node * p.rs_node;
    const int32_t *selg = p.selg + (size_t)node * 2 * kMaxV;
    double *utg = p.utg + (size_t)node * 32 * UTLD;
    const double *rtg = p.rtg + (size_t)node * 32 * 40;

    for (int e = tid; e < BW * (BW + 8); e += 256) (&Rt[0][0])[e] = rtg[e];
    if (tid < BW) sp[tid] = selg[kMaxV + jb + tid];
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int KS = (BW + 3) / 4;
    for (int c0 = 0; c0 < ncol; c0 += UPC) {
        if (tid < UPC) {
            const int cc = c0 + tid;
            if (cc < ncol) {
                const size_t col = (size_t)(tc0 + cc) * rc;
                for (int h = 0; h < BW; h += 8) {
                    double uv[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) uv[i] = (h + i < bwc) ? Sn[col + sp[h + i]] : 0.0;
                    for (int l = 0; l < h; ++l) {
                        const double ul = -Ut[l][tid];
#pragma unroll
                        for (int i = 0; i < 8; ++i) uv[i] -= Rt[l][h + i] * ul;
                    }
#pragma unroll
                    for (int l = 0; l < 8; ++l)
#pragma unroll
                        for (int i = l + 1; i < 8; ++i) uv[i] -= Rt[h + l][h + i] * uv[l];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        Ut[h + i][tid] = (h + i < bwc) ? -uv[i] : 0.0;
                        if (p.root && h + i < bwc) utg[(size_t)(h + i) * UTLD + cc] = uv[i];
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < BW; ++i) Ut[i][tid] = 0.0;
            }
        }
        __syncthreads();
        const int ctiles = (ncol - c0) < UPC ? (ncol - c0 + 63) / 64 : UPC / 64;
        for (int trow = 0; trow < tiles_r; ++trow) {
            const int r00 = trow * 64;
            if (r00 >= r) break;
            const int pr = r00 + wave * 16 + lr;
            const bool rowin = pr < r;
            const bool rowok = rowin && !rselg[pr];
            double bop[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int l = 4 * ks + lk;
                bop[ks] = (rowok && l < bwc) ? Sn[(size_t)(jb + l) * rc + pr] : 0.0;
            }
            for (int tc = 0; tc < ctiles; ++tc) {
                const int c00 = c0 + tc * 64;
                d4 acc[4];
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int cc = c00 + 16 * tt + lk + 4 * q;
                        acc[tt][q] = (cc < ncol && rowin) ? Sn[(size_t)(tc0 + cc) * rc + pr] : 0.0;
                    }
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const int l = 4 * ks + lk;
                        const double aop = (l < bwc) ? Ut[l][tc * 64 + 16 * tt + lr] : 0.0;
                        acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[ks], acc[tt], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int cc = c00 + 16 * tt + lk + 4 * q;
                        if (cc < ncol && rowin) Sn[(size_t)(tc0 + cc) * rc + pr] = acc[tt][q];
                    }
            }
        }
        __syncthreads();    // Ut is rewritten by the next column range
    }
}

// A whole node in one launch, for nodes of at most 512 rows (every merge
// node at v <= 256, and the short leaves of late panels): the workgroup
// runs the pivot steps of each column block and then the block's rank-BW
// update of the node's remaining columns itself on its own matrix cores
// (the node's block, at most 1 MiB, stays in L2).  The work per element is
// that of the two-launch scheme, so the selection and the values are the
// same bit for bit; what goes away is two launches per block, each with its
// own start-up (kernel code and node state fetched afresh).
template <int RPT, int NT>
__global__ __launch_bounds__(NT) void tslu_node_kernel(NodeArgs p, int tiles_r)
{
    static_assert(NT == 256, "the update takes 256 threads");
    __builtin_amdgcn_s_setprio(3);      // critical path (see tslu_panel_kernel)
    constexpr int BW = BlockW<RPT>::value;
    using L = Lds<BW, NT / 64>;
    static_assert(sizeof(L::tile) >= sizeof(double) * BW * (UPC + 2), "Ut fits the staging area");
    extern __shared__ double smem_raw[];
    L &s = *reinterpret_cast<L *>(smem_raw);
    UpdStage<BW> &u = *reinterpret_cast<UpdStage<BW> *>(reinterpret_cast<char *>(smem_raw) + sizeof(L));
    // the panel blocks use the staging area only at the root's last block
    double(*Ut)[UPC + 2] = reinterpret_cast<double(*)[UPC + 2]>(&s.tile[0]);
    const int node = blockIdx.x;
    const NodeRows nr = node_rows(p, node);
    const int nsel = nr.promoted ? 0 : (nr.r < p.vb ? nr.r : p.vb);
    const int nsteps = nr.promoted ? 1 : nsel;     // a promoted node only copies (at jb = 0)
    for (int jb = 0; jb < nsteps; jb += BW) {
        panel_block<RPT, NT>(p, node, jb, s);
        if (nsel - (jb + BW) <= 0) break;
        // the block's state written above (workspace) is read back below
        __threadfence_block();
        __syncthreads();
        update_node<BW>(p, node, jb, tiles_r, Ut, u);
        __threadfence_block();
        __syncthreads();
    }
}

// Gather of a level: the current-step panel values of every node's rows into
// its column-major scratch block, one 64 x 64 tile per workgroup (transposed
// through LDS); also clears the node's selected-row mask.
__global__ __launch_bounds__(256) void tslu_gather_kernel(NodeArgs p, int tiles_r, int tiles_c)
{
    __builtin_amdgcn_s_setprio(3);      // critical path (see tslu_panel_kernel)
    __shared__ double tile[64][65];
    __shared__ int64_t prow[64];        // physical rows of the tile's 64 rows
    const int per_node = tiles_r * tiles_c;
    const int node = blockIdx.x / per_node;
    const int t = blockIdx.x - node * per_node;
    const int trow = t / tiles_c, tcol = t - trow * tiles_c;
    const NodeRows nr = node_rows(p, node);
    if (nr.promoted) return;
    const int r = nr.r, r0 = trow * 64, c0 = tcol * 64;
    if (r0 >= r || c0 >= p.vb) return;
    const int tid = threadIdx.x;
    double *Sn = p.S + (size_t)node * p.s_node;
    // the rows' indices (candidate lists, row map) are looked up once per
    // row and shared through LDS, so that the value loads below are all in
    // flight together instead of each waiting for its row's index
    if (tid < 64 && r0 + tid < r) {
        const int g = node_gid(p, nr, r0 + tid);
        prow[tid] = p.rm ? (int64_t)p.rm[g] : (int64_t)(g - p.row0);
    }
    __syncthreads();
    constexpr int PER = 64 * 64 / 256;
    double v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + k * 256, i = e >> 6, c = e & 63;
        if (r0 + i < r && c0 + c < p.vb)
            v[k] = p.W[prow[i] * p.ldw + c0 + c];
        else
            v[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + k * 256, i = e >> 6, c = e & 63;
        tile[i][c] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + k * 256, c = e >> 6, i = e & 63;
        if (r0 + i < r && c0 + c < p.vb) Sn[(size_t)(c0 + c) * p.rc + r0 + i] = tile[i][c];
    }
    if (tcol == 0 && tid < 64 && r0 + tid < r) p.rsel[(size_t)node * p.rs_node + r0 + tid] = 0;
}

// The node kernels' dynamic LDS exceeds the default limit; the attribute is
// set once per device at handle creation (init_kernel_attributes), never on
// the launch path, so concurrent launches from several host threads never
// race on it.
template <int RPT, int NT>
int set_panel_attr()
{
    constexpr int BW = BlockW<RPT>::value;
    CFX_HIP(hipFuncSetAttribute((const void *)tslu_panel_kernel<RPT, NT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(Lds<BW, NT / 64>)));
    if constexpr (NT == 256)
        CFX_HIP(hipFuncSetAttribute((const void *)tslu_node_kernel<RPT, NT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(Lds<BW, NT / 64>) + sizeof(UpdStage<BW>))));
    return CFX_OK;
}

// Whole nodes in one launch each (nodes of at most 512 rows).
template <int RPT, int NT>
int launch_level_fused(NodeArgs a, int grid, int rows_cap, hipStream_t st)
{
    constexpr int BW = BlockW<RPT>::value;
    const size_t lds = sizeof(Lds<BW, NT / 64>) + sizeof(UpdStage<BW>);
    const int tiles_r = (rows_cap + 63) / 64;
    {
        const int tiles_v = (a.vb + 63) / 64;
        hipLaunchKernelGGL(tslu_gather_kernel, dim3(grid * tiles_r * tiles_v), dim3(256), 0, st, a, tiles_r,
                           tiles_v);
        CFX_HIP(hipGetLastError());
    }
    a.jb = 0;
    hipLaunchKernelGGL((tslu_node_kernel<RPT, NT>), dim3(grid), dim3(NT), lds, st, a, tiles_r);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

template <int RPT, int NT>
int launch_level(NodeArgs a, int grid, int rows_cap, hipStream_t st)
{
    constexpr int BW = BlockW<RPT>::value;
    const size_t lds = sizeof(Lds<BW, NT / 64>);
    const int nsel_max = rows_cap < a.vb ? rows_cap : a.vb;
    const int tiles_r = (rows_cap + 63) / 64;
    {
        const int tiles_v = (a.vb + 63) / 64;
        hipLaunchKernelGGL(tslu_gather_kernel, dim3(grid * tiles_r * tiles_v), dim3(256), 0, st, a, tiles_r,
                           tiles_v);
        CFX_HIP(hipGetLastError());
    }
    for (int jb = 0; jb < nsel_max; jb += BW) {
        a.jb = jb;
        hipLaunchKernelGGL((tslu_panel_kernel<RPT, NT>), dim3(grid), dim3(NT), lds, st, a);
        CFX_HIP(hipGetLastError());
        const int ncol_max = nsel_max - (jb + BW);
        if (ncol_max > 0) {
            const int tiles_c = (ncol_max + 63) / 64;
            hipLaunchKernelGGL(tslu_update_kernel<BW>, dim3(grid * tiles_r * tiles_c), dim3(256), 0, st, a,
                               tiles_r, tiles_c);
            CFX_HIP(hipGetLastError());
        }
    }
    return CFX_OK;
}

// Node kernel shape by node height: up to 512 rows one workgroup of 256
// threads; taller nodes 512 threads (two wavefronts per SIMD still leave
// each lane 256 registers), so that the register block x[RPT][BW] can be
// twice as wide as with 256 threads: fewer blocks, fewer update passes.
int launch_node_level(const NodeArgs &a, int grid, int rows_cap, int fuse_rows, hipStream_t st)
{
    if (rows_cap <= fuse_rows) {
        if (rows_cap <= 256) return launch_level_fused<1, 256>(a, grid, rows_cap, st);
        if (rows_cap <= 512) return launch_level_fused<2, 256>(a, grid, rows_cap, st);
    }
    if (rows_cap <= 256) return launch_level<1, 256>(a, grid, rows_cap, st);
    if (rows_cap <= 512) return launch_level<2, 256>(a, grid, rows_cap, st);
    if (rows_cap <= 1024) return launch_level<2, 512>(a, grid, rows_cap, st);
    if (rows_cap <= 2048) return launch_level<4, 512>(a, grid, rows_cap, st);
    if (rows_cap <= 4096) return launch_level<8, 512>(a, grid, rows_cap, st);
    if (rows_cap <= 8192) return launch_level<16, 512>(a, grid, rows_cap, st);
    return CFX_ENOTSUP;
}

}  // namespace

int init_kernel_attributes()
{
    int rc;
    if ((rc = set_panel_attr<1, 256>())) return rc;
    if ((rc = set_panel_attr<2, 256>())) return rc;
    if ((rc = set_panel_attr<2, 512>())) return rc;
    if ((rc = set_panel_attr<4, 512>())) return rc;
    if ((rc = set_panel_attr<8, 512>())) return rc;
    return set_panel_attr<16, 512>();
}

int launch_tslu(const double *W, int64_t ldw, int64_t row0, int64_t rows, int vb, int leaves,
                const Workspace &ws, int32_t *piv_out, int32_t *ipiv, int32_t *info, hipStream_t st,
                const int32_t *rm, int fuse_rows)
{
    int64_t h = (rows + leaves - 1) / leaves;
    if (h < vb) h = vb;
    if (h > kMaxLeafRows) return CFX_ENOTSUP;
    const int nl = (int)((rows + h - 1) / h);
    if (nl > ws.max_nodes) return CFX_ENOMEM;

    NodeArgs a{};
    a.W = W;
    a.ldw = ldw;
    a.row0 = row0;
    a.rows = rows;
    a.vb = vb;
    a.S = ws.S;
    a.s_node = ws.s_node;
    a.piv_out = piv_out;
    a.lu00 = ws.lu00;
    a.ipiv = ipiv;
    a.plan = ipiv ? ws.plan : nullptr;
    a.info = info;
    a.rm = rm;
    a.selg = ws.selg;
    a.rsel = ws.rsel;
    a.rs_node = (int)ws.rs_node;
    a.utg = ws.utg;
    a.rtg = ws.rtg;

    // leaves
    a.leaf = 1;
    a.h = h;
    a.cand_out = ws.cand[0];
    a.ccnt_out = ws.ccnt[0];
    a.rc = (int)h;
    a.root = nl == 1;
    int rc = launch_node_level(a, nl, (int)h, fuse_rows, st);
    if (rc) return rc;

    // playoff rounds
    int nn = nl, cur = 0;
    while (nn > 1) {
        const int nout = (nn + 1) / 2;
        a.leaf = 0;
        a.cand_in = ws.cand[cur];
        a.ccnt_in = ws.ccnt[cur];
        a.nn_in = nn;
        a.cand_out = ws.cand[cur ^ 1];
        a.ccnt_out = ws.ccnt[cur ^ 1];
        a.rc = 2 * vb;
        a.root = nout == 1;
        if ((rc = launch_node_level(a, nout, 2 * vb, fuse_rows, st))) return rc;
        nn = nout;
        cur ^= 1;
    }
    return CFX_OK;
}

}  // namespace cfx

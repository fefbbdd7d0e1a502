// Tournament pivoting (TournPivot of Alg. 1; Sec. 7.3 "Pivoting in COnfLUX";
// Sec. 7.4, Step 1) on gfx950.
//
// One workgroup of 256 threads runs one node of the tournament: a leaf (h
// consecutive rows of the panel) or a merge of two children's candidate
// rows, stacked left child first and taken with their current-step panel
// values.  The node selects min(vb, rows) rows by Gaussian elimination with
// partial pivoting, ties to the smallest global row.  A level of the tree is
// one launch.
//
// Layout inside a node: thread t owns physical rows t, t+256, ... (RPT rows)
// and keeps their values of the current inner block of BW <= 32 columns in
// registers.  The node's panel block lives in a column-major scratch block
// (element (c, p) at c*rc + p): a wavefront touching one column of 64
// consecutive rows makes one coalesced access, and the matrix-core tiles of
// the trailing update read and write 128-byte row runs.
//
// Per inner block:
//  B. pivot steps: each thread scores its unselected rows, a wavefront
//     shuffle reduction picks the wave's best, the winning lane publishes
//     its row into a double-buffered LDS slot, one barrier, and every thread
//     picks the overall winner from the 4 slots and eliminates its rows
//     against that row (registers only);
//  D. the block's pivot rows are extended to the trailing columns: U rows by
//     substitution with the block's unit-lower triangle, one column per
//     thread, in registers;
//  E. the rank-BW update of the trailing columns on the FP64 matrix cores,
//     in transposed form C^T -= U^T L^T (selected rows get zero
//     multipliers, so they are left unchanged).
// Rows are never moved: selected rows are marked, and the selection order is
// kept in LDS.  In exact arithmetic this is the unblocked elimination, so the
// selection is the same.
//
// The root also turns its selection into LAPACK-style interchanges (ipiv)
// and a row-move plan for the swap kernel, and copies its factored top
// vb x vb block (L00 and U00 of the panel) out.
#include <climits>
#include <utility>

#include "cfx_internal.h"

namespace cfx {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

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

__device__ __forceinline__ bool beats(double a, int g, double b, int gb)
{
    return a > b || (a == b && g < gb);
}

// (a, g) of the wavefront's best candidate, uniform across lanes: a DPP
// butterfly inside each row of 16 lanes (xor 1, xor 2, half-mirror,
// mirror), then the four row results combined through readlane.
__device__ __forceinline__ void wave_argmax(double &a, int &g)
{
    auto dpp_step = [&](auto CTRL) {
        constexpr int ctrl = decltype(CTRL)::value;
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(a), ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(a), ctrl, 0xF, 0xF, false);
        const int g2 = __builtin_amdgcn_update_dpp(0, g, ctrl, 0xF, 0xF, false);
        const double a2 = __hiloint2double(hi, lo);
        if (beats(a2, g2, a, g)) { a = a2; g = g2; }
    };
    dpp_step(std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
    dpp_step(std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
    dpp_step(std::integral_constant<int, 0x141>{});  // row_half_mirror
    dpp_step(std::integral_constant<int, 0x140>{});  // row_mirror
    double ba = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(a), 0),
                                 __builtin_amdgcn_readlane(__double2loint(a), 0));
    int bg = __builtin_amdgcn_readlane(g, 0);
#pragma unroll
    for (int row = 1; row < 4; ++row) {
        const double ra = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(a), 16 * row),
                                           __builtin_amdgcn_readlane(__double2loint(a), 16 * row));
        const int rg = __builtin_amdgcn_readlane(g, 16 * row);
        if (beats(ra, rg, ba, bg)) { ba = ra; bg = rg; }
    }
    a = ba;
    g = bg;
}

// Score of a candidate value: |a|; NaN ranks below every number but above
// "not a candidate" (-1), so a block of NaNs still yields a pivot.
__device__ __forceinline__ double score(double a)
{
    const double s = fabs(a);
    return s == s ? s : -0.5;
}

template <int BW>
struct Lds {
    static constexpr int UTLD = ((kMaxV - BW) + 15) & ~15;  // trailing columns
    d2 cand[2][NW][BW / 2 > 0 ? BW / 2 : 1];   // published pivot-row candidates
    double slot_a[2][NW];
    int slot_g[2][NW];
    int slot_t[2][NW];
    int slot_s[2][NW];
    double RT[BW][BW + 8];      // RT[l][i] = multiplier of block pivot i on pivot l
    union {
        double Ut[BW][UTLD];    // -U rows of the block at the trailing columns
        double tile[64 * 65];   // gather: transpose staging
        int plan_tmp[2 * kMaxV];
    };
    int sel[kMaxV];             // selected global rows, in order
    int selp[kMaxV];            // physical scratch row of each selected row
    unsigned char rowsel[kMaxLeafRows];   // physical row already selected
};

template <int RPT>
__global__ __launch_bounds__(NT) void tslu_node_kernel(NodeArgs p)
{
    constexpr int BW = (64 / RPT) < 32 ? (64 / RPT) : 32;
    using L = Lds<BW>;
    extern __shared__ double smem_raw[];
    L &s = *reinterpret_cast<L *>(smem_raw);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int node = blockIdx.x;
    const int vb = p.vb;
    const int rc = p.rc;

    // ---- node rows ---------------------------------------------------------
    int r;
    int64_t leaf_first = 0;
    const int32_t *cl_list = nullptr, *cr_list = nullptr;
    int cl = 0;
    if (p.leaf) {
        leaf_first = (int64_t)node * p.h;
        const int64_t last = leaf_first + p.h < p.rows ? leaf_first + p.h : p.rows;
        r = (int)(last - leaf_first);
    } else {
        const int a = 2 * node;
        if (a + 1 >= p.nn_in) {                 // unpaired: promoted unchanged
            const int c = p.ccnt_in[a];
            for (int i = tid; i < c; i += NT) p.cand_out[(size_t)node * vb + i] = p.cand_in[(size_t)a * vb + i];
            if (tid == 0) p.ccnt_out[node] = c;
            return;
        }
        cl = p.ccnt_in[a];
        r = cl + p.ccnt_in[a + 1];
        cl_list = p.cand_in + (size_t)a * vb;
        cr_list = p.cand_in + (size_t)(a + 1) * vb;
    }
    auto gid_of = [&](int pr) -> int {
        if (p.leaf) return (int)(p.row0 + leaf_first + pr);
        return pr < cl ? cl_list[pr] : cr_list[pr - cl];
    };

    double *Sn = p.S + (size_t)node * p.s_node;
    for (int i = tid; i < r; i += NT) s.rowsel[i] = 0;

    // ---- gather the current-step panel values, transposed through LDS ------
    // (a 64-row strip of all vb columns is loaded at once, then written out
    //  column-major one 64 x 64 tile at a time)
    {
        double *tile = s.tile;                  // 64 x 65 staging tile
        constexpr int PER = 64 * 64 / NT;       // 16 elements per thread per tile
        constexpr int NTL = 2;                  // tiles loaded per batch
        for (int r0 = 0; r0 < r; r0 += 64)
        for (int t0 = 0; t0 < vb; t0 += 64 * NTL) {
            double v[NTL][PER];
#pragma unroll
            for (int tl = 0; tl < NTL; ++tl)
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int e = tid + k * NT, i = e >> 6, c = t0 + tl * 64 + (e & 63);
                    v[tl][k] = (r0 + i < r && c < vb)
                                   ? p.W[(int64_t)(gid_of(r0 + i) - p.row0) * p.ldw + c] : 0.0;
                }
#pragma unroll
            for (int tl = 0; tl < NTL; ++tl) {
                if (t0 + tl * 64 < vb) {
#pragma unroll
                    for (int k = 0; k < PER; ++k) {
                        const int e = tid + k * NT, i = e >> 6, c = e & 63;
                        tile[i * 65 + c] = v[tl][k];
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < PER; ++k) {
                        const int e = tid + k * NT, c = e >> 6, i = e & 63;
                        if (r0 + i < r && t0 + tl * 64 + c < vb)
                            Sn[(size_t)(t0 + tl * 64 + c) * rc + r0 + i] = tile[i * 65 + c];
                    }
                    __syncthreads();
                }
            }
        }
    }

    int gid[RPT];
    bool live[RPT];     // a real row that is not selected yet
    static_for<RPT>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        const int pr = tid + q * NT;
        live[q] = pr < r;
        gid[q] = live[q] ? gid_of(pr) : INT_MAX;
    });

    const int nsel = r < vb ? r : vb;

    for (int jb = 0; jb < nsel; jb += BW) {
        const int bwc = (nsel - jb) < BW ? (nsel - jb) : BW;
        const int tc0 = jb + bwc;            // first trailing column
        const int ncol = nsel - tc0;         // trailing columns that matter

        {   // x: the block columns of this thread's rows, live only here
        double x[RPT][BW];
        static_for<RPT>([&](auto QC) {
            constexpr int q = decltype(QC)::value;
            const int pr = tid + q * NT;
#pragma unroll
            for (int c = 0; c < BW; ++c)
                x[q][c] = (pr < r && c < bwc) ? Sn[(size_t)(jb + c) * rc + pr] : 0.0;
        });

        // ---- B: pivot steps of the block --------------------------------
        static_for<BW>([&](auto JC) {
            constexpr int j = decltype(JC)::value;
            if (j < bwc) {
                const int par = j & 1;
                double ba = -1.0;
                int bg = INT_MAX, bq = -1;
                static_for<RPT>([&](auto QC) {
                    constexpr int q = decltype(QC)::value;
                    if (live[q]) {
                        const double a = score(x[q][j]);
                        if (beats(a, gid[q], ba, bg)) { ba = a; bg = gid[q]; bq = q; }
                    }
                });
                double wa = ba;
                int wg = bg;
                wave_argmax(wa, wg);
                // gids are unique, so exactly one lane owns the wave's best
                if (bq >= 0 && bg == wg) {
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        if (q == bq) {
#pragma unroll
                            for (int c = 0; c + 1 < BW; c += 2) s.cand[par][wave][c / 2] = d2{x[q][c], x[q][c + 1]};
                            if (BW & 1) s.cand[par][wave][BW / 2][0] = x[q][BW - 1];
                        }
                    });
                    s.slot_t[par][wave] = tid;
                    s.slot_s[par][wave] = bq;
                }
                if (lane == 0) {
                    s.slot_a[par][wave] = wa;
                    s.slot_g[par][wave] = wg;
                }
                __syncthreads();
                double ma = s.slot_a[par][0];
                int mg = s.slot_g[par][0], mw = 0;
#pragma unroll
                for (int w = 1; w < NW; ++w) {
                    const double aw = s.slot_a[par][w];
                    const int gw = s.slot_g[par][w];
                    if (beats(aw, gw, ma, mg)) { ma = aw; mg = gw; mw = w; }
                }
                const int ot = s.slot_t[par][mw], oq = s.slot_s[par][mw];
                const double *prow = reinterpret_cast<const double *>(&s.cand[par][mw][0]);
                if (tid == 0) {
                    s.sel[jb + j] = mg;
                    s.selp[jb + j] = ot + oq * NT;
                    s.rowsel[ot + oq * NT] = 1;
                }
                if (tid < j) s.RT[tid][j] = prow[tid];
                static_for<RPT>([&](auto QC) {
                    constexpr int q = decltype(QC)::value;
                    if (tid == ot && q == oq) live[q] = false;
                });
                const double piv = prow[j];
                if (piv != 0.0) {
                    d2 pv[BW / 2 > 0 ? BW / 2 : 1];
#pragma unroll
                    for (int c = 2 * ((j + 1) / 2); c + 1 < BW; c += 2) pv[c / 2] = s.cand[par][mw][c / 2];
                    static_for<RPT>([&](auto QC) {
                        constexpr int q = decltype(QC)::value;
                        if (live[q]) {
                            const double l = x[q][j] / piv;
                            x[q][j] = l;
#pragma unroll
                            for (int c = j + 1; c < BW; ++c)
                                x[q][c] -= l * ((c + 1 < BW || !(BW & 1)) ? pv[c / 2][c & 1] : prow[c]);
                        }
                    });
                }
            }
        });

        // block columns back to the scratch block (final for this block)
        static_for<RPT>([&](auto QC) {
            constexpr int q = decltype(QC)::value;
            const int pr = tid + q * NT;
            if (pr < r) {
#pragma unroll
                for (int c = 0; c < BW; ++c)
                    if (c < bwc) Sn[(size_t)(jb + c) * rc + pr] = x[q][c];
            }
        });
        }
        __syncthreads();

        if (ncol > 0) {
            // ---- D: U rows of the block at the trailing columns ---------
            // (unit-lower substitution, one column per thread, in chunks of
            //  8 rows held in registers; finished rows are kept in LDS)
            for (int c = tid; c < ncol; c += NT) {
                const size_t col = (size_t)(tc0 + c) * rc;
                for (int h = 0; h < bwc; h += 8) {
                    double u[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) u[i] = (h + i < bwc) ? Sn[col + s.selp[jb + h + i]] : 0.0;
                    for (int l = 0; l < h; ++l) {
                        const double ul = -s.Ut[l][c];
#pragma unroll
                        for (int i = 0; i < 8; ++i) u[i] -= s.RT[l][h + i] * ul;
                    }
#pragma unroll
                    for (int l = 0; l < 8; ++l)
#pragma unroll
                        for (int i = l + 1; i < 8; ++i) u[i] -= s.RT[h + l][h + i] * u[l];
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (h + i < bwc) {
                            s.Ut[h + i][c] = -u[i];
                            Sn[col + s.selp[jb + h + i]] = u[i];
                        }
                }
            }
            __syncthreads();

            // ---- E: C^T -= U^T L^T on the matrix cores ---------------------
            // A = -U^T (16 trailing columns x 4 pivots), B = L^T (4 pivots x
            // 16 rows, zero for selected rows), D = C^T tile (16 x 16).  A
            // wave walks (row block, 64-column chunk) pairs and keeps the
            // next chunk's loads in flight while the current one computes.
            const int lr = lane & 15, lk = lane >> 4;
            const int nrb = (r + 15) >> 4;
            const int nch = (ncol + 63) >> 6;
            const int my_nrb = nrb > wave ? (nrb - wave + NW - 1) / NW : 0;
            const int total = my_nrb * nch;
            constexpr int KS = (BW + 3) / 4;
            auto load = [&](int it, d4 (&acc)[4], double (&bo)[KS]) {
                const int rb = wave + NW * (it / nch);
                const int c0 = (it % nch) * 64;
                const int pr = rb * 16 + lr;
                const bool rowok = pr < r && !s.rowsel[pr];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int l = 4 * ks + lk;
                    bo[ks] = (rowok && l < bwc) ? Sn[(size_t)(jb + l) * rc + pr] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int cc = c0 + 16 * t + lk + 4 * q;
                        acc[t][q] = (cc < ncol && pr < r) ? Sn[(size_t)(tc0 + cc) * rc + pr] : 0.0;
                    }
            };
            d4 cur[4], nxt[4];
            double bc[KS], bn[KS];
            if (total > 0) load(0, cur, bc);
            for (int it = 0; it < total; ++it) {
                if (it + 1 < total) load(it + 1, nxt, bn);
                const int rb = wave + NW * (it / nch);
                const int c0 = (it % nch) * 64;
                const int pr = rb * 16 + lr;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (c0 + 16 * t < ncol) {
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks) {
                            const int l = 4 * ks + lk;
                            const int cc = c0 + 16 * t + lr;
                            const double aop = (l < bwc && cc < ncol) ? s.Ut[l][cc] : 0.0;
                            cur[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bc[ks], cur[t], 0, 0, 0);
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int cc = c0 + 16 * t + lk + 4 * q;
                            if (cc < ncol && pr < r) Sn[(size_t)(tc0 + cc) * rc + pr] = cur[t][q];
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) cur[t] = nxt[t];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) bc[ks] = bn[ks];
            }
        }
        __syncthreads();
    }

    // ---- outputs -----------------------------------------------------------
    for (int j = tid; j < nsel; j += NT) p.cand_out[(size_t)node * vb + j] = s.sel[j];
    if (tid == 0) p.ccnt_out[node] = nsel;
    if (!p.root) return;

    const int64_t k = p.row0;   // the panel's diagonal row
    if (p.piv_out)
        for (int j = tid; j < vb; j += NT) p.piv_out[j] = s.sel[j];
    for (int e = tid; e < vb * vb; e += NT) {
        const int j = e / vb, c = e - j * vb;
        p.lu00[e] = Sn[(size_t)c * rc + s.selp[j]];
    }
    if (tid == 0 && p.info) {
        for (int j = 0; j < vb; ++j)
            if (Sn[(size_t)j * rc + s.selp[j]] == 0.0) {
                if (*p.info == 0) *p.info = (int32_t)(k + j + 1);
                break;
            }
    }
    if (tid == 0 && p.ipiv && p.plan) {
        // Sequential interchanges k+j <-> (current position of pivot j).
        // loc[t]: current position of the row that started at k+t;
        // at[q]:  which starting top row sits at top position k+q.
        int *loc = s.plan_tmp;
        int *at = loc + vb;
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
        int *dst = p.plan + 1, *src = p.plan + 1 + 2 * kMaxV;
        int np = 0;
        for (int j = 0; j < vb; ++j)
            if (s.sel[j] != k + j) { dst[np] = (int)(k + j); src[np] = s.sel[j]; ++np; }
        for (int t = 0; t < vb; ++t)
            if (loc[t] >= k + vb) { dst[np] = loc[t]; src[np] = (int)(k + t); ++np; }
        p.plan[0] = np;
    }
}

template <int RPT>
int launch_level(const NodeArgs &a, int grid, hipStream_t st)
{
    constexpr int BW = (64 / RPT) < 32 ? (64 / RPT) : 32;
    static bool attr_set = false;
    const size_t lds = sizeof(Lds<BW>);
    if (!attr_set) {
        CFX_HIP(hipFuncSetAttribute((const void *)tslu_node_kernel<RPT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    hipLaunchKernelGGL(tslu_node_kernel<RPT>, dim3(grid), dim3(NT), lds, st, a);
    CFX_HIP(hipGetLastError());
    return CFX_OK;
}

int launch_node_level(const NodeArgs &a, int grid, int rows_cap, hipStream_t st)
{
    if (rows_cap <= 256) return launch_level<1>(a, grid, st);
    if (rows_cap <= 512) return launch_level<2>(a, grid, st);
    if (rows_cap <= 1024) return launch_level<4>(a, grid, st);
    if (rows_cap <= 2048) return launch_level<8>(a, grid, st);
    if (rows_cap <= 4096) return launch_level<16>(a, grid, st);
    if (rows_cap <= 8192) return launch_level<32>(a, grid, st);
    return CFX_ENOTSUP;
}

}  // namespace

int launch_tslu(const double *W, int64_t ldw, int64_t row0, int64_t rows, int vb, int leaves,
                const Workspace &ws, int32_t *piv_out, int32_t *ipiv, int32_t *info, hipStream_t st)
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

    // leaves
    a.leaf = 1;
    a.h = h;
    a.cand_out = ws.cand[0];
    a.ccnt_out = ws.ccnt[0];
    a.rc = (int)h;
    a.root = nl == 1;
    int rc = launch_node_level(a, nl, (int)h, st);
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
        if ((rc = launch_node_level(a, nout, 2 * vb, st))) return rc;
        nn = nout;
        cur ^= 1;
    }
    return CFX_OK;
}

}  // namespace cfx

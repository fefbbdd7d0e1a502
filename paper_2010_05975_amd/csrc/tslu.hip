// Tournament pivoting (TournPivot of Alg. 1; Sec. 7.3 "Pivoting in COnfLUX";
// Sec. 7.4, Step 1) on gfx950.
//
// One workgroup runs one node of the tournament: a leaf (h consecutive rows
// of the panel) or a merge of two children's candidate rows, stacked left
// child first and taken with their current-step panel values.  The node
// selects min(vb, rows) rows by Gaussian elimination with partial pivoting
// (ties to the smallest global row).  A level of the tree is one launch.
//
// Inside a node the elimination is blocked by inner panels of bw <= 32
// columns: the inner panel lives in LDS and is eliminated column by column
// (a wavefront shuffle argmax, then a cross-wave reduction), then the
// bw x (cols) block of U is formed by substitution and the rest of the node
// block (kept in a global scratch block, mostly L2-resident) receives the
// rank-bw update.  Rows are never moved in the scratch block: a logical ->
// physical row map in LDS is permuted instead.  In exact arithmetic this is
// the same elimination as the unblocked one, so the selection is the same.
//
// The root additionally turns its selection into LAPACK-style interchanges
// (ipiv), a row-move plan for the swap kernel, and copies its factored top
// vb x vb block (L00 and U00 of the panel) out.
#include <climits>

#include "cfx_internal.h"

namespace cfx {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int BW = 32;                       // widest inner panel
constexpr size_t kLdsBudget = 152 * 1024;    // dynamic LDS per node

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
    double *S;              // node scratch
    int64_t s_node;
    int bw;                 // inner panel width for this launch
    int r_cap;              // max rows of a node in this launch
    int root;               // this launch is the root
    int32_t *piv_out;       // root: selected global rows (may be null)
    double *lu00;           // root: factored top block (may be null)
    int32_t *ipiv;          // root: interchanges, global indexing (may be null)
    int32_t *plan;          // root: row-move plan (may be null)
    int32_t *info;          // root: first zero pivot (may be null)
};

__device__ __forceinline__ bool beats(double a, int g, double b, int gb)
{
    return a > b || (a == b && g < gb);
}

__global__ __launch_bounds__(NT) void tslu_node_kernel(NodeArgs p)
{
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ldp = p.bw + 1;

    double *P = smem;                                       // r_cap x ldp
    int *gid = reinterpret_cast<int *>(P + (size_t)p.r_cap * ldp);
    int *phys = gid + p.r_cap;
    double *red_a = reinterpret_cast<double *>(phys + p.r_cap + (p.r_cap & 1));
    int *red_g = reinterpret_cast<int *>(red_a + NW);
    int *red_i = red_g + NW;
    int *s_piv = red_i + NW;

    const int node = blockIdx.x;
    const int vb = p.vb;
    int r;

    // ---- node rows ------------------------------------------------------
    if (p.leaf) {
        int64_t first = (int64_t)node * p.h;
        int64_t last = first + p.h < p.rows ? first + p.h : p.rows;
        r = (int)(last - first);
        for (int i = tid; i < r; i += NT) gid[i] = (int)(p.row0 + first + i);
    } else {
        const int a = 2 * node;
        if (a + 1 >= p.nn_in) {                 // unpaired: promoted unchanged
            const int c = p.ccnt_in[a];
            for (int i = tid; i < c; i += NT) p.cand_out[(size_t)node * vb + i] = p.cand_in[(size_t)a * vb + i];
            if (tid == 0) p.ccnt_out[node] = c;
            return;
        }
        const int cl = p.ccnt_in[a], cr = p.ccnt_in[a + 1];
        r = cl + cr;
        for (int i = tid; i < cl; i += NT) gid[i] = p.cand_in[(size_t)a * vb + i];
        for (int i = tid; i < cr; i += NT) gid[cl + i] = p.cand_in[(size_t)(a + 1) * vb + i];
    }
    for (int i = tid; i < r; i += NT) phys[i] = i;
    __syncthreads();

    // ---- gather the current-step panel values into the scratch block -----
    double *Sn = p.S + (size_t)node * p.s_node;
    for (int i = 0; i < r; ++i) {
        const double *src = p.W + (gid[i] - p.row0) * p.ldw;
        for (int c = tid; c < vb; c += NT) Sn[(size_t)i * vb + c] = src[c];
    }
    __syncthreads();

    const int nsel = r < vb ? r : vb;

    // ---- blocked GEPP -----------------------------------------------------
    for (int jb = 0; jb < nsel; jb += p.bw) {
        const int bwc = (nsel - jb) < p.bw ? (nsel - jb) : p.bw;
        const int nrows = r - jb;

        // A: inner panel into LDS (logical rows jb .. r-1).
        for (int e = tid; e < nrows * bwc; e += NT) {
            const int i = e / bwc, c = e - i * bwc;
            P[i * ldp + c] = Sn[(size_t)phys[jb + i] * vb + jb + c];
        }
        __syncthreads();

        // B: unblocked elimination of the inner panel.
        for (int j = 0; j < bwc; ++j) {
            double ba = -1.0;
            int bg = INT_MAX, bi = -1;
            for (int i = j + tid; i < nrows; i += NT) {
                const double a = fabs(P[i * ldp + j]);
                const int g = gid[jb + i];
                if (beats(a, g, ba, bg)) { ba = a; bg = g; bi = i; }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double a2 = __shfl_xor(ba, off);
                const int g2 = __shfl_xor(bg, off);
                const int i2 = __shfl_xor(bi, off);
                if (beats(a2, g2, ba, bg)) { ba = a2; bg = g2; bi = i2; }
            }
            if (lane == 0) { red_a[wave] = ba; red_g[wave] = bg; red_i[wave] = bi; }
            __syncthreads();
            if (tid == 0) {
                double a = red_a[0];
                int g = red_g[0], bsel = red_i[0];
                for (int w = 1; w < NW; ++w)
                    if (beats(red_a[w], red_g[w], a, g)) { a = red_a[w]; g = red_g[w]; bsel = red_i[w]; }
                *s_piv = bsel < 0 ? j : bsel;   // all candidates NaN: keep order
            }
            __syncthreads();
            const int pr = *s_piv;
            if (pr != j) {
                for (int c = tid; c < bwc; c += NT) {
                    const double t = P[j * ldp + c];
                    P[j * ldp + c] = P[pr * ldp + c];
                    P[pr * ldp + c] = t;
                }
                if (tid == 0) {
                    int t = gid[jb + j]; gid[jb + j] = gid[jb + pr]; gid[jb + pr] = t;
                    t = phys[jb + j]; phys[jb + j] = phys[jb + pr]; phys[jb + pr] = t;
                }
            }
            __syncthreads();
            const double pv = P[j * ldp + j];
            if (pv != 0.0) {
                for (int i = j + 1 + tid; i < nrows; i += NT) {
                    const double l = P[i * ldp + j] / pv;
                    P[i * ldp + j] = l;
                    for (int c = j + 1; c < bwc; ++c) P[i * ldp + c] -= l * P[j * ldp + c];
                }
            }
            __syncthreads();
        }

        // C: inner panel back to the scratch block.
        for (int e = tid; e < nrows * bwc; e += NT) {
            const int i = e / bwc, c = e - i * bwc;
            Sn[(size_t)phys[jb + i] * vb + jb + c] = P[i * ldp + c];
        }

        // D: U block rows jb .. jb+bwc for the columns right of the panel
        //    (unit lower substitution with the inner panel's L).
        const int c0 = jb + bwc;
        for (int c = c0 + tid; c < nsel; c += NT) {
            double u[BW];
#pragma unroll
            for (int j = 0; j < BW; ++j)
                if (j < bwc) u[j] = Sn[(size_t)phys[jb + j] * vb + c];
#pragma unroll
            for (int j = 1; j < BW; ++j) {
                if (j < bwc) {
                    double s = u[j];
#pragma unroll
                    for (int l = 0; l < BW; ++l)
                        if (l < j) s -= P[j * ldp + l] * u[l];
                    u[j] = s;
                }
            }
#pragma unroll
            for (int j = 1; j < BW; ++j)
                if (j < bwc) Sn[(size_t)phys[jb + j] * vb + c] = u[j];
        }
        __syncthreads();

        // E: rank-bwc update of the remaining rows and columns.
        const int cc = tid & 31, grp = tid >> 5;
        for (int ct = c0; ct < nsel; ct += 32) {
            const int c = ct + cc;
            if (c < nsel) {
                double u[BW];
#pragma unroll
                for (int l = 0; l < BW; ++l)
                    if (l < bwc) u[l] = Sn[(size_t)phys[jb + l] * vb + c];
                for (int i = bwc + grp; i < nrows; i += NT / 32) {
                    double *s = Sn + (size_t)phys[jb + i] * vb + c;
                    double acc = *s;
                    const double *Pi = P + i * ldp;
#pragma unroll
                    for (int l = 0; l < BW; ++l)
                        if (l < bwc) acc -= Pi[l] * u[l];
                    *s = acc;
                }
            }
        }
        __syncthreads();
    }

    // ---- outputs ------------------------------------------------------------
    for (int j = tid; j < nsel; j += NT) p.cand_out[(size_t)node * vb + j] = gid[j];
    if (tid == 0) p.ccnt_out[node] = nsel;
    if (!p.root) return;

    const int64_t k = p.row0;   // the panel's diagonal row
    if (p.piv_out)
        for (int j = tid; j < vb; j += NT) p.piv_out[j] = gid[j];
    if (p.lu00)
        for (int j = 0; j < vb; ++j)
            for (int c = tid; c < vb; c += NT) p.lu00[(size_t)j * vb + c] = Sn[(size_t)phys[j] * vb + c];
    if (tid == 0 && p.info) {
        for (int j = 0; j < vb; ++j)
            if (Sn[(size_t)phys[j] * vb + j] == 0.0) {
                if (*p.info == 0) *p.info = (int32_t)(k + j + 1);
                break;
            }
    }
    if (tid == 0 && p.ipiv && p.plan) {
        // Sequential interchanges k+j <-> (current position of pivot j).
        // loc[t]: current position of the row that started at k+t;
        // at[q]:  which starting top row sits at top position k+q.
        int *loc = reinterpret_cast<int *>(P);
        int *at = loc + vb;
        for (int t = 0; t < vb; ++t) { loc[t] = (int)(k + t); at[t] = t; }
        for (int j = 0; j < vb; ++j) {
            const int pj = gid[j];
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
            if (gid[j] != k + j) { dst[np] = (int)(k + j); src[np] = gid[j]; ++np; }
        for (int t = 0; t < vb; ++t)
            if (loc[t] >= k + vb) { dst[np] = loc[t]; src[np] = (int)(k + t); ++np; }
        p.plan[0] = np;
    }
}

size_t node_lds_bytes(int r_cap, int bw)
{
    size_t b = (size_t)r_cap * (bw + 1) * sizeof(double);
    b += 2 * (size_t)r_cap * sizeof(int) + ((r_cap & 1) ? sizeof(int) : 0);
    b += NW * sizeof(double) + 2 * NW * sizeof(int) + 2 * sizeof(int);
    return b;
}

int pick_bw(int r_cap)
{
    for (int bw = BW; bw >= 1; --bw)
        if (node_lds_bytes(r_cap, bw) <= kLdsBudget) return bw;
    return 0;
}

}  // namespace

int launch_tslu(const double *W, int64_t ldw, int64_t row0, int64_t rows, int vb,
                int leaves, const Workspace &ws, int32_t *piv_out, int32_t *ipiv,
                int32_t *info, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        CFX_HIP(hipFuncSetAttribute((const void *)tslu_node_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    int64_t h = (rows + leaves - 1) / leaves;
    if (h < vb) h = vb;
    if (h > kMaxLeafRows) return CFX_ENOTSUP;
    int nl = (int)((rows + h - 1) / h);
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
    a.r_cap = (int)h;
    a.bw = pick_bw(a.r_cap);
    if (a.bw == 0) return CFX_ENOTSUP;
    a.root = nl == 1;
    hipLaunchKernelGGL(tslu_node_kernel, dim3(nl), dim3(NT), node_lds_bytes(a.r_cap, a.bw), st, a);
    CFX_HIP(hipGetLastError());

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
        a.r_cap = 2 * vb;
        a.bw = pick_bw(a.r_cap);
        a.root = nout == 1;
        hipLaunchKernelGGL(tslu_node_kernel, dim3(nout), dim3(NT), node_lds_bytes(a.r_cap, a.bw), st, a);
        CFX_HIP(hipGetLastError());
        nn = nout;
        cur ^= 1;
    }
    return CFX_OK;
}

}  // namespace cfx

// Internal declarations of the gfx950 LU library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cfx.h"

#define CFX_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return CFX_EHIP;          \
    } while (0)

namespace cfx {

constexpr int kMaxV = 256;        // largest supported panel width
constexpr int kMaxLeafRows = 8192; // largest supported tournament node height
constexpr int kBatchClasses = 5;   // batched size classes: n <= 32, 64, 128, 256, 512

// ---------------------------------------------------------------------------
// Workspace of one factorisation (carved out of the caller's `work`).
// ---------------------------------------------------------------------------
struct Workspace {
    double *S;          // node scratch: nodes x node_rows x v doubles
    int64_t s_node;     // doubles per node in S
    int32_t *cand[2];   // candidate lists, ping-pong: nodes x v
    int32_t *ccnt[2];   // candidate counts: nodes
    int32_t *plan;      // row-move plan: [0] = count, then dst[2v], src[2v]
    int32_t *plan_alt;  // a second plan buffer (panels of the lookahead schedule alternate)
    double *lu00;       // factored diagonal block, v x v
    int32_t *selg;      // tournament node state: selection [nodes x 2 x kMaxV]
    unsigned char *rsel; // tournament node state: selected-row mask [nodes x rs_node]
    int64_t rs_node;
    double *utg;        // tournament node state: U rows of a block [nodes x 32 x kMaxV]
    double *rtg;        // tournament node state: block triangle [nodes x 32 x 40]
    double *scratch;    // mixed precision: packed low-precision panels
    size_t scratch_bytes;
    int64_t max_nodes;
};

// Bytes of workspace for order n and options; and the carve-up.
// delay: panels per trailing update of the tile-stationary schedule (the
// low-precision packed operands then hold K = delay v).
size_t workspace_bytes(int64_t n, int v, int leaves, int precision, int delay = 1, int min_leaf = 0);
// Leaves of the tournament of a panel with `rows` rows: L, or with a
// minimum leaf height R > 0, min(L, max(1, ceil(rows / R))).
inline int panel_leaves(int leaves, int min_leaf, int64_t rows)
{
    if (min_leaf <= 0) return leaves;
    const int64_t k = (rows + min_leaf - 1) / min_leaf;
    return (int)(k < 1 ? 1 : (k < leaves ? k : leaves));
}
int carve_workspace(void *work, size_t bytes, int64_t n, int v, int leaves,
                    int precision, Workspace *ws, int delay = 1, int min_leaf = 0);

// Tournament pivoting of the rows x vb panel at W (stride ldw); panel row i
// is global row row0 + i.  When `ipiv` is set the root also turns the
// selection into LAPACK-style interchanges ipiv[row0 .. row0+vb) and a
// row-move plan (row0 is then the panel's diagonal row).  The root always
// copies its factored top block to ws.lu00.  `piv_out` (may be null)
// receives the selected global rows.
// fuse_rows: nodes of at most this many rows (<= 512) run as one launch each
// (pivot steps and the node's own updates in one workgroup); taller nodes
// take two launches per column block.  Same results either way.
constexpr int kFuseRows = 512;          // largest fusable node (2 v at v = 256)
constexpr int kFuseRowsDefault = 0;    // measured slower than two launches
int launch_tslu(const double *W, int64_t ldw, int64_t row0, int64_t rows, int vb,
                int leaves, const Workspace &ws, int32_t *piv_out, int32_t *ipiv,
                int32_t *info, hipStream_t st, const int32_t *rm = nullptr,
                int fuse_rows = kFuseRowsDefault);
// (rm: row masking; panel row i, global row row0 + i, is then physical row
// rm[row0 + i] of W, which points at row 0 of the panel's first column.)

// Kernel attributes (dynamic LDS limits) of the current device; called by
// cfx_create, so that no launch path sets them.
int init_kernel_attributes();

// Scratch of the allocation-free solve: a device array of this many bytes
// per GPU.  noalloc_scratch returns its device address on `device`, which
// must be the current device (looked up once per device, then cached).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
int noalloc_scratch(int device, void **ptr);
// The handle's spin limit of the one-launch triangular solves.
int solve_spin_limit(const cfx_handle *h);

// Polls of a one-launch triangular solve's wait before the block gives up
// (sets sync[4] and writes NaN for its rows).
constexpr int kSolveSpinLimit = 1 << 22;

// getrs pieces: permutation of ipiv, and the blocked triangular solves.
// rm (row masking): factor row i is physical row rm[i], and rm is also the
// permutation of P B (ipiv is then not read).  tmp holds n x max(nrhs, 2)
// doubles.
int launch_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                 const int32_t *ipiv, double *B, int64_t ldb, int32_t *perm,
                 double *tmp, int32_t *sync, hipStream_t st,
                 int spin_limit = kSolveSpinLimit, const int32_t *rm = nullptr);
// perm[i] = source row of row i of P B (ipiv interchanges composed).
int launch_perm(int64_t n, const int32_t *ipiv, int32_t *perm, hipStream_t st);
// T[i, :] = B[perm[i], :]  /  B[i, :] = T[i, :]   (n x nrhs).
int launch_gather_rows(int64_t n, int64_t nrhs, const double *B, int64_t ldb,
                       const int32_t *perm, double *T, int64_t ldt, hipStream_t st);
int launch_copy_rows(int64_t n, int64_t nrhs, const double *T, int64_t ldt,
                     double *B, int64_t ldb, hipStream_t st);
// X <- U^{-1} L^{-1} X in place (X n x nrhs, stride ldx).  `sync` (device,
// kTrsvSyncBytes) and Y (device, n doubles, the intermediate vector; its
// contents are overwritten) let one contiguous right-hand side take the
// one-launch-per-triangle solve; with either null it takes the blocked
// launches.  Calls sharing a sync buffer or Y must be stream-ordered.
// sync[4] is set (and stays set until the host clears it) when a wait of
// that solve gave up after spin_limit polls.
constexpr size_t kTrsvSyncBytes = 256;
int launch_trsv(int64_t n, int64_t nrhs, const double *LU, int64_t lda, double *X,
                int64_t ldx, int32_t *sync, double *Y, hipStream_t st,
                int spin_limit = kSolveSpinLimit, const int32_t *rm = nullptr);
// Host-blocking: *gave_up = sync[4] after `st` drains; sync[4] is cleared.
int read_solve_flag(int32_t *sync, hipStream_t st, bool *gave_up);

// Apply the row-move plan to the n columns of A (w1 <= w0), to the columns
// [w0, w1) only (window), or to all columns but those; the diagonal block of
// the panel (rows k..k+vb, columns k..k+vb) is written from ws.lu00 where
// its columns are covered.
int launch_laswp(double *A, int64_t lda, int64_t n, int64_t k, int vb,
                 const Workspace &ws, hipStream_t st, int64_t w0 = 0, int64_t w1 = 0, bool window = false);

// Row masking: the root's row-move plan applied to the row map rm (logical
// row -> physical row) instead of the rows, and L00\U00 written into the
// panel columns of the pivot rows where they are.
int launch_rowmap_apply(double *A, int64_t lda, int32_t *rm, int64_t k, int vb,
                        const Workspace &ws, hipStream_t st);
// rm[i] = i for i < n.
int launch_rowmap_init(int32_t *rm, int64_t n, hipStream_t st);

// FactorizeA10 and FactorizeA01: L21 = A21 U00^{-1} and U12 = L00^{-1} A12,
// in place, for the trailing m rows / columns of panel k.  rm: the row map
// of row masking (logical row i at physical row rm[i]), or null.
int launch_trsm(double *A, int64_t lda, int64_t k, int vb, int64_t m,
                hipStream_t st, const int32_t *rm = nullptr);
// L21 and the first n1 columns of U12 in one launch; the other columns of
// U12 (n1 .. m) separately.
int launch_trsm_first(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t n1,
                      hipStream_t st, const int32_t *rm = nullptr);
int launch_trsm_rest(double *A, int64_t lda, int64_t k, int vb, int64_t m, int64_t n1,
                     hipStream_t st, const int32_t *rm = nullptr);

// FactorizeA11: C[0:mr, 0:nc] -= L[0:mr, 0:K] * U[0:K, 0:nc]  (FP64 MFMA).
// max_wgs > 0 bounds the grid (persistent workgroups walk the tiles).
// Row maps (null: none): row i of L and of C is physical row rmap[i] (L, C
// then point at row 0 of their columns), row l of U physical row umap[l].
int launch_schur_f64(const double *L, int64_t ldl, const double *U, int64_t ldu,
                     double *C, int64_t ldc, int64_t mr, int64_t nc, int K,
                     int max_wgs, hipStream_t st, const int32_t *rmap = nullptr,
                     const int32_t *umap = nullptr);

// Mixed-precision FactorizeA11.  launch_pack_lp rounds L21 (m x K, stride
// ldl) and U12 (K x n, stride ldu) to the working precision (FP8: after the
// power-of-two row / column scaling) into `buf` (lp_pack_bytes bytes);
// launch_schur_lp then applies C[0:m, col0:col0+ncols] -= L21 U12[:, col0:
// col0+ncols] from the packed operands, FP32 accumulation, FP64 C.
// Row maps as for launch_schur_f64 (rmap: rows of L21 and C; umap: rows
// of U12).
size_t lp_pack_bytes(int precision, int64_t m, int64_t n, int K);
int launch_pack_lp(int precision, const double *L21, int64_t ldl, int64_t m, const double *U12,
                   int64_t ldu, int64_t n, int K, void *buf, hipStream_t st,
                   const int32_t *rmap = nullptr, const int32_t *umap = nullptr);
int launch_schur_lp(int precision, const void *buf, int64_t m, int64_t n, int K, int64_t col0,
                    int64_t ncols, double *C, int64_t ldc, int max_wgs, hipStream_t st,
                    const int32_t *rmap = nullptr);

int launch_set_int(int32_t *p, int32_t value, hipStream_t st);

// Batched LU + solve (one persistent launch after a one-workgroup sort).
// work: batched_work_bytes(count) bytes; vb_class: panel width per size
// class; grid: persistent workgroups.
size_t batched_work_bytes(int32_t count);
int launch_gesv_batched(int32_t count, const int32_t *n, const int32_t *nrhs, double *const *A,
                        const int64_t *lda, double *const *B, const int64_t *ldb,
                        int32_t *const *ipiv, int32_t *info, void *work,
                        const int32_t *vb_class, int grid, hipStream_t st);
// eta[i] = max over right-hand sides of the normwise backward error of X_i
// for A_i X_i = B_i (compensated residual rows).  One workgroup per system.
int launch_batched_eta(int count, const int32_t *n, const int32_t *nrhs, double *const *A,
                       const int64_t *lda, double *const *B, const int64_t *ldb,
                       double *const *X, const int64_t *ldx, double *eta, hipStream_t st);
// count systems of order n, contiguous (n x n each), for the tuner.
int launch_batched_synth(double *A, int n, int64_t count, uint64_t seed, hipStream_t st);

// ---------------------------------------------------------------------------
// Iterative refinement (GMRES-IR) pieces.
// ---------------------------------------------------------------------------
// y = A x (plain FP64), and r = b - A x with compensated row sums
// (rowabs_i = sum_j |A_ij| when rowabs is not null).
int launch_gemv(const double *A, int64_t lda, int64_t n, const double *x, double *y,
                hipStream_t st);
int launch_residual(const double *A, int64_t lda, int64_t n, const double *x,
                    const double *b, double *r, double *rowabs, hipStream_t st);

// Device vectors of one refinement: x, r, b are consecutive at stride ldv.
struct IrVectors {
    int64_t n;
    int restart;
    double *x, *r, *b, *w, *z, *rowabs, *tmp;
    double *ys;         // intermediate vector of the one-launch triangular solves
    double *V;          // restart + 1 Krylov vectors at stride ldv
    int64_t ldv;
    double *partial;    // block partial sums
    double *out;        // small reduction results
    int32_t *sync;      // counters of the triangular solves (kTrsvSyncBytes)
};
struct IrParams {
    double tol;
    int max_outer;
    double gmres_tol;
    int spin_limit = kSolveSpinLimit;   // of the one-launch triangular solves
};
struct IrResult {
    double eta, eta_first;
    int outer, inner, converged;
};
size_t ir_vec_bytes(int64_t n, int restart);
IrVectors carve_ir(void *base, int64_t n, int restart);
// Refine v.x (holding the initial solution) for the right-hand side v.b of
// A x = b, preconditioned by the factors F (stride ldf) with permutation
// perm.  Host-blocking on st.
int ir_refine(const double *A, int64_t lda, const double *F, int64_t ldf,
              const int32_t *perm, const IrVectors &v, const IrParams &p,
              IrResult *res, hipStream_t st);

}  // namespace cfx

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

// ---------------------------------------------------------------------------
// Workspace of one factorisation (carved out of the caller's `work`).
// ---------------------------------------------------------------------------
struct Workspace {
    double *S;          // node scratch: nodes x node_rows x v doubles
    int64_t s_node;     // doubles per node in S
    int32_t *cand[2];   // candidate lists, ping-pong: nodes x v
    int32_t *ccnt[2];   // candidate counts: nodes
    int32_t *plan;      // row-move plan: [0] = count, then dst[2v], src[2v]
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
size_t workspace_bytes(int64_t n, int v, int leaves, int precision);
int carve_workspace(void *work, size_t bytes, int64_t n, int v, int leaves,
                    int precision, Workspace *ws);

// Tournament pivoting of the rows x vb panel at W (stride ldw); panel row i
// is global row row0 + i.  When `ipiv` is set the root also turns the
// selection into LAPACK-style interchanges ipiv[row0 .. row0+vb) and a
// row-move plan (row0 is then the panel's diagonal row).  The root always
// copies its factored top block to ws.lu00.  `piv_out` (may be null)
// receives the selected global rows.
int launch_tslu(const double *W, int64_t ldw, int64_t row0, int64_t rows, int vb,
                int leaves, const Workspace &ws, int32_t *piv_out, int32_t *ipiv,
                int32_t *info, hipStream_t st);

// getrs pieces: permutation of ipiv, and the blocked triangular solves.
int launch_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                 const int32_t *ipiv, double *B, int64_t ldb, int32_t *perm,
                 double *tmp, hipStream_t st);

// Apply the row-move plan to all n columns of A; the diagonal block of the
// panel (rows k..k+vb, columns k..k+vb) is written from ws.lu00.
int launch_laswp(double *A, int64_t lda, int64_t n, int64_t k, int vb,
                 const Workspace &ws, hipStream_t st);

// FactorizeA10 and FactorizeA01: L21 = A21 U00^{-1} and U12 = L00^{-1} A12,
// in place, for the trailing m rows / columns of panel k.
int launch_trsm(double *A, int64_t lda, int64_t k, int vb, int64_t m,
                hipStream_t st);

// FactorizeA11: C[0:mr, 0:nc] -= L[0:mr, 0:K] * U[0:K, 0:nc]  (FP64 MFMA).
int launch_schur_f64(const double *L, int64_t ldl, const double *U, int64_t ldu,
                     double *C, int64_t ldc, int64_t mr, int64_t nc, int K,
                     hipStream_t st);

int launch_set_int(int32_t *p, int32_t value, hipStream_t st);

}  // namespace cfx

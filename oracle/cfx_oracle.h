/*
 * cfx_oracle.h -- CPU oracle for blocked LU with tournament pivoting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this library; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * library.
 *
 * All matrices are row-major FP64 with a row stride (lda >= n).  Row and
 * column indices are 0-based.
 */
#ifndef CFX_ORACLE_H
#define CFX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Operation counters, checked against the statement counts of the in-place
 * LU program (Sec. 6: |V_S1| divisions and |V_S2| multiply-subtracts). */
typedef struct {
    int64_t divisions;          /* S1: A[i,k] /= A[k,k]                 */
    int64_t multiply_subtracts; /* S2: A[i,j] -= A[i,k] * A[k,j]        */
} oracle_counters;

/* Tournament pivot selection for one panel (Sec. 7.3, "Pivoting in
 * COnfLUX"; Step 1 of the I/O-cost proof in Sec. 7.4).
 *   W      : rows x vb panel, row-major, stride ldw.  Row r of W is global
 *            row (row0 + r).
 *   L      : leaf count; leaf height h = max(vb, ceil(rows / L)).
 *   piv    : out, vb global row indices in selection order.
 *   margin : out, minimum pivot margin over every selection in the panel.
 * Returns 0, or a negative argument index. */
int oracle_tslu(int64_t rows, int64_t vb, const double *W, int64_t ldw,
                int64_t row0, int64_t L, int64_t *piv, double *margin);

/* Blocked right-looking LU, A = P L U, with tournament pivoting TP(v, L)
 * (Alg. 1 compute steps: TournPivot, FactorizeA10, FactorizeA01,
 * FactorizeA11), with explicit row interchanges.
 *   min_leaf : 0, or R > 0: a panel with r rows has min(L, max(1,
 *              ceil(r / R))) leaves (leaves of at least R rows; the leaf
 *              count follows the panel's height).
 *   A        : n x n, overwritten by L (strict lower, unit diagonal
 *              implicit) and U (upper).
 *   ipiv     : out int32[n]; row i was interchanged with row ipiv[i] >= i,
 *              applied in order i = 0 .. n-1.
 *   info     : out; 0, or j+1 for the first exactly zero U[j][j].
 *   margins  : out, one entry per panel (may be NULL): minimum pivot margin.
 *   npanels  : stop after this many panels (<= 0: all).  The untouched
 *              trailing part then holds partially updated values.
 *   cnt      : out counters (may be NULL).
 * Returns 0, or a negative argument index. */
int oracle_getrf(int64_t n, double *A, int64_t lda, int64_t v, int64_t L,
                 int64_t min_leaf, int32_t *ipiv, int32_t *info, double *margins,
                 int64_t npanels, oracle_counters *cnt);

/* Solve A X = B with the factors of oracle_getrf: apply ipiv to B in order,
 * forward substitution with unit L, back substitution with U.  B is
 * n x nrhs, row-major, stride ldb, overwritten with X. */
int oracle_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                 const int32_t *ipiv, double *B, int64_t ldb);

/* Normwise backward error of one solution column,
 *   eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf),
 * with every residual entry accumulated in doubled precision (the "Dot2"
 * scheme of Ogita, Rump and Oishi, 2005: Knuth's error-free TwoSum and
 * Dekker's TwoProduct with Veltkamp's splitting, no fused multiply-add).
 * x and b are strided columns (stride incx / incb).  Returns NaN when any
 * x_i, b_i or residual entry (hence any entry of A met by it) is not
 * finite, so a non-finite solution never scores as accurate. */
double oracle_eta(int64_t n, const double *A, int64_t lda, const double *x,
                  int64_t incx, const double *b, int64_t incb);

#ifdef __cplusplus
}
#endif
#endif

/*
 * cfx_oracle.c -- plain, slow CPU oracle for blocked LU with tournament
 * pivoting (COnfLUX, Kwasniewski et al., arXiv 2010.05975).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Everything is FP64 (the paper's element size is 8 bytes, Sec. 8).  The
 * loops follow the definitions directly: no blocking, no reordering of the
 * per-element reductions.  OpenMP only splits independent rows (or columns)
 * of a step, so every element sees the same operation sequence for any
 * thread count and the results are bitwise reproducible.
 *
 * Readings of the paper used here (the paper is silent on them):
 *  - leaf count L is fixed per run; leaf height h = max(vb, ceil(rows/L));
 *    the last leaf may be short;
 *  - the reduction tree pairs consecutive nodes (0,1), (2,3), ...; an unpaired
 *    last node is promoted unchanged; a merge stacks the left child's
 *    candidates before the right child's;
 *  - a merge works on the candidates' current-step panel values, not on the
 *    children's partially eliminated values;
 *  - the local candidate rule ("locally perform the LUP decomposition") is
 *    Gaussian elimination with partial pivoting (GEPP); ties go to the
 *    smallest global row index; an exactly zero pivot skips the scaling and
 *    the update;
 *  - pivot rows are physically interchanged (LAPACK-style ipiv) over all n
 *    columns instead of masked;
 *  - a zero U[j][j] is reported LAPACK-style through info and its column of
 *    L is left unscaled.
 */
#include "cfx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* GEPP row selection on a small dense block (the "local LUP decomposition"  */
/* of a tournament leaf, and the "playoff" of a merge; Sec. 7.3, Sec. 7.4    */
/* Step 1).                                                                  */
/*   blk  : rows x vb working copy, row-major, contiguous (destroyed).       */
/*   gid  : global row index of each block row (permuted in place).          */
/*   sel  : out, the first nsel = min(vb, rows) selected global rows.        */
/*   mmin : in/out running minimum of the pivot margins.                     */
/* ------------------------------------------------------------------------ */
static int64_t gepp_select(int64_t rows, int64_t vb, double *blk, int64_t *gid,
                           int64_t *sel, double *mmin)
{
    int64_t nsel = rows < vb ? rows : vb;
    for (int64_t j = 0; j < nsel; ++j) {
        /* Pivot: largest |value| in column j among rows j..rows-1; an exact
         * tie is broken towards the smallest global row index. */
        int64_t p = j;
        double best = fabs(blk[j * vb + j]);
        for (int64_t i = j + 1; i < rows; ++i) {
            double a = fabs(blk[i * vb + j]);
            if (a > best || (a == best && gid[i] < gid[p])) {
                best = a;
                p = i;
            }
        }
        /* Margin (|a1| - |a2|) / |a1| between the best and the runner-up. */
        double second = -1.0;
        for (int64_t i = j; i < rows; ++i) {
            if (i == p) continue;
            double a = fabs(blk[i * vb + j]);
            if (a > second) second = a;
        }
        double margin;
        if (second < 0.0) margin = 1.0;          /* single candidate */
        else if (best == 0.0) margin = 0.0;       /* all candidates zero */
        else margin = (best - second) / best;
        if (margin < *mmin) *mmin = margin;

        /* Interchange rows j and p of the working block. */
        if (p != j) {
            for (int64_t c = 0; c < vb; ++c) {
                double t = blk[j * vb + c];
                blk[j * vb + c] = blk[p * vb + c];
                blk[p * vb + c] = t;
            }
            int64_t t = gid[j];
            gid[j] = gid[p];
            gid[p] = t;
        }
        sel[j] = gid[j];

        /* Eliminate below the pivot (skipped for an exactly zero pivot). */
        double piv = blk[j * vb + j];
        if (piv != 0.0) {
            for (int64_t i = j + 1; i < rows; ++i) {
                double l = blk[i * vb + j] / piv;
                blk[i * vb + j] = l;
                for (int64_t c = j + 1; c < vb; ++c)
                    blk[i * vb + c] -= l * blk[j * vb + c];
            }
        }
    }
    return nsel;
}

/* Copy the current-step panel values of the listed global rows into blk. */
static void gather_rows(const double *W, int64_t ldw, int64_t row0,
                        const int64_t *g, int64_t cnt, int64_t vb, double *blk)
{
    for (int64_t i = 0; i < cnt; ++i)
        memcpy(blk + i * vb, W + (g[i] - row0) * ldw, (size_t)vb * sizeof(double));
}

int oracle_tslu(int64_t rows, int64_t vb, const double *W, int64_t ldw,
                int64_t row0, int64_t L, int64_t *piv, double *margin)
{
    if (rows < 0) return -1;
    if (vb < 1 || vb > rows) return -2;
    if (!W) return -3;
    if (ldw < vb) return -4;
    if (L < 1) return -6;
    if (!piv) return -7;

    double mmin = 1.0;
    /* Leaves: fixed count L, height h = max(vb, ceil(rows / L)). */
    int64_t h = (rows + L - 1) / L;
    if (h < vb) h = vb;
    int64_t nnodes = (rows + h - 1) / h;

    /* Each node keeps up to vb candidates (global rows, selection order). */
    int64_t *cand = (int64_t *)malloc((size_t)(nnodes * vb) * sizeof(int64_t));
    int64_t *ccnt = (int64_t *)malloc((size_t)nnodes * sizeof(int64_t));
    int64_t maxrows = (h > 2 * vb) ? h : 2 * vb;
    double *blk = (double *)malloc((size_t)(maxrows * vb) * sizeof(double));
    int64_t *gid = (int64_t *)malloc((size_t)maxrows * sizeof(int64_t));

    for (int64_t leaf = 0; leaf < nnodes; ++leaf) {
        int64_t r0 = leaf * h;
        int64_t r1 = r0 + h < rows ? r0 + h : rows;
        for (int64_t i = r0; i < r1; ++i) gid[i - r0] = row0 + i;
        gather_rows(W, ldw, row0, gid, r1 - r0, vb, blk);
        ccnt[leaf] = gepp_select(r1 - r0, vb, blk, gid, cand + leaf * vb, &mmin);
    }

    /* Playoff rounds: merge consecutive pairs until one node is left. */
    while (nnodes > 1) {
        int64_t next = 0;
        for (int64_t a = 0; a < nnodes; a += 2) {
            if (a + 1 == nnodes) {              /* unpaired: promoted */
                memmove(cand + next * vb, cand + a * vb, (size_t)vb * sizeof(int64_t));
                ccnt[next] = ccnt[a];
            } else {
                int64_t cl = ccnt[a], cr = ccnt[a + 1];
                for (int64_t i = 0; i < cl; ++i) gid[i] = cand[a * vb + i];
                for (int64_t i = 0; i < cr; ++i) gid[cl + i] = cand[(a + 1) * vb + i];
                gather_rows(W, ldw, row0, gid, cl + cr, vb, blk);
                int64_t *out = (int64_t *)malloc((size_t)vb * sizeof(int64_t));
                int64_t c = gepp_select(cl + cr, vb, blk, gid, out, &mmin);
                memcpy(cand + next * vb, out, (size_t)c * sizeof(int64_t));
                free(out);
                ccnt[next] = c;
            }
            ++next;
        }
        nnodes = next;
    }
    memcpy(piv, cand, (size_t)vb * sizeof(int64_t));
    if (margin) *margin = mmin;
    free(cand); free(ccnt); free(blk); free(gid);
    return 0;
}

int oracle_getrf(int64_t n, double *A, int64_t lda, int64_t v, int64_t L,
                 int64_t min_leaf, int32_t *ipiv, int32_t *info, double *margins,
                 int64_t npanels, oracle_counters *cnt)
{
    if (n < 0) return -1;
    if (!A && n > 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (v < 1) return -4;
    if (L < 1) return -5;
    if (min_leaf < 0) return -6;
    if (!ipiv && n > 0) return -7;
    if (!info) return -8;

    *info = 0;
    int64_t ndiv = 0, nms = 0;
    int64_t *piv = (int64_t *)malloc((size_t)(v > 0 ? v : 1) * sizeof(int64_t));
    /* row_at[q] = which of this panel's starting rows sits at position q,
     * where_is[r] = position of starting row r (both relative to row k). */
    int64_t *row_at = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *where_is = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));

    int64_t panel = 0;
    for (int64_t k = 0; k < n; k += v, ++panel) {
        if (npanels > 0 && panel >= npanels) break;
        int64_t vb = (n - k < v) ? n - k : v;
        int64_t m = n - k - vb;  /* trailing size */

        /* TournPivot on the current panel A[k:n, k:k+vb], over L leaves,
         * or with a minimum leaf height over ceil(rows / min_leaf) of them
         * (at most L, at least 1). */
        int64_t Lk = L;
        if (min_leaf > 0) {
            Lk = (n - k + min_leaf - 1) / min_leaf;
            if (Lk > L) Lk = L;
            if (Lk < 1) Lk = 1;
        }
        double mm = 1.0;
        oracle_tslu(n - k, vb, A + k * lda + k, lda, k, Lk, piv, &mm);
        if (margins) margins[panel] = mm;

        /* Row interchanges over all n columns, LAPACK-style, in order. */
        for (int64_t q = 0; q < n - k; ++q) { row_at[q] = q; where_is[q] = q; }
        for (int64_t j = 0; j < vb; ++j) {
            int64_t r = where_is[piv[j] - k];   /* current position of p_j */
            ipiv[k + j] = (int32_t)(k + r);
            if (r != j) {
                double *x = A + (k + j) * lda, *y = A + (k + r) * lda;
                for (int64_t c = 0; c < n; ++c) { double t = x[c]; x[c] = y[c]; y[c] = t; }
                int64_t a = row_at[j], b = row_at[r];
                row_at[j] = b; row_at[r] = a;
                where_is[b] = j; where_is[a] = r;
            }
        }

        /* A00: LU without pivoting of the vb x vb diagonal block, now in the
         * root's pivot order (the root's factored block in exact arithmetic). */
        for (int64_t j = 0; j < vb; ++j) {
            double u = A[(k + j) * lda + k + j];
            if (u == 0.0 && *info == 0) *info = (int32_t)(k + j + 1);
            for (int64_t i = j + 1; i < vb; ++i) {
                double *ri = A + (k + i) * lda + k;
                const double *rj = A + (k + j) * lda + k;
                if (u != 0.0) ri[j] /= u;
                ++ndiv;
                for (int64_t c = j + 1; c < vb; ++c) ri[c] -= ri[j] * rj[c];
                nms += vb - j - 1;
            }
        }

        /* FactorizeA10: L21 = A21 U00^{-1}, column by column. */
        #pragma omp parallel for schedule(static) reduction(+:ndiv, nms)
        for (int64_t i = k + vb; i < n; ++i) {
            double *ri = A + i * lda + k;
            for (int64_t j = 0; j < vb; ++j) {
                double s = ri[j];
                for (int64_t l = 0; l < j; ++l) s -= ri[l] * A[(k + l) * lda + k + j];
                nms += j;
                double u = A[(k + j) * lda + k + j];
                ri[j] = (u != 0.0) ? s / u : s;
                ++ndiv;
            }
        }

        /* FactorizeA01: U12 = L00^{-1} A12, column by column. */
        #pragma omp parallel for schedule(static) reduction(+:nms)
        for (int64_t c = k + vb; c < n; ++c) {
            for (int64_t j = 1; j < vb; ++j) {
                double s = A[(k + j) * lda + c];
                for (int64_t l = 0; l < j; ++l) s -= A[(k + j) * lda + k + l] * A[(k + l) * lda + c];
                A[(k + j) * lda + c] = s;
                nms += j;
            }
        }

        /* FactorizeA11: Schur complement A22 -= L21 U12, in l order. */
        #pragma omp parallel for schedule(static) reduction(+:nms)
        for (int64_t i = k + vb; i < n; ++i) {
            double *ri = A + i * lda;
            for (int64_t l = 0; l < vb; ++l) {
                double a = ri[k + l];
                const double *ul = A + (k + l) * lda;
                for (int64_t c = k + vb; c < n; ++c) ri[c] -= a * ul[c];
            }
            nms += vb * m;
        }
    }
    if (cnt) { cnt->divisions = ndiv; cnt->multiply_subtracts = nms; }
    free(piv); free(row_at); free(where_is);
    return 0;
}

int oracle_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                 const int32_t *ipiv, double *B, int64_t ldb)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (!LU && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (!ipiv && n > 0) return -5;
    if (!B && n > 0 && nrhs > 0) return -6;
    if (ldb < (nrhs > 1 ? nrhs : 1)) return -7;

    /* P b: the interchanges in order. */
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = ipiv[i];
        if (r != i)
            for (int64_t c = 0; c < nrhs; ++c) {
                double t = B[i * ldb + c]; B[i * ldb + c] = B[r * ldb + c]; B[r * ldb + c] = t;
            }
    }
    /* L y = P b (unit diagonal). */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < nrhs; ++c) {
            double s = B[i * ldb + c];
            for (int64_t l = 0; l < i; ++l) s -= LU[i * lda + l] * B[l * ldb + c];
            B[i * ldb + c] = s;
        }
    /* U x = y. */
    for (int64_t i = n - 1; i >= 0; --i)
        for (int64_t c = 0; c < nrhs; ++c) {
            double s = B[i * ldb + c];
            for (int64_t l = i + 1; l < n; ++l) s -= LU[i * lda + l] * B[l * ldb + c];
            B[i * ldb + c] = s / LU[i * lda + i];
        }
    return 0;
}

/* Error-free transformations: a + b = s + e exactly (Knuth's TwoSum), and
 * a * b = p + e exactly (Dekker's TwoProduct with Veltkamp's splitting,
 * valid barring overflow).  No fused multiply-add is needed. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b, z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void split(double a, double *hi, double *lo)
{
    double c = 134217729.0 * a;  /* 2^27 + 1 */
    double h = c - (c - a);
    *hi = h;
    *lo = a - h;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double ah, al, bh, bl;
    double x = a * b;
    split(a, &ah, &al);
    split(b, &bh, &bl);
    *e = al * bl - (((x - ah * bh) - al * bh) - ah * bl);
    *p = x;
}

double oracle_eta(int64_t n, const double *A, int64_t lda, const double *x,
                  int64_t incx, const double *b, int64_t incb)
{
    double rmax = 0.0, anorm = 0.0, xnorm = 0.0, bnorm = 0.0;
    int bad = 0;   /* some x_i, b_i or residual entry is not finite */
    for (int64_t i = 0; i < n; ++i) {
        double ax = fabs(x[i * incx]), ab = fabs(b[i * incb]);
        if (!isfinite(ax) || !isfinite(ab)) bad = 1;
        if (ax > xnorm) xnorm = ax;
        if (ab > bnorm) bnorm = ab;
    }
    #pragma omp parallel for schedule(static) reduction(max:rmax, anorm) reduction(|:bad)
    for (int64_t i = 0; i < n; ++i) {
        const double *ri = A + i * lda;
        /* r_i = b_i - sum_j a_ij x_j, accumulated as s + c (Dot2). */
        double s = b[i * incb], c = 0.0, rowabs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double p, pe, t, te;
            two_prod(-ri[j], x[j * incx], &p, &pe);
            two_sum(s, p, &t, &te);
            s = t;
            c += te + pe;
            rowabs += fabs(ri[j]);
        }
        double r = fabs(s + c);
        if (!isfinite(r) || !isfinite(rowabs)) bad = 1;
        if (r > rmax) rmax = r;
        if (rowabs > anorm) anorm = rowabs;
    }
    if (bad) return NAN;
    double den = anorm * xnorm + bnorm;
    return den > 0.0 ? rmax / den : 0.0;
}

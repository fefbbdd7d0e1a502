/*
 * cfx.h -- C ABI of an MI355X (gfx950) library for dense LU factorisation
 * with tournament pivoting, after COnfLUX (Kwasniewski et al., "On the
 * Parallel I/O Optimality of Linear Algebra Kernels: Near-Optimal LU
 * Factorization", arXiv 2010.05975).
 *
 * The problem (Sec. 2.2, Fig. 1, and Sec. 6 statements S1/S2): overwrite a
 * dense n x n matrix A in place with its factors, A = P L U, L unit lower
 * triangular (stored strictly below the diagonal), U upper triangular.  The
 * factorisation is blocked with panel width v (Alg. 1); each panel's v pivot
 * rows are chosen by tournament pivoting (Sec. 7.3): every leaf of L leaves
 * selects v candidate rows by Gaussian elimination with partial pivoting,
 * and a binary reduction tree of "playoff" rounds keeps v winners per node
 * (Sec. 7.4, Step 1).  FactorizeA10 and FactorizeA01 are the two triangular
 * solves and FactorizeA11 the Schur-complement update (Sec. 7.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are ROW-MAJOR FP64 with a row stride (lda >= number of
 *    columns), 0-based indices.
 *  - Pointers named A, B, X, ipiv, info, work are DEVICE pointers (memory
 *    from hipMalloc or a PyTorch CUDA tensor) unless stated otherwise.  The
 *    caller owns all of them; the library never frees or keeps them beyond
 *    the call, and never allocates device memory outside the handle.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Calls are asynchronous on it unless stated otherwise.
 *  - Return value: CFX_OK (0), -i when argument i (1-based) is invalid,
 *    or one of the named negative codes below.  Numerical singularity is
 *    reported through `info`, never through the return value.  No call
 *    throws across the ABI.
 *  - A handle is not thread-safe: serialise calls on one handle.
 */
#ifndef CFX_H
#define CFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CFX_OK = 0,
    CFX_PENDING = 1,          /* serving: result not ready yet             */
    CFX_ENOMEM = -1001,       /* workspace or arena too small              */
    CFX_EHIP = -1002,         /* a HIP runtime call failed                 */
    CFX_EBUSY = -1003,        /* serving: queue full                       */
    CFX_ENOTSUP = -1004,      /* shape outside the supported range         */
    CFX_ESOLVE = -1005,       /* a one-launch triangular solve gave up a
                                 wait (bounded spin); its result is NaN    */
};

enum {
    CFX_PREC_FP64 = 0,        /* every step in FP64                        */
    CFX_PREC_BF16 = 1,        /* Schur update with BF16 operands, FP32 acc */
    CFX_PREC_FP16 = 2,        /* Schur update with FP16 operands, FP32 acc */
    CFX_PREC_FP8 = 3,         /* Schur update with FP8 (OCP E4M3) operands,
                                 each row of L21 and column of U12 scaled by
                                 a power of two first, FP32 acc (an
                                 experiment: 3 fraction bits)              */
};

/* Options of the tournament-pivoted LU.
 *   v         : panel width (Alg. 1 blocking parameter v), 1..256.
 *   leaves    : leaf count L of the tournament; a panel with r rows left has
 *               L_r leaves of h = max(v, ceil(r / L_r)) rows (the last one
 *               may be shorter), L_r = L, or with min_leaf_rows = R > 0
 *               L_r = min(L, max(1, ceil(r / R))): leaves of at least R rows
 *               (TP(v, L_r), Sec. 7.3, with the leaf count following the
 *               panel's height: fewer tree levels for short panels).  h must
 *               not exceed 8192 rows.
 *   precision : CFX_PREC_*; the pivot search, row interchanges and both
 *               triangular solves are always FP64.  With BF16/FP16/FP8 each
 *               Schur update rounds L21 and U12 to that format (to nearest,
 *               ties to even, once from FP64; FP8 after scaling each row of
 *               L21 and each column of U12 by the power of two that brings
 *               its largest magnitude into [128, 256)), multiplies on the
 *               matrix cores with FP32 accumulation and subtracts the FP32
 *               sum (FP8: scaled back exactly) from the FP64 trailing
 *               matrix.
 *   lookahead : 0 or 1; 1 overlaps the next panel's tournament with the
 *               rest of the current Schur update on a second stream.
 *   min_leaf_rows : R above; 0 (fixed L) or 1..8192. */
typedef struct {
    int32_t v;
    int32_t leaves;
    int32_t precision;
    int32_t lookahead;
    int32_t min_leaf_rows;
} cfx_lu_opts;

typedef struct cfx_handle cfx_handle;

/* Create / destroy a handle on the current HIP device.  The handle owns a
 * second stream and a few events (for lookahead); nothing else. */
int cfx_create(cfx_handle **h);
int cfx_destroy(cfx_handle *h);

/* Overlap tuning of cfx_getrf with lookahead = 1 (host-side settings of the
 * handle; they change scheduling only, never a result bit).  While the next
 * panel's tournament runs on the second stream, the rest of the Schur update
 * is issued in launches of `chunk_cols` columns whose grid is bounded by
 * `schur_workgroups` workgroups that walk the tiles persistently (see also
 * cfx_set_reserved_cus, which keeps compute units free for the tournament).
 *   schur_workgroups : -1 = by precision (the default): no bound for FP64,
 *                      384 for BF16/FP16 (their update is bound by HBM and
 *                      loses little to a bound); 0 = one workgroup per tile
 *                      (no bound); else >= 8.
 *   chunk_cols       : >= 0; 0 (the default) = automatic: the whole rest in
 *                      one launch when compute units are reserved, 512
 *                      columns per launch otherwise (the tournament's
 *                      launches then start between two of them).
 *   one_stream       : 1 issues the same launches, in the same order, on
 *                      the caller's stream only (no overlap; for counter
 *                      collection by profilers that serialize dispatches
 *                      and cannot follow waits between streams); default 0.
 * Get: host int32 pointers (any may be NULL).  Set returns -2 / -3 / -4 for
 * an invalid value. */
int cfx_overlap_tuning(cfx_handle *h, int32_t *schur_workgroups, int32_t *chunk_cols,
                       int32_t *one_stream);
int cfx_set_overlap_tuning(cfx_handle *h, int32_t schur_workgroups, int32_t chunk_cols,
                           int32_t one_stream);

/* Triangular solves of cfx_getrf with lookahead = 1 (scheduling only: the
 * same bits).  L21 and the next panel's columns of U12 are solved in one
 * launch ahead of the next tournament; the rest of U12 is solved with the
 * rest of the update.  While the trailing matrix has at least `rows` rows
 * the update, not the next tournament, bounds each step, and all of U12 is
 * solved in the first launch instead (one launch less before the update).
 * The low-precision factorisations always solve all of U12 first.
 *   rows : >= 0; default 16384; 0 = always all of U12 first.
 * Get: host int32 pointer.  Set returns -2 for a negative value. */
int cfx_full_trsm_rows(cfx_handle *h, int32_t *rows);
int cfx_set_full_trsm_rows(cfx_handle *h, int32_t rows);

/* Launch shape of the tournament (scheduling only: the same selection and
 * values bit for bit).  Nodes of at most node_rows rows (every merge node
 * at v <= 256, and the short leaves of late panels, when node_rows = 512)
 * run as ONE launch each: one workgroup takes the node's pivot
 * steps block by block and applies each block's rank update to the node's
 * remaining columns itself.  Taller nodes, and every node when node_rows =
 * 0 (the default: one workgroup's update was measured slower than the
 * spread one), take two launches per 32-column block (the pivot steps in
 * one workgroup, the update spread over many).  node_rows in 0..512; set
 * returns -2 otherwise. */
int cfx_tournament_fusion(cfx_handle *h, int32_t *node_rows);
int cfx_set_tournament_fusion(cfx_handle *h, int32_t node_rows);

/* Tile-stationary schedule of cfx_getrf (rows interchanged; not used by
 * cfx_getrf_masked, which returns CFX_ENOTSUP when it is set): with delay
 * d > 1 the trailing matrix receives the Schur updates of d panels at once,
 * C -= [L21_1 .. L21_d] [U12_1; ..; U12_d] (K = d v), so every C tile is
 * read and written once per d panels instead of once per panel (the S2
 * subcomputations of the I/O-optimal schedule, Sec. 6, with K toward
 * sqrt(M); COnfLUX's per-step cost, Sec. 7.4).  Inside a batch each
 * panel's columns, and its pivot rows' trailing columns, first receive the
 * batch's earlier panels (thin updates).  The pivots and the arithmetic of
 * each element are those of Alg. 1 up to the grouping of the sums (d
 * panels' products accumulate together), so the factors agree with d = 1
 * to rounding.  d in 1..8 (default 1); the workspace of low-precision
 * factorisations grows with d (query cfx_getrf_buffer_size after setting
 * it).  Set returns -2 for an invalid d. */
int cfx_schur_delay(cfx_handle *h, int32_t *delay);
int cfx_set_schur_delay(cfx_handle *h, int32_t delay);

/* Compute units kept free of the overlapped Schur launches of cfx_getrf and
 * cfx_getrf_masked with lookahead (scheduling only: the same factors bit
 * for bit).  The rest of each panel's update runs on a handle stream whose
 * CU mask leaves `cus` compute units out, so the next panel's tournament
 * (the critical path of Sec. 7.3) starts its launches on them at once
 * instead of waiting for the update's workgroups to drain.  cus = 0 puts
 * the update on the caller's stream.  Default 32 (4 per XCD on a
 * 256-CU device).  cus in 0..(compute units / 4);
 * set returns -2 otherwise, and synchronises the handle's previous update
 * stream before replacing it. */
int cfx_reserved_cus(cfx_handle *h, int32_t *cus);
int cfx_set_reserved_cus(cfx_handle *h, int32_t cus);

/* Static description of the library build (host memory, NUL-terminated). */
const char *cfx_version(void);

/* Workspace bytes cfx_getrf needs for an n x n matrix with these options.
 * `bytes` is a host pointer. */
int cfx_getrf_buffer_size(cfx_handle *h, int64_t n, const cfx_lu_opts *opts,
                          size_t *bytes);

/* Blocked right-looking LU with tournament pivoting, A = P L U (Alg. 1,
 * compute steps TournPivot, FactorizeA10, FactorizeA01, FactorizeA11; the
 * pivot rows are interchanged explicitly rather than masked).
 *   n     : order of A, n >= 0.
 *   A     : device, n x n row-major, stride lda >= max(1, n); overwritten by
 *           L (strictly below the diagonal, unit diagonal implicit) and U.
 *   ipiv  : device int32[n]: row i was interchanged with row ipiv[i] >= i,
 *           interchanges applied in order i = 0 .. n-1 (LAPACK style, 0-based).
 *   info  : device int32: 0, or j+1 for the first exactly zero U[j][j]
 *           (the factorisation continues; that column of L is left unscaled).
 *   opts  : host pointer, see cfx_lu_opts.
 *   work  : device workspace of at least cfx_getrf_buffer_size bytes,
 *           256-byte aligned.
 * Asynchronous on `stream`. */
int cfx_getrf(cfx_handle *h, int64_t n, double *A, int64_t lda, int32_t *ipiv,
              int32_t *info, const cfx_lu_opts *opts, void *work,
              size_t work_bytes, void *stream);

/* The same factorisation with row masking instead of row interchanges
 * (Sec. 7.3, "Row Swapping vs. Row Masking"): the pivots are chosen
 * exactly as by cfx_getrf (the same ipiv, the same arithmetic), but no row
 * of A is moved; the library keeps, and returns, the row map
 *   rowmap : device int32[n]: row i of the factors L\U (in the order of
 *            cfx_getrf's output, i.e. of P A) is stored in physical row
 *            rowmap[i] of A; equivalently (P A)[i, :] = A_input[rowmap[i], :].
 * So A[rowmap, :] after this call equals, bit for bit, the A of cfx_getrf
 * on the same input and options.  Every kernel reaches rows through the
 * map (gather on read) instead of the interchange kernel moving 2 vb rows
 * of n columns per panel.  Arguments otherwise as cfx_getrf (rowmap is
 * argument 6; info 7, opts 8, work 9). */
int cfx_getrf_masked(cfx_handle *h, int64_t n, double *A, int64_t lda,
                     int32_t *ipiv, int32_t *rowmap, int32_t *info,
                     const cfx_lu_opts *opts, void *work, size_t work_bytes,
                     void *stream);

/* Tournament pivot selection of one panel (Sec. 7.3; Sec. 7.4 Step 1): the
 * panel is W = rows x vb at device pointer W with stride ldw; row i of W is
 * global row row0 + i.  Writes the vb selected global rows, in selection
 * order, to the device int32 array piv.  W is not modified.  `leaves` as in
 * cfx_lu_opts.  work as for cfx_getrf with n = rows, v = vb.
 * Asynchronous on `stream`. */
int cfx_tslu(cfx_handle *h, int64_t rows, int64_t vb, const double *W,
             int64_t ldw, int64_t row0, int32_t leaves, int32_t *piv,
             void *work, size_t work_bytes, void *stream);

/* The Schur-complement update alone (FactorizeA11 of Alg. 1, statement S2
 * of Sec. 6, which carries the 2N^3/3 flops of the factorisation):
 *     C[0:m, 0:n] -= L21[0:m, 0:K] U12[0:K, 0:n]
 * with the arithmetic cfx_getrf uses for `precision` (FP64: FP64 matrix
 * cores, FP64 accumulation; BF16/FP16/FP8: operands rounded as described
 * under cfx_lu_opts, FP32 accumulation, FP64 C).
 *   L21 : device, m x K row-major, stride ldl >= max(1, K).
 *   U12 : device, K x n row-major, stride ldu >= max(1, n).
 *   C   : device, m x n row-major, stride ldc >= max(1, n); must not
 *         overlap L21 or U12.
 *   max_workgroups : 0 = one workgroup per 128 x 128 tile; else (>= 8) a
 *         persistent grid of that many workgroups walks the tiles.
 *   work : device, cfx_schur_update_buffer_size bytes, 256-byte aligned
 *         (0 bytes, and work may be NULL, for FP64; the packed operands
 *         otherwise).
 * Asynchronous on `stream`. */
int cfx_schur_update_buffer_size(cfx_handle *h, int32_t precision, int64_t m,
                                 int64_t n, int64_t K, size_t *bytes);
int cfx_schur_update(cfx_handle *h, int32_t precision, int64_t m, int64_t n,
                     int64_t K, const double *L21, int64_t ldl,
                     const double *U12, int64_t ldu, double *C, int64_t ldc,
                     int32_t max_workgroups, void *work, size_t work_bytes,
                     void *stream);

/* Solve A X = B with the factors of cfx_getrf: apply the interchanges of
 * ipiv to B in order, forward substitution with unit L, back substitution
 * with U.
 *   LU   : device, n x n factors, stride lda.
 *   ipiv : device int32[n] as written by cfx_getrf (i <= ipiv[i] < n); an
 *          entry outside [i, n) is taken as no interchange.
 *   B    : device, n x nrhs row-major, stride ldb >= nrhs; overwritten by X.
 * Asynchronous on `stream`. */
int cfx_getrs(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU,
              int64_t lda, const int32_t *ipiv, double *B, int64_t ldb,
              void *stream);
/* cfx_getrs for the factors of cfx_getrf_masked: factor row i is physical
 * row rowmap[i] of LU, and rowmap is also the permutation of P B (so no
 * ipiv is needed).  Same results as cfx_getrs on the interchanged factors;
 * scratch, ordering and errors as cfx_getrs. */
int cfx_getrs_masked(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU,
                     int64_t lda, const int32_t *rowmap, double *B, int64_t ldb,
                     void *stream);

/* Scratch and ordering of cfx_getrs: the permutation and the gathered
 * right-hand sides (with one right-hand side, also the solve's intermediate
 * vector: n x max(nrhs, 2) doubles) live in a device buffer owned by the
 * handle, grown with
 * hipMalloc when a call needs more (hipFree of the old one waits for the
 * device).  Calls on one handle are ordered on the device through an event
 * of the handle, whatever streams they are issued on.
 *
 * A single contiguous right-hand side takes a one-launch-per-triangle solve
 * whose blocks wait for earlier blocks with a bounded spin.  The waits end
 * on a working device; if one ever gives up, that block writes NaN for its
 * rows and a sticky flag of the handle is set.  cfx_getrs_check
 * (host-blocking: it synchronises `stream`) returns CFX_ESOLVE and clears
 * the flag when any solve on the handle gave up since the last check, else
 * CFX_OK.  cfx_set_solve_spin_limit sets the number of polls before a wait
 * gives up (default 4194304; 0 gives up at once, which tests use to force
 * the error path while every kernel still exits normally); it also applies
 * to cfx_gesv_ir and to serving workers.  Returns -2 for polls < 0. */
int cfx_getrs_check(cfx_handle *h, void *stream);
int cfx_set_solve_spin_limit(cfx_handle *h, int32_t polls);

/* cfx_getrs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, with the same arguments, results and errors, but its
 * permutation, gathered right-hand sides and counters live in a fixed
 * device array of 32 MiB per GPU (set up by cfx_create; held until the
 * process ends) instead of the handle's growable scratch.  No call on this
 * path allocates or frees memory.
 *   Limit: 256 + 4 n (rounded up to 256) + 8 n max(nrhs, 2) bytes <= 32 MiB
 *   (e.g. n = 32768 with up to 127 right-hand sides); larger problems return
 *   CFX_ENOTSUP without doing anything.
 *   Every call on one GPU shares that array: calls that overlap on the
 *   device race (order them on one stream, or through events).  The
 *   give-up flag of its one-launch solve is cleared at the start of each
 *   call and read by cfx_getrs_check. */
int cfx_getrs_noalloc(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU,
                      int64_t lda, const int32_t *ipiv, double *B, int64_t ldb,
                      void *stream);

/* Mixed-precision solve with iterative refinement.  The paper computes the
 * factorisation only; refinement is the standard GMRES-IR of Carson and
 * Higham (SIAM J. Sci. Comput. 40(2), 2018): the tournament-pivoted LU of
 * Alg. 1, with its Schur updates (FactorizeA11) in lu.precision, is the
 * left preconditioner M = U^{-1} L^{-1} P of GMRES on M A d = M r; the
 * residual r = b - A x (compensated FP64 row sums), the GMRES iteration and
 * the update x += d are FP64.  Refinement of a right-hand side stops when
 * its normwise backward error
 *     eta = |b - A x|_inf / (|A|_inf |x|_inf + |b|_inf)
 * is <= tol, after max_outer refinement steps, or when eta has not halved
 * over the last two steps (stagnation: the factors are too inaccurate for
 * this matrix; converged is then 0).
 *   lu            : factorisation options (precision CFX_PREC_BF16/FP16 for
 *                   the mixed-precision factorisation; FP64 also allowed).
 *   tol           : target eta (>= 0), e.g. 5e-15.
 *   max_outer     : maximum refinement steps (0 .. 10000).
 *   gmres_restart : Krylov dimension of one GMRES solve (1 .. 64).
 *   gmres_tol     : relative reduction of the preconditioned residual that
 *                   ends one GMRES solve, in (0, 1). */
typedef struct {
    cfx_lu_opts lu;
    double tol;
    int32_t max_outer;
    int32_t gmres_restart;
    double gmres_tol;
} cfx_ir_opts;

typedef struct {
    double eta;          /* final eta, maximum over the right-hand sides     */
    double eta_first;    /* eta of the plain solve with the factors (max)    */
    int32_t outer;       /* refinement steps, maximum over right-hand sides  */
    int32_t inner;       /* GMRES iterations, summed over right-hand sides   */
    int32_t converged;   /* 1 if every right-hand side reached tol           */
    int32_t info;        /* info of the factorisation (see cfx_getrf)        */
} cfx_ir_report;

/* Workspace bytes of cfx_gesv_ir (host pointer `bytes`): an n x n factor
 * copy, pivots, the getrf workspace and (gmres_restart + 9) n-vectors (one
 * of them the intermediate vector of the one-launch triangular solves). */
int cfx_gesv_ir_buffer_size(cfx_handle *h, int64_t n, int64_t nrhs,
                            const cfx_ir_opts *opts, size_t *bytes);

/* Solve A X = B by factorisation + GMRES-IR.
 *   A    : device, n x n row-major, stride lda; NOT modified (the library
 *          factors a copy inside work).
 *   B    : device, n x nrhs row-major, stride ldb; not modified.
 *   X    : device, n x nrhs row-major, stride ldx; receives the solution.
 *   rep  : host pointer, filled before return.
 *   work : device, >= cfx_gesv_ir_buffer_size bytes, 256-byte aligned.
 * Host-blocking: returns when X and rep are final (it synchronises
 * `stream`, on which all of its work runs).  A singular factorisation is
 * reported through rep->info (and a non-finite eta), not the return value.
 * Returns CFX_ESOLVE (rep still filled, eta NaN) when a triangular solve of
 * the refinement gave up a wait (see cfx_getrs_check). */
int cfx_gesv_ir(cfx_handle *h, int64_t n, int64_t nrhs, const double *A,
                int64_t lda, const double *B, int64_t ldb, double *X,
                int64_t ldx, const cfx_ir_opts *opts, cfx_ir_report *rep,
                void *work, size_t work_bytes, void *stream);

/* Batched LU + solve of `count` independent systems A_i X_i = B_i in one
 * persistent launch (preceded by a one-workgroup sort of the systems by
 * size).  Each system is factored as cfx_getrf with leaves = 1 (TP(v, 1):
 * every panel's pivots come from GEPP of the whole panel, ties to the
 * smaller row, Sec. 7.3), with the panel width v taken per size class from
 * the handle's tuning table, then solved like cfx_getrs.
 * All array arguments are DEVICE arrays of `count` entries:
 *   n[i]     : order, 0 <= n[i] <= 512.
 *   nrhs[i]  : right-hand sides, 0 <= nrhs[i] <= 16.
 *   A[i]     : device pointer, n x n row-major, stride lda[i] >= max(1, n);
 *              overwritten by L and U (as cfx_getrf).
 *   B[i]     : device pointer, n x nrhs row-major, stride ldb[i] >=
 *              max(1, nrhs); overwritten by X.
 *   ipiv[i]  : device pointer to int32[n[i]] (as cfx_getrf).
 *   info[i]  : 0, j+1 for the first exactly zero U[j][j] (that system's X
 *              is then not finite), or -k when that system's k-th
 *              descriptor is invalid (1 n, 2 A/ipiv null, 3 lda, 4 nrhs,
 *              5 B null, 6 ldb); an invalid system is skipped.
 *   work     : device, cfx_gesv_batched_buffer_size bytes, 256-byte aligned.
 *   flags    : 0, or CFX_BATCHED_NO_GRAPH.  By default the launches are
 *              captured into a HIP graph on the first call and the graph is
 *              replayed by later calls with identical arguments (same
 *              count, array pointers and work); the array CONTENTS are read
 *              at run time, so new systems in the same buffers reuse it.
 * Asynchronous on `stream`. */
enum { CFX_BATCHED_NO_GRAPH = 1 };

int cfx_gesv_batched_buffer_size(cfx_handle *h, int32_t count, size_t *bytes);
int cfx_gesv_batched(cfx_handle *h, int32_t count, const int32_t *n,
                     const int32_t *nrhs, double *const *A, const int64_t *lda,
                     double *const *B, const int64_t *ldb, int32_t *const *ipiv,
                     int32_t *info, void *work, size_t work_bytes, int32_t flags,
                     void *stream);

/* Autotuner of the batched panel width: for each size class (n <= 32, 64,
 * 128, 256, 512) it times the batched launch on synthetic diagonally
 * shifted systems of the class's largest order with v in {8, 16, 32} and
 * keeps the fastest in the handle's table.  Allocates and frees its own
 * device buffers (about 2.2 GB); host-blocking on `stream`. */
int cfx_batched_tune(cfx_handle *h, void *stream);
/* Read / set the table (host int32[5], entries in {8, 16, 32}). */
int cfx_batched_tuning(cfx_handle *h, int32_t *vb);
int cfx_batched_set_tuning(cfx_handle *h, const int32_t *vb);

/* ------------------------------------------------------------------------
 * Serving: a request loop on one device.  Requests (solve A X = B, or solve
 * again with factors kept from an earlier request) are queued by
 * cfx_serve_submit from any thread; worker threads, one per slot, each with
 * its own stream, admit them in arrival order as soon as a slot is free and
 * the request's device memory fits in the caller's arena (resident factors
 * nobody is using are evicted, least recently used first, to make room).
 * Admitted requests run concurrently on their streams.  Consecutive queued
 * systems of order <= 512 are admitted together and solved by one
 * cfx_gesv_batched launch (FP64; their factors may be kept resident too).
 * Larger systems are factored by cfx_getrf with the configured precision
 * and solved with cfx_getrs semantics (FP64), refined by GMRES-IR
 * (BF16/FP16); when refinement from low-precision factors does not reach
 * ir.tol (it stops after ir.max_outer steps or on stagnation), the request
 * refactors in FP64 and solves again.  Every result reports its eta (as cfx_gesv_ir), and its
 * arithmetic does not depend on what else runs: a request gives the same
 * bits alone and in a mix.
 * ------------------------------------------------------------------------ */
typedef struct cfx_server cfx_server;

typedef struct {
    void *arena;             /* device memory owned by the caller           */
    size_t arena_bytes;      /* the HBM budget of the server                */
    int32_t max_slots;       /* concurrent requests (worker threads), 1..64 */
    cfx_ir_opts ir;          /* factorisation + refinement options; with
                                ir.lu.precision FP64, ir.max_outer = 0 gives
                                the plain solve                            */
    int32_t batch_max;       /* max systems per batched launch (0: 256)     */
    int64_t lowp_min_n;      /* with a low-precision ir.lu.precision: the
                                smallest order factored in that precision;
                                smaller requests are factored in FP64 (the
                                low-precision route only pays off for large
                                systems).  0: every request in ir.lu's
                                precision                                  */
} cfx_serve_cfg;

enum { CFX_SOLVE = 0, CFX_RESOLVE = 1 };

/* One request.  A, B, X are DEVICE pointers owned by the caller and must
 * stay valid (A and B unchanged) until the result has been polled.  The
 * server's streams do not wait for any stream of the caller: A and B must
 * be written, and no pending work may touch X, when the request is
 * submitted.
 *   kind          : CFX_SOLVE, or CFX_RESOLVE to reuse the resident factors
 *                   `factor_id` (refactored from A when they were evicted).
 *   n, nrhs       : order (1 .. INT32_MAX) and right-hand sides (>= 1).
 *   A / lda       : n x n row-major (read only).
 *   B / ldb       : n x nrhs row-major (read only).
 *   X / ldx       : n x nrhs row-major, receives the solution.
 *   keep_resident : keep the factors on the device after the request. */
typedef struct {
    int32_t kind;
    int32_t keep_resident;
    uint64_t factor_id;
    int64_t n, nrhs;
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    double *X;
    int64_t ldx;
} cfx_request;

typedef struct {
    int32_t status;      /* CFX_OK, or CFX_ENOMEM (does not fit the arena),
                            CFX_ESOLVE (a triangular solve gave up a wait)
                            or another error code of the solve             */
    int32_t info;        /* factorisation info                             */
    uint64_t factor_id;  /* id of the factors used (new or reused)         */
    int32_t resident_hit;/* RESOLVE found its factors on the device        */
    int32_t batched;     /* solved inside a batched launch                 */
    int32_t outer, inner;/* refinement steps / GMRES iterations            */
    double eta;          /* backward error of X (max over right-hand sides) */
    double t_submit, t_admit, t_start, t_done; /* seconds, steady clock,
                            from server creation                           */
    int32_t fallback;    /* 1: the low-precision factors did not reach the
                            refinement target, so the request refactored A
                            in FP64 (the resident factors are FP64 since)  */
} cfx_result;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t resident_hits, resident_misses, evictions;
    int64_t batches, batched_requests;
    int64_t resident_factors;
    size_t bytes_in_use, bytes_peak;
} cfx_serve_stats;

/* Start the workers (host threads) on the current device.  cfg is copied. */
int cfx_serve_create(const cfx_serve_cfg *cfg, cfx_server **out);
/* Queue a request (non-blocking, thread-safe); *ticket identifies it.
 * Returns -2 for an invalid request. */
int cfx_serve_submit(cfx_server *s, const cfx_request *req, uint64_t *ticket);
/* CFX_PENDING while the request is queued or running; CFX_OK once done,
 * with *out filled and the ticket retired.  -2: unknown ticket. */
int cfx_serve_poll(cfx_server *s, uint64_t ticket, cfx_result *out);
/* Drop resident factors (CFX_EBUSY while a request is using them). */
int cfx_serve_release(cfx_server *s, uint64_t factor_id);
int cfx_serve_stats_get(cfx_server *s, cfx_serve_stats *out);
/* Finish every queued request, stop the workers, free the server.  Results
 * not yet polled are discarded. */
int cfx_serve_destroy(cfx_server *s);

/* Per-phase device time of the factorisation steps, for measurement.
 * Between cfx_profile_begin and cfx_profile_end every cfx_getrf on the
 * handle records HIP events around each phase on the stream that runs it
 * (the column-chunk launches of one overlapped trailing update form one
 * timed span; schur_launches counts the launches inside the spans).
 * cfx_profile_end waits for those events (host-blocking), fills `out`
 * (host pointer) with the summed durations and stops recording.
 *   schur_flops : algorithmic flops of the Schur updates, 2 * rows * cols * K
 *                 summed over launches (statement S2 of Sec. 6, twice for
 *                 the multiply and the subtract). */
typedef struct {
    double tslu_ms;       /* TournPivot: leaves and playoff rounds        */
    double laswp_ms;      /* row interchanges                             */
    double trsm_ms;       /* FactorizeA10 + FactorizeA01                  */
    double schur_ms;      /* FactorizeA11                                 */
    double schur_flops;
    int64_t schur_launches;
    int64_t panels;
} cfx_profile;

int cfx_profile_begin(cfx_handle *h);
int cfx_profile_end(cfx_handle *h, cfx_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* CFX_H */

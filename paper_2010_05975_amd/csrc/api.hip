// C ABI entry points (include/cfx.h): argument checks, workspace carving and
// the host loop over panels of Alg. 1 (TournPivot, interchanges,
// FactorizeA10/A01, FactorizeA11 per panel).
#include <cmath>
#include <new>
#include <vector>

#include "cfx_internal.h"

namespace cfx {
enum Phase { PH_TSLU = 0, PH_LASWP, PH_TRSM, PH_SCHUR, PH_COUNT };

// Event-pair recorder behind cfx_profile_begin / cfx_profile_end.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int phase; hipEvent_t a, b; double flops; int launches; };
    std::vector<Rec> recs;
    int64_t panels = 0;

    hipEvent_t next()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    // Returns the begin event (or null when not recording).
    hipEvent_t begin(hipStream_t st)
    {
        if (!on) return nullptr;
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, st);
        return e;
    }
    void end(int phase, hipEvent_t a, hipStream_t st, double flops = 0.0, int launches = 1)
    {
        if (!on || !a) return;
        hipEvent_t e = next();
        if (!e) return;
        (void)hipEventRecord(e, st);
        recs.push_back({phase, a, e, flops, launches});
    }
};
}  // namespace cfx

namespace cfx {
constexpr int kLpSchurWgs = 384;
constexpr int64_t kLaChunk = 512;    // columns per overlapped launch without reserved compute units
constexpr int kReserveCus = 32;      // compute units kept free for the tournament by default
constexpr int64_t kFullTrsmRows = 16384;   // trailing size from which all of U12 is solved up front
}  // namespace cfx

struct cfx_handle {
    int device = 0;
    hipStream_t side = nullptr;     // lookahead stream (default priority)
    hipEvent_t ev_panel = nullptr;  // next panel's columns updated
    hipEvent_t ev_tslu = nullptr;   // next panel's tournament done
    // the rest of each overlapped update runs on `upd`, a stream whose CU
    // mask leaves `reserve_cus` compute units free: the tournament's
    // launches start there at once instead of waiting for the update's
    // workgroups to drain (null: the caller's stream)
    hipStream_t upd = nullptr;
    hipEvent_t ev_upd = nullptr;    // the rest of the last update done
    int64_t full_trsm_rows = cfx::kFullTrsmRows;   // all of U12 up front from this trailing size
    int reserve_cus = 0;

    void *scratch = nullptr;        // getrs permutation + gather buffer
    size_t scratch_bytes = 0;
    int32_t *gsync = nullptr;       // getrs: counters of the one-launch solves
                                    // (kTrsvSyncBytes; [4] = a wait gave up)
    hipEvent_t ev_getrs = nullptr;  // the last getrs on this handle (scratch reuse)
    bool getrs_issued = false;
    int spin_limit = cfx::kSolveSpinLimit;
    void *na_scratch = nullptr;     // this device's scratch of cfx_getrs_noalloc
    cfx::Profiler prof;
    int cu_count = 256;
    // grid bound of the Schur updates that overlap the next tournament
    // (0: one workgroup per tile; -1: by precision, none for FP64 and
    // kLpSchurWgs for the HBM-bound low-precision update, which then leaves
    // compute units to the tournament at little cost of its own)
    int schur_wgs = -1;
    int64_t la_chunk = 0;           // columns per overlapped Schur launch (0: automatic)
    int delay = 1;                  // panels per trailing update (tile-stationary schedule)
    int fuse_rows = cfx::kFuseRowsDefault;  // tournament nodes up to this height run as one launch
    bool one_stream = false;        // lookahead launches on the caller's stream only
    // batched: panel width per size class (the tuner's table) and the graph
    // of the last batched call, replayed when the arguments repeat
    int32_t bvb[cfx::kBatchClasses] = {8, 16, 16, 32, 32};
    int64_t bvb_version = 0;
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    struct {
        int32_t count;
        const void *p[10];
        int64_t version;
    } bkey{};
};

namespace cfx {

int solve_spin_limit(const cfx_handle *h) { return h->spin_limit; }

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }


struct Layout {
    int64_t max_nodes, node_rows;
    size_t off_S, off_cand0, off_cand1, off_cnt0, off_cnt1, off_plan, off_plan2, off_lu00, off_selg, off_rsel,
        off_utg, off_rtg, off_mp, total;
};

static Layout layout(int64_t n, int v, int leaves, int precision, int delay, int min_leaf)
{
    Layout L{};
    int64_t h0 = (n + leaves - 1) / leaves;
    if (h0 < v) h0 = v;
    // with a minimum leaf height R, panels shorter than L R rows have
    // fewer leaves of up to R rows
    if (min_leaf > 0 && (n < min_leaf ? n : min_leaf) > h0) h0 = n < min_leaf ? n : min_leaf;
    // A panel with r rows has ceil(r / max(vb, ceil(r / leaves))) <= leaves
    // nodes; that count is not monotone in r, so bound it by leaves (and n).
    L.max_nodes = leaves < n ? leaves : n;
    if (L.max_nodes < 1) L.max_nodes = 1;
    L.node_rows = h0 > 2 * v ? h0 : 2 * v;
    size_t o = 0;
    L.off_S = o;     o = align_up(o + (size_t)L.max_nodes * L.node_rows * v * sizeof(double));
    L.off_cand0 = o; o = align_up(o + (size_t)L.max_nodes * v * sizeof(int32_t));
    L.off_cand1 = o; o = align_up(o + (size_t)L.max_nodes * v * sizeof(int32_t));
    L.off_cnt0 = o;  o = align_up(o + (size_t)L.max_nodes * sizeof(int32_t));
    L.off_cnt1 = o;  o = align_up(o + (size_t)L.max_nodes * sizeof(int32_t));
    L.off_plan = o;  o = align_up(o + (size_t)(1 + 4 * kMaxV) * sizeof(int32_t));
    L.off_plan2 = o; o = align_up(o + (size_t)(1 + 4 * kMaxV) * sizeof(int32_t));
    L.off_lu00 = o;  o = align_up(o + (size_t)v * v * sizeof(double));
    L.off_selg = o;  o = align_up(o + (size_t)L.max_nodes * 2 * kMaxV * sizeof(int32_t));
    L.off_rsel = o;  o = align_up(o + (size_t)L.max_nodes * L.node_rows);
    L.off_utg = o;   o = align_up(o + (size_t)L.max_nodes * 32 * kMaxV * sizeof(double));
    L.off_rtg = o;   o = align_up(o + (size_t)L.max_nodes * 32 * 40 * sizeof(double));
    L.off_mp = o;
    // packed operands of the widest low-precision update (K = delay v)
    if (precision != CFX_PREC_FP64) o = align_up(o + lp_pack_bytes(precision, n, n, v * delay));
    L.total = o;
    return L;
}

size_t workspace_bytes(int64_t n, int v, int leaves, int precision, int delay, int min_leaf)
{
    return layout(n, v, leaves, precision, delay, min_leaf).total;
}

int carve_workspace(void *work, size_t bytes, int64_t n, int v, int leaves, int precision,
                    Workspace *ws, int delay, int min_leaf)
{
    Layout L = layout(n, v, leaves, precision, delay, min_leaf);
    if (bytes < L.total) return CFX_ENOMEM;
    char *b = static_cast<char *>(work);
    ws->S = reinterpret_cast<double *>(b + L.off_S);
    ws->s_node = L.node_rows * v;
    ws->cand[0] = reinterpret_cast<int32_t *>(b + L.off_cand0);
    ws->cand[1] = reinterpret_cast<int32_t *>(b + L.off_cand1);
    ws->ccnt[0] = reinterpret_cast<int32_t *>(b + L.off_cnt0);
    ws->ccnt[1] = reinterpret_cast<int32_t *>(b + L.off_cnt1);
    ws->plan = reinterpret_cast<int32_t *>(b + L.off_plan);
    ws->plan_alt = reinterpret_cast<int32_t *>(b + L.off_plan2);
    ws->lu00 = reinterpret_cast<double *>(b + L.off_lu00);
    ws->selg = reinterpret_cast<int32_t *>(b + L.off_selg);
    ws->rsel = reinterpret_cast<unsigned char *>(b + L.off_rsel);
    ws->rs_node = L.node_rows;
    ws->utg = reinterpret_cast<double *>(b + L.off_utg);
    ws->rtg = reinterpret_cast<double *>(b + L.off_rtg);
    ws->scratch = reinterpret_cast<double *>(b + L.off_mp);
    ws->scratch_bytes = bytes - L.off_mp;
    ws->max_nodes = L.max_nodes;
    return CFX_OK;
}

static int check_opts(const cfx_lu_opts *o)
{
    if (!o) return 1;
    if (o->v < 1 || o->v > kMaxV) return 1;
    if (o->leaves < 1) return 1;
    if (o->precision != CFX_PREC_FP64 && o->precision != CFX_PREC_BF16 && o->precision != CFX_PREC_FP16 &&
        o->precision != CFX_PREC_FP8)
        return 2;
    if (o->lookahead < 0 || o->lookahead > 1) return 1;
    if (o->min_leaf_rows < 0 || o->min_leaf_rows > kMaxLeafRows) return 1;
    return 0;
}

static int ensure_scratch(cfx_handle *h, size_t bytes)
{
    if (h->scratch_bytes >= bytes) return CFX_OK;
    // hipFree waits for the device, so no earlier getrs still reads it
    if (h->scratch) CFX_HIP(hipFree(h->scratch));
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    CFX_HIP(hipMalloc(&h->scratch, bytes));
    h->scratch_bytes = bytes;
    return CFX_OK;
}

static int check_ir_opts(const cfx_ir_opts *o)
{
    if (!o) return 1;
    if (int c = check_opts(&o->lu)) return c;
    if (!(o->tol >= 0)) return 1;
    if (o->max_outer < 0 || o->max_outer > 10000) return 1;
    if (o->gmres_restart < 1 || o->gmres_restart > 64) return 1;
    if (!(o->gmres_tol > 0 && o->gmres_tol < 1)) return 1;
    return 0;
}

// Workspace of cfx_gesv_ir: factor copy, ipiv, perm, info, the getrf
// workspace and the refinement vectors.
struct IrLayout {
    size_t off_F, off_ipiv, off_perm, off_info, off_getrf, getrf_bytes, off_vec, total;
};

static IrLayout ir_layout(int64_t n, const cfx_ir_opts *o, int delay)
{
    IrLayout L{};
    size_t p = 0;
    L.off_F = p;     p = align_up(p + (size_t)n * n * sizeof(double));
    L.off_ipiv = p;  p = align_up(p + (size_t)n * sizeof(int32_t));
    L.off_perm = p;  p = align_up(p + (size_t)n * sizeof(int32_t));
    L.off_info = p;  p = align_up(p + sizeof(int32_t));
    L.off_getrf = p;
    L.getrf_bytes = workspace_bytes(n, o->lu.v, o->lu.leaves, o->lu.precision, delay, o->lu.min_leaf_rows);
    p = align_up(p + L.getrf_bytes);
    L.off_vec = p;   p = align_up(p + ir_vec_bytes(n, o->gmres_restart));
    L.total = p;
    return L;
}

}  // namespace cfx

using namespace cfx;

extern "C" {

const char *cfx_version(void)
{
    return "cfx 0.1 gfx950: TP(v,L) blocked LU, FP64 MFMA Schur update";
}

int cfx_create(cfx_handle **h)
{
    if (!h) return -1;
    cfx_handle *p = new (std::nothrow) cfx_handle();
    if (!p) return CFX_ENOMEM;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_panel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_tslu, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_upd, hipEventDisableTiming) != hipSuccess) {
        cfx_destroy(p);
        return CFX_EHIP;
    }
    if (hipEventCreateWithFlags(&p->ev_getrs, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&p->gsync, kTrsvSyncBytes) != hipSuccess ||
        hipMemset(p->gsync, 0, kTrsvSyncBytes) != hipSuccess) {
        cfx_destroy(p);
        return CFX_EHIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
        cus > 0)
        p->cu_count = cus;
    if (int rc = init_kernel_attributes()) {
        cfx_destroy(p);
        return rc;
    }
    if (int rc = cfx_set_reserved_cus(p, p->cu_count >= 4 * kReserveCus ? kReserveCus : p->cu_count / 4)) {
        cfx_destroy(p);
        return rc;
    }
    if (int rc = noalloc_scratch(p->device, &p->na_scratch)) {
        cfx_destroy(p);
        return rc;
    }

    *h = p;
    return CFX_OK;
}

int cfx_profile_begin(cfx_handle *h)
{
    if (!h) return -1;
    h->prof.on = true;
    h->prof.used = 0;
    h->prof.recs.clear();
    h->prof.panels = 0;
    return CFX_OK;
}

int cfx_profile_end(cfx_handle *h, cfx_profile *out)
{
    if (!h) return -1;
    if (!out) return -2;
    Profiler &pf = h->prof;
    cfx_profile r{};
    double ms[PH_COUNT] = {0, 0, 0, 0};
    for (const auto &rec : pf.recs) {
        CFX_HIP(hipEventSynchronize(rec.b));
        float t = 0.f;
        CFX_HIP(hipEventElapsedTime(&t, rec.a, rec.b));
        ms[rec.phase] += t;
        if (rec.phase == PH_SCHUR) {
            r.schur_flops += rec.flops;
            r.schur_launches += rec.launches;
        }
    }
    r.tslu_ms = ms[PH_TSLU];
    r.laswp_ms = ms[PH_LASWP];
    r.trsm_ms = ms[PH_TRSM];
    r.schur_ms = ms[PH_SCHUR];
    r.panels = pf.panels;
    *out = r;
    pf.on = false;
    pf.recs.clear();
    pf.used = 0;
    return CFX_OK;
}

int cfx_destroy(cfx_handle *h)
{
    if (!h) return -1;
    for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
    if (h->scratch) (void)hipFree(h->scratch);
    if (h->gsync) (void)hipFree(h->gsync);
    if (h->ev_getrs) (void)hipEventDestroy(h->ev_getrs);
    if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
    if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->ev_tslu) (void)hipEventDestroy(h->ev_tslu);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->upd) (void)hipStreamDestroy(h->upd);
    if (h->ev_upd) (void)hipEventDestroy(h->ev_upd);
    delete h;
    return CFX_OK;
}

int cfx_getrf_buffer_size(cfx_handle *h, int64_t n, const cfx_lu_opts *opts, size_t *bytes)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (check_opts(opts)) return check_opts(opts) == 2 ? CFX_ENOTSUP : -3;
    if (!bytes) return -4;
    *bytes = workspace_bytes(n, opts->v, opts->leaves, opts->precision, h->delay, opts->min_leaf_rows);
    return CFX_OK;
}

}  // extern "C"

namespace cfx {

// The tile-stationary schedule (the handle's delay d > 1): the trailing
// matrix receives the Schur updates of d panels at once, C -= [L21 ...]
// [U12; ...] with K = d v, so each C tile is read and written once per d
// panels while it accumulates d v products in registers: the S2
// subcomputations of the I/O-optimal schedule (Sec. 6, X-partition with
// rho = sqrt(M)/2; COnfLUX's per-step cost, Sec. 7.4) take K toward
// sqrt(M).  Inside a batch only what the next steps read is brought up to
// date: panel k's columns receive the batch's earlier panels before its
// tournament, and its pivot rows' trailing columns before U12 (both K =
// k - K0 updates of thin blocks).  Interchanges move whole rows, so the
// batch's L21 columns stay aligned with the rows of the trailing matrix.
// The first tournament of each batch runs beside the batch-end update
// (lookahead); the others have only the thin updates beside them.
static int getrf_run_delayed(cfx_handle *h, int64_t n, double *A, int64_t lda, int32_t *ipiv, int32_t *info,
                             const cfx_lu_opts *opts, const Workspace &ws, hipStream_t st)
{
    const int prec = opts->precision, v = opts->v, Lv = opts->leaves, d = h->delay;
    const bool la = opts->lookahead != 0;
    hipStream_t side = h->one_stream ? st : h->side;
    Profiler &pf = h->prof;
    auto at = [&](int64_t r, int64_t c) { return A + r * lda + c; };
    // A[r:r+m, c:c+nc] -= A[r:r+m, k0:k0+K] A[k0:k0+K, c:c+nc], one launch
    auto update = [&](int64_t r, int64_t c, int64_t m, int64_t nc, int64_t k0, int64_t K, hipStream_t s) -> int {
        if (m <= 0 || nc <= 0 || K <= 0) return CFX_OK;
        hipEvent_t e = pf.begin(s);
        int rc;
        if (prec == CFX_PREC_FP64) {
            rc = launch_schur_f64(at(r, k0), lda, at(k0, c), lda, at(r, c), lda, m, nc, (int)K, 0, s);
        } else {
            rc = launch_pack_lp(prec, at(r, k0), lda, m, at(k0, c), lda, nc, (int)K, ws.scratch, s);
            if (!rc) rc = launch_schur_lp(prec, ws.scratch, m, nc, (int)K, 0, nc, at(r, c), lda, 0, s);
        }
        pf.end(PH_SCHUR, e, s, 2.0 * (double)m * (double)nc * (double)K);
        return rc;
    };
    auto tslu = [&](int64_t k, hipStream_t s) -> int {
        const int vb = (int)((n - k) < v ? (n - k) : v);
        hipEvent_t e = pf.begin(s);
        const int rc = launch_tslu(at(k, k), lda, k, n - k, vb, panel_leaves(Lv, opts->min_leaf_rows, n - k), ws,
                                   nullptr, ipiv, info, s, nullptr, h->fuse_rows);
        pf.end(PH_TSLU, e, s);
        return rc;
    };
    int rc;
    if ((rc = tslu(0, st))) return rc;
    bool tslu_on_side = false;
    for (int64_t K0 = 0; K0 < n; K0 += (int64_t)d * v) {
        const int64_t kE = (K0 + (int64_t)d * v) < n ? K0 + (int64_t)d * v : n;
        for (int64_t k = K0; k < kE; k += v) {
            const int vb = (int)((n - k) < v ? (n - k) : v);
            const int64_t m = n - k - vb;
            if (k > K0) {
                // panel k's columns receive the batch's earlier panels
                if ((rc = update(k, k, n - k, vb, K0, k - K0, st))) return rc;
                if ((rc = tslu(k, st))) return rc;
            } else if (tslu_on_side) {
                CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
                tslu_on_side = false;
            } else if (k > 0) {
                if ((rc = tslu(k, st))) return rc;
            }
            hipEvent_t e = pf.begin(st);
            if ((rc = launch_laswp(A, lda, n, k, vb, ws, st))) return rc;
            pf.end(PH_LASWP, e, st);
            if (m > 0) {
                if (k == K0) {
                    e = pf.begin(st);
                    if ((rc = launch_trsm(A, lda, k, vb, m, st))) return rc;
                    pf.end(PH_TRSM, e, st);
                } else {
                    e = pf.begin(st);
                    if ((rc = launch_trsm_first(A, lda, k, vb, m, 0, st))) return rc;   // L21
                    pf.end(PH_TRSM, e, st);
                    // the pivot rows' trailing columns receive the batch's earlier panels
                    if ((rc = update(k, k + vb, vb, m, K0, k - K0, st))) return rc;
                    e = pf.begin(st);
                    if ((rc = launch_trsm_rest(A, lda, k, vb, m, 0, st))) return rc;    // U12
                    pf.end(PH_TRSM, e, st);
                }
            }
            if (pf.on) ++pf.panels;
        }
        // the batch-end update of rows and columns kE.. with K = kE - K0
        const int64_t m = n - kE, K = kE - K0;
        if (m <= 0) break;
        const int vbn = (int)(m < v ? m : v);
        const double *Lb = at(kE, K0), *Ub = at(K0, kE);
        double *Cb = at(kE, kE);
        auto part = [&](int64_t c0, int64_t cw, int wgs, hipStream_t s) -> int {
            if (prec == CFX_PREC_FP64)
                return launch_schur_f64(Lb, lda, Ub + c0, lda, Cb + c0, lda, m, cw, (int)K, wgs, s);
            return launch_schur_lp(prec, ws.scratch, m, m, (int)K, c0, cw, Cb, lda, wgs, s);
        };
        hipEvent_t e = pf.begin(st);
        if (prec != CFX_PREC_FP64 && (rc = launch_pack_lp(prec, Lb, lda, m, Ub, lda, m, (int)K, ws.scratch, st)))
            return rc;
        if ((rc = part(0, vbn, 0, st))) return rc;       // the next panel's columns first
        pf.end(PH_SCHUR, e, st, 2.0 * (double)m * vbn * (double)K);
        if (la) {
            CFX_HIP(hipEventRecord(h->ev_panel, st));
            CFX_HIP(hipStreamWaitEvent(side, h->ev_panel, 0));
            if ((rc = tslu(kE, side))) return rc;
            CFX_HIP(hipEventRecord(h->ev_tslu, side));
            tslu_on_side = true;
        }
        const int64_t chunk = la ? (h->la_chunk > 0 ? h->la_chunk : kLaChunk) : m;
        const int wgs = la ? (h->schur_wgs >= 0 ? h->schur_wgs : (prec == CFX_PREC_FP64 ? 0 : cfx::kLpSchurWgs)) : 0;
        if (vbn < m) {
            e = pf.begin(st);
            int nl = 0;
            for (int64_t c0 = vbn; c0 < m; c0 += chunk, ++nl) {
                const int64_t cw = (m - c0) < chunk ? (m - c0) : chunk;
                if ((rc = part(c0, cw, wgs, st))) return rc;
            }
            pf.end(PH_SCHUR, e, st, 2.0 * (double)m * (double)(m - vbn) * (double)K, nl);
        }
    }
    if (tslu_on_side) CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
    return CFX_OK;
}

// The host loop of Alg. 1 shared by cfx_getrf (rm null: rows interchanged)
// and cfx_getrf_masked (rm: the row map, rows never moved).  Arguments are
// checked by the callers.
static int getrf_run(cfx_handle *h, int64_t n, double *A, int64_t lda, int32_t *ipiv, int32_t *rm,
                     int32_t *info, const cfx_lu_opts *opts, void *work, size_t work_bytes, hipStream_t st)
{
    int rc = launch_set_int(info, 0, st);
    if (rc || n == 0) return rc;

    const int v = opts->v, L = opts->leaves, ml = opts->min_leaf_rows;
    {
        int64_t h0 = (n + L - 1) / L;
        if (h0 < v) h0 = v;
        if (h0 > kMaxLeafRows) return CFX_ENOTSUP;
    }
    Workspace ws;
    if ((rc = carve_workspace(work, work_bytes, n, v, L, opts->precision, &ws, h->delay, opts->min_leaf_rows)))
        return rc;
    if (rm && (rc = launch_rowmap_init(rm, n, st))) return rc;
    if (h->delay > 1) {
        if (rm) return CFX_ENOTSUP;
        return getrf_run_delayed(h, n, A, lda, ipiv, info, opts, ws, st);
    }

    // Per panel k: the tournament's panel (W, row0 = k; with a row map W
    // points at row 0 of column k), the interchanges (or the row-map update),
    // and the blocks of the Schur update: L21 / C rows k+vb.., U12 rows
    // k..k+vb; with a row map the blocks point at row 0 of their columns and
    // their rows go through the map.
    auto panel_w = [&](int64_t k) -> double * { return rm ? A + k : A + k * lda + k; };
    // The row-move plan of panel k: panels alternate between two buffers,
    // so a panel's interchanges that are still being applied beside the
    // next panel's tournament never read the plan that tournament writes.
    auto wsk = [&](int64_t k) -> Workspace {
        Workspace w = ws;
        if ((k / v) & 1) w.plan = ws.plan_alt;
        return w;
    };
    auto swap = [&](int64_t k, int vb, hipStream_t s) -> int {
        return rm ? launch_rowmap_apply(A, lda, rm, k, vb, wsk(k), s) : launch_laswp(A, lda, n, k, vb, wsk(k), s);
    };
    struct Blocks {
        double *L21, *U12, *C;
        const int32_t *rmap, *umap;
    };
    auto blocks = [&](int64_t k, int vb) -> Blocks {
        if (rm) return {A + k, A + k + vb, A + k + vb, rm + k + vb, rm + k};
        double *panel = A + k * lda + k;
        return {panel + vb * lda, panel + vb, panel + vb * lda + vb, nullptr, nullptr};
    };
    auto schur = [&](const Blocks &b, int64_t m, int64_t col0, int64_t ncols, int vb, int max_wgs,
                     hipStream_t s) -> int {
        if (opts->precision == CFX_PREC_FP64)
            return launch_schur_f64(b.L21, lda, b.U12 + col0, lda, b.C + col0, lda, m, ncols, vb, max_wgs, s,
                                    b.rmap, b.umap);
        return launch_schur_lp(opts->precision, ws.scratch, m, m, vb, col0, ncols, b.C, lda, max_wgs, s, b.rmap);
    };
    auto pack = [&](const Blocks &b, int64_t m, int vb, hipStream_t s) -> int {
        if (opts->precision == CFX_PREC_FP64) return CFX_OK;
        return launch_pack_lp(opts->precision, b.L21, lda, m, b.U12, lda, m, vb, ws.scratch, s, b.rmap, b.umap);
    };

    Profiler &pf = h->prof;
    const int prec = opts->precision;
    if (!opts->lookahead) {
        for (int64_t k = 0; k < n; k += v) {
            const int vb = (int)((n - k) < v ? (n - k) : v);
            const int64_t m = n - k - vb;
            hipEvent_t e = pf.begin(st);
            if ((rc = launch_tslu(panel_w(k), lda, k, n - k, vb, panel_leaves(L, ml, n - k), wsk(k), nullptr, ipiv,
                                  info, st, rm,
                                  h->fuse_rows)))
                return rc;
            pf.end(PH_TSLU, e, st);
            e = pf.begin(st);
            if ((rc = swap(k, vb, st))) return rc;
            pf.end(PH_LASWP, e, st);
            if (m > 0) {
                e = pf.begin(st);
                if ((rc = launch_trsm(A, lda, k, vb, m, st, rm))) return rc;
                pf.end(PH_TRSM, e, st);
                const Blocks b = blocks(k, vb);
                e = pf.begin(st);
                if ((rc = pack(b, m, vb, st))) return rc;
                if ((rc = schur(b, m, 0, m, vb, 0, st))) return rc;
                pf.end(PH_SCHUR, e, st, 2.0 * (double)m * (double)m * vb);
            }
            if (pf.on) ++pf.panels;
        }
        return CFX_OK;
    }

    // Lookahead (depth 1): the Schur update of panel k is split into the
    // next panel's columns (A22[:, 0:vb']) and the rest.  The next panel's
    // tournament only reads those columns, so it runs on the side stream
    // while the main stream finishes the rest of the update; the next
    // interchanges wait for both.
    hipStream_t side = h->one_stream ? st : h->side;
    {
        const int vb0 = (int)(n < v ? n : v);
        hipEvent_t e = pf.begin(st);
        if ((rc = launch_tslu(panel_w(0), lda, 0, n, vb0, panel_leaves(L, ml, n), wsk(0), nullptr, ipiv, info, st, rm,
                              h->fuse_rows)))
            return rc;
        pf.end(PH_TSLU, e, st);
    }
    bool tslu_on_side = false, upd_pending = false;
    for (int64_t k = 0; k < n; k += v) {
        const int vb = (int)((n - k) < v ? (n - k) : v);
        const int64_t m = n - k - vb;
        if (tslu_on_side) CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
        if (upd_pending) CFX_HIP(hipStreamWaitEvent(st, h->ev_upd, 0));
        tslu_on_side = upd_pending = false;
        // While the next tournament bounds the step (U12 split between the
        // first solve and the rest of the update), only the columns of this
        // panel and the next one are interchanged ahead of it; the others go
        // with the rest of the update, before the rest of U12.
        const int vbn0 = (int)(m < v ? m : v);
        const bool split_swap = !rm && m > 0 && prec == CFX_PREC_FP64 && m < h->full_trsm_rows;
        hipEvent_t e = pf.begin(st);
        if (split_swap) rc = launch_laswp(A, lda, n, k, vb, wsk(k), st, k, k + vb + vbn0, true);
        else rc = swap(k, vb, st);
        if (rc) return rc;
        pf.end(PH_LASWP, e, st);
        if (m > 0) {
            const int vbn = vbn0;                          // next panel width
            // FP64: L21 and the next panel's columns of U12 first (one
            // launch), the rest of U12 with the rest of the update; the
            // low-precision pack needs all of U12 at once.  (The rest of U12
            // needs only the interchanges, but launched beside the first
            // solve it holds that solve back: neither grid fits the device
            // at once, and the first waits for the second to drain.)  While
            // the trailing matrix is large the update, not the next
            // tournament, bounds the step: then all of U12 is solved in the
            // first launch, which starts the update about one solve earlier
            // and the tournament a fraction of one later.
            const int64_t n1 = (prec == CFX_PREC_FP64 && m < h->full_trsm_rows) ? vbn : m;
            e = pf.begin(st);
            if ((rc = launch_trsm_first(A, lda, k, vb, m, n1, st, rm))) return rc;
            pf.end(PH_TRSM, e, st);
            const Blocks b = blocks(k, vb);
            e = pf.begin(st);
            if ((rc = pack(b, m, vb, st))) return rc;
            if ((rc = schur(b, m, 0, vbn, vb, 0, st))) return rc;
            pf.end(PH_SCHUR, e, st, 2.0 * (double)m * vbn * vb);
            // the rest of the update on the CU-masked stream when there is
            // one, then the next panel's tournament on the side stream.  The
            // rest is queued first: the tournament is a long run of small
            // launches, and a host that is held back by the depth of the
            // side stream's queue would otherwise reach the update only
            // after most of the tournament had been dispatched
            hipStream_t ts = side, us = (h->upd && !h->one_stream) ? h->upd : st;
            CFX_HIP(hipEventRecord(h->ev_panel, st));
            if (ts != st) CFX_HIP(hipStreamWaitEvent(ts, h->ev_panel, 0));
            if (us != st) CFX_HIP(hipStreamWaitEvent(us, h->ev_panel, 0));
            const int64_t kn = k + vb;
            auto tournament = [&]() -> int {
                hipEvent_t et = pf.begin(ts);
                const int r = launch_tslu(panel_w(kn), lda, kn, n - kn, vbn, panel_leaves(L, ml, n - kn), wsk(kn),
                                          nullptr, ipiv, info, ts, rm, h->fuse_rows);
                if (r) return r;
                pf.end(PH_TSLU, et, ts);
                CFX_HIP(hipEventRecord(h->ev_tslu, ts));
                tslu_on_side = true;
                return CFX_OK;
            };
            // on one stream the tournament goes first: it is the next
            // panel's critical path and the rest only has to end before the
            // next interchanges
            if (us == ts && (rc = tournament())) return rc;
            if (split_swap) {
                e = pf.begin(us);
                if ((rc = launch_laswp(A, lda, n, k, vb, wsk(k), us, k, k + vb + vbn, false))) return rc;
                pf.end(PH_LASWP, e, us);
            }
            if (n1 < m) {
                e = pf.begin(us);
                if ((rc = launch_trsm_rest(A, lda, k, vb, m, n1, us, rm))) return rc;
                pf.end(PH_TRSM, e, us);
            }
            // the rest of the update, in column chunks when the update shares
            // the device with the tournament without reserved compute units:
            // between two chunks the dispatcher can start the tournament's
            // launches instead of leaving them behind one huge grid (one
            // event pair around all chunks: events between the launches
            // would cost the step about 2 %)
            const int64_t chunk = h->la_chunk > 0 ? h->la_chunk : (us != st ? m : kLaChunk);
            const int wgs = h->schur_wgs >= 0 ? h->schur_wgs : (prec == CFX_PREC_FP64 ? 0 : cfx::kLpSchurWgs);
            if (vbn < m) {
                e = pf.begin(us);
                int nl = 0;
                for (int64_t c0 = vbn; c0 < m; c0 += chunk, ++nl) {
                    const int64_t cw = (m - c0) < chunk ? (m - c0) : chunk;
                    if ((rc = schur(b, m, c0, cw, vb, wgs, us))) return rc;
                }
                pf.end(PH_SCHUR, e, us, 2.0 * (double)m * (double)(m - vbn) * vb, nl);
            }
            if (us != st) {
                CFX_HIP(hipEventRecord(h->ev_upd, us));
                upd_pending = true;
            }
            if (us != ts && (rc = tournament())) return rc;
        }
        if (pf.on) ++pf.panels;
    }
    if (tslu_on_side) CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
    if (upd_pending) CFX_HIP(hipStreamWaitEvent(st, h->ev_upd, 0));
    return CFX_OK;
}

}  // namespace cfx

extern "C" {

int cfx_getrf(cfx_handle *h, int64_t n, double *A, int64_t lda, int32_t *ipiv, int32_t *info,
              const cfx_lu_opts *opts, void *work, size_t work_bytes, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (!A && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (!ipiv && n > 0) return -5;
    if (!info) return -6;
    if (int c = check_opts(opts)) return c == 2 ? CFX_ENOTSUP : -7;
    if (!work && n > 0) return -8;
    if (reinterpret_cast<uintptr_t>(work) & 255) return -8;
    return getrf_run(h, n, A, lda, ipiv, nullptr, info, opts, work, work_bytes, static_cast<hipStream_t>(stream));
}

int cfx_getrf_masked(cfx_handle *h, int64_t n, double *A, int64_t lda, int32_t *ipiv, int32_t *rowmap,
                     int32_t *info, const cfx_lu_opts *opts, void *work, size_t work_bytes, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (!A && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (!ipiv && n > 0) return -5;
    if (!rowmap && n > 0) return -6;
    if (!info) return -7;
    if (int c = check_opts(opts)) return c == 2 ? CFX_ENOTSUP : -8;
    if (!work && n > 0) return -9;
    if (reinterpret_cast<uintptr_t>(work) & 255) return -9;
    return getrf_run(h, n, A, lda, ipiv, rowmap, info, opts, work, work_bytes, static_cast<hipStream_t>(stream));
}

int cfx_gesv_ir_buffer_size(cfx_handle *h, int64_t n, int64_t nrhs, const cfx_ir_opts *opts, size_t *bytes)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (int c = check_ir_opts(opts)) return c == 2 ? CFX_ENOTSUP : -4;
    if (!bytes) return -5;
    *bytes = ir_layout(n, opts, h->delay).total;
    return CFX_OK;
}

int cfx_gesv_ir(cfx_handle *h, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                int64_t ldb, double *X, int64_t ldx, const cfx_ir_opts *opts, cfx_ir_report *rep, void *work,
                size_t work_bytes, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (nrhs < 0) return -3;
    if (!A && n > 0) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!B && n > 0 && nrhs > 0) return -6;
    if (ldb < (nrhs > 1 ? nrhs : 1)) return -7;
    if (!X && n > 0 && nrhs > 0) return -8;
    if (ldx < (nrhs > 1 ? nrhs : 1)) return -9;
    if (int c = check_ir_opts(opts)) return c == 2 ? CFX_ENOTSUP : -10;
    if (!rep) return -11;
    const IrLayout lay = ir_layout(n, opts, h->delay);
    if (n > 0 && (!work || (reinterpret_cast<uintptr_t>(work) & 255))) return -12;
    if (n > 0 && work_bytes < lay.total) return CFX_ENOMEM;
    cfx_ir_report r{};
    if (n == 0) {
        r.converged = 1;
        *rep = r;
        return CFX_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(work);
    double *F = reinterpret_cast<double *>(w + lay.off_F);
    int32_t *ipiv = reinterpret_cast<int32_t *>(w + lay.off_ipiv);
    int32_t *perm = reinterpret_cast<int32_t *>(w + lay.off_perm);
    int32_t *dinfo = reinterpret_cast<int32_t *>(w + lay.off_info);
    CFX_HIP(hipMemcpy2DAsync(F, (size_t)n * sizeof(double), A, (size_t)lda * sizeof(double),
                             (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, st));
    int rc = cfx_getrf(h, n, F, n, ipiv, dinfo, &opts->lu, w + lay.off_getrf, lay.getrf_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_perm(n, ipiv, perm, st))) return rc;
    CFX_HIP(hipMemcpyAsync(&r.info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CFX_HIP(hipStreamSynchronize(st));
    const IrVectors v = carve_ir(w + lay.off_vec, n, opts->gmres_restart);
    IrParams p{opts->tol, opts->max_outer, opts->gmres_tol};
    p.spin_limit = h->spin_limit;
    r.converged = 1;
    r.eta = 0.0;
    r.eta_first = 0.0;
    // a NaN backward error of any right-hand side makes the aggregate NaN
    auto worst = [](double acc, double e) { return (acc != acc || e != e) ? NAN : std::fmax(acc, e); };
    // the give-up flag of the solves (sticky; work may hold anything)
    if ((rc = launch_set_int(v.sync + 4, 0, st))) return rc;
    int status = CFX_OK;
    for (int64_t c = 0; c < nrhs; ++c) {
        if ((rc = launch_copy_rows(n, 1, B + c, ldb, v.b, 1, st))) return rc;
        if ((rc = launch_gather_rows(n, 1, v.b, 1, perm, v.x, 1, st))) return rc;
        if ((rc = launch_trsv(n, 1, F, n, v.x, 1, v.sync, v.ys, st, p.spin_limit))) return rc;
        IrResult res{};
        rc = ir_refine(A, lda, F, n, perm, v, p, &res, st);
        if (rc == CFX_ESOLVE) {         // X is NaN: report it, go on with the others
            status = CFX_ESOLVE;
            res.eta = NAN;
            res.converged = 0;
        } else if (rc) {
            return rc;
        }
        if ((rc = launch_copy_rows(n, 1, v.x, 1, X + c, ldx, st))) return rc;
        r.eta = worst(r.eta, res.eta);
        r.eta_first = worst(r.eta_first, res.eta_first);
        if (res.outer > r.outer) r.outer = res.outer;
        r.inner += res.inner;
        r.converged &= res.converged;
    }
    CFX_HIP(hipStreamSynchronize(st));
    *rep = r;
    return status;
}

int cfx_gesv_batched_buffer_size(cfx_handle *h, int32_t count, size_t *bytes)
{
    if (!h) return -1;
    if (count < 0) return -2;
    if (!bytes) return -3;
    *bytes = batched_work_bytes(count);
    return CFX_OK;
}

int cfx_gesv_batched(cfx_handle *h, int32_t count, const int32_t *n, const int32_t *nrhs, double *const *A,
                     const int64_t *lda, double *const *B, const int64_t *ldb, int32_t *const *ipiv,
                     int32_t *info, void *work, size_t work_bytes, int32_t flags, void *stream)
{
    if (!h) return -1;
    if (count < 0) return -2;
    if (count == 0) return CFX_OK;
    if (!n) return -3;
    if (!nrhs) return -4;
    if (!A) return -5;
    if (!lda) return -6;
    if (!B) return -7;
    if (!ldb) return -8;
    if (!ipiv) return -9;
    if (!info) return -10;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -11;
    if (work_bytes < batched_work_bytes(count)) return CFX_ENOMEM;
    if (flags & ~CFX_BATCHED_NO_GRAPH) return -13;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = h->cu_count;   // one resident workgroup per compute unit
    if (flags & CFX_BATCHED_NO_GRAPH)
        return launch_gesv_batched(count, n, nrhs, A, lda, B, ldb, ipiv, info, work, h->bvb, grid, st);
    const void *key[10] = {n, nrhs, A, lda, B, ldb, ipiv, info, work, nullptr};
    bool same = h->bexec && h->bkey.count == count && h->bkey.version == h->bvb_version;
    for (int i = 0; same && i < 10; ++i) same = h->bkey.p[i] == key[i];
    if (!same) {
        if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
        if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
        h->bexec = nullptr;
        h->bgraph = nullptr;
        CFX_HIP(hipStreamBeginCapture(h->side, hipStreamCaptureModeThreadLocal));
        int rc = launch_gesv_batched(count, n, nrhs, A, lda, B, ldb, ipiv, info, work, h->bvb, grid, h->side);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->side, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess || !g) return CFX_EHIP;
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return CFX_EHIP;
        }
        h->bgraph = g;
        h->bexec = x;
        h->bkey.count = count;
        h->bkey.version = h->bvb_version;
        for (int i = 0; i < 10; ++i) h->bkey.p[i] = key[i];
    }
    CFX_HIP(hipGraphLaunch(h->bexec, st));
    return CFX_OK;
}

int cfx_batched_tune(cfx_handle *h, void *stream)
{
    if (!h) return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int grid = h->cu_count;
    const int count = 4 * grid;
    const int reps[kBatchClasses] = {32, 64, 128, 256, 512};
    const int cands[3] = {8, 16, 32};
    const int nmax = reps[kBatchClasses - 1];
    double *A = nullptr, *B = nullptr;
    int32_t *ipiv = nullptr, *info = nullptr, *nv = nullptr, *rv = nullptr;
    int64_t *ldav = nullptr, *ldbv = nullptr;
    double **Ap = nullptr, **Bp = nullptr;
    int32_t **Ip = nullptr;
    void *work = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CFX_OK;
    std::vector<double *> hA(count), hB(count);
    std::vector<int32_t *> hI(count);
    std::vector<int32_t> hn(count), hr(count, 1);
    std::vector<int64_t> hlda(count), hldb(count, 1);
    int32_t table[kBatchClasses];
    for (int c = 0; c < kBatchClasses; ++c) table[c] = h->bvb[c];
    auto fail = [&](int code) { rc = code; };
    if (hipMalloc(&A, (size_t)count * nmax * nmax * sizeof(double)) != hipSuccess ||
        hipMalloc(&B, (size_t)count * nmax * sizeof(double)) != hipSuccess ||
        hipMalloc(&ipiv, (size_t)count * nmax * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&info, (size_t)count * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&nv, (size_t)count * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&rv, (size_t)count * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&ldav, (size_t)count * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&ldbv, (size_t)count * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&Ap, (size_t)count * sizeof(double *)) != hipSuccess ||
        hipMalloc(&Bp, (size_t)count * sizeof(double *)) != hipSuccess ||
        hipMalloc(&Ip, (size_t)count * sizeof(int32_t *)) != hipSuccess ||
        hipMalloc(&work, batched_work_bytes(count)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        fail(CFX_ENOMEM);
    for (int c = 0; c < kBatchClasses && rc == CFX_OK; ++c) {
        const int n = reps[c];
        for (int i = 0; i < count; ++i) {
            hA[i] = A + (size_t)i * n * n;
            hB[i] = B + (size_t)i * n;
            hI[i] = ipiv + (size_t)i * n;
            hn[i] = n;
            hlda[i] = n;
        }
        if (hipMemcpyAsync(Ap, hA.data(), count * sizeof(double *), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(Bp, hB.data(), count * sizeof(double *), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(Ip, hI.data(), count * sizeof(int32_t *), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(nv, hn.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(rv, hr.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(ldav, hlda.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(ldbv, hldb.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            fail(CFX_EHIP);
            break;
        }
        float best = 0.f;
        int bestv = table[c];
        for (int ci = 0; ci < 3 && rc == CFX_OK; ++ci) {
            table[c] = cands[ci];
            float tmin = 0.f;
            for (int rep = 0; rep < 2 && rc == CFX_OK; ++rep) {
                int r2 = launch_batched_synth(A, n, count, 1234 + rep, st);
                if (!r2) r2 = launch_batched_synth(B, 1, (int64_t)count * n, 99, st);
                if (!r2 && hipEventRecord(e0, st) != hipSuccess) r2 = CFX_EHIP;
                if (!r2) r2 = launch_gesv_batched(count, nv, rv, Ap, ldav, Bp, ldbv, Ip, info, work, table, grid, st);
                if (!r2 && hipEventRecord(e1, st) != hipSuccess) r2 = CFX_EHIP;
                float ms = 0.f;
                if (!r2 && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    r2 = CFX_EHIP;
                if (r2) fail(r2);
                else if (rep == 0 || ms < tmin) tmin = ms;
            }
            if (rc == CFX_OK && (ci == 0 || tmin < best)) {
                best = tmin;
                bestv = cands[ci];
            }
        }
        table[c] = bestv;
    }
    if (rc == CFX_OK) {
        for (int c = 0; c < kBatchClasses; ++c) h->bvb[c] = table[c];
        ++h->bvb_version;
    }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void *p : {(void *)A, (void *)B, (void *)ipiv, (void *)info, (void *)nv, (void *)rv, (void *)ldav,
                    (void *)ldbv, (void *)Ap, (void *)Bp, (void *)Ip, work})
        if (p) (void)hipFree(p);
    return rc;
}

int cfx_batched_tuning(cfx_handle *h, int32_t *vb)
{
    if (!h) return -1;
    if (!vb) return -2;
    for (int c = 0; c < kBatchClasses; ++c) vb[c] = h->bvb[c];
    return CFX_OK;
}

int cfx_overlap_tuning(cfx_handle *h, int32_t *schur_workgroups, int32_t *chunk_cols, int32_t *one_stream)
{
    if (!h) return -1;
    if (schur_workgroups) *schur_workgroups = h->schur_wgs;
    if (chunk_cols) *chunk_cols = (int32_t)h->la_chunk;
    if (one_stream) *one_stream = h->one_stream ? 1 : 0;
    return CFX_OK;
}

int cfx_set_overlap_tuning(cfx_handle *h, int32_t schur_workgroups, int32_t chunk_cols, int32_t one_stream)
{
    if (!h) return -1;
    if (schur_workgroups < -1 || (schur_workgroups > 0 && schur_workgroups < 8)) return -2;
    if (chunk_cols < 0) return -3;
    if (one_stream != 0 && one_stream != 1) return -4;
    h->schur_wgs = schur_workgroups;
    h->la_chunk = chunk_cols;
    h->one_stream = one_stream != 0;
    return CFX_OK;
}

int cfx_full_trsm_rows(cfx_handle *h, int32_t *rows)
{
    if (!h) return -1;
    if (!rows) return -2;
    *rows = (int32_t)h->full_trsm_rows;
    return CFX_OK;
}

int cfx_set_full_trsm_rows(cfx_handle *h, int32_t rows)
{
    if (!h) return -1;
    if (rows < 0) return -2;
    h->full_trsm_rows = rows;
    return CFX_OK;
}

int cfx_tournament_fusion(cfx_handle *h, int32_t *node_rows)
{
    if (!h) return -1;
    if (!node_rows) return -2;
    *node_rows = h->fuse_rows;
    return CFX_OK;
}

int cfx_set_tournament_fusion(cfx_handle *h, int32_t node_rows)
{
    if (!h) return -1;
    if (node_rows < 0 || node_rows > kFuseRows) return -2;
    h->fuse_rows = node_rows;
    return CFX_OK;
}

int cfx_schur_delay(cfx_handle *h, int32_t *delay)
{
    if (!h) return -1;
    if (!delay) return -2;
    *delay = h->delay;
    return CFX_OK;
}

int cfx_set_schur_delay(cfx_handle *h, int32_t delay)
{
    if (!h) return -1;
    if (delay < 1 || delay > 8) return -2;
    h->delay = delay;
    return CFX_OK;
}

int cfx_reserved_cus(cfx_handle *h, int32_t *cus)
{
    if (!h) return -1;
    if (!cus) return -2;
    *cus = h->upd ? h->reserve_cus : 0;
    return CFX_OK;
}

int cfx_set_reserved_cus(cfx_handle *h, int32_t cus)
{
    if (!h) return -1;
    if (cus < 0 || cus > h->cu_count / 4) return -2;
    if (h->upd) {
        // work queued on the old stream ends before it goes away
        CFX_HIP(hipStreamSynchronize(h->upd));
        CFX_HIP(hipStreamDestroy(h->upd));
        h->upd = nullptr;
    }
    h->reserve_cus = 0;
    if (cus == 0) return CFX_OK;
    // mask bits are logical compute units, consecutive bits spread over the
    // XCDs: clearing the lowest `cus` bits leaves about cus / 8 compute
    // units free on every XCD
    std::vector<uint32_t> mask((size_t)(h->cu_count + 31) / 32, 0u);
    for (int c = cus; c < h->cu_count; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
    CFX_HIP(hipExtStreamCreateWithCUMask(&h->upd, (uint32_t)mask.size(), mask.data()));
    h->reserve_cus = cus;
    return CFX_OK;
}

int cfx_batched_set_tuning(cfx_handle *h, const int32_t *vb)
{
    if (!h) return -1;
    if (!vb) return -2;
    for (int c = 0; c < kBatchClasses; ++c)
        if (vb[c] != 8 && vb[c] != 16 && vb[c] != 32) return -2;
    for (int c = 0; c < kBatchClasses; ++c) h->bvb[c] = vb[c];
    ++h->bvb_version;
    return CFX_OK;
}

int cfx_tslu(cfx_handle *h, int64_t rows, int64_t vb, const double *W, int64_t ldw, int64_t row0,
             int32_t leaves, int32_t *piv, void *work, size_t work_bytes, void *stream)
{
    if (!h) return -1;
    if (rows < 1 || rows > INT32_MAX) return -2;
    if (vb < 1 || vb > kMaxV || vb > rows) return -3;
    if (!W) return -4;
    if (ldw < vb) return -5;
    if (row0 < 0 || row0 + rows > INT32_MAX) return -6;
    if (leaves < 1) return -7;
    if (!piv) return -8;
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -9;
    Workspace ws;
    int rc = carve_workspace(work, work_bytes, rows, (int)vb, leaves, CFX_PREC_FP64, &ws);
    if (rc) return rc;
    return launch_tslu(W, ldw, row0, rows, (int)vb, leaves, ws, piv, nullptr, nullptr,
                       static_cast<hipStream_t>(stream), nullptr, h->fuse_rows);
}

int cfx_getrs(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
              const int32_t *ipiv, double *B, int64_t ldb, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (nrhs < 0) return -3;
    if (!LU && n > 0) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!ipiv && n > 0) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < (nrhs > 1 ? nrhs : 1)) return -8;
    if (n == 0 || nrhs == 0) return CFX_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t need = align_up((size_t)n * sizeof(int32_t)) + (size_t)n * (nrhs > 1 ? nrhs : 2) * sizeof(double);
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    // calls on one handle share its scratch and counters: each one waits for
    // the previous one, whatever streams they are issued on
    if (h->getrs_issued) CFX_HIP(hipStreamWaitEvent(st, h->ev_getrs, 0));
    int32_t *perm = static_cast<int32_t *>(h->scratch);
    double *tmp = reinterpret_cast<double *>(static_cast<char *>(h->scratch) +
                                             align_up((size_t)n * sizeof(int32_t)));
    rc = launch_getrs(n, nrhs, LU, lda, ipiv, B, ldb, perm, tmp, h->gsync, st, h->spin_limit);
    if (rc) return rc;
    CFX_HIP(hipEventRecord(h->ev_getrs, st));
    h->getrs_issued = true;
    return CFX_OK;
}

int cfx_schur_update_buffer_size(cfx_handle *h, int32_t precision, int64_t m, int64_t n, int64_t K,
                                 size_t *bytes)
{
    if (!h) return -1;
    if (precision < CFX_PREC_FP64 || precision > CFX_PREC_FP8) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (K < 0 || K > INT32_MAX / 2) return -5;
    if (!bytes) return -6;
    *bytes = precision == CFX_PREC_FP64 ? 0 : lp_pack_bytes(precision, m, n, (int)K);
    return CFX_OK;
}

int cfx_schur_update(cfx_handle *h, int32_t precision, int64_t m, int64_t n, int64_t K, const double *L21,
                     int64_t ldl, const double *U12, int64_t ldu, double *C, int64_t ldc, int32_t max_workgroups,
                     void *work, size_t work_bytes, void *stream)
{
    if (!h) return -1;
    if (precision < CFX_PREC_FP64 || precision > CFX_PREC_FP8) return -2;
    if (m < 0 || m > INT32_MAX) return -3;
    if (n < 0 || n > INT32_MAX) return -4;
    if (K < 0 || K > INT32_MAX / 2) return -5;
    const bool any = m > 0 && n > 0 && K > 0;
    if (any && !L21) return -6;
    if (ldl < (K > 1 ? K : 1)) return -7;
    if (any && !U12) return -8;
    if (ldu < (n > 1 ? n : 1)) return -9;
    if (m > 0 && n > 0 && !C) return -10;
    if (ldc < (n > 1 ? n : 1)) return -11;
    if (max_workgroups < 0 || (max_workgroups > 0 && max_workgroups < 8)) return -12;
    if (!any) return CFX_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == CFX_PREC_FP64)
        return launch_schur_f64(L21, ldl, U12, ldu, C, ldc, m, n, (int)K, max_workgroups, st);
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -13;
    if (work_bytes < lp_pack_bytes(precision, m, n, (int)K)) return CFX_ENOMEM;
    int rc = launch_pack_lp(precision, L21, ldl, m, U12, ldu, n, (int)K, work, st);
    if (rc) return rc;
    return launch_schur_lp(precision, work, m, n, (int)K, 0, n, C, ldc, max_workgroups, st);
}

int cfx_getrs_noalloc(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                      const int32_t *ipiv, double *B, int64_t ldb, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (nrhs < 0) return -3;
    if (!LU && n > 0) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!ipiv && n > 0) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < (nrhs > 1 ? nrhs : 1)) return -8;
    if (n == 0 || nrhs == 0) return CFX_OK;
    // counters | permutation | gathered right-hand sides, all in the
    // device's fixed scratch (no allocation on this path)
    const size_t off_perm = kTrsvSyncBytes;
    const size_t off_tmp = off_perm + align_up((size_t)n * sizeof(int32_t));
    const size_t cols = nrhs > 1 ? (size_t)nrhs : 2;   // one right-hand side: its solve's intermediate vector
    if (cols > (kNoAllocScratchBytes - off_tmp) / sizeof(double) / (size_t)n) return CFX_ENOTSUP;
    if (!h->na_scratch) return CFX_EHIP;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(h->na_scratch);
    int32_t *sync = reinterpret_cast<int32_t *>(base);
    // the give-up flag starts at zero for this call (the tickets and solved
    // counts are cleared by the solve itself); a fill kernel, not a memset
    int rc = launch_set_int(sync + 4, 0, st);
    if (rc) return rc;
    return launch_getrs(n, nrhs, LU, lda, ipiv, B, ldb, reinterpret_cast<int32_t *>(base + off_perm),
                        reinterpret_cast<double *>(base + off_tmp), sync, st, h->spin_limit);
}

int cfx_getrs_masked(cfx_handle *h, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                     const int32_t *rowmap, double *B, int64_t ldb, void *stream)
{
    if (!h) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (nrhs < 0) return -3;
    if (!LU && n > 0) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (!rowmap && n > 0) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < (nrhs > 1 ? nrhs : 1)) return -8;
    if (n == 0 || nrhs == 0) return CFX_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t need = (size_t)n * (nrhs > 1 ? nrhs : 2) * sizeof(double);
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    if (h->getrs_issued) CFX_HIP(hipStreamWaitEvent(st, h->ev_getrs, 0));
    rc = launch_getrs(n, nrhs, LU, lda, nullptr, B, ldb, nullptr, static_cast<double *>(h->scratch), h->gsync, st,
                      h->spin_limit, rowmap);
    if (rc) return rc;
    CFX_HIP(hipEventRecord(h->ev_getrs, st));
    h->getrs_issued = true;
    return CFX_OK;
}

int cfx_getrs_check(cfx_handle *h, void *stream)
{
    if (!h) return -1;
    bool gave_up = false, na_gave_up = false;
    int rc = read_solve_flag(h->gsync, static_cast<hipStream_t>(stream), &gave_up);
    if (rc) return rc;
    if (h->na_scratch &&
        (rc = read_solve_flag(static_cast<int32_t *>(h->na_scratch), static_cast<hipStream_t>(stream),
                              &na_gave_up)))
        return rc;
    return (gave_up || na_gave_up) ? CFX_ESOLVE : CFX_OK;
}

int cfx_set_solve_spin_limit(cfx_handle *h, int32_t polls)
{
    if (!h) return -1;
    if (polls < 0) return -2;
    h->spin_limit = polls;
    return CFX_OK;
}

}  // extern "C"

// C ABI entry points (include/cfx.h): argument checks, workspace carving and
// the host loop over panels of Alg. 1 (TournPivot, interchanges,
// FactorizeA10/A01, FactorizeA11 per panel).
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
    struct Rec { int phase; hipEvent_t a, b; double flops; };
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
    void end(int phase, hipEvent_t a, hipStream_t st, double flops = 0.0)
    {
        if (!on || !a) return;
        hipEvent_t e = next();
        if (!e) return;
        (void)hipEventRecord(e, st);
        recs.push_back({phase, a, e, flops});
    }
};
}  // namespace cfx

struct cfx_handle {
    int device = 0;
    hipStream_t side = nullptr;     // lookahead stream (default priority)
    hipEvent_t ev_panel = nullptr;  // next panel's columns updated
    hipEvent_t ev_tslu = nullptr;   // next panel's tournament done
    void *scratch = nullptr;        // getrs permutation + gather buffer
    size_t scratch_bytes = 0;
    cfx::Profiler prof;
};

namespace cfx {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    int64_t max_nodes, node_rows;
    size_t off_S, off_cand0, off_cand1, off_cnt0, off_cnt1, off_plan, off_lu00, off_selg, off_rsel,
        off_utg, off_rtg, off_mp, total;
};

static Layout layout(int64_t n, int v, int leaves, int precision)
{
    Layout L{};
    int64_t h0 = (n + leaves - 1) / leaves;
    if (h0 < v) h0 = v;
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
    L.off_lu00 = o;  o = align_up(o + (size_t)v * v * sizeof(double));
    L.off_selg = o;  o = align_up(o + (size_t)L.max_nodes * 2 * kMaxV * sizeof(int32_t));
    L.off_rsel = o;  o = align_up(o + (size_t)L.max_nodes * L.node_rows);
    L.off_utg = o;   o = align_up(o + (size_t)L.max_nodes * 32 * kMaxV * sizeof(double));
    L.off_rtg = o;   o = align_up(o + (size_t)L.max_nodes * 32 * 40 * sizeof(double));
    L.off_mp = o;
    (void)precision;
    L.total = o;
    return L;
}

size_t workspace_bytes(int64_t n, int v, int leaves, int precision)
{
    return layout(n, v, leaves, precision).total;
}

int carve_workspace(void *work, size_t bytes, int64_t n, int v, int leaves, int precision,
                    Workspace *ws)
{
    Layout L = layout(n, v, leaves, precision);
    if (bytes < L.total) return CFX_ENOMEM;
    char *b = static_cast<char *>(work);
    ws->S = reinterpret_cast<double *>(b + L.off_S);
    ws->s_node = L.node_rows * v;
    ws->cand[0] = reinterpret_cast<int32_t *>(b + L.off_cand0);
    ws->cand[1] = reinterpret_cast<int32_t *>(b + L.off_cand1);
    ws->ccnt[0] = reinterpret_cast<int32_t *>(b + L.off_cnt0);
    ws->ccnt[1] = reinterpret_cast<int32_t *>(b + L.off_cnt1);
    ws->plan = reinterpret_cast<int32_t *>(b + L.off_plan);
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
    if (o->precision != CFX_PREC_FP64) return 2;   // mixed precision: not in this build yet
    if (o->lookahead < 0 || o->lookahead > 1) return 1;
    return 0;
}

static int ensure_scratch(cfx_handle *h, size_t bytes)
{
    if (h->scratch_bytes >= bytes) return CFX_OK;
    if (h->scratch) CFX_HIP(hipFree(h->scratch));
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    CFX_HIP(hipMalloc(&h->scratch, bytes));
    h->scratch_bytes = bytes;
    return CFX_OK;
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
        hipEventCreateWithFlags(&p->ev_tslu, hipEventDisableTiming) != hipSuccess) {
        delete p;
        return CFX_EHIP;
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
            ++r.schur_launches;
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
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->ev_tslu) (void)hipEventDestroy(h->ev_tslu);
    if (h->side) (void)hipStreamDestroy(h->side);
    delete h;
    return CFX_OK;
}

int cfx_getrf_buffer_size(cfx_handle *h, int64_t n, const cfx_lu_opts *opts, size_t *bytes)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (check_opts(opts)) return check_opts(opts) == 2 ? CFX_ENOTSUP : -3;
    if (!bytes) return -4;
    *bytes = workspace_bytes(n, opts->v, opts->leaves, opts->precision);
    return CFX_OK;
}

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
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = launch_set_int(info, 0, st);
    if (rc || n == 0) return rc;

    const int v = opts->v, L = opts->leaves;
    {
        int64_t h0 = (n + L - 1) / L;
        if (h0 < v) h0 = v;
        if (h0 > kMaxLeafRows) return CFX_ENOTSUP;
    }
    Workspace ws;
    if ((rc = carve_workspace(work, work_bytes, n, v, L, opts->precision, &ws))) return rc;

    Profiler &pf = h->prof;
    if (!opts->lookahead) {
        for (int64_t k = 0; k < n; k += v) {
            const int vb = (int)((n - k) < v ? (n - k) : v);
            const int64_t m = n - k - vb;
            double *panel = A + k * lda + k;
            hipEvent_t e = pf.begin(st);
            if ((rc = launch_tslu(panel, lda, k, n - k, vb, L, ws, nullptr, ipiv, info, st))) return rc;
            pf.end(PH_TSLU, e, st);
            e = pf.begin(st);
            if ((rc = launch_laswp(A, lda, n, k, vb, ws, st))) return rc;
            pf.end(PH_LASWP, e, st);
            if (m > 0) {
                e = pf.begin(st);
                if ((rc = launch_trsm(A, lda, k, vb, m, st))) return rc;
                pf.end(PH_TRSM, e, st);
                e = pf.begin(st);
                if ((rc = launch_schur_f64(panel + vb * lda, lda, panel + vb, lda, panel + vb * lda + vb,
                                           lda, m, m, vb, st)))
                    return rc;
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
    hipStream_t side = h->side;
    {
        const int vb0 = (int)(n < v ? n : v);
        hipEvent_t e = pf.begin(st);
        if ((rc = launch_tslu(A, lda, 0, n, vb0, L, ws, nullptr, ipiv, info, st))) return rc;
        pf.end(PH_TSLU, e, st);
    }
    bool tslu_on_side = false;
    for (int64_t k = 0; k < n; k += v) {
        const int vb = (int)((n - k) < v ? (n - k) : v);
        const int64_t m = n - k - vb;
        double *panel = A + k * lda + k;
        if (tslu_on_side) CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
        tslu_on_side = false;
        hipEvent_t e = pf.begin(st);
        if ((rc = launch_laswp(A, lda, n, k, vb, ws, st))) return rc;
        pf.end(PH_LASWP, e, st);
        if (m > 0) {
            e = pf.begin(st);
            if ((rc = launch_trsm(A, lda, k, vb, m, st))) return rc;
            pf.end(PH_TRSM, e, st);
            const int vbn = (int)(m < v ? m : v);          // next panel width
            double *L21 = panel + vb * lda, *U12 = panel + vb, *C = panel + vb * lda + vb;
            e = pf.begin(st);
            if ((rc = launch_schur_f64(L21, lda, U12, lda, C, lda, m, vbn, vb, st))) return rc;
            pf.end(PH_SCHUR, e, st, 2.0 * (double)m * vbn * vb);
            // next panel's tournament on the side stream
            CFX_HIP(hipEventRecord(h->ev_panel, st));
            CFX_HIP(hipStreamWaitEvent(side, h->ev_panel, 0));
            const int64_t kn = k + vb;
            e = pf.begin(side);
            if ((rc = launch_tslu(A + kn * lda + kn, lda, kn, n - kn, vbn, L, ws, nullptr, ipiv, info, side)))
                return rc;
            pf.end(PH_TSLU, e, side);
            CFX_HIP(hipEventRecord(h->ev_tslu, side));
            tslu_on_side = true;
            // the rest of the update
            if (m > vbn) {
                e = pf.begin(st);
                if ((rc = launch_schur_f64(L21, lda, U12 + vbn, lda, C + vbn, lda, m, m - vbn, vb, st)))
                    return rc;
                pf.end(PH_SCHUR, e, st, 2.0 * (double)m * (double)(m - vbn) * vb);
            }
        }
        if (pf.on) ++pf.panels;
    }
    if (tslu_on_side) CFX_HIP(hipStreamWaitEvent(st, h->ev_tslu, 0));
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
                       static_cast<hipStream_t>(stream));
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
    const size_t need = align_up((size_t)n * sizeof(int32_t)) + (size_t)n * nrhs * sizeof(double);
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    int32_t *perm = static_cast<int32_t *>(h->scratch);
    double *tmp = reinterpret_cast<double *>(static_cast<char *>(h->scratch) +
                                             align_up((size_t)n * sizeof(int32_t)));
    return launch_getrs(n, nrhs, LU, lda, ipiv, B, ldb, perm, tmp, static_cast<hipStream_t>(stream));
}

}  // extern "C"
